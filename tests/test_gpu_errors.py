"""Every BC_ERR_* code provoked through the C ABI, and the noise budget.

Each failing call must return its code, leave a message, launch nothing and
leave the context usable: a correct call right after it still matches the
oracle-pinned results (decryptions checked).  The allocation failure is
forced from the host with the pool's test hook; no case makes the GPU fault.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import Params

pytestmark = pytest.mark.gpu


def make(prm, seed=3, rot=()):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(rot))
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], rot)


def enc(dev, dk, count, seed, hi=None):
    vals = synth.slot_values(seed, count, dev.M, 0, hi or dev.p)
    r = synth.encrypt_randomness(seed + 1, count, dev.N)
    return vals, dev.encrypt(dk, vals, r["u"], r["e"])


def expect(code, fn, *args):
    import paper_2407_07308_amd as bc

    with pytest.raises(bc.BoostcomError) as ei:
        fn(*args)
    assert ei.value.code == code, (ei.value.code, str(ei.value))
    assert str(ei.value)
    return ei.value


PRM = Params(10, 257, 8, 50, 4, 50, 2)


def test_level_errors_and_noise_budget():
    import paper_2407_07308_amd as bc

    dev, dk = make(PRM)
    vals, x = enc(dev, dk, 2, 10)
    x0 = x
    while x0.level > 0:
        x0 = dev.mod_switch(x0)
    # modulus switch at level 0
    expect(bc.BC_ERR_LEVEL, dev.mod_switch, x0)
    # one multiplication at level 0 fits the budget, a second does not
    m = dev.mul_relin(dk, x0, x0)
    assert m.level == 0 and m.noise > x0.noise
    assert np.array_equal(dev.decrypt(dk, m), vals.astype(np.int64) ** 2 % dev.p)
    err = expect(bc.BC_ERR_LEVEL, dev.mul_relin, dk, m, m)
    assert "noise" in str(err)
    # a comparison circuit deeper than what is left of the chain
    _, y = enc(dev, dk, 2, 12)
    x3, y3 = dev.mod_switch(dev.mod_switch(x)), dev.mod_switch(dev.mod_switch(y))
    expect(bc.BC_ERR_LEVEL, dev.compare_lt, dk, [x3], [y3])
    expect(bc.BC_ERR_LEVEL, dev.compare_levels, 3, 1)
    # the context still works
    xs, a = enc(dev, dk, 2, 14, 129)
    ys, b = enc(dev, dk, 2, 16, 129)
    assert np.array_equal(dev.decrypt(dk, dev.compare_lt(dk, [a], [b])), (xs < ys).astype(np.uint32))


def test_noise_estimates_travel_with_the_batches():
    import paper_2407_07308_amd as bc

    dev, dk = make(PRM)
    _, x = enc(dev, dk, 1, 20)
    prm = bc.bc_params(PRM.logN, PRM.p, PRM.nQ, PRM.bitsQ, PRM.nP, PRM.bitsP, PRM.dnum)
    out = ctypes.c_double()
    assert dev.L.bc_noise_estimate(ctypes.byref(prm), bc.BC_NOISE_FRESH, PRM.nQ - 1, 0.0, 0.0, ctypes.byref(out)) == 0
    assert x.noise == pytest.approx(out.value, abs=1e-3)
    m = dev.mul_relin(dk, x, x)
    assert dev.L.bc_noise_estimate(ctypes.byref(prm), bc.BC_NOISE_MUL, PRM.nQ - 1, x.noise, x.noise,
                                   ctypes.byref(out)) == 0
    assert m.noise == pytest.approx(out.value, abs=1e-3)
    lt = dev.compare_lt(dk, [x], [x])
    want_lt = ctypes.c_double()
    assert dev.L.bc_noise_compare(ctypes.byref(prm), PRM.nQ - 1, x.noise, 1, ctypes.byref(want_lt), None) == 0
    assert lt.noise == pytest.approx(want_lt.value, abs=1e-3)


def test_key_shape_context_and_null_errors():
    import paper_2407_07308_amd as bc

    dev, dk = make(PRM, rot=(1,))
    other, ok = make(PRM, seed=4)
    _, x = enc(dev, dk, 2, 30)
    L = dev.L
    # no rotation key for step 2
    expect(bc.BC_ERR_KEY, dev.rotate, dk, x, 2)
    # keys of another context
    expect(bc.BC_ERR_PARAM, dev.mul_relin, ok, x, x)
    expect(bc.BC_ERR_PARAM, dev.compare_lt, ok, [x], [x])
    # mismatched shapes: count not dividing, output of the wrong level
    _, y3 = enc(dev, dk, 3, 32)
    expect(bc.BC_ERR_ARG, dev.add, x, y3)
    wrong = dev.new_batch(2, x.level, 2)  # a product lands one level lower
    ca, cw = x.ctb(), wrong.ctb()
    rc = L.bc_mul_relin(dev.handle, dk.handle, ctypes.byref(ca), ctypes.byref(ca), ctypes.byref(cw), None)
    assert rc == bc.BC_ERR_ARG and L.bc_last_error()
    # planes of different levels in one comparison (the C call itself: the
    # binding would size the output from the first plane's level)
    x1 = dev.mod_switch(x)
    lt = dev.new_batch(2, 0, 2)
    pa, pb, co = bc._ctb_array([x, x1]), bc._ctb_array([x, x]), lt.ctb()
    assert L.bc_compare_lt(dev.handle, dk.handle, 2, pa, pb, ctypes.byref(co), None) == bc.BC_ERR_ARG
    assert b"level" in L.bc_last_error()
    # null pointers
    assert L.bc_mul_relin(dev.handle, dk.handle, None, ctypes.byref(ca), ctypes.byref(cw), None) == bc.BC_ERR_ARG
    assert L.bc_mul_relin(None, dk.handle, ctypes.byref(ca), ctypes.byref(ca), ctypes.byref(cw), None) == bc.BC_ERR_ARG
    assert L.bc_rotate(dev.handle, None, ctypes.byref(ca), 1, ctypes.byref(cw), None) == bc.BC_ERR_ARG
    null_data = bc.bc_ctb(None, 2, x.level, 2, 0.0)
    assert L.bc_add(dev.handle, ctypes.byref(null_data), ctypes.byref(ca), ctypes.byref(cw), None) == bc.BC_ERR_ARG
    assert L.bc_decrypt(dev.handle, dk.handle, ctypes.byref(ca), None, None) == bc.BC_ERR_ARG
    # bad parameter sets are refused before any device work
    h = ctypes.c_void_p()
    for bad in [(9, 257, 8, 50, 4, 50, 2), (10, 256, 8, 50, 4, 50, 2), (10, 257, 8, 50, 4, 50, 9),
                (10, 257, 30, 50, 20, 50, 2), (10, 257, 8, 70, 4, 50, 2)]:
        assert L.bc_ctx_create(ctypes.byref(bc.bc_params(*bad)), ctypes.byref(h)) == bc.BC_ERR_PARAM, bad
    # nothing above broke the context
    vals, z = enc(dev, dk, 2, 34)
    assert np.array_equal(dev.decrypt(dk, dev.rotate(dk, z, 1)),
                          np.concatenate([np.roll(vals[:, :64], -1, 1), np.roll(vals[:, 64:], -1, 1)], 1))


def test_forced_allocation_failure_is_reported_and_recovers():
    import paper_2407_07308_amd as bc

    dev, dk = make(PRM)
    vals, x = enc(dev, dk, 2, 40)
    ref = dev.export(dev.mul_relin(dk, x, x))
    import torch

    torch.cuda.synchronize()
    dev.trim()  # no cached block: the next workspace request allocates
    dev.set_tuning(bc.BC_TUNE_TEST_FAIL_ALLOC, 1)
    e = expect(bc.BC_ERR_OOM, dev.mul_relin, dk, x, x)
    assert "allocation" in str(e)
    assert dev.get_tuning(bc.BC_TUNE_TEST_FAIL_ALLOC) == 0  # the hook switched itself off
    torch.cuda.synchronize()
    assert np.array_equal(dev.export(dev.mul_relin(dk, x, x)), ref)
    assert np.array_equal(dev.decrypt(dk, dev.mul_relin(dk, x, x)), vals.astype(np.int64) ** 2 % dev.p)
