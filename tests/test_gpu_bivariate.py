"""The bivariate circuit on the device (bc_compare_bivariate): full-range
base-p digits, byte-identical to the oracle's evaluation of the same
schedule on the same seeded inputs (N = 2^12), and exact on uint16 as two
base-257 digits at the workload's N = 2^15 chain (decryptions of LT, max and
min, edge cases included)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params

pytestmark = pytest.mark.gpu

P = 257


def setup(prm, seed):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], ()), rnd


def uint16_pairs(seed, G, M):
    xs = synth.integers(seed, (G, M), 0, 65536)
    ys = synth.integers(seed, (G, M), 0, 65536, index=1)
    # edge cases: equal values, extremes, equal top digits, digit 256
    xs[0, :8] = [0, 65535, 65535, 256, 257, 300, 12345, 65279]
    ys[0, :8] = [65535, 0, 65535, 257, 256, 300, 12346, 65280]
    return xs, ys


def encrypt_planes(dev, dk, vals, nd, seed):
    out = []
    for d, pl in enumerate(oracle.to_digits(vals, P, nd)):
        r = synth.encrypt_randomness(seed + d, pl.shape[0], dev.N)
        out.append(dev.encrypt(dk, pl, r["u"], r["e"]))
    return out


def test_bivariate_matches_oracle_n4096():
    import paper_2407_07308_amd as bc

    prm = Params(12, P, 13, 50, 4, 50, 4)
    print("bivariate: N=2^12 oracle parity", flush=True)
    dev, dk, rnd = setup(prm, 71)
    G, nd = 2, 2
    xs, ys = uint16_pairs(72, G, dev.M)
    A = encrypt_planes(dev, dk, xs, nd, 80)
    B = encrypt_planes(dev, dk, ys, nd, 90)
    lt, mx, mn = dev.compare_max_min(dk, A, B, circuit=bc.BC_CIRCUIT_BIVARIATE)
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    dec = lambda planes: sum(dev.decrypt(dk, p).astype(np.int64) * P ** (nd - 1 - d) for d, p in enumerate(planes))
    assert np.array_equal(dec(mx), np.maximum(xs, ys))
    assert np.array_equal(dec(mn), np.minimum(xs, ys))
    # the oracle on group 0 (same keys, same encryption randomness)
    orc = Oracle(prm)
    orc.keygen(rnd)
    xd, yd = oracle.to_digits(xs, P, nd), oracle.to_digits(ys, P, nd)
    oa, ob = [], []
    for d in range(nd):
        ra = synth.encrypt_randomness(80 + d, G, prm.N)
        rb = synth.encrypt_randomness(90 + d, G, prm.N)
        oa.append(orc.encrypt(xd[d][0], ra["u"][0], ra["e"][0]))
        ob.append(orc.encrypt(yd[d][0], rb["u"][0], rb["e"][0]))
    ev = CtEvaluator(orc)
    o_lt = oracle.compare_lt_bivariate(ev, oa, ob, P)
    assert ev.mults == nd * 518 + nd - 1
    o_mx, o_mn = oracle.max_min(ev, oa, ob, o_lt)
    assert lt.level == o_lt.level and mx[0].level == o_mx[0].level
    assert np.array_equal(dev.export(lt)[0], o_lt.data)
    for d in range(nd):
        assert np.array_equal(dev.export(mx[d])[0], o_mx[d].data), f"max plane {d}"
        assert np.array_equal(dev.export(mn[d])[0], o_mn[d].data), f"min plane {d}"


def test_bivariate_uint16_two_digits_full_size():
    import paper_2407_07308_amd as bc

    prm = Params(15, P, 14, 50, 5, 50, 3)
    print("bivariate: N=2^15, 2 base-257 digits", flush=True)
    dev, dk, _ = setup(prm, 73)
    G, nd = 2, 2
    xs, ys = uint16_pairs(74, G, dev.M)
    A = encrypt_planes(dev, dk, xs, nd, 100)
    B = encrypt_planes(dev, dk, ys, nd, 110)
    lt, mx, mn = dev.compare_max_min(dk, A, B, circuit=bc.BC_CIRCUIT_BIVARIATE)
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    dec = lambda planes: sum(dev.decrypt(dk, p).astype(np.int64) * P ** (nd - 1 - d) for d, p in enumerate(planes))
    assert np.array_equal(dec(mx), np.maximum(xs, ys))
    assert np.array_equal(dec(mn), np.minimum(xs, ys))
    ltl, mml = dev.compare_levels(prm.nQ - 1, nd, bc.BC_CIRCUIT_BIVARIATE)
    assert (lt.level, mx[0].level) == (ltl, mml) == (prm.nQ - 1 - 10, prm.nQ - 1 - 11)
    # the same call again gives the same bytes (the workspace pool reuses blocks)
    lt2 = dev.compare_max_min(dk, A, B, True, False, False, circuit=bc.BC_CIRCUIT_BIVARIATE)[0]
    assert np.array_equal(dev.export(lt2), dev.export(lt))


@pytest.mark.parametrize("p,prm", [(257, Params(12, 257, 13, 50, 4, 50, 4)), (17, Params(12, 17, 9, 36, 2, 36, 3))])
def test_matrix_core_combination_equals_vector_units(p, prm):
    """The g_k(S) combinations on the matrix cores (split-int8 products) and
    in fp64 on the vector units give the same ciphertext bytes."""
    import paper_2407_07308_amd as bc

    print(f"bivariate: matrix cores vs vector units, p={p}", flush=True)
    dev, dk, _ = setup(prm, 75)
    G = 3
    x = synth.slot_values(76, G, dev.M, 0, p)
    y = synth.slot_values(77, G, dev.M, 0, p)
    x[0, :4], y[0, :4] = [0, p - 1, 5, p - 1], [p - 1, 0, 5, p - 1]
    rx, ry = synth.encrypt_randomness(78, G, dev.N), synth.encrypt_randomness(79, G, dev.N)
    A, B = [dev.encrypt(dk, x, rx["u"], rx["e"])], [dev.encrypt(dk, y, ry["u"], ry["e"])]
    out = {}
    for mfma in (1, 0):
        dev.set_tuning(bc.BC_TUNE_MFMA, mfma)
        out[mfma] = dev.compare_max_min(dk, A, B, True, False, False, circuit=bc.BC_CIRCUIT_BIVARIATE)[0]
    assert np.array_equal(dev.export(out[1]), dev.export(out[0]))
    assert np.array_equal(dev.decrypt(dk, out[1]), (x < y).astype(np.uint32))
