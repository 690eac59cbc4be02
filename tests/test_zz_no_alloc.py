"""The allocation-free multiplication (bc_mul_relin_noalloc) against
bc_mul_relin: same bytes on two calls in a row, the second with a smaller
input, at the workload's N = 2^15 chain; nothing is taken from the workspace
pool; calls beyond the fixed scratch are refused before any launch."""
import numpy as np
import pytest

import synth
from oracle import Params

pytestmark = pytest.mark.gpu

PRM = Params(15, 257, 14, 50, 5, 50, 3)


def first(dev, b, n):
    """The first n ciphertexts of a batch (a view)."""
    import paper_2407_07308_amd as bc

    return bc.Batch(b.tensor[: dev.ct_words(b.level, b.ncomp) * n], n, b.level, b.ncomp, b.noise)


def test_noalloc_matches_the_pooled_multiplication():
    import torch

    import paper_2407_07308_amd as bc

    print("no-alloc: N=2^15, 14x50 + 5x50, dnum 3", flush=True)
    dev = bc.Context.from_params(PRM)
    rnd = synth.keygen_randomness(61, PRM.N, PRM.nQ, PRM.nP, PRM.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    vals = synth.slot_values(62, 2, dev.M, 0, PRM.p)
    r = synth.encrypt_randomness(63, 2, PRM.N)
    x = dev.encrypt(dk, vals, r["u"], r["e"])
    x1 = first(dev, x, 1)
    want = (vals.astype(np.int64) ** 2) % PRM.p
    # first call: one ciphertext at the top level (44.25 MiB of workspace)
    ref = dev.mul_relin(dk, x1, x1)
    torch.cuda.synchronize()
    held = dev.pool_bytes()
    got = dev.mul_relin_noalloc(dk, x1, x1)
    assert got.level == ref.level and got.noise == pytest.approx(ref.noise)
    assert np.array_equal(dev.export(got), dev.export(ref))
    # second call, smaller input: a product two levels down (the scratch
    # still holds the first call's words)
    y = first(dev, dev.mul_relin(dk, ref, ref), 1)
    ref2 = dev.mul_relin(dk, y, y)
    torch.cuda.synchronize()
    held = dev.pool_bytes()
    got2 = dev.mul_relin_noalloc(dk, y, y)
    torch.cuda.synchronize()
    assert dev.pool_bytes() == held  # no workspace block was taken or added
    assert got2.level == ref2.level == PRM.nQ - 4
    assert np.array_equal(dev.export(got2), dev.export(ref2))
    x8 = (want[:1] ** 2 % PRM.p) ** 2 % PRM.p  # ref2 = ((x^2)^2)^2
    assert np.array_equal(dev.decrypt(dk, got2), x8)
    assert np.array_equal(dev.decrypt(dk, got), want[:1])
    # two ciphertexts at the top need 88.5 MiB: refused, nothing launched
    with pytest.raises(bc.BoostcomError) as ei:
        dev.mul_relin_noalloc(dk, x, x)
    assert ei.value.code == bc.BC_ERR_ARG and "scratch" in str(ei.value)
    # the pooled path still works after the refusal, and so does the scratch
    assert np.array_equal(dev.export(dev.mul_relin_noalloc(dk, x1, x1)), dev.export(ref))


def test_noalloc_at_level_zero_and_small_ring():
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)
    print("no-alloc: N=2^10, level 0 (key switch without a modulus switch)", flush=True)
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(64, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    vals = synth.slot_values(65, 3, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(66, 3, prm.N)
    x = dev.encrypt(dk, vals, r["u"], r["e"])
    while x.level > 0:
        x = dev.mod_switch(x)
    for cnt in (3, 1):  # a smaller second call
        xs = first(dev, x, cnt)
        ref = dev.mul_relin(dk, xs, xs)
        got = dev.mul_relin_noalloc(dk, xs, xs)
        assert got.level == 0
        assert np.array_equal(dev.export(got), dev.export(ref))
        assert np.array_equal(dev.decrypt(dk, got), (vals[:cnt].astype(np.int64) ** 2) % prm.p)
