"""Modulus raising on the matrix cores (BC_TUNE_MFMA_MODUP): the split-int8
contraction with the folded forward stages gives the same bytes as the fp64
kernel and as the oracle.

At N = 2^12 with four primes per digit (alpha 4, no folded stage) products
against the oracle; at the workload's N = 2^15 chain (alpha 5, two folded
stages, the reduced fp64 hand-off on and off) products at the top level and
after a modulus switch, and a whole comparison, against the fp64 kernel;
the tuning errors."""
import numpy as np
import pytest

import synth
from oracle import Oracle, Params

pytestmark = pytest.mark.gpu


def ctx_and_keys(prm, seed):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], ()), rnd


def test_products_match_oracle_alpha4():
    import paper_2407_07308_amd as bc

    prm = Params(12, 257, 13, 50, 4, 50, 4)
    print("modup mfma: N=2^12 alpha 4 oracle parity", flush=True)
    dev, dk, rnd = ctx_and_keys(prm, 21)
    count = 2
    a = synth.slot_values(22, count, dev.M, 0, prm.p)
    b = synth.slot_values(23, count, dev.M, 0, prm.p)
    ra, rb = synth.encrypt_randomness(24, count, prm.N), synth.encrypt_randomness(25, count, prm.N)
    ca, cb = dev.encrypt(dk, a, ra["u"], ra["e"]), dev.encrypt(dk, b, rb["u"], rb["e"])
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 1)
    assert dev.get_tuning(bc.BC_TUNE_MFMA_MODUP) == 1
    p1 = dev.mul_relin(dk, ca, cb)
    p2 = dev.mul_relin(dk, p1, p1)
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
    q1 = dev.mul_relin(dk, ca, cb)
    q2 = dev.mul_relin(dk, q1, q1)
    assert np.array_equal(dev.export(p1), dev.export(q1))
    assert np.array_equal(dev.export(p2), dev.export(q2))
    want = (a.astype(np.int64) * b % prm.p) ** 2 % prm.p
    assert np.array_equal(dev.decrypt(dk, p2), want.astype(np.uint32))
    orc = Oracle(prm)
    orc.keygen(rnd)
    oa = orc.encrypt(a[1], ra["u"][1], ra["e"][1])
    ob = orc.encrypt(b[1], rb["u"][1], rb["e"][1])
    o1 = orc.mul(oa, ob)
    assert np.array_equal(dev.export(p1)[1], o1.data)
    assert np.array_equal(dev.export(p2)[1], orc.mul(o1, o1).data)


@pytest.mark.parametrize("raw", [1, 0])
def test_workload_chain_matches_fp64_kernel(raw):
    import paper_2407_07308_amd as bc

    prm = Params(15, 257, 14, 50, 5, 50, 3)
    print(f"modup mfma: N=2^15 alpha 5, fp64 hand-off {raw}", flush=True)
    dev, dk, _ = ctx_and_keys(prm, 26)
    assert dev.get_tuning(bc.BC_TUNE_NTT_PARTS) == 2
    dev.set_tuning(bc.BC_TUNE_RAW_HANDOFF, raw)
    count = 3
    a = synth.slot_values(27, count, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(28, count, prm.N)
    ca = dev.encrypt(dk, a, r["u"], r["e"])
    low = dev.mod_switch(dev.mod_switch(ca))

    def run():
        p1 = dev.mul_relin(dk, ca, ca)
        p2 = dev.mul_relin(dk, low, p1)
        return dev.export(p1), dev.export(p2)

    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 1)
    m1, m2 = run()
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
    f1, f2 = run()
    assert np.array_equal(m1, f1)
    assert np.array_equal(m2, f2)


def test_comparison_on_the_matrix_cores():
    import paper_2407_07308_amd as bc

    prm = Params(15, 257, 14, 50, 5, 50, 3)
    print("modup mfma: N=2^15 uint16 comparison", flush=True)
    dev, dk, _ = ctx_and_keys(prm, 29)
    G, nd, base = 2, 3, 129
    xs = synth.integers(30, (G, dev.M), 0, 1 << 16)
    ys = synth.integers(30, (G, dev.M), 0, 1 << 16, index=1)

    def planes(v, seed):
        out = []
        for d in range(nd):
            digit = (v // base ** (nd - 1 - d)) % base
            r = synth.encrypt_randomness(seed + d, G, prm.N)
            out.append(dev.encrypt(dk, digit.astype(np.uint32), r["u"], r["e"]))
        return out

    A, B = planes(xs, 31), planes(ys, 41)
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 1)
    lt, mx, _ = dev.compare_max_min(dk, A, B, True, True, False)
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
    lt0, mx0, _ = dev.compare_max_min(dk, A, B, True, True, False)
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    assert np.array_equal(dev.export(lt), dev.export(lt0))
    for d in range(nd):
        assert np.array_equal(dev.export(mx[d]), dev.export(mx0[d])), d


def test_tuning_errors():
    import paper_2407_07308_amd as bc

    # 60-bit special primes: no fp64 arithmetic, no tables
    dev = bc.Context.from_params(Params(12, 257, 4, 50, 1, 60, 4))
    with pytest.raises(bc.BoostcomError) as ei:
        dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 1)
    assert ei.value.code == bc.BC_ERR_ARG
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
    # 30-bit primes: 2^32 is not a residue below them
    dev = bc.Context.from_params(Params(12, 257, 4, 30, 2, 30, 2))
    with pytest.raises(bc.BoostcomError) as ei:
        dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 1)
    assert ei.value.code == bc.BC_ERR_ARG
