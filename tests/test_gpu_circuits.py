"""Comparison circuits on the device vs the oracle.

Ciphertexts of the circuit outputs are compared bit for bit with the oracle's
evaluation of the same Paterson-Stockmeyer schedule (the schedule is fixed,
so every intermediate ciphertext is determined); decryptions are checked
against the plaintext semantics (integer '<', max, min on digits in
[0, (p-1)/2]).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params

pytestmark = pytest.mark.gpu


def make(prm, seed=5):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    orc = Oracle(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    orc.keygen(rnd)
    return dev, dk, orc


def enc_planes(dev, dk, orc, planes, seed):
    """planes: list over digits of uint32 [count][M]; returns device batches and oracle lists."""
    D, O = [], []
    for d, pl in enumerate(planes):
        r = synth.encrypt_randomness(seed + d, pl.shape[0], dev.N)
        D.append(dev.encrypt(dk, pl, r["u"], r["e"]))
        O.append([orc.encrypt(pl[i], r["u"][i], r["e"][i]) for i in range(pl.shape[0])])
    return D, O


def check(dev, d, o):
    got = dev.export(d)
    want = np.stack([c.data for c in o])
    assert got.shape == want.shape
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} residues differ"


@pytest.mark.parametrize("full_range", [False, True])
def test_single_digit_lt_p17(full_range):
    prm = Params(10, 17, 6, 36, 1, 60, 3)
    dev, dk, orc = make(prm)
    G, hi = 3, (17 if full_range else 9)
    x = synth.slot_values(60, G, orc.M, 0, hi)
    y = synth.slot_values(60, G, orc.M, 0, hi, index=1)
    x[0, :2] = y[0, :2]
    (Dx, Dy), (Ox, Oy) = zip(*[enc_planes(dev, dk, orc, [v], s) for v, s in ((x, 61), (y, 62))])
    lt = dev.compare_lt(dk, Dx, Dy)
    ev = CtEvaluator(orc)
    o_lt = [oracle.compare_lt(ev, [Ox[0][i]], [Oy[0][i]], 17) for i in range(G)]
    check(dev, lt, o_lt)
    z = (x.astype(np.int64) - y) % 17
    assert np.array_equal(dev.decrypt(dk, lt), (z >= 9).astype(np.uint32))


def test_lexicographic_max_min_p17_two_digits():
    prm = Params(10, 17, 9, 36, 1, 60, 3)
    dev, dk, orc = make(prm)
    G, base, nd = 2, 9, 2
    xs = synth.integers(70, (G, orc.M), 0, base ** nd)
    ys = synth.integers(70, (G, orc.M), 0, base ** nd, index=1)
    xs[0, 0] = ys[0, 0]
    xd, yd = oracle.to_digits(xs, base, nd), oracle.to_digits(ys, base, nd)
    DA, OA = enc_planes(dev, dk, orc, xd, 71)
    DB, OB = enc_planes(dev, dk, orc, yd, 81)
    lt, mx, mn = dev.compare_max_min(dk, DA, DB)
    ev = CtEvaluator(orc)
    for i in range(G):
        a = [OA[d][i] for d in range(nd)]
        b = [OB[d][i] for d in range(nd)]
        o_lt = oracle.compare_lt(ev, a, b, 17)
        o_mx, o_mn = oracle.max_min(ev, a, b, o_lt)
        check(dev, dev_slice(dev, lt, i), [o_lt])
        for d in range(nd):
            check(dev, dev_slice(dev, mx[d], i), [o_mx[d]])
            check(dev, dev_slice(dev, mn[d], i), [o_mn[d]])
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    val = lambda planes: sum(dev.decrypt(dk, p).astype(np.int64) * base ** (nd - 1 - k) for k, p in enumerate(planes))
    assert np.array_equal(val(mx), np.maximum(xs, ys))
    assert np.array_equal(val(mn), np.minimum(xs, ys))


def dev_slice(dev, b, i):
    import paper_2407_07308_amd as bc

    w = dev.ct_words(b.level, b.ncomp)
    return bc.Batch(b.tensor[i * w:(i + 1) * w], 1, b.level, b.ncomp)


def test_per_op_path_equals_batched():
    """One ciphertext per launch gives the same bytes as the batched launches."""
    import paper_2407_07308_amd as bc

    prm = Params(10, 17, 6, 36, 1, 60, 3)
    dev, dk, orc = make(prm)
    G, base, nd = 3, 9, 2
    xs = synth.integers(95, (G, orc.M), 0, base ** nd)
    ys = synth.integers(95, (G, orc.M), 0, base ** nd, index=1)
    DA, _ = enc_planes(dev, dk, orc, oracle.to_digits(xs, base, nd), 96)
    DB, _ = enc_planes(dev, dk, orc, oracle.to_digits(ys, base, nd), 97)
    lt, mx, mn = dev.compare_max_min(dk, DA, DB)
    dev.set_exec_mode(bc.BC_EXEC_PER_OP)
    lt2, mx2, mn2 = dev.compare_max_min(dk, DA, DB)
    dev.set_exec_mode(bc.BC_EXEC_BATCHED)
    for x, y in [(lt, lt2)] + list(zip(mx, mx2)) + list(zip(mn, mn2)):
        assert np.array_equal(dev.export(x), dev.export(y))


def test_lt_p257_matches_oracle_and_graph_replay():
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)  # all primes < 2^50: fp64 transforms
    dev, dk, orc = make(prm)
    G = 2
    x = synth.slot_values(90, G, orc.M, 0, 129)
    y = synth.slot_values(90, G, orc.M, 0, 129, index=1)
    (Dx, Dy), (Ox, Oy) = zip(*[enc_planes(dev, dk, orc, [v], s) for v, s in ((x, 91), (y, 92))])
    lt = dev.compare_lt(dk, Dx, Dy)
    ev = CtEvaluator(orc)
    check(dev, lt, [oracle.compare_lt(ev, [Ox[0][i]], [Oy[0][i]], 257) for i in range(G)])
    assert np.array_equal(dev.decrypt(dk, lt), (x < y).astype(np.uint32))
    # graph mode: first call records, later calls replay; every replay equals eager
    ref = dev.export(lt)
    dev.set_exec_mode(bc.BC_EXEC_GRAPH)
    outs = dev.compare_max_min(dk, Dx, Dy, True, False, False)
    for _ in range(3):
        assert np.array_equal(dev.export(outs[0]), ref)
        outs[0].tensor.zero_()
        dev.compare_max_min(dk, Dx, Dy, True, False, False, outs=outs)
    assert np.array_equal(dev.export(outs[0]), ref)
    dev.set_exec_mode(bc.BC_EXEC_BATCHED)
