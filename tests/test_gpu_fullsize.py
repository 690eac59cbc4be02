"""Bit-exact parity with the oracle at the workload sizes.

The device runs each workload as the benchmark does (autotuned transform
schedule, every group batched into one launch sequence); the oracle evaluates
sampled groups one by one on the same seeded inputs, and the sampled output
ciphertexts must agree residue for residue.  Decryptions of the whole batch
are checked against the plaintext answers.

  N = 2^12, p = 17, 4 x 36-bit primes: one pair, single-digit LT
  N = 2^14, p = 257, 8 x 50-bit primes, dnum 2: 16 pairs, pairs 0 and 15 sampled
  N = 2^15, p = 257, 14 x 50-bit primes, dnum 3: uint16 as 3 base-129 digit
        planes, LT + max + min over 4 groups, group 0 sampled (about 12 s of
        oracle work on 16 cores)
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle

pytestmark = pytest.mark.gpu


def setup(name, seed):
    import paper_2407_07308_amd as bc

    prm = oracle.PARAMS[name]
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    dev.autotune()
    orc = Oracle(prm)
    orc.keygen(rnd)
    return prm, dev, dk, orc


def planes_both(dev, dk, orc, planes, seed, sample):
    """Device batches of every plane, oracle ciphertexts of the sampled groups."""
    D, O = [], []
    for d, pl in enumerate(planes):
        r = synth.encrypt_randomness(seed + d, pl.shape[0], dev.N)
        D.append(dev.encrypt(dk, pl, r["u"], r["e"]))
        O.append({i: orc.encrypt(pl[i], r["u"][i], r["e"][i]) for i in sample})
    return D, O


def same_ct(dev, batch, i, ct):
    got = dev.export(batch)[i]
    assert got.shape == ct.data.shape
    assert np.array_equal(got, ct.data), f"{np.count_nonzero(got != ct.data)} residues differ"


@pytest.mark.parametrize("name,G,sample,seed", [("n12_p17", 1, (0,), 101), ("n14_p257", 16, (0, 15), 102)])
def test_single_digit_lt_at_workload_size(name, G, sample, seed):
    prm, dev, dk, orc = setup(name, seed)
    print(f"\n[fullsize] {name}: {G} pairs, oracle on {sample}", flush=True)
    hi = (prm.p + 1) // 2
    x = synth.slot_values(seed, G, dev.M, 0, hi)
    y = synth.slot_values(seed, G, dev.M, 0, hi, index=1)
    (Dx, Ox), (Dy, Oy) = planes_both(dev, dk, orc, [x], seed + 10, sample), planes_both(dev, dk, orc, [y], seed + 20, sample)
    lt = dev.compare_lt(dk, Dx, Dy)
    assert np.array_equal(dev.decrypt(dk, lt), (x < y).astype(np.uint32))
    ev = CtEvaluator(orc)
    for i in sample:
        same_ct(dev, lt, i, oracle.compare_lt(ev, [Ox[0][i]], [Oy[0][i]], prm.p))


def test_uint16_lt_max_min_at_workload_size():
    prm, dev, dk, orc = setup("n15_p257", 103)
    G, base, nd = 4, 129, 3
    print(f"\n[fullsize] n15_p257: {G} uint16 groups, oracle on group 0", flush=True)
    xs = synth.integers(103, (G, dev.M), 0, 65536)
    ys = synth.integers(103, (G, dev.M), 0, 65536, index=1)
    xs[0, :4] = ys[0, :4]  # equal pairs in the sampled group
    A, OA = planes_both(dev, dk, orc, oracle.to_digits(xs, base, nd), 110, (0,))
    B, OB = planes_both(dev, dk, orc, oracle.to_digits(ys, base, nd), 120, (0,))
    lt, mx, mn = dev.compare_max_min(dk, A, B)
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    val = lambda planes: sum(dev.decrypt(dk, p).astype(np.int64) * base ** (nd - 1 - i) for i, p in enumerate(planes))
    assert np.array_equal(val(mx), np.maximum(xs, ys))
    assert np.array_equal(val(mn), np.minimum(xs, ys))
    ev = CtEvaluator(orc)
    oa, ob = [OA[d][0] for d in range(nd)], [OB[d][0] for d in range(nd)]
    o_lt = oracle.compare_lt(ev, oa, ob, prm.p)
    o_mx, o_mn = oracle.max_min(ev, oa, ob, o_lt)
    same_ct(dev, lt, 0, o_lt)
    for d in range(nd):
        same_ct(dev, mx[d], 0, o_mx[d])
        same_ct(dev, mn[d], 0, o_mn[d])


@pytest.mark.parametrize("name,seed", [("n14_p257", 104), ("n15_p257", 105)])
def test_rotation_and_level0_mul_at_workload_size(name, seed):
    """Rotation at the workload ring sizes takes the key-switching route of
    those sizes (part-limb raising transforms, then whole-limb ModDown and
    the key-switch combination): compared with the oracle for a one-slot
    rotation and the row swap, at the top level and one level down; then one
    multiplication at level 0 (no modulus switch) at full size."""
    import paper_2407_07308_amd as bc

    prm = oracle.PARAMS[name]
    steps = (1, bc.BC_ROW_SWAP)
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(steps))
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps)
    dev.autotune()
    orc = Oracle(prm)
    orc.keygen(rnd, rot_steps=steps)
    G = 3
    vals = synth.slot_values(seed, G, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(seed + 1, G, dev.N)
    x = dev.encrypt(dk, vals, r["u"], r["e"])
    ox = orc.encrypt(vals[0], r["u"][0], r["e"][0])
    print(f"\n[fullsize] {name}: rotations {steps} of {G} ciphertexts, oracle on ciphertext 0", flush=True)
    h = dev.M // 2
    for step in steps:
        y = dev.rotate(dk, x, step)
        same_ct(dev, y, 0, orc.rotate(ox, step))
        want = np.concatenate([vals[:, h:], vals[:, :h]], axis=1) if step == bc.BC_ROW_SWAP else np.concatenate(
            [np.roll(vals[:, :h], -step, axis=1), np.roll(vals[:, h:], -step, axis=1)], axis=1)
        assert np.array_equal(dev.decrypt(dk, y), want)
    x1, ox1 = dev.mod_switch(x), orc.mod_switch(ox)
    same_ct(dev, dev.rotate(dk, x1, 1), 0, orc.rotate(ox1, 1))
    # down to level 0, then one multiplication there
    x0, ox0 = x1, ox1
    while x0.level > 0:
        x0, ox0 = dev.mod_switch(x0), orc.mod_switch(ox0)
    m = dev.mul_relin(dk, x0, x0)
    assert m.level == 0
    same_ct(dev, m, 0, orc.mul(ox0, ox0))
    assert np.array_equal(dev.decrypt(dk, m), vals.astype(np.int64) ** 2 % prm.p)
