"""Pins of the slot-packed comparison and the window tournament.

The paper combines per-digit LT and EQ lexicographically, the digits of one
integer sitting in slots of one ciphertext, by ShiftMul (shift the ciphertext,
multiply by the equality result) and ShiftAdd (sum by shifting) (Background,
"Word-wise Universal FHE Scheme").  Pinned here:
  * the slot evaluator's rotation against the encrypted oracle's rotation
    (itself pinned as an automorphism that rotates slot rows);
  * the packed LT against integer '<' over every pair of small integers, for
    both digit circuits and every block length up to 8 digits;
  * the tournament against numpy's minimum / maximum over every cyclic window;
  * both on encrypted slots at small N, with the rotation keys of the shifts;
  * the multiplication, rotation and level counts of both schedules.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params, SlotEvaluator


def _rows(M, ints_per_row, l):
    """positions of integer k's first digit, k over both rows"""
    h = M // 2
    return [r * h + k * l for r in range(2) for k in range(ints_per_row)]


def pack(values, base, l, M):
    """integers -> slot vector: l digits each (most significant first), rows filled in order"""
    h = M // 2
    per_row = h // l
    assert len(values) == 2 * per_row
    out = np.zeros(M, dtype=np.int64)
    for idx, v in enumerate(values):
        r, k = divmod(idx, per_row)
        for i, d in enumerate(oracle.to_digits([v], base, l)):
            out[r * h + k * l + i] = int(d[0])
    return out


def test_slot_evaluator_rotation_matches_encrypted_rotation():
    prm = Params(5, 17, 3, 36, 1, 60, 3)
    o = Oracle(prm)
    o.keygen(synth.keygen_randomness(11, prm.N, prm.nQ, prm.nP, prm.dnum, 3), rot_steps=(1, 2, 3))
    x = synth.slot_values(12, 1, o.M, 0, 17)[0]
    r = synth.encrypt_randomness(13, 1, o.N)
    ct = o.encrypt(x, r["u"][0], r["e"][0])
    ev = SlotEvaluator(17, o.M)
    for s in (1, 2, 3):
        assert np.array_equal(o.decrypt(o.rotate(ct, s)).astype(np.int64), ev.rotate(x, s)), s
    # and by hand: slot j of a row receives slot j + s of the same row
    h = o.M // 2
    want = np.array([x[(j // h) * h + (j % h + 1) % h] for j in range(o.M)])
    assert np.array_equal(ev.rotate(x, 1), want)


@pytest.mark.parametrize("circuit,base", [("univariate", 9), ("bivariate", 17)])
@pytest.mark.parametrize("l", [1, 2, 4])
def test_packed_lt_every_pair_p17(circuit, base, l):
    """every pair of l'-digit integers (l' = min(l, 2) significant digits,
    leading zero digits above): LT at the first slot of each block"""
    p = 17
    nd = min(l, 2)
    vals = list(range(base ** nd))
    pairs = list(itertools.product(vals, vals))
    per_row = 64  # integers per row of the simulated vector
    M = 2 * per_row * l
    ev = SlotEvaluator(p, M)
    chunk = 2 * per_row
    for c0 in range(0, len(pairs), chunk):
        part = pairs[c0:c0 + chunk]
        part = part + [(0, 0)] * (chunk - len(part))
        a = pack([x for x, _ in part], base, l, M)
        b = pack([y for _, y in part], base, l, M)
        lt = oracle.compare_lt_packed(ev, a, b, p, l, circuit)
        got = lt[_rows(M, per_row, l)]
        want = np.array([int(x < y) for x, y in part])
        assert np.array_equal(got, want), (c0, circuit, l)


@pytest.mark.parametrize("l", [2, 4, 8])
def test_packed_lt_random_p257(l):
    p, base = 257, 129
    M = 128
    per_row = (M // 2) // l
    rng = np.random.default_rng(l)
    for trial in range(20):
        xs = rng.integers(0, base ** l, 2 * per_row)
        ys = xs.copy()
        # equal prefixes of every length, then a difference
        for i in range(len(ys)):
            j = rng.integers(0, l + 1)
            if j < l:
                ys[i] = xs[i] + rng.choice([-1, 1]) * base ** j
        ys = np.clip(ys, 0, base ** l - 1)
        ev = SlotEvaluator(p, M)
        lt = oracle.compare_lt_packed(ev, pack(xs, base, l, M), pack(ys, base, l, M), p, l)
        assert np.array_equal(lt[_rows(M, per_row, l)], (xs < ys).astype(np.int64)), trial


@pytest.mark.parametrize("p,mults_lt", [(17, 8), (257, 30)])
@pytest.mark.parametrize("l", [1, 2, 4, 8])
def test_packed_schedule_counts(p, mults_lt, l):
    """LT and EQ of the digits, then 2 log2(l) - 1 products and rotations
    (none for l = 1); depth: the digit circuit's plus log2(l)"""
    M = 2 * 8
    from test_oracle_circuits import LevelEvaluator

    class Lev(LevelEvaluator):
        def __init__(self, p):
            super().__init__(p)
            self.rotations = 0

        def rotate(self, a, s):
            self.rotations += 1
            return a

    ev = Lev(p)
    lt = oracle.compare_lt_packed(ev, (3, 0), (5, 0), p, l)
    r = l.bit_length() - 1
    assert ev.mults == mults_lt + max(0, 2 * r - 1)
    assert ev.rotations == max(0, 2 * r - 1)
    depth_lt = (p - 1).bit_length() - 1
    assert -lt[1] == depth_lt + r


@pytest.mark.parametrize("circuit,vmax", [("univariate", 9), ("bivariate", 17)])
@pytest.mark.parametrize("k", [2, 4, 8])
@pytest.mark.parametrize("want_max", [False, True])
def test_tournament_every_window(circuit, vmax, k, want_max):
    p, M = 17, 64
    h = M // 2
    rng = np.random.default_rng(k + 10 * want_max)
    for trial in range(10):
        x = rng.integers(0, vmax, M)
        ev = SlotEvaluator(p, M)
        got = oracle.tournament(ev, x, p, k, want_max, circuit)
        rows = x.reshape(2, h)
        win = np.array([[rows[r][(j + np.arange(k)) % h] for j in range(h)] for r in range(2)])
        want = (win.max(axis=2) if want_max else win.min(axis=2)).reshape(-1)
        assert np.array_equal(got, want), trial
        assert ev.rotations == k.bit_length() - 1


def _oracle(prm, steps, seed=21):
    o = Oracle(prm)
    o.keygen(synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(steps)), rot_steps=steps)
    return o


def test_encrypted_packed_lt_p17():
    """two base-9 digits per integer in pairs of slots (l = 2) and four-slot
    blocks holding 3 digits under a zero digit (l = 4), N = 2^5 (4 slots a row)"""
    prm = Params(5, 17, 8, 36, 1, 60, 8)  # one prime per digit: below the 60-bit P
    o = _oracle(prm, (1, 2))
    p, base = 17, 9
    for l, nd in ((2, 2), (4, 3)):
        per_row = (o.M // 2) // l
        xs = synth.integers(30 + l, (2 * per_row,), 0, base ** nd)
        ys = synth.integers(30 + l, (2 * per_row,), 0, base ** nd, index=1)
        xs[0] = ys[0]
        r = synth.encrypt_randomness(40 + l, 2, o.N)
        ca = o.encrypt(pack(xs, base, l, o.M), r["u"][0], r["e"][0])
        cb = o.encrypt(pack(ys, base, l, o.M), r["u"][1], r["e"][1])
        ev = CtEvaluator(o)
        lt = oracle.compare_lt_packed(ev, ca, cb, p, l)
        dec = o.decrypt(lt).astype(np.int64)
        assert np.array_equal(dec[_rows(o.M, per_row, l)], (xs < ys).astype(np.int64)), l
        assert lt.level == prm.nQ - 1 - 4 - (l.bit_length() - 1)
        assert o.budget_bits(lt) > 5


def test_encrypted_tournament_p17():
    """minimum and maximum over windows of 4 slots (two rounds), N = 2^5"""
    prm = Params(5, 17, 12, 36, 1, 60, 12)
    o = _oracle(prm, (1, 2), seed=22)
    x = synth.slot_values(50, 1, o.M, 0, 9)[0].astype(np.int64)
    r = synth.encrypt_randomness(51, 1, o.N)
    ct = o.encrypt(x, r["u"][0], r["e"][0])
    h = o.M // 2
    rows = x.reshape(2, h)
    win = np.array([[rows[rr][(j + np.arange(4)) % h] for j in range(h)] for rr in range(2)])
    for want_max in (False, True):
        ev = CtEvaluator(o)
        out = oracle.tournament(ev, ct, 17, 4, want_max)
        want = (win.max(axis=2) if want_max else win.min(axis=2)).reshape(-1)
        assert np.array_equal(o.decrypt(out).astype(np.int64), want), want_max
        assert out.level == prm.nQ - 1 - 2 * 5
        assert o.budget_bits(out) > 5
