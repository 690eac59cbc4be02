"""Pins of the bivariate comparison circuit.

The paper's bivariate circuit compares two digits of F_p exactly, whatever
their values (Introduction: 2p - 6 non-scalar multiplications; Background,
"Word-wise Universal FHE Scheme": LT and EQ per digit, combined in
lexicographic order).  Its polynomial is fixed by its values on all of
Z_p x Z_p, so brute force pins every coefficient; an independent evaluation
(Vandermonde products instead of the interpolation formula) checks all 66049
pairs at p = 257; the schedule is pinned on plain integers (values,
multiplications, depth) and on encrypted digits at small N.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, IntEvaluator, Oracle, Params

from test_oracle_circuits import LevelEvaluator


@pytest.mark.parametrize("p", [3, 5, 7, 17])
def test_bivariate_table_brute_force(p):
    c = oracle.lt_bivariate_table(p)
    for x in range(p):
        for y in range(p):
            s, z = (x + y) % p, (x - y) % p
            v = sum(int(c[m, k]) * pow(s, m, p) * pow(z, k, p) for m in range(p) for k in range(p)) % p
            assert v == int(x < y), (x, y)


def test_bivariate_table_p257_every_pair():
    p = 257
    c = oracle.lt_bivariate_table(p)
    # evaluate G(s, z) at every point by Vandermonde products
    V = np.array([[pow(t, j, p) for j in range(p)] for t in range(p)], dtype=np.int64)
    G = (V @ c) % p
    G = (G @ V.T) % p  # G[s][z] = sum_m,k c[m][k] s^m z^k
    xs, ys = np.meshgrid(np.arange(p), np.arange(p), indexing="ij")
    want = (xs < ys).astype(np.int64)
    assert np.array_equal(G[(xs + ys) % p, (xs - ys) % p], want)


@pytest.mark.parametrize("p", [5, 17, 257])
def test_bivariate_even_part_is_half_z_to_p_minus_1(p):
    """LT(X,Y) + LT(Y,X) = (X - Y)^(p-1): the part of G even in Z is
    (p+1)/2 Z^(p-1), the rest is odd in Z (what the schedule relies on)."""
    c = oracle.lt_bivariate_table(p)
    for k in range(0, p, 2):
        for m in range(p):
            want = (p + 1) // 2 if (m, k) == (0, p - 1) else 0
            assert c[m, k] == want, (m, k)


@pytest.mark.parametrize("p,mults,depth", [(17, 34, 5), (257, 518, 9)])
def test_bivariate_schedule_on_integers(p, mults, depth):
    rng = np.random.default_rng(p)
    pairs = [(x, y) for x in range(p) for y in range(p)] if p < 50 else \
        [(0, 0), (0, p - 1), (p - 1, 0), (p - 1, p - 1), (128, 129), (129, 128)] + \
        [tuple(int(v) for v in rng.integers(0, p, 2)) for _ in range(40)]
    for x, y in pairs:
        ev = LevelEvaluator(p)
        lt, top = oracle.lt_bivariate(ev, (x, 0), (y, 0), p)
        assert lt[0] == int(x < y), (x, y)
        assert (1 - top[0]) % p == int(x == y)
        assert ev.mults == mults
        assert -lt[1] == depth
    # against the paper's 2p - 6 for the bivariate circuit: the same order
    assert mults <= 2 * p + 4


def test_bivariate_lexicographic_base_p_p17():
    """Two base-17 digits (every integer in [0, 289)): LT is integer '<'."""
    p, nd = 17, 2
    ev = IntEvaluator(p)
    rng = np.random.default_rng(3)
    vals = list(range(0, p ** nd, 5)) + [p - 1, p, p ** nd - 1]
    ys = list(rng.choice(p ** nd, 40)) + [0, p, p ** nd - 1]
    for x in vals:
        for y in ys:
            xd = [int(d[0]) for d in oracle.to_digits([x], p, nd)]
            yd = [int(d[0]) for d in oracle.to_digits([y], p, nd)]
            assert oracle.compare_lt_bivariate(ev, xd, yd, p) == int(x < y), (x, y)


def _setup(prm, seed=37):
    o = Oracle(prm)
    o.keygen(synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0))
    return o


def test_encrypted_bivariate_lexicographic_max_min_p17():
    o = _setup(Params(5, 17, 9, 36, 1, 60, 3))
    p, nd = 17, 2
    xs = synth.integers(47, (o.M,), 0, p ** nd)
    ys = synth.integers(47, (o.M,), 0, p ** nd, index=1)
    xs[0] = ys[0]
    xd, yd = oracle.to_digits(xs, p, nd), oracle.to_digits(ys, p, nd)
    r = synth.encrypt_randomness(48, 2 * nd, o.N)
    ca = [o.encrypt(pl, r["u"][i], r["e"][i]) for i, pl in enumerate(xd)]
    cb = [o.encrypt(pl, r["u"][nd + i], r["e"][nd + i]) for i, pl in enumerate(yd)]
    ev = CtEvaluator(o)
    lt = oracle.compare_lt_bivariate(ev, ca, cb, p)
    assert np.array_equal(o.decrypt(lt), (xs < ys).astype(np.uint32))
    mx, mn = oracle.max_min(ev, ca, cb, lt)
    dec = lambda planes: sum(o.decrypt(c).astype(np.int64) * p ** (nd - 1 - i) for i, c in enumerate(planes))
    assert np.array_equal(dec(mx), np.maximum(xs, ys))
    assert np.array_equal(dec(mn), np.minimum(xs, ys))
    assert ev.mults == 2 * 34 + 1 + 2 * nd
    assert min(o.budget_bits(c) for c in mx + mn) > 5


def test_encrypted_bivariate_p257_full_range():
    """Full-range digits of F_257: the bivariate LT is integer '<' on every
    pair (where the univariate f(x - y) is not)."""
    o = _setup(Params(7, 257, 11, 50, 3, 60, 4))
    x = synth.slot_values(49, 1, o.M, 0, 257)[0]
    y = synth.slot_values(49, 1, o.M, 0, 257, 1)[0]
    x[:3], y[:3] = [0, 256, 200], [256, 0, 200]
    r = synth.encrypt_randomness(50, 2, o.N)
    cx, cy = o.encrypt(x, r["u"][0], r["e"][0]), o.encrypt(y, r["u"][1], r["e"][1])
    ev = CtEvaluator(o)
    lt, top = oracle.lt_bivariate(ev, cx, cy, 257)
    assert np.array_equal(o.decrypt(lt), (x < y).astype(np.uint32))
    assert np.array_equal(o.decrypt(oracle.eq_from_top(ev, top)), (x == y).astype(np.uint32))
    assert ev.mults == 518 and lt.level == 11 - 1 - 9
    assert o.budget_bits(lt) > 5
