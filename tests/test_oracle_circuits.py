"""Pins of the comparison circuit.

The paper's univariate circuit evaluates LT(X, Y) = f(X - Y) with about
sqrt(p-3) + O(log p) non-scalar multiplications (Introduction) and combines
per-digit LT and EQ lexicographically (Background, "Word-wise Universal FHE
Scheme").  f is fixed by its values on all of Z_p, so brute force over Z_p pins
every coefficient; the schedule is pinned by evaluating it on plain integers.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, IntEvaluator, Oracle, Params


@pytest.mark.parametrize("p", [3, 5, 7, 17, 257])
def test_lt_polynomial_brute_force(p):
    c = oracle.lt_coefficients(p)
    for z in range(p):
        val = sum(ck * pow(z, k, p) for k, ck in enumerate(c)) % p
        assert val == (1 if z >= (p + 1) // 2 else 0), (p, z)
    assert all(c[k] == 0 for k in range(0, p - 1, 2))
    assert c[p - 1] == (p + 1) // 2


@pytest.mark.parametrize("p,nz", [(17, 8), (257, 113)])
def test_lt_polynomial_sparsity(p, nz):
    assert sum(1 for x in oracle.lt_coefficients(p) if x) == nz


@pytest.mark.parametrize("p", [17, 257])
def test_lt_on_domain_is_less_than(p):
    h = (p - 1) // 2
    c = oracle.lt_coefficients(p)
    for x in range(h + 1):
        for y in range(h + 1):
            z = (x - y) % p
            assert sum(ck * pow(z, k, p) for k, ck in enumerate(c)) % p == int(x < y)


class LevelEvaluator(IntEvaluator):
    """Integers mod p carrying the multiplicative depth (level = -depth)."""

    def mul(self, a, b):
        self.mults += 1
        return (a[0] * b[0] % self.p, min(a[1], b[1]) - 1)

    def mul_add(self, a, b, c):
        self.mults += 1
        return ((a[0] * b[0] + c[0]) % self.p, min(a[1], b[1], c[1]) - 1)

    def add(self, a, b):
        return ((a[0] + b[0]) % self.p, min(a[1], b[1]))

    def sub(self, a, b):
        return ((a[0] - b[0]) % self.p, min(a[1], b[1]))

    def mul_scalar(self, a, c):
        return (a[0] * c % self.p, a[1])

    def add_const(self, a, c):
        return ((a[0] + c) % self.p, a[1])

    def level(self, a):
        return a[1]

    def to_level(self, a, lv):
        return (a[0], min(a[1], lv))


@pytest.mark.parametrize("p,mults,depth", [(17, 8, 4), (257, 30, 8)])
def test_paterson_stockmeyer_schedule(p, mults, depth):
    c = oracle.lt_coefficients(p)
    for z in range(p):
        ev = LevelEvaluator(p)
        f, top = oracle.lt_univariate(ev, (z, 0), p)
        assert f[0] == sum(ck * pow(z, k, p) for k, ck in enumerate(c)) % p
        assert top[0] == pow(z, p - 1, p)
        assert ev.mults == mults
        assert -f[1] == depth
    # against the paper's sqrt(p-3) + O(log p) count for the univariate circuit
    assert mults <= math.sqrt(p - 3) + 2 * math.log2(p)


@pytest.mark.parametrize("ndig", [1, 2, 3])
def test_lexicographic_lt_max_min_brute_force_p17(ndig):
    p, base = 17, 9
    ev = IntEvaluator(p)
    vals = range(base ** ndig) if ndig < 3 else range(0, base ** ndig, 7)
    vals = list(vals)
    rng = np.random.default_rng(ndig)
    ys = vals if ndig == 1 else list(rng.choice(vals, 60))
    for x in vals:
        for y in ys:
            xd = [int(d[0]) for d in oracle.to_digits([x], base, ndig)]
            yd = [int(d[0]) for d in oracle.to_digits([y], base, ndig)]
            lt = oracle.compare_lt(ev, xd, yd, p)
            assert lt == int(x < y)
            mx, mn = oracle.max_min(ev, xd, yd, lt)
            assert sum(d * base ** (ndig - 1 - i) for i, d in enumerate(mx)) == max(x, y)
            assert sum(d * base ** (ndig - 1 - i) for i, d in enumerate(mn)) == min(x, y)


def test_lexicographic_uint16_base129_p257():
    p, base = 257, 129
    ev = IntEvaluator(p)
    xs = synth.integers(5, (400,), 0, 65536)
    ys = synth.integers(5, (400,), 0, 65536, index=1)
    xs[:5] = ys[:5]  # ties
    for x, y in zip(xs, ys):
        xd = [int(d[0]) for d in oracle.to_digits([x], base, 3)]
        yd = [int(d[0]) for d in oracle.to_digits([y], base, 3)]
        lt = oracle.compare_lt(ev, xd, yd, p)
        assert lt == int(x < y)


def _setup(prm, seed=31):
    o = Oracle(prm)
    o.keygen(synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0))
    return o


def _enc_planes(o, planes, seed):
    r = synth.encrypt_randomness(seed, len(planes), o.N)
    return [o.encrypt(pl, r["u"][i], r["e"][i]) for i, pl in enumerate(planes)]


def test_encrypted_lt_p17_tiny():
    o = _setup(Params(5, 17, 6, 36, 1, 60, 3))
    h = 8
    x = synth.slot_values(40, 1, o.M, 0, h + 1)[0]
    y = synth.slot_values(40, 1, o.M, 0, h + 1, 1)[0]
    cx, cy = _enc_planes(o, [x, y], 41)
    ev = CtEvaluator(o)
    f, top = oracle.lt_univariate(ev, o.sub(cx, cy), 17)
    assert np.array_equal(o.decrypt(f), (x < y).astype(np.uint32))
    assert np.array_equal(o.decrypt(oracle.eq_from_top(ev, top)), (x == y).astype(np.uint32))
    assert ev.mults == 8 and o.budget_bits(f) > 10


def test_encrypted_lexicographic_max_min_p17_tiny():
    o = _setup(Params(5, 17, 9, 36, 1, 60, 3))
    base, nd = 9, 2
    xs = synth.integers(42, (o.M,), 0, base ** nd)
    ys = synth.integers(42, (o.M,), 0, base ** nd, index=1)
    xs[0] = ys[0]
    xd, yd = oracle.to_digits(xs, base, nd), oracle.to_digits(ys, base, nd)
    ca = _enc_planes(o, xd, 43)
    cb = _enc_planes(o, yd, 44)
    ev = CtEvaluator(o)
    lt = oracle.compare_lt(ev, ca, cb, 17)
    assert np.array_equal(o.decrypt(lt), (xs < ys).astype(np.uint32))
    mx, mn = oracle.max_min(ev, ca, cb, lt)
    dec = lambda planes: sum(o.decrypt(c).astype(np.int64) * base ** (nd - 1 - i) for i, c in enumerate(planes))
    assert np.array_equal(dec(mx), np.maximum(xs, ys))
    assert np.array_equal(dec(mn), np.minimum(xs, ys))
    assert min(o.budget_bits(c) for c in mx + mn) > 5


def test_encrypted_lt_p257_full_range_matches_polynomial():
    """Full-range digits: the decryption is f(x - y) slot-wise (integer '<' only
    where |x - y| <= (p-1)/2)."""
    o = _setup(Params(7, 257, 8, 50, 3, 60, 2))
    x = synth.slot_values(45, 1, o.M, 0, 257)[0]
    y = synth.slot_values(45, 1, o.M, 0, 257, 1)[0]
    cx, cy = _enc_planes(o, [x, y], 46)
    ev = CtEvaluator(o)
    f, _ = oracle.lt_univariate(ev, o.sub(cx, cy), 257)
    z = (x.astype(np.int64) - y) % 257
    assert np.array_equal(o.decrypt(f), (z >= 129).astype(np.uint32))
    assert ev.mults == 30 and f.level == 0
