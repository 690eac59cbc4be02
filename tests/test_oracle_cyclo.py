"""Pins of the non-power-of-two cyclotomic rings (the rings the paper's
BluesteinNTT serves; Background, "Efficient Polynomial and NTT").

Phi_m against textbook values and the identity prod_{d | m} Phi_d = X^m - 1;
the roots of unity against their order; the evaluation representation
against closed forms (monomials, constants) and against the ring's own
multiplication (a schoolbook product reduced by long division: forward maps
it to the slotwise product, inverse brings it back); the inverse against the
forward on random inputs; all at small m and at the workload's m = 18157.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import CycloRing


def polymul(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def test_cyclotomic_textbook_values():
    assert oracle.cyclotomic(3) == [1, 1, 1]
    assert oracle.cyclotomic(7) == [1] * 7
    assert oracle.cyclotomic(9) == [1, 0, 0, 1, 0, 0, 1]
    assert oracle.cyclotomic(15) == [1, -1, 0, 1, -1, 1, 0, -1, 1]
    # Phi_105 is the first with a coefficient -2 (at X^7 and X^41)
    c105 = oracle.cyclotomic(105)
    assert len(c105) == 49 and c105[7] == -2 and c105[41] == -2 and min(c105) == -2


@pytest.mark.parametrize("m", [15, 21, 45, 63, 105, 255])
def test_product_of_cyclotomics_is_x_m_minus_1(m):
    prod = [1]
    for d in range(1, m + 1):
        if m % d == 0:
            prod = polymul(prod, oracle.cyclotomic(d))
    assert prod == [-1] + [0] * (m - 1) + [1]
    assert len(oracle.cyclotomic(m)) - 1 == len(oracle.zm_star(m)) == sum(
        1 for k in range(1, m + 1) if math.gcd(k, m) == 1)


@pytest.mark.parametrize("m", [105, 1023, 18157])
def test_roots_have_order_m_and_are_roots_of_phi(m):
    r = CycloRing(m, 2, 50)
    assert r.N == len(r.zm)
    for q, w in zip(r.moduli, r.omega):
        assert q % (2 * r.L * m) == 1 and q < 2 ** 50
        assert pow(w, m, q) == 1
        for f in {f for f in range(2, m + 1) if m % f == 0 and all(f % g for g in range(2, f))}:
            assert pow(w, m // f, q) != 1
        ev = lambda x: sum(c * pow(x, j, q) for j, c in enumerate(r.phi)) % q
        assert ev(pow(w, r.zm[1], q)) == 0  # a primitive root
        k_bad = next(k for k in range(1, m) if math.gcd(k, m) > 1)
        assert ev(pow(w, k_bad, q)) != 0  # not a primitive root


@pytest.mark.parametrize("m", [105, 1023])
def test_forward_closed_forms(m):
    r = CycloRing(m, 1, 50)
    q, w = r.moduli[0], r.omega[0]
    one = np.zeros((1, r.N), np.uint64)
    one[0, 0] = 1
    assert np.all(r.forward(one) == 1)
    for j in (1, 2, r.N - 1):
        xj = np.zeros((1, r.N), np.uint64)
        xj[0, j] = 1
        assert np.array_equal(r.forward(xj)[0], np.array([pow(w, j * k, q) for k in r.zm], np.uint64)), j
    assert np.array_equal(r.inverse(np.ones((1, r.N), np.uint64)), one)


@pytest.mark.parametrize("m", [105, 1023, 4369])
def test_ring_product_round_trip(m):
    r = CycloRing(m, 2, 50)
    rng = np.random.default_rng(m)
    a = np.stack([rng.integers(0, q, r.N, dtype=np.uint64) for q in r.moduli])
    b = np.stack([rng.integers(0, q, r.N, dtype=np.uint64) for q in r.moduli])
    fa, fb = r.forward(a), r.forward(b)
    prod = np.stack([np.array([int(x) * int(y) % q for x, y in zip(fa[i], fb[i])], np.uint64)
                     for i, q in enumerate(r.moduli)])
    ab = r.mul(a, b)
    assert np.array_equal(r.forward(ab), prod)
    assert np.array_equal(r.inverse(prod), ab)
    assert np.array_equal(r.inverse(fa), a)


def test_workload_ring_round_trip():
    """m = 18157 = 67 x 271: phi(m) = 17820, convolution length 2^16"""
    r = CycloRing(18157, 1, 50)
    assert (r.N, r.L) == (17820, 65536)
    assert set(r.phi) <= {-1, 0, 1}
    rng = np.random.default_rng(5)
    a = rng.integers(0, r.moduli[0], (1, r.N), dtype=np.uint64)
    fa = r.forward(a)
    assert np.array_equal(r.inverse(fa), a)
    # X * X^(N-1) = X^N, reduced: -(Phi_m - X^N)
    x1 = np.zeros((1, r.N), np.uint64)
    x1[0, 1] = 1
    xt = np.zeros((1, r.N), np.uint64)
    xt[0, r.N - 1] = 1
    q = r.moduli[0]
    want = np.array([(-c) % q for c in r.phi[:-1]], np.uint64)
    assert np.array_equal(r.mul(x1, xt)[0], want)
