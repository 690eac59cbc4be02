"""Pins of the slot encoding and of the digit-base reading.

The paper packs integers into SIMD slots and compares them digit by digit
(Background, "Word-wise Universal FHE Scheme"); the slot structure of
Z_p[x]/(x^N + 1) used here is fixed by the factorisation of t^M + 1 over F_p.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Oracle, Params

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/table3_parameters.txt"


def test_slot_counts():
    assert oracle.slot_count(17) == 8
    assert oracle.slot_count(257) == 128
    assert oracle.slot_count(5) == 2
    assert oracle.slot_count(13) == 2


@pytest.mark.parametrize("p", [17, 257])
def test_slot_roots_are_all_roots_of_t_m_plus_one(p):
    M = oracle.slot_count(p)
    roots = oracle.slot_roots(p, M)
    assert len(set(roots)) == M
    for z in roots:
        assert pow(z, M, p) == p - 1
    # the least primitive root is 3 for both Fermat primes
    assert oracle.primitive_root(p) == 3


def py_negacyclic_mod_p(a, b, p):
    N = len(a)
    out = [0] * N
    for i in np.nonzero(a)[0]:
        for j in np.nonzero(b)[0]:
            k = int(i) + int(j)
            t = int(a[i]) * int(b[j])
            if k < N:
                out[k] = (out[k] + t) % p
            else:
                out[k - N] = (out[k - N] - t) % p
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("p,N", [(17, 8), (17, 64), (257, 128), (257, 512)])
def test_encode_decode_round_trip_and_slot_product(p, N):
    M = oracle.slot_count(p)
    rng = np.random.default_rng(p + N)
    for _ in range(3):
        u = rng.integers(0, p, M)
        v = rng.integers(0, p, M)
        mu = oracle.encode_poly(u, p, N)
        mv = oracle.encode_poly(v, p, N)
        assert np.array_equal(oracle.decode_poly(mu, p, N), u)
        d = N // M
        assert not np.any(np.delete(mu, np.arange(0, N, d)))  # zero off multiples of d
        prod = py_negacyclic_mod_p(mu, mv, p)
        assert np.array_equal(oracle.decode_poly(prod, p, N), (u * v) % p)


def py_automorphism_mod_p(m, g, p):
    N = len(m)
    out = np.zeros(N, dtype=np.int64)
    for i in range(N):
        j = (i * g) % (2 * N)
        if j < N:
            out[j] = m[i]
        else:
            out[j - N] = (-int(m[i])) % p
    return out


@pytest.mark.parametrize("p,N", [(17, 16), (257, 256)])
def test_rotation_by_galois_element(p, N):
    """x -> x^(5^r) rotates each half-row left by r; x -> x^(2N-1) swaps rows."""
    M = oracle.slot_count(p)
    h = M // 2
    rng = np.random.default_rng(5)
    v = rng.integers(0, p, M)
    m = oracle.encode_poly(v, p, N)
    for r in (1, 2, h - 1):
        out = oracle.decode_poly(py_automorphism_mod_p(m, oracle.galois_element(r, N), p), p, N)
        expect = np.concatenate([np.roll(v[:h], -r), np.roll(v[h:], -r)])
        assert np.array_equal(out, expect)
    out = oracle.decode_poly(py_automorphism_mod_p(m, oracle.galois_element(-1, N), p), p, N)
    assert np.array_equal(out, np.concatenate([v[h:], v[:h]]))


def _phi(m):
    r, n, f = m, m, 2
    while f * f <= n:
        if n % f == 0:
            while n % f == 0:
                n //= f
            r -= r // f
        f += 1
    if n > 1:
        r -= r // n
    return r


def _order(p, m):
    k, x = 1, p % m
    while x != 1:
        x = x * p % m
        k += 1
    return k


def test_table3_digit_base_reading():
    """Table 3: N = phi(m); slots = phi(m)/ord_m(p); 'no of int' = floor(slots/l);
    and d*l digits cover a 64-bit integer with base p for the bivariate circuit
    but base (p+1)/2 for the univariate one -- the univariate LT is exact on
    digits in [0, (p-1)/2], which is why the digit planes use base (p+1)/2."""
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 20
    tight_u = 0
    for name, p, m, N, circ, d, l, logq, lam, nint in rows:
        p, m, N, d, l, nint = map(int, (p, m, N, d, l, nint))
        assert _phi(m) == N
        slots = N // _order(p, m)
        assert slots // l == nint, name
        base = p if circ == "B" else (p + 1) // 2
        assert d * l * math.log2(base) >= 64 - 1e-9, (name, circ)
        if circ == "U" and d * l * math.log2(p) >= 64 and d * l * math.log2(base) < 64.1:
            tight_u += 1
    # several univariate rows are exactly tight at base (p+1)/2 (e.g. p1: 16*4 bits)
    assert tight_u >= 2
