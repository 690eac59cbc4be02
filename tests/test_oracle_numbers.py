"""Pins of the oracle's number theory and transforms against the mathematics.

Residue-number arithmetic and the NTT follow the paper's background section
("Efficient Polynomial and NTT"); these checks tie the oracle to independent
facts: trial division, the defining equations of a 2N-th root of unity, direct
polynomial evaluation, and schoolbook negacyclic products.
"""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import Oracle, Params

L = oracle.lib()


def trial_prime(n: int) -> bool:
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    r = math.isqrt(n)
    f = 3
    while f <= r:
        if n % f == 0:
            return False
        f += 2
    return True


def strong_probable_prime(n: int, bases=(2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47)) -> bool:
    """Independent check with Python's pow (more bases than the oracle uses)."""
    if n < 2:
        return False
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in bases:
        if a % n == 0:
            continue
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_is_prime_small_range_matches_trial_division():
    for n in range(0, 30000):
        assert bool(L.or_is_prime(n)) == trial_prime(n), n


def test_is_prime_rejects_pseudoprimes():
    # Carmichael numbers and strong pseudoprimes to base 2 (and to 2,3,5,7).
    for n in (561, 1105, 1729, 2465, 41041, 825265, 2047, 3215031751, 3474749660383, 341550071728321):
        assert not L.or_is_prime(n), n


def test_is_prime_random_36bit_matches_trial_division():
    rng = random.Random(7)
    hits = 0
    for _ in range(40):
        n = rng.randrange(2**35, 2**36) | 1
        t = trial_prime(n)
        hits += t
        assert bool(L.or_is_prime(n)) == t
    for n in (68719403009, 68718428161, 68717592577):  # primes of the N=2^12, p=17 chain
        assert trial_prime(n) and L.or_is_prime(n)


@pytest.mark.parametrize("name", sorted(oracle.PARAMS))
def test_prime_chain_definition(name):
    """q_i prime, = 1 mod 2N p, below 2^bits, strictly decreasing, and no
    qualifying prime skipped above the smallest one (the chain is the largest
    such primes)."""
    prm = oracle.PARAMS[name]
    o = Oracle(prm)
    step = 2 * prm.N * prm.p
    for chain, bits, exclude in ((o.q, prm.bitsQ, []), (o.special, prm.bitsP, o.q)):
        assert chain == sorted(chain, reverse=True)
        for q in chain:
            assert q % step == 1 and q < 2**bits and strong_probable_prime(q)
        c = ((2**bits - 2) // step) * step + 1
        expect = []
        while len(expect) < len(chain):
            if strong_probable_prime(c) and c not in exclude:
                expect.append(c)
            c -= step
        assert expect == chain
    assert not set(o.q) & set(o.special)


@pytest.mark.parametrize("name", sorted(oracle.PARAMS))
def test_psi_is_primitive_2n_th_root(name):
    prm = oracle.PARAMS[name]
    o = Oracle(prm)
    for i, q in enumerate(o.moduli):
        psi = int(L.or_ctx_psi(o.ctx, i))
        assert pow(psi, prm.N, q) == q - 1
        assert pow(psi, 2 * prm.N, q) == 1


def small_ctx(logN=4, p=17):
    return Oracle(Params(logN, p, 3, 36, 1, 60, 3))


def test_ntt_forward_is_evaluation_at_odd_powers():
    o = small_ctx(4)
    N = o.N
    rng = np.random.default_rng(1)
    for m, q in enumerate(o.moduli):
        psi = int(L.or_ctx_psi(o.ctx, m))
        a = rng.integers(0, q, N, dtype=np.uint64)
        f = a.copy()
        L.or_ntt_forward(o.ctx, m, oracle._p(f))
        for k in range(N):
            x = pow(psi, 2 * k + 1, q)
            assert int(f[k]) == sum(int(a[i]) * pow(x, i, q) for i in range(N)) % q


def py_schoolbook(a, b, q):
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            t = int(a[i]) * int(b[j])
            if k < N:
                out[k] = (out[k] + t) % q
            else:
                out[k - N] = (out[k - N] - t) % q
    return out


def test_c_schoolbook_matches_python_schoolbook():
    q = 68719403009
    rng = np.random.default_rng(2)
    for N in (1, 2, 8, 32):
        a = rng.integers(0, q, N, dtype=np.uint64)
        b = rng.integers(0, q, N, dtype=np.uint64)
        out = np.zeros(N, np.uint64)
        L.or_schoolbook_negacyclic(oracle._p(a), oracle._p(b), oracle._p(out), N, q)
        assert [int(x) for x in out] == py_schoolbook(a, b, q)


@pytest.mark.parametrize("logN,p", [(3, 17), (6, 17), (8, 257), (10, 257)])
def test_ntt_product_matches_schoolbook_every_prime(logN, p):
    o = Oracle(Params(logN, p, 4, 50, 2, 60, 2))
    rng = np.random.default_rng(logN)
    for m, q in enumerate(o.moduli):
        a = rng.integers(0, q, o.N, dtype=np.uint64)
        b = rng.integers(0, q, o.N, dtype=np.uint64)
        ref = np.zeros(o.N, np.uint64)
        L.or_schoolbook_negacyclic(oracle._p(a), oracle._p(b), oracle._p(ref), o.N, q)
        assert np.array_equal(o.negacyclic_mul(m, a, b), ref)


def test_x_to_the_n_is_minus_one_and_monomials():
    o = small_ctx(5)
    N, q = o.N, o.moduli[0]
    for i, j in ((N - 1, 1), (3, 7), (N - 2, N - 3), (0, 5)):
        a = np.zeros(N, np.uint64)
        b = np.zeros(N, np.uint64)
        a[i] = 1
        b[j] = 1
        r = o.negacyclic_mul(0, a, b)
        k = i + j
        expect = np.zeros(N, np.uint64)
        if k < N:
            expect[k] = 1
        else:
            expect[k - N] = q - 1
        assert np.array_equal(r, expect)


def test_ntt_round_trip_full_size():
    o = Oracle(oracle.PARAMS["n12_p17"])
    rng = np.random.default_rng(3)
    for m, q in enumerate(o.moduli):
        a = rng.integers(0, q, o.N, dtype=np.uint64)
        f = a.copy()
        L.or_ntt_forward(o.ctx, m, oracle._p(f))
        L.or_ntt_inverse(o.ctx, m, oracle._p(f))
        assert np.array_equal(a, f)


def test_ntt_product_is_ring_homomorphism_full_size():
    """(a*b)*c == a*(b*c) and a*(b+c) == a*b + a*c at N = 2^12."""
    o = Oracle(oracle.PARAMS["n12_p17"])
    rng = np.random.default_rng(4)
    q = o.moduli[1]
    a, b, c = (rng.integers(0, q, o.N, dtype=np.uint64) for _ in range(3))
    ab_c = o.negacyclic_mul(1, o.negacyclic_mul(1, a, b), c)
    a_bc = o.negacyclic_mul(1, a, o.negacyclic_mul(1, b, c))
    assert np.array_equal(ab_c, a_bc)
    bc = ((b.astype(object) + c.astype(object)) % q).astype(np.uint64)
    lhs = o.negacyclic_mul(1, a, bc)
    rhs = ((o.negacyclic_mul(1, a, b).astype(object) + o.negacyclic_mul(1, a, c).astype(object)) % q).astype(np.uint64)
    assert np.array_equal(lhs, rhs)
