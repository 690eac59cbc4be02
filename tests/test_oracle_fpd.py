"""Pins of the F_{p^d} slots and their digit extraction (Background, "Word-wise
Universal FHE Scheme": integers as elements of F_{p^d}^l, split into F_p
digits by the mod-extract step).

The slot structure against number theory (d is the order of p mod 2N, the
Frobenius steps against their closed form), the power-basis encoding against
the CRT definition (decode is reduction modulo x^d - zeta_j, independent of
the encoder), the slots as fields (products of plaintexts are slotwise
products; the automorphism x -> x^p is the slotwise p-th power), the trace
of monomials against the full sum over the Frobenius group, the monomial
product of a ciphertext against the plaintext definition, and the encrypted
extraction against the coordinates it must return."""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params


def order_mod(p, n):
    x, k = p % n, 1
    while x != 1:
        x, k = x * p % n, k + 1
    return k


@pytest.mark.parametrize("p,logN", [(17, 10), (17, 12), (257, 10), (257, 13), (257, 15)])
def test_degree_is_the_order_of_p(p, logN):
    N = 1 << logN
    d = oracle.fpd_degree(p, N)
    assert d == order_mod(p, 2 * N)
    assert d * oracle.slot_count(p) == N


@pytest.mark.parametrize("p,logN", [(17, 10), (17, 12), (257, 10), (257, 15)])
def test_frobenius_steps_closed_form(p, logN):
    N = 1 << logN
    steps = oracle.frobenius_steps(p, N)
    assert 2 ** len(steps) == oracle.fpd_degree(p, N)
    for b, r in enumerate(steps):
        assert 0 <= r < N // 2
        assert pow(5, r, 2 * N) == pow(p, 2 ** b, 2 * N)
        assert oracle.galois_element(r, N) == pow(p, 2 ** b, 2 * N)


def random_fpd(rng, p, N):
    M, d = oracle.slot_count(p), oracle.fpd_degree(p, N)
    return rng.integers(0, p, (M, d))


@pytest.mark.parametrize("p,logN", [(17, 10), (257, 10), (257, 12)])
def test_encode_decode(p, logN):
    N = 1 << logN
    rng = np.random.default_rng(logN + p)
    E = random_fpd(rng, p, N)
    m = oracle.encode_fpd(E, p, N)
    assert np.array_equal(oracle.decode_fpd(m, p, N), E)
    # the F_p subfield: a constant element in every slot is the ordinary slot encoding
    v = rng.integers(0, p, oracle.slot_count(p))
    E0 = np.zeros_like(E)
    E0[:, 0] = v
    assert np.array_equal(oracle.encode_fpd(E0, p, N), oracle.encode_poly(v, p, N))
    assert np.array_equal(oracle.decode_poly(oracle.encode_fpd(E0, p, N), p, N), v)


def negacyclic_mod_p(a, b, N, p):
    c = np.convolve(np.asarray(a, np.int64), np.asarray(b, np.int64)) % p
    out = c[:N].copy()
    out[: N - 1] = (out[: N - 1] - c[N:]) % p
    return out


@pytest.mark.parametrize("p,logN", [(17, 10), (257, 10)])
def test_slots_are_the_crt_fields(p, logN):
    """decode(m1 m2) is the slotwise product in F_p[x]/(x^d - zeta_j), and
    decode(m(x^p)) the slotwise p-th power (the Frobenius)."""
    N = 1 << logN
    rng = np.random.default_rng(7 * logN + p)
    A, B = random_fpd(rng, p, N), random_fpd(rng, p, N)
    ma, mb = oracle.encode_fpd(A, p, N), oracle.encode_fpd(B, p, N)
    prod = oracle.decode_fpd(negacyclic_mod_p(ma, mb, N, p), p, N)
    roots = oracle.slot_roots(p, oracle.slot_count(p))
    for j, z in enumerate(roots):
        assert np.array_equal(prod[j], oracle.fpd_slot_mul(A[j], B[j], z, p)), j
    frob = oracle.decode_fpd(oracle.plain_automorphism(ma, p % (2 * N), N, p), p, N)
    for j, z in enumerate(roots):
        acc = np.zeros(len(A[j]), np.int64)
        acc[0] = 1
        for _ in range(p):
            acc = oracle.fpd_slot_mul(acc, A[j], z, p)
        assert np.array_equal(frob[j], acc), j


@pytest.mark.parametrize("p,logN", [(17, 10), (257, 10)])
def test_trace_of_monomials(p, logN):
    """sum over all d Frobenius powers of x^j: d x^j when d | j, else 0; and
    the log2(d) doublings give the same sum on a random plaintext."""
    N = 1 << logN
    d = oracle.fpd_degree(p, N)
    group = [pow(p, i, 2 * N) for i in range(d)]
    assert len(set(group)) == d
    for j in (0, 1, 3, d - 1, d, 2 * d + 5, 3 * d, N - 1):
        xj = np.zeros(N, np.int64)
        xj[j] = 1
        tr = sum(oracle.plain_automorphism(xj, g, N, p) for g in group) % p
        want = np.zeros(N, np.int64)
        if j % d == 0:
            want[j] = d % p
        assert np.array_equal(tr, want), j
    rng = np.random.default_rng(11)
    m = rng.integers(0, p, N)
    full = sum(oracle.plain_automorphism(m, g, N, p) for g in group) % p
    z = m.copy()
    for r in oracle.frobenius_steps(p, N):
        z = (z + oracle.plain_automorphism(z, oracle.galois_element(r, N), N, p)) % p
    assert np.array_equal(z, full)


def test_mul_monomial_matches_plaintext_product():
    prm = Params(10, 17, 6, 36, 1, 60, 3)
    o = Oracle(prm)
    rnd = synth.keygen_randomness(31, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    o.keygen(rnd)
    rng = np.random.default_rng(3)
    m = rng.integers(0, 17, prm.N).astype(np.uint32)
    r = synth.encrypt_randomness(32, 1, prm.N)
    ct = o.encrypt_poly(m, r["u"][0], r["e"][0])
    for e in (0, 1, 5, prm.N - 1, prm.N, prm.N + 7, 2 * prm.N - 3):
        xe = np.zeros(2 * prm.N, np.int64)
        xe[e] = 1
        want = negacyclic_mod_p(m, (xe[: prm.N] - xe[prm.N:]) % 17, prm.N, 17)
        assert np.array_equal(o.decrypt_poly(o.mul_monomial(ct, e)), want), e
    # the noise is unchanged (a signed permutation of the coefficients)
    assert o.noise_bits(o.mul_monomial(ct, 9)) == o.noise_bits(ct)


@pytest.mark.parametrize("prm", [Params(10, 17, 6, 36, 1, 60, 3), Params(10, 257, 8, 50, 4, 50, 2)])
def test_extract_digit_returns_the_coordinates(prm):
    p, N = prm.p, prm.N
    steps = oracle.frobenius_steps(p, N)
    o = Oracle(prm)
    rnd = synth.keygen_randomness(41, N, prm.nQ, prm.nP, prm.dnum, len(steps))
    o.keygen(rnd, rot_steps=steps)
    rng = np.random.default_rng(prm.p)
    E = random_fpd(rng, p, N)
    r = synth.encrypt_randomness(42, 1, N)
    ct = o.encrypt_poly(oracle.encode_fpd(E, p, N), r["u"][0], r["e"][0])
    d = oracle.fpd_degree(p, N)
    ev = CtEvaluator(o)
    for k in sorted({0, 1, d // 2 + 1, d - 1}):
        z = oracle.extract_digit(ev, o, ct, k, p)
        assert z.level == ct.level
        assert np.array_equal(o.decrypt(z), E[:, k]), k
        # the result is an ordinary slot encoding: nothing off the multiples of d
        poly = o.decrypt_poly(z)
        assert not np.delete(poly, np.arange(0, N, d)).any(), k


def test_extract_digit_planted_mistakes_fail():
    """A wrong sign of the monomial or one doubling short leaves other
    coordinates mixed in: the check above would catch either."""
    p, N = 17, 1 << 10
    rng = np.random.default_rng(5)
    E = random_fpd(rng, p, N)
    m = oracle.encode_fpd(E, p, N).astype(np.int64)
    d = oracle.fpd_degree(p, N)

    def plain_extract(m, k, shift_sign, nsteps):
        xk = np.zeros(N, np.int64)
        e = (shift_sign * k) % (2 * N)
        xk[e % N] = 1 if e < N else p - 1
        z = negacyclic_mod_p(m, xk, N, p)
        for r in oracle.frobenius_steps(p, N)[:nsteps]:
            z = (z + oracle.plain_automorphism(z, oracle.galois_element(r, N), N, p)) % p
        return oracle.decode_poly(z * pow(d, -1, p) % p, p, N)

    t = len(oracle.frobenius_steps(p, N))
    assert np.array_equal(plain_extract(m, 3, -1, t), E[:, 3])
    assert not np.array_equal(plain_extract(m, 3, +1, t), E[:, 3])
    assert not np.array_equal(plain_extract(m, 3, -1, t - 1), E[:, 3])
