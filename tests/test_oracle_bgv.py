"""Pins of the oracle's BGV operations.

Each operation is checked against what BGV fixes mathematically (Background,
"Word-wise Universal FHE Scheme": ciphertexts over R_Q x R_Q that decrypt
through [c0 + c1 s]_Q mod p, with addition, multiplication and rotation acting
slot-wise): decryptions equal the plaintext operation, exact divisibility of
the base conversions checked with Python big integers, and noise bounds.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import Ct, Oracle, Params

TINY = {
    "p17": Params(5, 17, 6, 36, 1, 60, 3),
    "p17_alpha1": Params(4, 17, 5, 36, 1, 60, 5),
    "p257": Params(7, 257, 8, 50, 3, 60, 2),
    "p257_d3": Params(7, 257, 7, 50, 4, 60, 3),
}


def setup(name, rot=(1,), seed=11):
    prm = TINY[name]
    o = Oracle(prm)
    o.keygen(synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(rot)), rot_steps=rot)
    return o


def enc(o, vals, seed, idx=0):
    r = synth.encrypt_randomness(seed, idx + 1, o.N)
    return o.encrypt(vals, r["u"][idx], r["e"][idx])


def rand_slots(o, seed, lo=0, hi=None, index=0):
    return synth.slot_values(seed, 1, o.M, lo, o.p if hi is None else hi, index)[0].astype(np.int64)


@pytest.fixture(scope="module", params=sorted(TINY))
def ctx(request):
    return setup(request.param)


def test_fresh_round_trip_and_noise(ctx):
    o = ctx
    v = rand_slots(o, 1)
    c = enc(o, v, 2)
    assert np.array_equal(o.decrypt(c), v)
    # fresh noise: |m + p(e u' ...)| <= p (|e0| + |e|*|u|_1 + ...) ~ p * 19 * (2N + 1) + p
    bound = o.p * 19 * (2 * o.N + 2)
    assert o.noise_bits(c) <= math.log2(bound)
    poly = o.decrypt_poly(c)
    d = o.N // o.M
    assert not np.any(np.delete(poly, np.arange(0, o.N, d)))


def test_add_sub_scalar_const(ctx):
    o = ctx
    u, v = rand_slots(o, 3), rand_slots(o, 4)
    cu, cv = enc(o, u, 5, 0), enc(o, v, 5, 1)
    p = o.p
    assert np.array_equal(o.decrypt(o.add(cu, cv)), (u + v) % p)
    assert np.array_equal(o.decrypt(o.sub(cu, cv)), (u - v) % p)
    for c in (0, 1, p - 1, (p - 1) // 2, (p + 1) // 2, 7):
        assert np.array_equal(o.decrypt(o.mul_scalar(cu, c)), (u * c) % p)
        assert np.array_equal(o.decrypt(o.add_const(cu, c)), (u + c) % p)


def _crt(o, res, level):
    return o.crt_centred(res, level)


def test_tensor_decrypts_to_product_with_s_squared(ctx):
    o = ctx
    u, v = rand_slots(o, 6), rand_slots(o, 7)
    cu, cv = enc(o, u, 8, 0), enc(o, v, 8, 1)
    t = o.tensor(cu, cv)
    assert t.ncomp == 3
    assert np.array_equal(o.decrypt(t), (u * v) % o.p)


def test_relin_keeps_plaintext_and_is_a_key_switch(ctx):
    o = ctx
    u, v = rand_slots(o, 9), rand_slots(o, 10)
    t = o.tensor(enc(o, u, 11, 0), enc(o, v, 11, 1))
    r = o.relin(t)
    assert r.ncomp == 2 and r.level == t.level
    assert np.array_equal(o.decrypt(r), (u * v) % o.p)
    # ks0 + ks1 s - d2 s^2 is small compared with Q: a genuine key switch
    d2 = t.data[2]
    ks = o.key_switch(o.keys["rlk"], d2, t.level)
    lv = t.level
    diff = np.zeros((lv + 1, o.N), np.uint64)
    for i in range(lv + 1):
        q = o.moduli[i]
        s = o.keys["sk"][i]
        s2 = o.negacyclic_mul(i, s, s)
        ks1s = o.negacyclic_mul(i, ks[1, i], s)
        d2s2 = o.negacyclic_mul(i, d2[i], s2)
        diff[i] = ((ks[0, i].astype(object) + ks1s.astype(object) - d2s2.astype(object)) % q).astype(np.uint64)
    vals = _crt(o, diff, lv)
    Q = math.prod(o.q[: lv + 1])
    noise = max(abs(x) for x in vals)
    assert noise < Q >> 40
    assert all(x % o.p == 0 for x in vals)  # the switching noise is a multiple of p


def test_mul_relin_and_modswitch_levels(ctx):
    o = ctx
    u, v, w = rand_slots(o, 12), rand_slots(o, 13), rand_slots(o, 14)
    cu, cv, cw = enc(o, u, 15, 0), enc(o, v, 15, 1), enc(o, w, 15, 2)
    top = o.prm.nQ - 1
    m1 = o.mul(cu, cv)
    assert m1.level == top - 1
    assert np.array_equal(o.decrypt(m1), (u * v) % o.p)
    m2 = o.mul(m1, cw)  # operands at different levels: cw is switched down
    assert m2.level == top - 2
    assert np.array_equal(o.decrypt(m2), (u * v * w) % o.p)


def test_mul_add_levels_and_values(ctx):
    """a b + c with the addition before the product's switch: one level
    below the lower of the tensor and the addend, decrypting to the slotwise
    a b + c, whichever operand sits higher."""
    o = ctx
    u, v, w = rand_slots(o, 18), rand_slots(o, 19), rand_slots(o, 20)
    cu, cv, cw = enc(o, u, 21, 0), enc(o, v, 21, 1), enc(o, w, 21, 2)
    top = o.prm.nQ - 1
    m = o.mul_add(cu, cv, cw)
    assert m.level == top - 1
    assert np.array_equal(o.decrypt(m), (u * v + w) % o.p)
    m1 = o.mul(cu, cv)
    hi = o.mul_add(m1, cw, cu)  # addend above the tensor: switched down to it
    assert hi.level == top - 2
    assert np.array_equal(o.decrypt(hi), (u * v * w + u) % o.p)
    lo = o.mul_add(cu, cv, m1)  # addend below the tensor: the tensor is switched down
    assert lo.level == top - 2
    assert np.array_equal(o.decrypt(lo), (2 * u * v) % o.p)
    assert o.budget_bits(m) >= o.budget_bits(o.add(cw, o.mul(cu, cv))) - 1


def test_to_level_drops_primes(ctx):
    """Level alignment keeps the residues modulo the remaining primes: the
    same plaintext at every lower level, with the noise budget of the smaller
    modulus (a product's noise sits at the switching floor)."""
    o = ctx
    u, v = rand_slots(o, 22), rand_slots(o, 23)
    m = o.mul(enc(o, u, 24, 0), enc(o, v, 24, 1))
    for lv in range(m.level - 1, -1, -1):
        d = o.to_level(m, lv)
        assert d.level == lv and d.data.shape[1] == lv + 1
        assert np.array_equal(o.decrypt(d), (u * v) % o.p)
        if lv > 0:
            assert o.budget_bits(d) > 10


def test_mod_switch_exact_division(ctx):
    """c' q_l = c - p t exactly, with t = [c_l p^-1]_{q_l} in (-q_l/2, q_l/2]."""
    o = ctx
    c = enc(o, rand_slots(o, 16), 17)
    lv = c.level
    ql = o.q[lv]
    s = o.mod_switch(c)
    assert s.level == lv - 1
    Qlo = math.prod(o.q[:lv])
    for comp in range(2):
        for n in range(0, o.N, 3):
            full = _big(o, [int(c.data[comp, i, n]) for i in range(lv + 1)], o.q[: lv + 1])
            low = _big(o, [int(s.data[comp, i, n]) for i in range(lv)], o.q[:lv])
            # D = c - q_l c' must be p t with t = c_l p^-1 mod q_l, |t| <= q_l/2 (mod Q_{l-1})
            D = (full - ql * low) % Qlo
            if D > Qlo // 2:
                D -= Qlo
            assert D % o.p == 0
            t = D // o.p
            assert abs(t) <= ql // 2
            assert t % ql == int(c.data[comp, lv, n]) * pow(o.p, ql - 2, ql) % ql
    assert np.array_equal(o.decrypt(s), o.decrypt(c))
    # |[c0' + c1' s]| <= |[c0 + c1 s]| / q_l + p (N + 1) / 2  (rounding term p(t0 + t1 s)/q_l)
    bound = 2 ** o.noise_bits(c) / ql + o.p * (o.N + 1) / 2
    assert o.noise_bits(s) <= math.log2(bound) + 1e-9


def _big(o, res, mods):
    Q = math.prod(mods)
    x = 0
    for r, q in zip(res, mods):
        qh = Q // q
        x += r * qh * pow(qh % q, q - 2, q)
    return x % Q


def test_modup_is_fast_base_conversion(ctx):
    """u_m = X + k Q_j (mod q_m) for one k in [0, alpha) per coefficient, where
    X in [0, Q_j) is the digit's CRT value; digit limbs are copied exactly."""
    o = ctx
    rng = np.random.default_rng(18)
    for lv in (o.prm.nQ - 1, o.prm.nQ // 2):
        x = np.stack([rng.integers(0, q, o.N, dtype=np.uint64) for q in o.q[: lv + 1]])
        ext = list(o.q[: lv + 1]) + o.special
        for j in range(o.prm.dnum):
            lo, hi = j * o.alpha, min((j + 1) * o.alpha, o.prm.nQ, lv + 1)
            if lo >= hi:
                continue
            u = o.modup(x, lv, j)
            Qj = math.prod(o.q[lo:hi])
            for n in range(0, o.N, 5):
                X = _big(o, [int(x[i, n]) for i in range(lo, hi)], o.q[lo:hi])
                ks = set()
                for e, m in enumerate(ext):
                    if lo <= e < hi:
                        assert u[e, n] == x[e, n]
                        continue
                    cands = [k for k in range(hi - lo) if (X + k * Qj) % m == int(u[e, n])]
                    assert len(cands) == 1
                    ks.add(cands[0])
                assert len(ks) == 1


@pytest.mark.parametrize("sign", [1, -1])
def test_moddown_divides_by_p_exactly(ctx, sign):
    """acc = P Y + p e (mod Q_l P) maps to Y - k p (mod Q_l) with 0 <= k < nP
    (k = 0 or the wrap of the representative sum): the exact division by P that
    keeps the plaintext."""
    o = ctx
    rng = np.random.default_rng(19 if sign > 0 else 20)
    lv = o.prm.nQ - 1
    Ql = math.prod(o.q[: lv + 1])
    P = math.prod(o.special)
    mods = list(o.q[: lv + 1]) + o.special
    nP = o.prm.nP
    Ys = [int(rng.integers(0, 2**62)) * int(rng.integers(0, 2**62)) % Ql for _ in range(o.N)]
    es = [sign * int(rng.integers(0, 50)) for _ in range(o.N)]
    acc = np.zeros((len(mods), o.N), np.uint64)
    for n in range(o.N):
        A = (P * Ys[n] + o.p * es[n]) % (Ql * P)
        for e, m in enumerate(mods):
            acc[e, n] = A % m
    out = o.moddown(acc, lv)
    for n in range(o.N):
        got = _big(o, [int(out[i, n]) for i in range(lv + 1)], o.q[: lv + 1])
        k = ((Ys[n] - got) % Ql)
        assert k % o.p == 0 and 0 <= k // o.p < nP + (1 if sign < 0 else 0), (n, k)


def test_rotation_decrypts_rotated_and_composes(ctx):
    o = setup(next(k for k, v in TINY.items() if v == ctx.prm), rot=(1, 2, -1))
    v = rand_slots(o, 21)
    c = enc(o, v, 22)
    h = o.M // 2
    r1 = o.rotate(c, 1)
    assert np.array_equal(o.decrypt(r1), np.concatenate([np.roll(v[:h], -1), np.roll(v[h:], -1)]))
    r11 = o.rotate(r1, 1)
    assert np.array_equal(o.decrypt(r11), o.decrypt(o.rotate(c, 2)))
    sw = o.rotate(c, -1)
    assert np.array_equal(o.decrypt(sw), np.concatenate([v[h:], v[:h]]))
    assert r1.level == c.level


def test_automorphism_is_ring_homomorphism():
    o = setup("p17")
    rng = np.random.default_rng(23)
    g = oracle.galois_element(1, o.N)
    q = o.q[0]
    a = rng.integers(0, q, o.N, dtype=np.uint64)
    b = rng.integers(0, q, o.N, dtype=np.uint64)
    ca = Ct(np.stack([a[None], a[None]]).reshape(2, 1, o.N).copy(), 0)
    cb = Ct(np.stack([b[None], b[None]]).reshape(2, 1, o.N).copy(), 0)
    ab = o.negacyclic_mul(0, a, b)
    cab = Ct(np.stack([ab, ab]).reshape(2, 1, o.N).copy(), 0)
    sa = o.automorphism(ca, g).data[0, 0]
    sb = o.automorphism(cb, g).data[0, 0]
    assert np.array_equal(o.automorphism(cab, g).data[0, 0], o.negacyclic_mul(0, sa, sb))


def test_key_material_shapes_and_secret_is_ternary():
    o = setup("p257")
    sk = o.keys["sk"]
    for i, q in enumerate(o.moduli):
        assert set(np.unique(sk[i]).tolist()) <= {0, 1, q - 1}
    # pk0 + pk1 s = p e (small, a multiple of p)
    pk = o.keys["pk"]
    res = np.zeros((o.prm.nQ, o.N), np.uint64)
    for i, q in enumerate(o.q):
        t = o.negacyclic_mul(i, pk[1, i], sk[i])
        res[i] = ((pk[0, i].astype(object) + t.astype(object)) % q).astype(np.uint64)
    vals = o.crt_centred(res, o.prm.nQ - 1)
    assert all(v % o.p == 0 and abs(v) <= o.p * 19 for v in vals)


def test_encryption_uses_the_given_randomness():
    """c1 - pk1 u = p e1 and c0 - pk0 u - m = p e0 limb by limb (public-key
    encryption with randomness (u, e0, e1))."""
    o = setup("p17")
    r = synth.encrypt_randomness(50, 1, o.N)
    v = rand_slots(o, 51)
    m = oracle.encode_poly(v, o.p, o.N)
    c = o.encrypt_poly(m, r["u"][0], r["e"][0])
    pk = o.keys["pk"]
    for i, q in enumerate(o.q):
        u = np.array([int(x) % q for x in r["u"][0]], dtype=np.uint64)
        for comp, extra in ((0, m.astype(object)), (1, 0)):
            t = o.negacyclic_mul(i, pk[comp, i], u).astype(object)
            d = (c.data[comp, i].astype(object) - t - extra) % q
            e = r["e"][0][comp].astype(object) * o.p % q
            assert np.array_equal(d, e)
