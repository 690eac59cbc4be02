"""CPU oracle for the BGV less-than hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the device library and never
imports it; the two meet only through the seeded inputs of ``synth``.

Layers:
  * ``bgv_oracle.c`` (built into ``liboracle.so``): plain residue arithmetic,
    textbook NTT products, key switching, modulus switching, automorphisms.
  * this module: parameters, Python big-integer CRT decryption, the slot
    encoding, and the comparison circuits written on top of the C ops.

Paper passages followed: BGV ciphertexts, RNS residue matrices and the NTT
(Background, "Word-wise Universal FHE Scheme" and "Efficient Polynomial and
NTT"); digit-wise LT/EQ combined in lexicographic order (same section, the
comparison paragraph); the univariate circuit and its sqrt(p-3)+O(log p)
non-scalar multiplication count (Introduction).  The paper prints no LT
polynomial, prime choice or representative convention; the reading used is
restated at each function.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, OpenMP over limbs)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "bgv_oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        V, P, I, L, U = ctypes.c_void_p, u64p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "or_mulmod": (U, [U, U, U]),
            "or_powmod": (U, [U, U, U]),
            "or_invmod": (U, [U, U]),
            "or_is_prime": (I, [U]),
            "or_gen_primes": (I, [U, I, I, P, I, P]),
            "or_find_psi": (U, [U, I]),
            "or_ctx_new": (V, [I, U, I, I, I, I, I]),
            "or_ctx_free": (None, [V]),
            "or_ctx_nmod": (I, [V]),
            "or_ctx_moduli": (None, [V, P]),
            "or_ctx_psi": (U, [V, I]),
            "or_ntt_forward": (None, [V, I, P]),
            "or_ntt_inverse": (None, [V, I, P]),
            "or_negacyclic_mul": (None, [V, I, P, P, P]),
            "or_schoolbook_negacyclic": (None, [P, P, P, I, U]),
            "or_keygen": (None, [V, V, P, V, i64p, I, P, P, P, P]),
            "or_encrypt": (None, [V, P, V, V, V, V, P]),
            "or_decrypt_residues": (None, [V, P, P, I, I, P]),
            "or_add": (None, [V, P, P, I, I, P]),
            "or_sub": (None, [V, P, P, I, I, P]),
            "or_mul_scalar": (None, [V, P, I, I, L, P]),
            "or_add_const": (None, [V, P, I, I, L, P]),
            "or_tensor": (None, [V, P, P, I, P]),
            "or_mod_switch": (None, [V, P, I, I, P]),
            "or_modup": (None, [V, P, I, I, P]),
            "or_moddown": (None, [V, P, I, P]),
            "or_key_switch": (None, [V, P, P, I, P]),
            "or_relin": (None, [V, P, P, I, P]),
            "or_automorphism": (None, [V, P, I, I, L, P]),
            "or_rotate": (None, [V, P, P, I, L, P]),
            "or_find_root_m": (U, [U, U]),
            "or_poly_eval": (None, [P, I, P, I, U, P]),
            "or_poly_mod_monic": (None, [P, I, i64p, I, U, P]),
            "or_cyclo_mul": (None, [P, P, I, i64p, U, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def lib():
    return _load()


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(u64p)


def _v(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# number theory helpers (plain Python, used by tests and the encoding)
# ---------------------------------------------------------------------------

def primitive_root(p: int) -> int:
    """Least primitive root of the prime p (trial over the factors of p-1)."""
    phi = p - 1
    fac, n, f = [], phi, 2
    while f * f <= n:
        if n % f == 0:
            fac.append(f)
            while n % f == 0:
                n //= f
        f += 1
    if n > 1:
        fac.append(n)
    for g in range(2, p):
        if all(pow(g, phi // f, p) != 1 for f in fac):
            return g
    raise ValueError(p)


def slot_count(p: int) -> int:
    """M = 2^(s-1) where 2^s exactly divides p-1: x^N+1 splits over F_p into M
    factors x^d - zeta (zeta^M = -1), giving M slots when M <= N."""
    s = ((p - 1) & -(p - 1)).bit_length() - 1
    return 1 << (s - 1)


def slot_roots(p: int, M: int) -> list[int]:
    """zeta_j: slot j < M/2 <-> zeta^(5^j), slot M/2 + j <-> zeta^(-5^j), with
    zeta = g^((p-1)/2M) for g the least primitive root mod p."""
    g = primitive_root(p)
    zeta = pow(g, (p - 1) // (2 * M), p)
    roots = []
    for j in range(M):
        if j < M // 2:
            e = pow(5, j, 2 * M)
        else:
            e = (-pow(5, j - M // 2, 2 * M)) % (2 * M)
        roots.append(pow(zeta, e, p))
    return roots


def decode_poly(m: np.ndarray, p: int, N: int) -> np.ndarray:
    """Slots of the plaintext m(x) = mu(x^d): v_j = mu(zeta_j) mod p."""
    M = slot_count(p)
    d = N // M
    mu = [int(m[k * d]) % p for k in range(M)]
    out = np.zeros(M, dtype=np.uint32)
    for j, z in enumerate(slot_roots(p, M)):
        acc, zk = 0, 1
        for k in range(M):
            acc = (acc + mu[k] * zk) % p
            zk = zk * z % p
        out[j] = acc
    return out


def encode_poly(v, p: int, N: int) -> np.ndarray:
    """Inverse of ``decode_poly``: mu_k = M^-1 sum_j v_j zeta_j^-k (the zeta_j are
    the M distinct roots of t^M + 1, so the evaluation matrix is orthogonal up to
    the factor M); m has coefficient mu_k at x^(k d) and zero elsewhere."""
    M = slot_count(p)
    d = N // M
    roots = slot_roots(p, M)
    minv = pow(M, p - 2, p)
    out = np.zeros(N, dtype=np.uint32)
    for k in range(M):
        acc = 0
        for j, z in enumerate(roots):
            acc = (acc + int(v[j]) * pow(z, (p - 1 - k) % (p - 1), p)) % p
        out[k * d] = acc * minv % p
    return out


def galois_element(step: int, N: int) -> int:
    """Rotation by ``step`` slots: g = 5^step mod 2N; step -1 means the row swap g = 2N-1."""
    if step == -1:
        return 2 * N - 1
    return pow(5, step, 2 * N)


# ---------------------------------------------------------------------------
# parameters and context
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Params:
    logN: int
    p: int
    nQ: int
    bitsQ: int
    nP: int
    bitsP: int
    dnum: int

    @property
    def N(self) -> int:
        return 1 << self.logN


# Parameter sets of the workloads.  Readings: four 36-bit primes for the N=2^12
# case because a depth-four circuit does not fit in three; for the p=257
# chains as many 50-bit special primes as one digit has primes (P no smaller
# than a digit's modulus), because fewer leave key-switching noise far above
# the modulus.  Every prime stays below 2^50.
PARAMS = {
    "n12_p17": Params(12, 17, 4, 36, 1, 50, 4),
    "n13_p257": Params(13, 257, 8, 50, 4, 50, 2),
    "n14_p257": Params(14, 257, 8, 50, 4, 50, 2),
    "n15_p257": Params(15, 257, 14, 50, 5, 50, 3),
}


@dataclass
class Ct:
    data: np.ndarray  # uint64 [ncomp][level+1][N], coefficient domain
    level: int

    @property
    def ncomp(self) -> int:
        return self.data.shape[0]


class Oracle:
    def __init__(self, prm: Params):
        self.prm = prm
        self.lib = _load()
        self.ctx = self.lib.or_ctx_new(prm.logN, prm.p, prm.nQ, prm.bitsQ, prm.nP, prm.bitsP, prm.dnum)
        if not self.ctx:
            raise ValueError(f"oracle: cannot build parameters {prm}")
        n = self.lib.or_ctx_nmod(self.ctx)
        mods = np.zeros(n, dtype=np.uint64)
        self.lib.or_ctx_moduli(self.ctx, _p(mods))
        self.moduli = [int(x) for x in mods]
        self.q = self.moduli[: prm.nQ]
        self.special = self.moduli[prm.nQ:]
        self.N = prm.N
        self.p = prm.p
        self.M = slot_count(prm.p)
        self.alpha = -(-prm.nQ // prm.dnum)
        self.keys = None

    def __del__(self):
        if getattr(self, "ctx", None) and self.lib is not None:
            self.lib.or_ctx_free(self.ctx)
            self.ctx = None

    # ---------------- keys ----------------
    def keygen(self, rnd: dict, rot_steps=()):
        """Keys from the synth randomness (secret, pk, relin key, rotation keys)."""
        prm, N = self.prm, self.N
        nm = len(self.moduli)
        gal = np.array([galois_element(r, N) for r in rot_steps], dtype=np.int64)
        s = np.ascontiguousarray(rnd["s"], dtype=np.int8)
        a = np.ascontiguousarray(rnd["a"], dtype=np.uint64)
        e = np.ascontiguousarray(rnd["e"], dtype=np.int32)
        need_a = prm.nQ * N + (1 + len(gal)) * prm.dnum * nm * N
        need_e = N + (1 + len(gal)) * prm.dnum * N
        assert a.size == need_a and e.size == need_e, (a.size, need_a, e.size, need_e)
        sk = np.zeros((nm, N), np.uint64)
        pk = np.zeros((2, prm.nQ, N), np.uint64)
        rlk = np.zeros((prm.dnum, 2, nm, N), np.uint64)
        gk = np.zeros((max(len(gal), 1), prm.dnum, 2, nm, N), np.uint64)
        self.lib.or_keygen(self.ctx, _v(s), _p(a), _v(e), gal.ctypes.data_as(i64p), len(gal),
                           _p(sk), _p(pk), _p(rlk), _p(gk))
        self.keys = {"sk": sk, "s": s, "pk": pk, "rlk": rlk,
                     "gk": {int(r): gk[i] for i, r in enumerate(rot_steps)}}
        return self.keys

    # ---------------- encryption ----------------
    def encrypt_poly(self, m: np.ndarray, u: np.ndarray, e: np.ndarray) -> Ct:
        N, nQ = self.N, self.prm.nQ
        out = np.zeros((2, nQ, N), np.uint64)
        m = np.ascontiguousarray(m, dtype=np.uint32)
        u = np.ascontiguousarray(u, dtype=np.int8)
        e0 = np.ascontiguousarray(e[0], dtype=np.int32)
        e1 = np.ascontiguousarray(e[1], dtype=np.int32)
        self.lib.or_encrypt(self.ctx, _p(self.keys["pk"]), _v(m), _v(u), _v(e0), _v(e1), _p(out))
        return Ct(out, nQ - 1)

    def encrypt(self, slots, u, e) -> Ct:
        return self.encrypt_poly(encode_poly(slots, self.p, self.N), u, e)

    def decrypt_residues(self, ct: Ct) -> np.ndarray:
        out = np.zeros((ct.level + 1, self.N), np.uint64)
        self.lib.or_decrypt_residues(self.ctx, _p(self.keys["sk"]), _p(np.ascontiguousarray(ct.data)),
                                     ct.level, ct.ncomp, _p(out))
        return out

    def crt_centred(self, res: np.ndarray, level: int) -> list[int]:
        """Integer in (-Q/2, Q/2] with the given residues: sum_i r_i Qhat_i [Qhat_i^-1]_{q_i} mod Q."""
        qs = self.q[: level + 1]
        Q = math.prod(qs)
        terms = []
        for i, q in enumerate(qs):
            qh = Q // q
            terms.append((qh * pow(qh % q, q - 2, q), q))
        out = []
        for n in range(self.N):
            x = sum(int(res[i, n]) * t for i, (t, _) in enumerate(terms)) % Q
            if x > Q // 2:
                x -= Q
            out.append(x)
        return out

    def decrypt_poly(self, ct: Ct) -> np.ndarray:
        vals = self.crt_centred(self.decrypt_residues(ct), ct.level)
        return np.array([v % self.p for v in vals], dtype=np.uint32)

    def decrypt(self, ct: Ct) -> np.ndarray:
        return decode_poly(self.decrypt_poly(ct), self.p, self.N)

    def noise_bits(self, ct: Ct) -> float:
        """log2 of the largest |[c0 + c1 s]_Q| coefficient (noise plus message)."""
        vals = self.crt_centred(self.decrypt_residues(ct), ct.level)
        return math.log2(max(1, max(abs(v) for v in vals)))

    def budget_bits(self, ct: Ct) -> float:
        Q = math.prod(self.q[: ct.level + 1])
        return math.log2(Q / 2) - self.noise_bits(ct)

    # ---------------- elementary ops ----------------
    def _new(self, ncomp, level):
        return np.zeros((ncomp, level + 1, self.N), np.uint64)

    def mod_switch(self, ct: Ct) -> Ct:
        assert ct.level > 0
        out = self._new(ct.ncomp, ct.level - 1)
        self.lib.or_mod_switch(self.ctx, _p(ct.data), ct.level, ct.ncomp, _p(out))
        return Ct(out, ct.level - 1)

    def to_level(self, ct: Ct, level: int) -> Ct:
        """ct brought down to `level` for level alignment by dropping its top
        primes: the residues modulo the smaller modulus, no rescaling.  It
        decrypts to the same plaintext while its noise is below half the
        smaller modulus; the operands aligned in the circuit carry noise near
        the modulus-switching floor, where switching would not lower it."""
        assert level <= ct.level
        if ct.level == level:
            return ct
        return Ct(np.ascontiguousarray(ct.data[:, : level + 1]), level)

    def align(self, a: Ct, b: Ct):
        lv = min(a.level, b.level)
        return self.to_level(a, lv), self.to_level(b, lv)

    def add(self, a: Ct, b: Ct) -> Ct:
        a, b = self.align(a, b)
        out = self._new(a.ncomp, a.level)
        self.lib.or_add(self.ctx, _p(a.data), _p(b.data), a.level, a.ncomp, _p(out))
        return Ct(out, a.level)

    def sub(self, a: Ct, b: Ct) -> Ct:
        a, b = self.align(a, b)
        out = self._new(a.ncomp, a.level)
        self.lib.or_sub(self.ctx, _p(a.data), _p(b.data), a.level, a.ncomp, _p(out))
        return Ct(out, a.level)

    def centred(self, c: int) -> int:
        c %= self.p
        return c - self.p if c > (self.p - 1) // 2 else c

    def mul_scalar(self, a: Ct, c: int) -> Ct:
        """Multiply by the centred representative of c in Z_p."""
        out = self._new(a.ncomp, a.level)
        self.lib.or_mul_scalar(self.ctx, _p(a.data), a.level, a.ncomp, self.centred(c), _p(out))
        return Ct(out, a.level)

    def add_const(self, a: Ct, c: int) -> Ct:
        """Add the constant c (all slots) as its centred representative on x^0 of c0."""
        out = self._new(a.ncomp, a.level)
        self.lib.or_add_const(self.ctx, _p(a.data), a.level, a.ncomp, self.centred(c), _p(out))
        return Ct(out, a.level)

    def tensor(self, a: Ct, b: Ct) -> Ct:
        a, b = self.align(a, b)
        out = self._new(3, a.level)
        self.lib.or_tensor(self.ctx, _p(a.data), _p(b.data), a.level, _p(out))
        return Ct(out, a.level)

    def relin(self, ct3: Ct) -> Ct:
        out = self._new(2, ct3.level)
        self.lib.or_relin(self.ctx, _p(self.keys["rlk"]), _p(ct3.data), ct3.level, _p(out))
        return Ct(out, ct3.level)

    def mul(self, a: Ct, b: Ct) -> Ct:
        """Align, tensor, relinearise, then drop one prime unless at level 0."""
        r = self.relin(self.tensor(a, b))
        return self.mod_switch(r) if r.level > 0 else r

    def mul_add(self, a: Ct, b: Ct, c: Ct) -> Ct:
        """a b + c with the addition before the product's relinearisation and
        modulus switch: tensor a and b, bring the tensor and c to their lower
        level, add c to the first two components, relinearise, then drop one
        prime unless at level 0 (one switch for the sum instead of one for the
        product and another for c)."""
        t = self.tensor(a, b)
        lv = min(t.level, c.level)
        t, c = self.to_level(t, lv), self.to_level(c, lv)
        d01 = np.ascontiguousarray(t.data[:2])
        s = self._new(2, lv)
        self.lib.or_add(self.ctx, _p(d01), _p(c.data), lv, 2, _p(s))
        t3 = np.concatenate([s, t.data[2:]], axis=0)
        r = self.relin(Ct(t3, lv))
        return self.mod_switch(r) if r.level > 0 else r

    def modup(self, x: np.ndarray, level: int, digit: int) -> np.ndarray:
        out = np.zeros((level + 1 + self.prm.nP, self.N), np.uint64)
        self.lib.or_modup(self.ctx, _p(np.ascontiguousarray(x)), level, digit, _p(out))
        return out

    def moddown(self, acc: np.ndarray, level: int) -> np.ndarray:
        out = np.zeros((level + 1, self.N), np.uint64)
        self.lib.or_moddown(self.ctx, _p(np.ascontiguousarray(acc)), level, _p(out))
        return out

    def key_switch(self, ksk: np.ndarray, d: np.ndarray, level: int) -> np.ndarray:
        out = np.zeros((2, level + 1, self.N), np.uint64)
        self.lib.or_key_switch(self.ctx, _p(ksk), _p(np.ascontiguousarray(d)), level, _p(out))
        return out

    def automorphism(self, ct: Ct, g: int) -> Ct:
        out = self._new(ct.ncomp, ct.level)
        self.lib.or_automorphism(self.ctx, _p(ct.data), ct.level, ct.ncomp, g, _p(out))
        return Ct(out, ct.level)

    def rotate(self, ct: Ct, step: int) -> Ct:
        g = galois_element(step, self.N)
        out = self._new(2, ct.level)
        self.lib.or_rotate(self.ctx, _p(self.keys["gk"][step]), _p(ct.data), ct.level, g, _p(out))
        return Ct(out, ct.level)

    def mul_monomial(self, ct: Ct, e: int) -> Ct:
        """ct times the monomial x^e (any integer e; x^N = -1): every
        coefficient a_i of every component and limb moves to x^(i+e), negated
        when i + e wraps past N an odd number of times.  No noise growth."""
        N = self.N
        idx = (np.arange(N, dtype=np.int64) + e) % (2 * N)
        pos, neg = idx % N, idx >= N
        out = np.zeros_like(ct.data)
        for i in range(ct.level + 1):
            q = np.uint64(self.q[i])
            a = ct.data[:, i, :]
            out[:, i, pos] = np.where(neg, (q - a) % q, a)
        return Ct(out, ct.level)

    def negacyclic_mul(self, prime: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        out = np.zeros(self.N, np.uint64)
        self.lib.or_negacyclic_mul(self.ctx, prime, _p(np.ascontiguousarray(a, np.uint64)),
                                   _p(np.ascontiguousarray(b, np.uint64)), _p(out))
        return out


# ---------------------------------------------------------------------------
# the comparison circuit (Introduction: univariate circuit; Background:
# digit-wise LT/EQ combined lexicographically)
# ---------------------------------------------------------------------------

@lru_cache(maxsize=None)
def _lt_coefficients(p: int) -> tuple:
    """Coefficients c_0..c_{p-1} of the degree p-1 polynomial f over F_p with
    f(z) = 1 for z in [(p+1)/2, p-1] and 0 elsewhere (so f(x - y) = [x < y] for
    x, y in [0, (p-1)/2]).  Interpolating the indicator with (z-a)^(p-1) gives
    c_k = sum_{b=1}^{(p-1)/2} b^(p-1-k) for odd k, c_{p-1} = (p+1)/2, and zero for
    the even k (the half power sums vanish)."""
    c = [0] * p
    h = (p - 1) // 2
    for k in range(1, p - 1, 2):
        c[k] = sum(pow(b, p - 1 - k, p) for b in range(1, h + 1)) % p
    c[p - 1] = (p + 1) // 2
    return tuple(c)


def lt_coefficients(p: int) -> list[int]:
    return list(_lt_coefficients(p))


class IntEvaluator:
    """Plain Z_p arithmetic with the evaluator interface (for checking schedules)."""

    def __init__(self, p):
        self.p = p
        self.mults = 0

    def mul(self, a, b):
        self.mults += 1
        return a * b % self.p

    def mul_add(self, a, b, c):
        self.mults += 1
        return (a * b + c) % self.p

    def add(self, a, b):
        return (a + b) % self.p

    def sub(self, a, b):
        return (a - b) % self.p

    def mul_scalar(self, a, c):
        return a * c % self.p

    def add_const(self, a, c):
        return (a + c) % self.p

    def level(self, a):
        return 0

    def to_level(self, a, lv):
        return a


class CtEvaluator:
    """Evaluator over oracle ciphertexts."""

    def __init__(self, orc: Oracle):
        self.o = orc
        self.mults = 0

    def mul(self, a, b):
        self.mults += 1
        return self.o.mul(a, b)

    def mul_add(self, a, b, c):
        self.mults += 1
        return self.o.mul_add(a, b, c)

    def add(self, a, b):
        return self.o.add(a, b)

    def sub(self, a, b):
        return self.o.sub(a, b)

    def mul_scalar(self, a, c):
        return self.o.mul_scalar(a, c)

    def add_const(self, a, c):
        return self.o.add_const(a, c)

    def level(self, a):
        return a.level

    def to_level(self, a, lv):
        return self.o.to_level(a, lv)

    def rotate(self, a, step):
        return self.o.rotate(a, step)


class SlotEvaluator:
    """Plain slot vectors over F_p with the evaluator interface: M values,
    two rows of M/2 slots, rotate(x, s)[j] = x[j + s] within the row (what the
    automorphism x -> x^(5^s) does to the slots, see ``slot_roots``).  For
    checking the slot-packed schedules without encryption."""

    def __init__(self, p, M):
        self.p, self.M = p, M
        self.mults = 0
        self.rotations = 0
        self.depth_of = {}

    def _arr(self, a):
        return np.asarray(a, dtype=np.int64) % self.p

    def mul(self, a, b):
        self.mults += 1
        return self._arr(a) * self._arr(b) % self.p

    def mul_add(self, a, b, c):
        self.mults += 1
        return (self._arr(a) * self._arr(b) + self._arr(c)) % self.p

    def add(self, a, b):
        return (self._arr(a) + self._arr(b)) % self.p

    def sub(self, a, b):
        return (self._arr(a) - self._arr(b)) % self.p

    def mul_scalar(self, a, c):
        return self._arr(a) * c % self.p

    def add_const(self, a, c):
        return (self._arr(a) + c) % self.p

    def level(self, a):
        return 0

    def to_level(self, a, lv):
        return a

    def rotate(self, a, step):
        self.rotations += 1
        h = self.M // 2
        x = self._arr(a).reshape(2, h)
        return np.roll(x, -step, axis=1).reshape(-1)


def lt_univariate(ev, Z, p: int):
    """Paterson-Stockmeyer evaluation of f(Z) for p - 1 = 2^e (p = 17, 257).

    Baby steps Z^k for odd k < b (b = 2^ceil(e/2)) from the squares
    Z^2, ..., Z^(b/2) and products Z^(2^a + r) = Z^(2^a) Z^r; giant steps
    Z^b, Z^2b, ..., Z^(p-1) by squaring; blocks B_t = sum_{k odd < b} c_{tb+k} Z^k
    (scalar multiplications only, all babies first brought to the lowest baby
    level); the blocks are joined by a binary tree
    H[t0, t0 + 2^r) = H[t0, t0 + 2^(r-1)) + H[t0 + 2^(r-1), t0 + 2^r) Z^(2^(r-1) b),
    each node one multiply-accumulate (the lower half added before the
    product's modulus switch, see Oracle.mul_add); finally
    f = H + c_{p-1} Z^(p-1).

    Returns (f(Z), Z^(p-1)); Z^(p-1) gives EQ = 1 - Z^(p-1)."""
    e = (p - 1).bit_length() - 1
    assert 1 << e == p - 1, "schedule written for p - 1 a power of two"
    b = 1 << ((e + 1) // 2)
    c = lt_coefficients(p)
    pw = {1: Z}
    a = 1
    while 2 * a <= b // 2:
        pw[2 * a] = ev.mul(pw[a], pw[a])
        a *= 2
    for k in range(3, b, 2):
        hi = 1 << (k.bit_length() - 1)
        pw[k] = ev.mul(pw[hi], pw[k - hi])
    giants = [ev.mul(pw[b // 2], pw[b // 2])] if b > 1 else [Z]
    while b << len(giants) <= p - 1:
        giants.append(ev.mul(giants[-1], giants[-1]))
    odd = list(range(1, b, 2))
    lv = min(ev.level(pw[k]) for k in odd)
    baby = {k: ev.to_level(pw[k], lv) for k in odd}
    nblk = (p - 1) // b
    H = []
    for t in range(nblk):
        acc = ev.mul_scalar(baby[1], c[t * b + 1])
        for k in odd[1:]:
            acc = ev.add(acc, ev.mul_scalar(baby[k], c[t * b + k]))
        H.append(acc)
    r = 0
    while len(H) > 1:
        G = giants[r]
        H = [ev.mul_add(H[2 * i + 1], G, H[2 * i]) for i in range(len(H) // 2)]
        r += 1
    top = giants[-1]
    f = ev.add(H[0], ev.mul_scalar(top, c[p - 1]))
    return f, top


def eq_from_top(ev, top):
    """EQ = 1 - Z^(p-1)."""
    return ev.add_const(ev.mul_scalar(top, -1), 1)


def compare_lt(ev, a_digits, b_digits, p: int):
    """Lexicographic LT over digit planes, most significant first:
    LT = LT_0 + EQ_0 (LT_1 + EQ_1 (... LT_{n-1})), each step one
    multiply-accumulate."""
    lts, eqs = [], []
    for a, b in zip(a_digits, b_digits):
        f, top = lt_univariate(ev, ev.sub(a, b), p)
        lts.append(f)
        eqs.append(eq_from_top(ev, top))
    acc = lts[-1]
    for i in range(len(lts) - 2, -1, -1):
        acc = ev.mul_add(eqs[i], acc, lts[i])
    return acc


def max_min(ev, a_digits, b_digits, lt):
    """max_d = a_d + LT (b_d - a_d), min_d = b_d + LT (a_d - b_d), per plane,
    each one multiply-accumulate; a_d and b_d are first brought to LT's level
    (the differences are formed there)."""
    lv = ev.level(lt)
    al = [ev.to_level(a, lv) for a in a_digits]
    bl = [ev.to_level(b, lv) for b in b_digits]
    mx = [ev.mul_add(lt, ev.sub(b, a), a) for a, b in zip(al, bl)]
    mn = [ev.mul_add(lt, ev.sub(a, b), b) for a, b in zip(al, bl)]
    return mx, mn


# ---------------------------------------------------------------------------
# the bivariate circuit (Introduction: the bivariate comparison circuit, exact
# on every pair of digits of F_p; Background: LT and EQ per digit, combined in
# lexicographic order)
# ---------------------------------------------------------------------------

@lru_cache(maxsize=None)
def _lt_bivariate_table(p: int) -> tuple:
    """The bivariate interpolant of [x < y] over all (x, y) in [0, p-1]^2, in
    the variables S = X + Y and Z = X - Y (p odd, so (x, y) -> (s, z) is a
    bijection of F_p^2): the unique G(S, Z) = sum_{m, k < p} c[m][k] S^m Z^k
    with G(x + y, x - y) = [x < y].

    Interpolation written out from its definition: the indicator of a point
    a is 1 - (t - a)^(p-1), and (t - a)^(p-1) = sum_j a^(p-1-j) t^j in F_p
    (binomial(p-1, j) = (-1)^j mod p), so the coefficient of t^j in the
    interpolant of h is [j = 0] sum_a h(a) - sum_a h(a) a^(p-1-j) (0^0 = 1);
    in two variables c = L^T F L with L[a][j] = [j = 0] - a^(p-1-j) and
    F[s][z] = [x < y] for x = (s + z)/2, y = (s - z)/2."""
    inv2 = (p + 1) // 2
    L = np.zeros((p, p), np.int64)
    for a in range(p):
        for j in range(p):
            L[a, j] = ((1 if j == 0 else 0) - pow(a, p - 1 - j, p)) % p
    F = np.zeros((p, p), np.int64)
    for sv in range(p):
        for zv in range(p):
            x, y = (sv + zv) * inv2 % p, (sv - zv) * inv2 % p
            F[sv, zv] = 1 if x < y else 0
    c = (L.T @ F) % p
    c = (c @ L) % p
    return tuple(tuple(int(v) for v in row) for row in c)


def lt_bivariate_table(p: int) -> np.ndarray:
    """c[m][k]: coefficient of S^m Z^k (see _lt_bivariate_table)."""
    return np.array(_lt_bivariate_table(p), dtype=np.int64)


def _power_ladder(ev, X, top: int, odd_only: bool):
    """X^k for k = 1 .. top (top = 2^e), or for the odd k < top and top
    itself: X^(2^a) by squaring, and X^(2^a + r) = X^(2^a) X^r (r < 2^a; odd r
    when odd_only) block by block, so every power has depth ceil(log2 k)."""
    pw = {1: X}
    a = 1
    while a < top:
        pw[2 * a] = ev.mul(pw[a], pw[a])
        a *= 2
    a = 2
    while a < top:
        for r in range(1, a):
            if odd_only and r % 2 == 0:
                continue
            pw[a + r] = ev.mul(pw[a], pw[r])
        a *= 2
    return pw


def lt_bivariate(ev, X, Y, p: int):
    """The bivariate interpolant of [x < y] evaluated on X, Y (exact for every
    pair of digits in [0, p-1], p - 1 a power of two).

    The interpolant satisfies LT(X, Y) + LT(Y, X) = (X - Y)^(p-1) (the two
    orders plus equality cover every pair), so in S = X + Y, Z = X - Y its part
    even in Z is (p+1)/2 Z^(p-1) and the rest is odd in Z:
    LT = (p+1)/2 Z^(p-1) + sum_{k odd} Z^k g_k(S), g_k(S) = sum_m c[m][k] S^m.
    Schedule: S^1 .. S^(p-1) (p - 2 products), Z^k for odd k and Z^(p-1)
    (squarings plus one product per odd k >= 3), g_k(S) as scalar linear
    combinations of the S powers (all brought to the level of S^(p-1)), one
    product T_k = Z^k g_k(S) per odd k (Z^k brought to the same level), and
    LT = (p+1)/2 Z^(p-1) + sum_k T_k (at T's level).  2p + 4 products for
    p = 257 (518), depth log2(p-1) + 1.

    Returns (LT, Z^(p-1)); Z^(p-1) gives EQ = 1 - Z^(p-1)."""
    e = (p - 1).bit_length() - 1
    assert 1 << e == p - 1, "schedule written for p - 1 a power of two"
    c = lt_bivariate_table(p)
    Z = ev.sub(X, Y)
    S = ev.add(X, Y)
    sp = _power_ladder(ev, S, p - 1, False)
    zp = _power_ladder(ev, Z, p - 1, True)
    lv = ev.level(sp[p - 1])
    sl = {m: ev.to_level(sp[m], lv) for m in range(1, p)}
    odd = list(range(1, p - 1, 2))
    terms = []
    for k in odd:
        g = None
        for m in range(1, p):
            if c[m, k] == 0:
                continue
            t = ev.mul_scalar(sl[m], int(c[m, k]))
            g = t if g is None else ev.add(g, t)
        if g is None:
            g = ev.mul_scalar(sl[1], 0)
        g = ev.add_const(g, int(c[0, k]))
        terms.append(ev.mul(ev.to_level(zp[k], lv), g))
    lt_lv = ev.level(terms[0])
    acc = ev.mul_scalar(ev.to_level(zp[p - 1], lt_lv), (p + 1) // 2)
    for t in terms:
        acc = ev.add(acc, t)
    return acc, zp[p - 1]


def compare_lt_bivariate(ev, a_digits, b_digits, p: int):
    """Lexicographic LT over base-p digit planes (most significant first)
    with the bivariate circuit per digit:
    LT = LT_0 + EQ_0 (LT_1 + EQ_1 (... LT_{n-1})), EQ_d = 1 - (a_d - b_d)^(p-1)."""
    lts, eqs = [], []
    for a, b in zip(a_digits, b_digits):
        f, top = lt_bivariate(ev, a, b, p)
        lts.append(f)
        eqs.append(eq_from_top(ev, top))
    acc = lts[-1]
    for i in range(len(lts) - 2, -1, -1):
        acc = ev.mul_add(eqs[i], acc, lts[i])
    return acc


# ---------------------------------------------------------------------------
# slot-packed digits (Background, "Word-wise Universal FHE Scheme": the
# lexicographic combination by ShiftMul -- shift the ciphertext and multiply
# by the equality result -- and ShiftAdd -- a summation done by shifting)
# ---------------------------------------------------------------------------

def digit_lt_eq(ev, a, b, p: int, circuit: str = "univariate"):
    """Per-slot (LT, EQ) of two ciphertexts of digits: the univariate f(a - b)
    (digits in [0, (p-1)/2]) or the bivariate interpolant (any digits), with
    EQ = 1 - (a - b)^(p-1) from the same schedule."""
    if circuit == "bivariate":
        f, top = lt_bivariate(ev, a, b, p)
    else:
        f, top = lt_univariate(ev, ev.sub(a, b), p)
    return f, eq_from_top(ev, top)


def compare_lt_packed(ev, a, b, p: int, l: int, circuit: str = "univariate"):
    """LT of integers packed l digits each into consecutive slots of one
    ciphertext: integer k of a slot row at positions k l .. k l + l - 1, most
    significant digit first, l a power of two dividing the row length.

    Per-slot (L, E) = (LT, EQ) of the digits, then one round per shift
    s = 1, 2, ..., l/2 (rot(X, s) holds at slot j the value of slot j + s of
    its row):
        L <- L + E rot(L, s)     (ShiftMul: shift, multiply by EQ; ShiftAdd)
        E <- E rot(E, s)         (skipped in the last round)
    After the round with shift s, slot k l + i (i a multiple of 2s) holds the
    lexicographic (LT, EQ) of digits i .. i + 2s - 1 of integer k, so slot k l
    ends with the integer's LT (the other slots hold values of no meaning).
    Each L update is one multiply-accumulate."""
    assert l >= 1 and l & (l - 1) == 0, "l must be a power of two"
    L, E = digit_lt_eq(ev, a, b, p, circuit)
    s = 1
    while s < l:
        Lr = ev.rotate(L, s)
        last = 2 * s >= l
        Er = None if last else ev.rotate(E, s)
        L = ev.mul_add(E, Lr, L)
        if not last:
            E = ev.mul(E, Er)
        s *= 2
    return L


def tournament(ev, x, p: int, k: int, want_max: bool = False, circuit: str = "univariate"):
    """Minimum (maximum) over windows of k = 2^r consecutive slots of a row,
    by r rounds of comparisons between the ciphertext and its own shifts:
    round t, s = 2^t:
        Y = rot(X, s);  L = LT(X, Y) per slot;
        X <- Y + L (X - Y)   (min)   or   X <- X + L (Y - X)   (max)
    with X and Y first brought to L's level.  After the rounds slot j holds
    the min (max) of slots j .. j + k - 1 of its row (cyclically): the
    windows starting at multiples of k are tournaments over disjoint arrays
    of k values, the winner landing in the array's first slot."""
    assert k >= 1 and k & (k - 1) == 0, "k must be a power of two"
    X = x
    s = 1
    while s < k:
        Y = ev.rotate(X, s)
        L, _ = digit_lt_eq(ev, X, Y, p, circuit)
        lv = ev.level(L)
        Xl, Yl = ev.to_level(X, lv), ev.to_level(Y, lv)
        X = ev.mul_add(L, ev.sub(Yl, Xl), Xl) if want_max else ev.mul_add(L, ev.sub(Xl, Yl), Yl)
        s *= 2
    return X


# ---------------------------------------------------------------------------
# F_{p^d} slots and the "mod extract" of their F_p digits (Background,
# "Word-wise Universal FHE Scheme": an integer is an element of F_{p^d}^l,
# each F_{p^d} component split into F_p digits before the per-digit LT/EQ)
# ---------------------------------------------------------------------------

def fpd_degree(p: int, N: int) -> int:
    """d = N / M.  Over F_p, x^N + 1 = prod_j (x^d - zeta_j) with the slot
    roots zeta_j of ``slot_roots``; d is the order of p modulo 2N, so each
    factor is irreducible and slot j holds an element of
    F_p[x]/(x^d - zeta_j), a field of p^d elements."""
    return N // slot_count(p)


def encode_fpd(E, p: int, N: int) -> np.ndarray:
    """Plaintext whose slot j holds sum_k E[j][k] x^k in F_p[x]/(x^d - zeta_j)
    (the power basis 1, x, ..., x^(d-1)): m = sum_k x^k mu_k(x^d), mu_k the
    slot encoding of column k (``encode_poly``), so coefficient d i + k of m
    is coefficient d i of column k's encoding."""
    M = slot_count(p)
    d = N // M
    E = np.asarray(E, dtype=np.int64).reshape(M, d) % p
    out = np.zeros(N, dtype=np.uint32)
    for k in range(d):
        if E[:, k].any():
            out[k::d] = encode_poly(E[:, k], p, N)[0::d]
    return out


def decode_fpd(m, p: int, N: int) -> np.ndarray:
    """The slots of m as F_{p^d} elements, by definition: m mod (x^d - zeta_j),
    with x^(d i + k) = zeta_j^i x^k; row j holds its power-basis coordinates."""
    M = slot_count(p)
    d = N // M
    rows = np.asarray(m, dtype=np.int64).reshape(M, d) % p  # row i: coefficients d i .. d i + d - 1
    out = np.zeros((M, d), dtype=np.int64)
    for j, z in enumerate(slot_roots(p, M)):
        zi = np.array([pow(z, i, p) for i in range(M)], dtype=np.int64)
        out[j] = (zi[:, None] * rows).sum(axis=0) % p
    return out


def fpd_slot_mul(a, b, z: int, p: int) -> np.ndarray:
    """Product in F_p[x]/(x^d - z): the full product, then x^(d + k) = z x^k."""
    a, b = np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64)
    d = len(a)
    c = np.convolve(a, b) % p
    out = c[:d].copy()
    out[: d - 1] = (out[: d - 1] + z * c[d:]) % p
    return out


def plain_automorphism(m, g: int, N: int, p: int) -> np.ndarray:
    """m(x^g) mod (x^N + 1, p), g odd: coefficient i moves to x^(i g)."""
    out = np.zeros(N, dtype=np.int64)
    for i, c in enumerate(np.asarray(m, dtype=np.int64)):
        j = i * g % (2 * N)
        if j < N:
            out[j] = (out[j] + c) % p
        else:
            out[j - N] = (out[j - N] - c) % p
    return out


def frobenius_steps(p: int, N: int) -> list[int]:
    """Rotation steps r_b with 5^(r_b) = p^(2^b) mod 2N, b < log2(d): the
    automorphisms x -> x^(p^(2^b)) are Frobenius powers on every F_{p^d} slot
    (p = 1 mod 4, so p lies in the cyclic group <5> of order N/2 mod 2N and
    the rotation keys serve them).  Found by walking the powers of 5."""
    twoN = 2 * N
    log5, x = {}, 1
    for r in range(N // 2):
        log5[x] = r
        x = x * 5 % twoN
    t = fpd_degree(p, N).bit_length() - 1
    return [log5[pow(p, 1 << b, twoN)] for b in range(t)]


def extract_digit(ev, orc: "Oracle", ct: Ct, k: int, p: int) -> Ct:
    """Coordinate k of every slot's F_{p^d} element, as the F_p slot values of
    a new ciphertext: d^-1 Tr(x^-k m).  The trace Tr = sum over the Frobenius
    group <p> (order d) of x -> x^g fixes mu(x^d) and takes x^j, 0 < |j| < d,
    to zero (x^j is a root of unity of order above 2M in each slot, whose
    minimal polynomial over F_p is a binomial of degree > 1, so its conjugates
    sum to zero); so Tr(x^-k m) = d mu_k(x^d).  The sum over the group is taken
    as log2(d) doublings z <- z + sigma_{p^(2^b)}(z), each a rotation."""
    N = orc.N
    z = orc.mul_monomial(ct, 2 * N - k)  # x^-k = -x^(N-k)
    for r in frobenius_steps(p, N):
        z = ev.add(z, ev.rotate(z, r))
    return ev.mul_scalar(z, pow(fpd_degree(p, N), -1, p))


def to_digits(values, base: int, ndigits: int):
    """Integer -> digit planes, most significant first."""
    v = np.asarray(values, dtype=np.int64)
    return [((v // base ** (ndigits - 1 - i)) % base).astype(np.uint32) for i in range(ndigits)]


# ---------------------------------------------------------------------------
# non-power-of-two cyclotomic rings Z_q[X]/(Phi_m(X)), m odd (Background,
# "Efficient Polynomial and NTT": polynomials in the integer DFT
# representation, a (L+1) x phi(m) matrix; the BluesteinNTT converts between
# coefficients and that representation when the degree phi(m) is not a power
# of two).  The representation is the values at the primitive m-th roots of
# unity omega^k, k in Z_m^* ascending; here it is computed by its
# definition (polynomial evaluation), independently of any fast transform.
# ---------------------------------------------------------------------------

def _mobius(n: int) -> int:
    r, k, f = 1, n, 2
    while f * f <= k:
        if k % f == 0:
            k //= f
            if k % f == 0:
                return 0
            r = -r
        f += 1
    return -r if k > 1 else r


def cyclotomic(m: int) -> list:
    """Coefficients of Phi_m, lowest first: the product over d | m of
    (X^d - 1)^mu(m/d) (multiplications first, then the exact divisions)."""
    divs = [d for d in range(1, m + 1) if m % d == 0]
    poly = [1]
    for d in divs:  # multiply by (X^d - 1)
        if _mobius(m // d) == 1:
            out = [0] * (len(poly) + d)
            for i, c in enumerate(poly):
                out[i + d] += c
                out[i] -= c
            poly = out
    for d in divs:  # divide by (X^d - 1): q_i = q_(i-d) - p_i, from the bottom
        if _mobius(m // d) == -1:
            n = len(poly) - d
            q = [0] * n
            for i in range(n):
                q[i] = -poly[i] + (q[i - d] if i >= d else 0)
            assert all(poly[n + i] == q[n + i - d] for i in range(d)), "inexact division"
            poly = q
    while len(poly) > 1 and poly[-1] == 0:
        poly.pop()
    return poly


def zm_star(m: int) -> list:
    """The k in [0, m) prime to m, ascending: the positions the DFT
    representation keeps."""
    return [k for k in range(m) if math.gcd(k, m) == 1]


def bluestein_length(m: int) -> int:
    """The power-of-two length of Bluestein's convolution: at least 2m - 1,
    and at least 2^10 (the reading: the smallest transform length the device
    library runs; the primes, 1 mod 2 L m, follow from it)."""
    L = 1024
    while L < 2 * m - 1:
        L *= 2
    return L


class CycloRing:
    """Z_q[X]/(Phi_m) for `nprimes` primes: the largest below 2^bits that are
    1 mod 2 L m (an m-th root of unity, and a power-of-two transform of
    length L), omega_i the smallest x^((q_i - 1)/m) of order exactly m."""

    def __init__(self, m: int, nprimes: int, bits: int):
        assert m % 2 == 1 and m >= 3
        self.m = m
        self.L = bluestein_length(m)
        self.phi = cyclotomic(m)
        self.N = len(self.phi) - 1
        self.zm = zm_star(m)
        assert len(self.zm) == self.N
        L = lib()
        out = np.zeros(nprimes, dtype=np.uint64)
        n = L.or_gen_primes(2 * self.L * m, bits, nprimes, _p(np.zeros(1, np.uint64)), 0, _p(out))
        assert n == nprimes, "not enough primes"
        self.moduli = [int(q) for q in out]
        self.omega = [int(L.or_find_root_m(q, m)) for q in self.moduli]
        self._phi = np.array(self.phi, dtype=np.int64)

    def forward(self, a: np.ndarray) -> np.ndarray:
        """a[nprimes][N] coefficients -> values a(omega^k), k in Z_m^* ascending."""
        out = np.zeros_like(a, dtype=np.uint64)
        for i, (q, w) in enumerate(zip(self.moduli, self.omega)):
            pts = np.array([pow(w, k, q) for k in self.zm], dtype=np.uint64)
            self_a = np.ascontiguousarray(a[i], dtype=np.uint64)
            lib().or_poly_eval(_p(self_a), self.N, _p(pts), self.N, q, _p(out[i]))
        return out

    def inverse(self, A: np.ndarray) -> np.ndarray:
        """Values at the primitive roots -> the coefficients of the unique
        polynomial of degree < N taking them: the inverse length-m DFT of the
        values placed at k in Z_m^* (zero elsewhere), b_j = m^-1 sum_k A_k
        omega^(-jk), is a polynomial of degree < m with those values at the
        primitive roots; its remainder modulo Phi_m is the answer."""
        out = np.zeros_like(A, dtype=np.uint64)
        m = self.m
        for i, (q, w) in enumerate(zip(self.moduli, self.omega)):
            c = np.zeros(m, dtype=np.uint64)
            c[self.zm] = A[i]
            wi = pow(w, q - 2, q)
            pts = np.array([pow(wi, j, q) for j in range(m)], dtype=np.uint64)
            b = np.zeros(m, dtype=np.uint64)
            lib().or_poly_eval(_p(c), m, _p(pts), m, q, _p(b))
            minv = pow(m, q - 2, q)
            b = np.array([int(x) * minv % q for x in b], dtype=np.uint64)
            lib().or_poly_mod_monic(_p(b), m, self._phi.ctypes.data_as(i64p), self.N, q, _p(out[i]))
        return out

    def mul(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        """a b mod (Phi_m, q_i): schoolbook product and long division."""
        out = np.zeros_like(a, dtype=np.uint64)
        for i, q in enumerate(self.moduli):
            x = np.ascontiguousarray(a[i], dtype=np.uint64)
            y = np.ascontiguousarray(b[i], dtype=np.uint64)
            lib().or_cyclo_mul(_p(x), _p(y), self.N, self._phi.ctypes.data_as(i64p), q, _p(out[i]))
        return out
