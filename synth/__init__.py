"""Seeded synthetic inputs shared by the CPU oracle and the device path.

This module draws random numbers and nothing else: it holds none of the
scheme's arithmetic (no moduli, no reductions, no transforms).  Every array it
returns is handed, unchanged, to both implementations, which then reduce and
transform it themselves.

Generator: numpy's Philox4x32-10 counter-based bit generator, keyed by a
``SeedSequence`` built from ``(seed, purpose, index)`` so that every stream is
independent of how many numbers any other stream consumed.

Distributions (BGV as in the paper's background section on the word-wise
scheme; the error width and tail cut follow the workload recipe):

* secret and encryption randomness ``u``: i.i.d. uniform on {-1, 0, 1};
* errors: rounded normal, sigma = 3.2, rejected beyond 6 sigma;
* uniform ring elements: raw uniform 64-bit words (each side reduces them
  modulo its own primes);
* slot values and integers: uniform on the stated range.
"""
from __future__ import annotations

import numpy as np

SIGMA = 3.2
TAIL = 6.0

_PURPOSES = {
    "secret": 1,
    "pk_a": 2,
    "pk_e": 3,
    "ksk_a": 4,
    "ksk_e": 5,
    "enc_u": 6,
    "enc_e": 7,
    "slots": 8,
    "ints": 9,
    "schedule": 10,
    "poly": 11,
    "fpd": 12,
}


def generator(seed: int, purpose: str, index: int = 0) -> np.random.Generator:
    """Independent Philox stream for (seed, purpose, index)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF,
                                 _PURPOSES[purpose], int(index)])
    return np.random.Generator(np.random.Philox(ss))


def ternary(g: np.random.Generator, shape) -> np.ndarray:
    return (g.integers(0, 3, size=shape, dtype=np.int64) - 1).astype(np.int8)


def gaussian(g: np.random.Generator, shape, sigma: float = SIGMA, tail: float = TAIL) -> np.ndarray:
    """Rounded normal with rejection beyond ``tail * sigma``."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.int32)
    bound = int(np.floor(tail * sigma))
    filled = 0
    while filled < n:
        draw = np.rint(g.normal(0.0, sigma, size=n - filled)).astype(np.int64)
        keep = draw[np.abs(draw) <= bound]
        out[filled:filled + keep.size] = keep
        filled += keep.size
    return out.reshape(shape)


def words(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 2**64 - 1, size=shape, dtype=np.uint64, endpoint=True)


def uniform(g: np.random.Generator, lo: int, hi: int, shape) -> np.ndarray:
    """Uniform integers in [lo, hi) as uint32."""
    return g.integers(lo, hi, size=shape, dtype=np.int64).astype(np.uint32)


def keygen_randomness(seed: int, N: int, nQ: int, nP: int, dnum: int, nrot: int) -> dict:
    """Randomness consumed by key generation, in the layout the key generators take.

    * ``s``: int8[N] ternary secret;
    * ``a``: uint64 words: public key ``[nQ][N]``, then for the relinearisation key
      and each rotation key in order, ``dnum`` blocks of ``[nQ+nP][N]``;
    * ``e``: int32 errors: public key ``[N]``, then ``dnum`` blocks of ``[N]`` per
      switching key, same key order.
    """
    nkeys = 1 + nrot
    s = ternary(generator(seed, "secret"), (N,))
    a_pk = words(generator(seed, "pk_a"), (nQ * N,))
    e_pk = gaussian(generator(seed, "pk_e"), (N,))
    a_ks = [words(generator(seed, "ksk_a", k * 64 + j), ((nQ + nP) * N,))
            for k in range(nkeys) for j in range(dnum)]
    e_ks = [gaussian(generator(seed, "ksk_e", k * 64 + j), (N,))
            for k in range(nkeys) for j in range(dnum)]
    a = np.concatenate([a_pk] + a_ks) if a_ks else a_pk
    e = np.concatenate([e_pk] + e_ks) if e_ks else e_pk
    return {"s": s, "a": np.ascontiguousarray(a), "e": np.ascontiguousarray(e)}


def encrypt_randomness(seed: int, count: int, N: int) -> dict:
    """``u``: int8[count][N] ternary; ``e``: int32[count][2][N] errors."""
    u = ternary(generator(seed, "enc_u"), (count, N))
    e = gaussian(generator(seed, "enc_e"), (count, 2, N))
    return {"u": u, "e": e}


def slot_values(seed: int, count: int, nslots: int, lo: int, hi: int, index: int = 0) -> np.ndarray:
    """uint32[count][nslots] uniform in [lo, hi)."""
    return uniform(generator(seed, "slots", index), lo, hi, (count, nslots))


def integers(seed: int, shape, lo: int, hi: int, index: int = 0) -> np.ndarray:
    """uint32 integers uniform in [lo, hi) (e.g. uint16 operands)."""
    return uniform(generator(seed, "ints", index), lo, hi, shape)
