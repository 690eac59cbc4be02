"""Python binding of the gfx950 BGV less-than library (``libboostcom.so``).

Argument marshalling only: every computation happens in the library's HIP
kernels.  PyTorch provides device memory (ciphertext batches are int64 CUDA
tensors reinterpreted as uint64 residues) and the current HIP stream.  The C
functions keep their names (``bc_ctx_create`` ...); ``Context`` bundles them
for convenience.  Importing never compiles anything; if the shared library is
missing the first call raises ``BoostcomUnavailable``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libboostcom.so")

BC_OK, BC_ERR_ARG, BC_ERR_PARAM, BC_ERR_LEVEL, BC_ERR_OOM, BC_ERR_HIP, BC_ERR_KEY = 0, -1, -2, -3, -4, -5, -6
BC_ROW_SWAP = -1
BC_EXEC_BATCHED, BC_EXEC_GRAPH, BC_EXEC_PER_OP = 0, 1, 2
BC_GROUP_FORK_JOIN, BC_GROUP_PERSISTENT = 0, 1
BC_CIRCUIT_UNIVARIATE, BC_CIRCUIT_BIVARIATE = 0, 1
BC_PROF_NTT_FWD, BC_PROF_NTT_INV, BC_PROF_NTT_FWD_COMBINE, BC_PROF_NTT_FWD_PART, BC_PROF_NTT_INV_PART = 0, 1, 2, 3, 4
BC_PROF_TENSOR, BC_PROF_MODUP, BC_PROF_KS_INNER, BC_PROF_RELIN_MS, BC_PROF_LINCOMB, BC_PROF_MUL = 5, 6, 7, 8, 9, 10
BC_TUNE_NTT_CHUNK_BYTES, BC_TUNE_NTT_SINGLE_PASS, BC_TUNE_FP64, BC_TUNE_POOL_LIMIT_BYTES = 0, 1, 2, 3
BC_TUNE_NTT_PARTS, BC_TUNE_SPLIT_STREAMS = 4, 5
BC_TUNE_TEST_FAIL_ALLOC = 6
BC_TUNE_PERSISTENT = 7
BC_TUNE_MFMA = 8
BC_TUNE_RAW_HANDOFF = 9
BC_TUNE_MFMA_MODUP = 10
BC_NOISE_FRESH, BC_NOISE_BUDGET, BC_NOISE_ADD, BC_NOISE_TENSOR, BC_NOISE_MUL, BC_NOISE_MOD_SWITCH, BC_NOISE_ROTATE = range(7)


class BoostcomUnavailable(RuntimeError):
    pass


class BoostcomError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


class bc_params(ctypes.Structure):
    _fields_ = [("logN", ctypes.c_int32), ("p", ctypes.c_int32), ("nQ", ctypes.c_int32), ("bitsQ", ctypes.c_int32),
                ("nP", ctypes.c_int32), ("bitsP", ctypes.c_int32), ("dnum", ctypes.c_int32)]


class bc_ctb(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("count", ctypes.c_int32), ("level", ctypes.c_int32),
                ("ncomp", ctypes.c_int32), ("noise_bits", ctypes.c_float)]


_lib = None

# name -> (restype, argtypes)
_V, _P, _I, _S = ctypes.c_void_p, ctypes.POINTER, ctypes.c_int32, ctypes.c_size_t
_SIGS = {
    "bc_ctx_create": (_I, [_P(bc_params), _P(_V)]),
    "bc_ctx_destroy": (_I, [_V]),
    "bc_ctx_moduli": (_I, [_V, _P(ctypes.c_uint64), _I]),
    "bc_ctx_slots": (_I, [_V]),
    "bc_ct_words": (_S, [_V, _I, _I]),
    "bc_ctx_pool_bytes": (_S, [_V]),
    "bc_ctx_trim": (_I, [_V]),
    "bc_keygen_rand_sizes": (_I, [_V, _I, _P(_S), _P(_S)]),
    "bc_keygen": (_I, [_V, _V, _V, _V, _V, _I, _P(_V)]),
    "bc_keys_destroy": (_I, [_V]),
    "bc_keys_export": (_I, [_V, _V, _V, _S, _P(_S)]),
    "bc_keys_import": (_I, [_V, _V, _S, _P(_V)]),
    "bc_encrypt": (_I, [_V, _V, _V, _V, _V, _P(bc_ctb), _V]),
    "bc_decrypt": (_I, [_V, _V, _P(bc_ctb), _V, _V]),
    "bc_decrypt_poly": (_I, [_V, _V, _P(bc_ctb), _V, _V]),
    "bc_export": (_I, [_V, _P(bc_ctb), _V, _V]),
    "bc_import": (_I, [_V, _V, _P(bc_ctb), _V]),
    "bc_tensor": (_I, [_V, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_relin": (_I, [_V, _V, _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_mod_switch": (_I, [_V, _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_mul_relin": (_I, [_V, _V, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_mul_relin_noalloc": (_I, [_V, _V, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_rotate": (_I, [_V, _V, _P(bc_ctb), _I, _P(bc_ctb), _V]),
    "bc_add": (_I, [_V, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_sub": (_I, [_V, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_mul_scalar": (_I, [_V, _P(bc_ctb), _I, _P(bc_ctb), _V]),
    "bc_add_const": (_I, [_V, _P(bc_ctb), _I, _P(bc_ctb), _V]),
    "bc_compare_levels": (_I, [_V, _I, _I, _P(_I), _P(_I)]),
    "bc_compare_lt": (_I, [_V, _V, _I, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_compare_max_min": (_I, [_V, _V, _I, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_compare_bivariate": (_I, [_V, _V, _I, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_compare_levels_circuit": (_I, [_V, _I, _I, _I, _P(_I), _P(_I)]),
    "bc_compare_packed": (_I, [_V, _V, _I, _I, _P(bc_ctb), _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_packed_levels": (_I, [_V, _I, _I, _I, _P(_I)]),
    "bc_tournament": (_I, [_V, _V, _I, _I, _I, _P(bc_ctb), _P(bc_ctb), _V]),
    "bc_tournament_levels": (_I, [_V, _I, _I, _I, _P(_I)]),
    "bc_noise_compare_circuit": (_I, [_P(bc_params), _I, _I, ctypes.c_double, _I, _P(ctypes.c_double),
                                      _P(ctypes.c_double), _P(_I), _P(_I)]),
    "bc_set_exec_mode": (_I, [_V, _I]),
    "bc_group_create": (_I, [_I, _P(_V), _P(_V)]),
    "bc_group_destroy": (_I, [_V]),
    "bc_group_compare": (_I, [_V, _P(_V), _P(_I), _P(_P(bc_ctb)), _P(_P(bc_ctb)), _P(_P(bc_ctb)),
                              _P(_P(bc_ctb)), _P(_P(bc_ctb)), _V]),
    "bc_group_set_mode": (_I, [_V, _I]),
    "bc_group_get_mode": (_I, [_V, _P(_I), _P(_I), _P(_I), _P(_I)]),
    "bc_set_tuning": (_I, [_V, _I, ctypes.c_int64]),
    "bc_autotune": (_I, [_V, _V]),
    "bc_autotune_mul": (_I, [_V, _V, _V]),
    "bc_get_tuning": (_I, [_V, _I, _P(ctypes.c_int64)]),
    "bc_profile_enable": (_I, [_V, _I]),
    "bc_profile_read": (_I, [_V, _I, _P(ctypes.c_double), _P(ctypes.c_int64), _P(ctypes.c_double)]),
    "bc_noise_estimate": (_I, [_P(bc_params), _I, _I, ctypes.c_double, ctypes.c_double, _P(ctypes.c_double)]),
    "bc_noise_compare": (_I, [_P(bc_params), _I, ctypes.c_double, _I, _P(ctypes.c_double), _P(ctypes.c_double)]),
    "bc_fpd_info": (_I, [_V, _P(_I), _P(_I), _P(_I), _I]),
    "bc_encode_fpd": (_I, [_V, _V, _I, _V]),
    "bc_decode_fpd": (_I, [_V, _V, _I, _V]),
    "bc_encrypt_poly": (_I, [_V, _V, _V, _V, _V, _P(bc_ctb), _V]),
    "bc_extract_digits": (_I, [_V, _V, _P(bc_ctb), _V, _I, _P(bc_ctb), _V]),
    "bc_bluestein_create": (_I, [_I, _I, _I, _P(_V)]),
    "bc_bluestein_destroy": (_I, [_V]),
    "bc_bluestein_info": (_I, [_V, _P(_I), _P(_I), _P(ctypes.c_uint64)]),
    "bc_bluestein_forward": (_I, [_V, _V, _V, _I, _V]),
    "bc_bluestein_inverse": (_I, [_V, _V, _V, _I, _V]),
    "bc_strerror": (ctypes.c_char_p, [_I]),
    "bc_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Loads the in-tree shared library (never builds it)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same SONAME as the system
        # one; loading torch first makes the library bind to that single
        # runtime, so torch's device memory and streams are valid here.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise BoostcomUnavailable(f"{LIB_PATH} is missing: build it with `python -m paper_2407_07308_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def _check(rc: int):
    if rc != BC_OK:
        L = lib()
        raise BoostcomError(rc, f"{L.bc_strerror(rc).decode()}: {L.bc_last_error().decode()}")


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------

@dataclass
class Batch:
    """``count`` ciphertexts [count][ncomp][level+1][N] uint64 in a CUDA tensor,
    with the library's noise estimate (log2 bits; 0 = unknown)."""
    tensor: object  # torch.Tensor (int64, cuda)
    count: int
    level: int
    ncomp: int
    noise: float = 0.0

    def ctb(self) -> bc_ctb:
        return bc_ctb(self.tensor.data_ptr(), self.count, self.level, self.ncomp, self.noise)

    def take(self, c: bc_ctb) -> "Batch":
        """Adopts the level, components and noise estimate a call wrote to ``c``."""
        self.level, self.ncomp, self.noise = c.level, c.ncomp, float(c.noise_bits)
        return self

    def split(self, parts: int) -> list["Batch"]:
        """``parts`` batches of count / parts ciphertexts each, viewing
        consecutive ranges of this one (no copy)."""
        assert self.count % parts == 0
        n = self.count // parts
        w = self.tensor.numel() // parts
        return [Batch(self.tensor[i * w:(i + 1) * w], n, self.level, self.ncomp, self.noise) for i in range(parts)]


def _ctb_array(batches):
    arr = (bc_ctb * len(batches))()
    for i, b in enumerate(batches):
        arr[i] = b.ctb()
    return arr


def _take_array(batches, arr):
    for i, b in enumerate(batches):
        b.take(arr[i])


class Keys:
    def __init__(self, ctx: "Context", handle: ctypes.c_void_p, rot_steps):
        self.ctx = ctx
        self.handle = handle
        self.rot_steps = tuple(rot_steps)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bc_keys_destroy(self.handle)
            self.handle = None


class Context:
    def __init__(self, logN: int, p: int, nQ: int, bitsQ: int, nP: int, bitsP: int, dnum: int):
        self.prm = bc_params(logN, p, nQ, bitsQ, nP, bitsP, dnum)
        self.L = lib()
        h = ctypes.c_void_p()
        _check(self.L.bc_ctx_create(ctypes.byref(self.prm), ctypes.byref(h)))
        self.handle = h
        self.N = 1 << logN
        self.p = p
        self.nQ, self.nP, self.dnum = nQ, nP, dnum
        self.M = self.L.bc_ctx_slots(h)
        mods = (ctypes.c_uint64 * (nQ + nP))()
        _check(self.L.bc_ctx_moduli(h, mods, nQ + nP))
        self.moduli = [int(x) for x in mods]

    @classmethod
    def from_params(cls, prm) -> "Context":
        return cls(prm.logN, prm.p, prm.nQ, prm.bitsQ, prm.nP, prm.bitsP, prm.dnum)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bc_ctx_destroy(self.handle)
            self.handle = None

    # ------------------------------------------------------------ memory
    def ct_words(self, level: int, ncomp: int = 2) -> int:
        return int(self.L.bc_ct_words(self.handle, level, ncomp))

    def new_batch(self, count: int, level: int, ncomp: int = 2) -> Batch:
        import torch

        words = self.ct_words(level, ncomp) * count
        return Batch(torch.empty(words, dtype=torch.int64, device="cuda"), count, level, ncomp)

    def pool_bytes(self) -> int:
        return int(self.L.bc_ctx_pool_bytes(self.handle))

    def trim(self):
        _check(self.L.bc_ctx_trim(self.handle))

    # -------------------------------------------------------------- keys
    def keygen_sizes(self, nrot: int):
        w, e = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self.L.bc_keygen_rand_sizes(self.handle, nrot, ctypes.byref(w), ctypes.byref(e)))
        return w.value, e.value

    def keygen(self, s, a_words, errors, rot_steps=()) -> Keys:
        s = np.ascontiguousarray(s, dtype=np.int8)
        a = np.ascontiguousarray(a_words, dtype=np.uint64)
        e = np.ascontiguousarray(errors, dtype=np.int32)
        nw, ne = self.keygen_sizes(len(rot_steps))
        if s.size != self.N or a.size != nw or e.size != ne:
            raise BoostcomError(BC_ERR_ARG, f"keygen randomness sizes {s.size},{a.size},{e.size} != {self.N},{nw},{ne}")
        steps = (ctypes.c_int32 * max(1, len(rot_steps)))(*rot_steps)
        h = ctypes.c_void_p()
        _check(self.L.bc_keygen(self.handle, _np_ptr(s), _np_ptr(a), _np_ptr(e), steps, len(rot_steps),
                                ctypes.byref(h)))
        return Keys(self, h, rot_steps)

    def export_keys(self, keys: Keys) -> bytes:
        """The key set as a coefficient-domain blob (``bc_keys_export``)."""
        n = ctypes.c_size_t()
        _check(self.L.bc_keys_export(self.handle, keys.handle, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self.L.bc_keys_export(self.handle, keys.handle, buf, n.value, ctypes.byref(n)))
        return buf.raw

    def import_keys(self, blob: bytes) -> Keys:
        """A key set from a blob of ``export_keys`` (``bc_keys_import``)."""
        h = ctypes.c_void_p()
        _check(self.L.bc_keys_import(self.handle, blob, len(blob), ctypes.byref(h)))
        nrot = int(np.frombuffer(blob, dtype=np.int32, count=1, offset=36)[0])
        steps = np.frombuffer(blob, dtype=np.int32, count=nrot, offset=40).tolist()
        return Keys(self, h, steps)

    # ------------------------------------------------------- client side
    def encrypt(self, keys: Keys, slots, u, errors, out: Batch | None = None) -> Batch:
        slots = np.ascontiguousarray(slots, dtype=np.uint32).reshape(-1, self.M)
        count = slots.shape[0]
        u = np.ascontiguousarray(u, dtype=np.int8).reshape(count, self.N)
        e = np.ascontiguousarray(errors, dtype=np.int32).reshape(count, 2, self.N)
        out = out or self.new_batch(count, self.nQ - 1, 2)
        c = out.ctb()
        _check(self.L.bc_encrypt(self.handle, keys.handle, _np_ptr(slots), _np_ptr(u), _np_ptr(e), ctypes.byref(c),
                                 _stream()))
        return out.take(c)

    def decrypt(self, keys: Keys, b: Batch) -> np.ndarray:
        out = np.zeros((b.count, self.M), dtype=np.uint32)
        c = b.ctb()
        _check(self.L.bc_decrypt(self.handle, keys.handle, ctypes.byref(c), _np_ptr(out), _stream()))
        return out

    def decrypt_poly(self, keys: Keys, b: Batch) -> np.ndarray:
        out = np.zeros((b.count, self.N), dtype=np.uint32)
        c = b.ctb()
        _check(self.L.bc_decrypt_poly(self.handle, keys.handle, ctypes.byref(c), _np_ptr(out), _stream()))
        return out

    def export(self, b: Batch) -> np.ndarray:
        out = np.zeros((b.count, b.ncomp, b.level + 1, self.N), dtype=np.uint64)
        c = b.ctb()
        _check(self.L.bc_export(self.handle, ctypes.byref(c), _np_ptr(out), _stream()))
        return out

    def import_(self, host: np.ndarray, level: int, ncomp: int = 2, noise: float = 0.0) -> Batch:
        host = np.ascontiguousarray(host, dtype=np.uint64).reshape(-1, ncomp, level + 1, self.N)
        out = self.new_batch(host.shape[0], level, ncomp)
        out.noise = noise
        c = out.ctb()
        _check(self.L.bc_import(self.handle, _np_ptr(host), ctypes.byref(c), _stream()))
        return out

    # ------------------------------------------------------- server side
    def _binary(self, fn, a: Batch, b: Batch, level: int, ncomp: int, *extra) -> Batch:
        out = self.new_batch(a.count, level, ncomp)
        ca, cb, co = a.ctb(), b.ctb(), out.ctb()
        _check(fn(self.handle, *extra, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co), _stream()))
        return out.take(co)

    def tensor(self, a: Batch, b: Batch) -> Batch:
        return self._binary(self.L.bc_tensor, a, b, min(a.level, b.level), 3)

    def add(self, a: Batch, b: Batch) -> Batch:
        return self._binary(self.L.bc_add, a, b, min(a.level, b.level), a.ncomp)

    def sub(self, a: Batch, b: Batch) -> Batch:
        return self._binary(self.L.bc_sub, a, b, min(a.level, b.level), a.ncomp)

    def mul_relin(self, keys: Keys, a: Batch, b: Batch) -> Batch:
        lv = min(a.level, b.level)
        out = self.new_batch(a.count, lv - 1 if lv > 0 else 0, 2)
        ca, cb, co = a.ctb(), b.ctb(), out.ctb()
        _check(self.L.bc_mul_relin(self.handle, keys.handle, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co),
                                   _stream()))
        return out.take(co)

    def mul_relin_noalloc(self, keys: Keys, a: Batch, b: Batch, out: Batch = None) -> Batch:
        """bc_mul_relin_noalloc: the library allocates nothing (its workspace
        is the fixed per-GPU scratch array); ``out`` may be passed in."""
        lv = min(a.level, b.level)
        if out is None:
            out = self.new_batch(a.count, lv - 1 if lv > 0 else 0, 2)
        ca, cb, co = a.ctb(), b.ctb(), out.ctb()
        _check(self.L.bc_mul_relin_noalloc(self.handle, keys.handle, ctypes.byref(ca), ctypes.byref(cb),
                                           ctypes.byref(co), _stream()))
        return out.take(co)

    def relin(self, keys: Keys, a: Batch) -> Batch:
        out = self.new_batch(a.count, a.level, 2)
        ca, co = a.ctb(), out.ctb()
        _check(self.L.bc_relin(self.handle, keys.handle, ctypes.byref(ca), ctypes.byref(co), _stream()))
        return out.take(co)

    def mod_switch(self, a: Batch) -> Batch:
        out = self.new_batch(a.count, a.level - 1, 2)
        ca, co = a.ctb(), out.ctb()
        _check(self.L.bc_mod_switch(self.handle, ctypes.byref(ca), ctypes.byref(co), _stream()))
        return out.take(co)

    def rotate(self, keys: Keys, a: Batch, steps: int) -> Batch:
        out = self.new_batch(a.count, a.level, 2)
        ca, co = a.ctb(), out.ctb()
        _check(self.L.bc_rotate(self.handle, keys.handle, ctypes.byref(ca), steps, ctypes.byref(co), _stream()))
        return out.take(co)

    def mul_scalar(self, a: Batch, c: int) -> Batch:
        out = self.new_batch(a.count, a.level, a.ncomp)
        ca, co = a.ctb(), out.ctb()
        _check(self.L.bc_mul_scalar(self.handle, ctypes.byref(ca), int(c), ctypes.byref(co), _stream()))
        return out.take(co)

    def add_const(self, a: Batch, c: int) -> Batch:
        out = self.new_batch(a.count, a.level, a.ncomp)
        ca, co = a.ctb(), out.ctb()
        _check(self.L.bc_add_const(self.handle, ctypes.byref(ca), int(c), ctypes.byref(co), _stream()))
        return out.take(co)

    # ------------------------------------------------------ comparisons
    def compare_levels(self, in_level: int, ndigits: int, circuit: int = BC_CIRCUIT_UNIVARIATE):
        lt, mm = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.bc_compare_levels_circuit(self.handle, circuit, in_level, ndigits, ctypes.byref(lt),
                                                ctypes.byref(mm)))
        return lt.value, mm.value

    def packed_levels(self, in_level: int, digits_per_int: int, circuit: int = BC_CIRCUIT_UNIVARIATE) -> int:
        lv = ctypes.c_int32()
        _check(self.L.bc_packed_levels(self.handle, circuit, in_level, digits_per_int, ctypes.byref(lv)))
        return lv.value

    def compare_packed(self, keys: Keys, a: Batch, b: Batch, digits_per_int: int,
                       circuit: int = BC_CIRCUIT_UNIVARIATE, out: Batch = None) -> Batch:
        """LT of slot-packed integers (``bc_compare_packed``): valid at the first
        slot of every block of ``digits_per_int`` slots."""
        if out is None:
            out = self.new_batch(a.count, self.packed_levels(a.level, digits_per_int, circuit), 2)
        ca, cb, co = a.ctb(), b.ctb(), out.ctb()
        _check(self.L.bc_compare_packed(self.handle, keys.handle, circuit, digits_per_int, ctypes.byref(ca),
                                        ctypes.byref(cb), ctypes.byref(co), _stream()))
        return out.take(co)

    def tournament_levels(self, in_level: int, window: int, circuit: int = BC_CIRCUIT_UNIVARIATE) -> int:
        lv = ctypes.c_int32()
        _check(self.L.bc_tournament_levels(self.handle, circuit, in_level, window, ctypes.byref(lv)))
        return lv.value

    def tournament(self, keys: Keys, x: Batch, window: int, want_max: bool = False,
                   circuit: int = BC_CIRCUIT_UNIVARIATE, out: Batch = None) -> Batch:
        """Minimum (maximum) over every window of ``window`` slots of a row
        (``bc_tournament``)."""
        if out is None:
            out = self.new_batch(x.count, self.tournament_levels(x.level, window, circuit), 2)
        cx, co = x.ctb(), out.ctb()
        _check(self.L.bc_tournament(self.handle, keys.handle, circuit, window, 1 if want_max else 0,
                                    ctypes.byref(cx), ctypes.byref(co), _stream()))
        return out.take(co)

    # ------------------------------------------------ F_{p^d} slots
    def fpd_info(self):
        """(d, Frobenius rotation steps) of ``bc_fpd_info``."""
        d, n = ctypes.c_int32(), ctypes.c_int32()
        steps = (ctypes.c_int32 * 32)()
        _check(self.L.bc_fpd_info(self.handle, ctypes.byref(d), ctypes.byref(n), steps, 32))
        return d.value, list(steps[: n.value])

    def encode_fpd(self, elems) -> np.ndarray:
        """elems[count][M][d] -> plaintext coefficients [count][N] (``bc_encode_fpd``)."""
        d = self.N // self.M
        elems = np.ascontiguousarray(elems, dtype=np.uint32).reshape(-1, self.M, d)
        out = np.zeros((elems.shape[0], self.N), dtype=np.uint32)
        _check(self.L.bc_encode_fpd(self.handle, _np_ptr(elems), elems.shape[0], _np_ptr(out)))
        return out

    def decode_fpd(self, coeffs) -> np.ndarray:
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint32).reshape(-1, self.N)
        out = np.zeros((coeffs.shape[0], self.M, self.N // self.M), dtype=np.uint32)
        _check(self.L.bc_decode_fpd(self.handle, _np_ptr(coeffs), coeffs.shape[0], _np_ptr(out)))
        return out

    def encrypt_poly(self, keys: Keys, coeffs, u, errors, out: Batch | None = None) -> Batch:
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint32).reshape(-1, self.N)
        count = coeffs.shape[0]
        u = np.ascontiguousarray(u, dtype=np.int8).reshape(count, self.N)
        e = np.ascontiguousarray(errors, dtype=np.int32).reshape(count, 2, self.N)
        out = out or self.new_batch(count, self.nQ - 1, 2)
        c = out.ctb()
        _check(self.L.bc_encrypt_poly(self.handle, keys.handle, _np_ptr(coeffs), _np_ptr(u), _np_ptr(e),
                                      ctypes.byref(c), _stream()))
        return out.take(c)

    def extract_digits(self, keys: Keys, x: Batch, digits, out: Batch = None) -> Batch:
        """Coordinates ``digits`` of every F_{p^d} slot as F_p slot values
        (``bc_extract_digits``): digit-major, len(digits) * x.count ciphertexts."""
        dg = np.ascontiguousarray(digits, dtype=np.int32).reshape(-1)
        if out is None:
            out = self.new_batch(x.count * len(dg), x.level, 2)
        cx, co = x.ctb(), out.ctb()
        _check(self.L.bc_extract_digits(self.handle, keys.handle, ctypes.byref(cx), _np_ptr(dg), len(dg),
                                        ctypes.byref(co), _stream()))
        return out.take(co)

    def compare_fpd(self, keys: Keys, a: Batch, b: Batch, ndigits: int, circuit: int = BC_CIRCUIT_BIVARIATE,
                    want_max: bool = False, want_min: bool = False):
        """Integers packed as F_{p^d} slot elements (coordinate ndigits - 1 the
        most significant base-p digit): both operands' digits extracted
        (``bc_extract_digits``), then the lexicographic comparison of the
        digit planes (``bc_compare_max_min``).  Returns (lt, [max planes],
        [min planes]) as ``compare_max_min`` does."""
        order = list(range(ndigits - 1, -1, -1))
        A = self.extract_digits(keys, a, order).split(ndigits)
        B = self.extract_digits(keys, b, order).split(ndigits)
        return self.compare_max_min(keys, A, B, True, want_max, want_min, circuit=circuit)

    def set_exec_mode(self, mode: int):
        _check(self.L.bc_set_exec_mode(self.handle, mode))

    def set_tuning(self, key: int, value: int):
        _check(self.L.bc_set_tuning(self.handle, key, int(value)))

    def autotune(self) -> dict:
        """Picks the fastest transform schedule for this context; returns it."""
        _check(self.L.bc_autotune(self.handle, _stream()))
        return {"single_pass": self.get_tuning(BC_TUNE_NTT_SINGLE_PASS),
                "chunk_bytes": self.get_tuning(BC_TUNE_NTT_CHUNK_BYTES),
                "fp64": self.get_tuning(BC_TUNE_FP64),
                "parts_log": self.get_tuning(BC_TUNE_NTT_PARTS)}

    def autotune_mul(self, keys: Keys) -> dict:
        """Picks the fastest arithmetic, transform schedule and key-switching
        forms for a whole multiplication (``bc_autotune_mul``); returns them."""
        _check(self.L.bc_autotune_mul(self.handle, keys.handle, _stream()))
        return {"single_pass": self.get_tuning(BC_TUNE_NTT_SINGLE_PASS),
                "chunk_bytes": self.get_tuning(BC_TUNE_NTT_CHUNK_BYTES),
                "fp64": self.get_tuning(BC_TUNE_FP64),
                "parts_log": self.get_tuning(BC_TUNE_NTT_PARTS),
                "raw_handoff": self.get_tuning(BC_TUNE_RAW_HANDOFF),
                "mfma_modup": self.get_tuning(BC_TUNE_MFMA_MODUP)}

    def get_tuning(self, key: int) -> int:
        v = ctypes.c_int64()
        _check(self.L.bc_get_tuning(self.handle, key, ctypes.byref(v)))
        return v.value

    def profile_enable(self, on: bool):
        _check(self.L.bc_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, kind: int):
        """(milliseconds, launch pairs, algorithmic bytes) for BC_PROF_* `kind`."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(self.L.bc_profile_read(self.handle, kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    def compare_max_min(self, keys: Keys, a_digits, b_digits, want_lt=True, want_max=True, want_min=True, outs=None,
                        circuit: int = BC_CIRCUIT_UNIVARIATE):
        """Returns (lt, [max planes], [min planes]); ``outs`` reuses earlier output batches.
        circuit: BC_CIRCUIT_UNIVARIATE (digits in [0, (p-1)/2]) or
        BC_CIRCUIT_BIVARIATE (full-range digits, ``bc_compare_bivariate``)."""
        nd = len(a_digits)
        G = a_digits[0].count
        ltl, mml = self.compare_levels(a_digits[0].level, nd, circuit)
        if outs is None:
            lt = self.new_batch(G, ltl) if want_lt else None
            mx = [self.new_batch(G, mml) for _ in range(nd)] if want_max else None
            mn = [self.new_batch(G, mml) for _ in range(nd)] if want_min else None
        else:
            lt, mx, mn = outs
        A, B = _ctb_array(a_digits), _ctb_array(b_digits)
        clt = lt.ctb() if lt is not None else None
        cmx = _ctb_array(mx) if mx is not None else None
        cmn = _ctb_array(mn) if mn is not None else None
        fn = self.L.bc_compare_bivariate if circuit == BC_CIRCUIT_BIVARIATE else self.L.bc_compare_max_min
        _check(fn(self.handle, keys.handle, nd, A, B, ctypes.byref(clt) if clt is not None else None, cmx, cmn,
                  _stream()))
        if lt is not None:
            lt.take(clt)
        if mx is not None:
            _take_array(mx, cmx)
        if mn is not None:
            _take_array(mn, cmn)
        return lt, mx, mn

    def compare_lt(self, keys: Keys, a_digits, b_digits) -> Batch:
        return self.compare_max_min(keys, a_digits, b_digits, True, False, False)[0]


class Group:
    """Several contexts (ring sizes) whose comparison batches run together
    (``bc_group_*``): as a fork/join of ordinary launches (the default) or as
    one persistent launch draining a device work queue (BC_GROUP_PERSISTENT);
    either is recorded into a hipGraph."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        self.L = lib()
        arr = (ctypes.c_void_p * len(self.contexts))(*[c.handle.value for c in self.contexts])
        h = ctypes.c_void_p()
        _check(self.L.bc_group_create(len(self.contexts), arr, ctypes.byref(h)))
        self.handle = h
        self._keep = []

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bc_group_destroy(self.handle)
            self.handle = None

    def set_mode(self, mode: int):
        _check(self.L.bc_group_set_mode(self.handle, mode))

    def mode(self):
        """(mode, stages, tickets, workgroups) of the last persistent launch."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(self.L.bc_group_get_mode(self.handle, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def compare_max_min(self, requests, outs=None, want_lt=True, want_max=True, want_min=True):
        """requests: list over members of (keys, a_digits, b_digits).  Returns
        per member (lt, [max planes], [min planes]); ``outs`` reuses earlier outputs."""
        n = len(self.contexts)
        assert len(requests) == n
        if outs is None:
            outs = []
            for c, (k, a, b) in zip(self.contexts, requests):
                ltl, mml = c.compare_levels(a[0].level, len(a))
                G = a[0].count
                outs.append((c.new_batch(G, ltl) if want_lt else None,
                             [c.new_batch(G, mml) for _ in a] if want_max else None,
                             [c.new_batch(G, mml) for _ in a] if want_min else None))
        keys = (ctypes.c_void_p * n)(*[k.handle.value for (k, _, _) in requests])
        nd = (ctypes.c_int32 * n)(*[len(a) for (_, a, _) in requests])
        PA = ctypes.POINTER(bc_ctb)
        A = [_ctb_array(a) for (_, a, _) in requests]
        B = [_ctb_array(b) for (_, _, b) in requests]
        LT = [ctypes.pointer(o[0].ctb()) if o[0] is not None else None for o in outs]
        MX = [_ctb_array(o[1]) if o[1] is not None else None for o in outs]
        MN = [_ctb_array(o[2]) if o[2] is not None else None for o in outs]
        self._keep = [A, B, LT, MX, MN]
        pa = (PA * n)(*[ctypes.cast(x, PA) for x in A])
        pb = (PA * n)(*[ctypes.cast(x, PA) for x in B])
        plt = (PA * n)(*[ctypes.cast(x, PA) if x is not None else PA() for x in LT]) if want_lt else None
        pmx = (PA * n)(*[ctypes.cast(x, PA) if x is not None else PA() for x in MX]) if want_max else None
        pmn = (PA * n)(*[ctypes.cast(x, PA) if x is not None else PA() for x in MN]) if want_min else None
        _check(self.L.bc_group_compare(self.handle, keys, nd, pa, pb, plt, pmx, pmn, _stream()))
        for o, lt_c, mx_c, mn_c in zip(outs, LT, MX, MN):
            if o[0] is not None:
                o[0].take(lt_c.contents)
            if o[1] is not None:
                _take_array(o[1], mx_c)
            if o[2] is not None:
                _take_array(o[2], mn_c)
        return outs


class Bluestein:
    """Transforms of Z_q[X]/(Phi_m(X)), m odd (``bc_bluestein_*``): polynomials
    as torch uint64 tensors [count][nprimes][n] on the device."""

    def __init__(self, m: int, nprimes: int, bits: int = 50):
        self.L = lib()
        h = ctypes.c_void_p()
        _check(self.L.bc_bluestein_create(m, nprimes, bits, ctypes.byref(h)))
        self.handle = h
        n, conv = ctypes.c_int32(), ctypes.c_int32()
        mods = (ctypes.c_uint64 * nprimes)()
        _check(self.L.bc_bluestein_info(h, ctypes.byref(n), ctypes.byref(conv), mods))
        self.m, self.n, self.conv_len, self.nprimes = m, n.value, conv.value, nprimes
        self.moduli = [int(x) for x in mods]

    def __del__(self):
        if getattr(self, "handle", None):
            self.L.bc_bluestein_destroy(self.handle)
            self.handle = None

    def new(self, count: int):
        import torch

        return torch.zeros((count, self.nprimes, self.n), dtype=torch.uint64, device="cuda")

    def _run(self, fn, x, out):
        import torch

        assert x.dtype == torch.uint64 and x.is_cuda and x.is_contiguous() and tuple(x.shape[1:]) == (self.nprimes, self.n)
        if out is None:
            out = self.new(x.shape[0])
        _check(fn(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.shape[0], _stream()))
        return out

    def forward(self, x, out=None):
        return self._run(self.L.bc_bluestein_forward, x, out)

    def inverse(self, x, out=None):
        return self._run(self.L.bc_bluestein_inverse, x, out)
