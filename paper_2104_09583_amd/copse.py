"""Thin ctypes binding of libcopse (include/copse.h).

Every function here only marshals arguments into the C ABI of the same name;
all computation happens in the HIP library.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcopse.so")

COPSE_OK = 0
COPSE_EINVAL = -1
COPSE_ECAPACITY = -2
COPSE_ENOMEM = -3
COPSE_EDEVICE = -4
COPSE_ENOISE = -5
COPSE_EKEY = -6
COPSE_ETIMEOUT = -7

OP_ADD, OP_SUB, OP_TENSOR, OP_RELIN, OP_MODSWITCH, OP_MUL, OP_ROTATE, OP_MUL_PLAIN, OP_ADD_PLAIN = range(1, 10)

(PROF_NTT_FWD_ROWS, PROF_NTT_FWD_COLS, PROF_NTT_INV_ROWS, PROF_NTT_INV_COLS, PROF_KS_INNER, PROF_BCONV,
 PROF_ELEMENTWISE, PROF_NTT_FWD_ROWS_MODDOWN, PROF_NTT_FWD_ROWS_MODSWITCH, PROF_MATMUL_INNER,
 PROF_NTT_INV_ROWS_GATHER, PROF_STAGE_COMPARISON, PROF_STAGE_RESHUFFLE, PROF_STAGE_LEVELS,
 PROF_STAGE_AGGREGATION) = range(15)
PROF_KERNEL_KINDS = 11                 # kernel classes 0..10
PROF_STAGES = (11, 12, 13, 14)         # comparison, reshuffle, levels, aggregation
PROF_MORE_KERNEL_KINDS = (15, 16)      # relinearization inner products, giant-step sums
PROF_KINDS = 17


class CopseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"copse error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("t", ctypes.c_uint64), ("n_data_primes", ctypes.c_uint32),
                ("q0_max", ctypes.c_uint64), ("data_max", ctypes.c_uint64), ("alpha", ctypes.c_uint32),
                ("special_max", ctypes.c_uint64), ("device", ctypes.c_int)]


class CompileOptions(ctypes.Structure):
    _fields_ = [("fold", ctypes.c_int), ("n1_R", ctypes.c_uint32), ("n1_L", ctypes.c_uint32),
                ("n1_F", ctypes.c_uint32), ("server_replication", ctypes.c_int), ("result_privacy", ctypes.c_int),
                ("privacy_seed", ctypes.c_uint8 * 32), ("n_pad", ctypes.c_uint32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("top_level", ctypes.c_uint32), ("batch_lo", ctypes.c_uint32),
                ("batch_hi", ctypes.c_uint32), ("model", ctypes.c_int32), ("mm_cap", ctypes.c_int32),
                ("mm_waves", ctypes.c_int32), ("ks_jobs", ctypes.c_int32), ("bridge_wgs", ctypes.c_int32),
                ("gsum_b", ctypes.c_int32)]


TUNE_KNOBS = ("mm_cap", "mm_waves", "ks_jobs", "bridge_wgs", "gsum_b")
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def load_tuning(path: str = TUNING_PATH) -> list:
    """The committed autotuner choices (a list of dicts with log_n, top_level, batch [lo, hi], model and
    knobs); [] when there is no file."""
    import json
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f).get("entries", [])


class Meta(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "n_features", "precision", "K", "q", "b", "m", "d", "n_trees", "block_w", "queries_per_ct",
        "n1_R", "n1_L", "fold", "depth", "log_n", "server_rep", "n1_F")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_SHUTTING_DOWN = False


def _mark_shutdown():
    global _SHUTTING_DOWN
    _SHUTTING_DOWN = True


atexit.register(_mark_shutdown)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_09583_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, u8p, u32p, u64p, i32p, i64p = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8),
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64))
    PP = ctypes.POINTER(ctypes.c_void_p)
    sz, i32, u32, u64, dbl = ctypes.c_size_t, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "copse_ctx_create": [ctypes.POINTER(Params), PP],
        "copse_ctx_primes": [P, u64p, sz, ctypes.POINTER(sz)],
        "copse_ctx_set_stream": [P, P],
        "copse_ctx_sync": [P],
        "copse_ctx_set_tuning": [P, ctypes.POINTER(TuneEntry), sz],
        "copse_forest_compile": [ctypes.c_char_p, sz, u32, u32, u32, i32, u32, u32, PP, ctypes.POINTER(Meta)],
        "copse_compiled_rotations": [ctypes.POINTER(Meta), i32p, sz, ctypes.POINTER(sz)],
        "copse_forest_compile_private": [ctypes.c_char_p, sz, u32, u32, u32, i32, u32, u32, u8p, u32, PP,
                                         ctypes.POINTER(Meta)],
        "copse_compiled_codebook": [P, u32p, sz, ctypes.POINTER(sz)],
        "copse_forest_compile_ex": [ctypes.c_char_p, sz, u32, u32, u32, ctypes.POINTER(CompileOptions), PP,
                                    ctypes.POINTER(Meta)],
        "copse_keygen": [P, u8p, i32p, sz, i32, PP],
        "copse_keys_export_eval": [P, P, PP],
        "copse_model_encode": [P, P, P, i32, u8p, PP],
        "copse_query_encrypt": [P, P, ctypes.POINTER(Meta), u32p, sz, u8p, u32, PP],
        "copse_cts_level": [P, sz],
        "copse_evaluate": [P, P, P, P, PP],
        "copse_evaluate_batch": [P, P, P, PP, sz, PP],
        "copse_evaluate_plain": [P, P, P, P, PP],
        "copse_evaluate_noalloc": [P, P, P, P, P],
        "copse_exec_create": [P, P, P, sz, PP],
        "copse_exec_run": [P, PP, sz, PP],
        "copse_decrypt_labels": [P, P, ctypes.POINTER(Meta), P, sz, u8p, sz],
        "copse_encrypt_slots": [P, P, u64p, i32, u8p, u64, PP],
        "copse_decrypt_slots": [P, P, P, sz, u64p],
        "copse_cts_export": [P, P, u64p, sz, ctypes.POINTER(sz)],
        "copse_cts_import": [P, u64p, sz, PP],
        "copse_ct_op": [P, P, i32, P, sz, P, sz, ctypes.c_int32, u64p, PP],
        "copse_ct_rotate_many": [P, P, P, sz, i32p, sz, PP],
        "copse_poly_mul": [P, i32, u64p, u64p, u64p],
        "copse_profile_enable": [P, i32],
        "copse_profile_read": [P, i32, u64p, ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32],
        "copse_test_shake256": [u8p, sz, u8p, sz],
        "copse_chain_primes": [ctypes.POINTER(Params), u64p, sz, ctypes.POINTER(sz)],
        "copse_calib_copy": [P, sz],
        "copse_test_encode": [u32, u64, u64p, i64p],
        "copse_test_sample": [u8p, ctypes.c_char_p, u64, u32, i32, u64, sz, i64p],
        "copse_server_create": [P, sz, i32, PP],
        "copse_server_add_model": [P, P, P, ctypes.POINTER(ctypes.c_int)],
        "copse_server_submit": [P, i32, P, u64p],
        "copse_server_wait": [P, u64, i32, PP],
        "copse_server_latency": [P, u64, ctypes.POINTER(dbl)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("copse_ctx_destroy", "copse_compiled_destroy", "copse_keys_destroy", "copse_model_destroy",
                 "copse_cts_destroy", "copse_server_destroy", "copse_exec_destroy"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = None
    L.copse_ctx_stream.argtypes = [P]
    L.copse_ctx_stream.restype = P
    L.copse_ctx_device_bytes.argtypes = [P]
    L.copse_ctx_device_bytes.restype = sz
    L.copse_keys_bytes.argtypes = [P]
    L.copse_keys_bytes.restype = sz
    L.copse_model_bytes.argtypes = [P]
    L.copse_model_bytes.restype = sz
    L.copse_cts_count.argtypes = [P]
    L.copse_cts_count.restype = sz
    L.copse_last_error.argtypes = []
    L.copse_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != COPSE_OK:
        raise CopseError(rc, lib().copse_last_error().decode())


def _u8(b: bytes):
    assert len(b) >= 1
    return (ctypes.c_uint8 * len(b)).from_buffer_copy(b)


def _arr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ---------------------------------------------------------------- handles
class _Handle:
    _destroy = None

    def __init__(self, ptr: ctypes.c_void_p, owner=None):
        self.ptr = ptr
        self.owner = owner

    def close(self):
        if self.ptr and self.ptr.value:
            getattr(lib(), self._destroy)(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        if _SHUTTING_DOWN:
            return   # the process is exiting: leave the memory to the OS
        try:
            self.close()
        except Exception:
            pass


class Cts(_Handle):
    _destroy = "copse_cts_destroy"

    def __len__(self):
        return lib().copse_cts_count(self.ptr)

    def level(self, i: int = 0) -> int:
        return lib().copse_cts_level(self.ptr, i)

    def release(self) -> ctypes.c_void_p:
        p = self.ptr
        self.ptr = ctypes.c_void_p()
        return p


class Keys(_Handle):
    _destroy = "copse_keys_destroy"

    def nbytes(self) -> int:
        return lib().copse_keys_bytes(self.ptr)


class Compiled(_Handle):
    _destroy = "copse_compiled_destroy"


class Model(_Handle):
    _destroy = "copse_model_destroy"

    def nbytes(self) -> int:
        return lib().copse_model_bytes(self.ptr)


class Context(_Handle):
    _destroy = "copse_ctx_destroy"

    def __init__(self, log_n: int, n_data_primes: int, q0_max: int, data_max: int, alpha: int,
                 special_max: int, t: int = 65537, device: int = 0, tuning: bool = True):
        p = Params(log_n, t, n_data_primes, q0_max, data_max, alpha, special_max, device)
        h = ctypes.c_void_p()
        check(lib().copse_ctx_create(ctypes.byref(p), ctypes.byref(h)))
        super().__init__(h)
        self.N = 1 << log_n
        self.log_n = log_n
        self.t = t
        self.L = n_data_primes - 1
        self.alpha = alpha
        if tuning:
            # the committed autotuner choices for this ring and chain length
            self.set_tuning([e for e in load_tuning() if e["log_n"] == log_n and e["top_level"] == self.L])

    def set_tuning(self, entries: Sequence[dict]) -> None:
        """Installs launch-shape knobs (copse_ctx_set_tuning); each entry: log_n, top_level, batch [lo, hi],
        model (-1 any, 0 plaintext, 1 encrypted) and knobs {name: value} (missing or 0: built in)."""
        arr = (TuneEntry * max(1, len(entries)))()
        for i, e in enumerate(entries):
            k = e.get("knobs", {})
            arr[i] = TuneEntry(e["log_n"], e["top_level"], e["batch"][0], e["batch"][1], e.get("model", -1),
                               *[int(k.get(n, 0)) for n in TUNE_KNOBS])
        check(lib().copse_ctx_set_tuning(self.ptr, arr, len(entries)))

    # context
    def primes(self) -> List[int]:
        n = ctypes.c_size_t()
        check(lib().copse_ctx_primes(self.ptr, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.uint64)
        check(lib().copse_ctx_primes(self.ptr, _arr(out, ctypes.c_uint64), n.value, ctypes.byref(n)))
        return [int(x) for x in out]

    def stream(self) -> int:
        return lib().copse_ctx_stream(self.ptr)

    def set_stream(self, stream: Optional[int]) -> None:
        check(lib().copse_ctx_set_stream(self.ptr, ctypes.c_void_p(stream) if stream else None))

    def sync(self) -> None:
        check(lib().copse_ctx_sync(self.ptr))

    def device_bytes(self) -> int:
        return lib().copse_ctx_device_bytes(self.ptr)

    # keys
    def keygen(self, seed: bytes, rotations: Sequence[int], relin: bool = True) -> Keys:
        r = np.ascontiguousarray(np.array(list(rotations), dtype=np.int32))
        h = ctypes.c_void_p()
        check(lib().copse_keygen(self.ptr, _u8(seed), _arr(r, ctypes.c_int32), len(r), int(relin), ctypes.byref(h)))
        return Keys(h, self)

    def export_eval(self, keys: Keys) -> Keys:
        h = ctypes.c_void_p()
        check(lib().copse_keys_export_eval(self.ptr, keys.ptr, ctypes.byref(h)))
        return Keys(h, self)

    # model
    def model_encode(self, compiled: Compiled, keys: Optional[Keys] = None, encrypt: bool = False,
                     seed: Optional[bytes] = None) -> Model:
        h = ctypes.c_void_p()
        check(lib().copse_model_encode(self.ptr, compiled.ptr, keys.ptr if keys else None, int(encrypt),
                                       _u8(seed) if seed else None, ctypes.byref(h)))
        return Model(h, self)

    # queries
    def query_encrypt(self, keys: Keys, meta: Meta, features: np.ndarray, seed: bytes, group: int = 0) -> Cts:
        f = np.ascontiguousarray(np.asarray(features, dtype=np.uint32))
        h = ctypes.c_void_p()
        check(lib().copse_query_encrypt(self.ptr, keys.ptr, ctypes.byref(meta), _arr(f, ctypes.c_uint32),
                                        f.shape[0], _u8(seed), group, ctypes.byref(h)))
        return Cts(h, self)

    def evaluate(self, model: Model, keys: Keys, query: Cts) -> Cts:
        h = ctypes.c_void_p()
        check(lib().copse_evaluate(self.ptr, model.ptr, keys.ptr, query.ptr, ctypes.byref(h)))
        return Cts(h, self)

    def evaluate_noalloc(self, model: Model, keys: Keys, query: Cts, result: Cts) -> None:
        """copse_evaluate into the existing one-ciphertext handle `result`, every temporary in the library's
        scratch array (no device allocation); returns after the device has finished."""
        check(lib().copse_evaluate_noalloc(self.ptr, model.ptr, keys.ptr, query.ptr, result.ptr))

    def evaluate_plain(self, model: Model, keys: Keys, query: Cts) -> Cts:
        h = ctypes.c_void_p()
        check(lib().copse_evaluate_plain(self.ptr, model.ptr, keys.ptr, query.ptr, ctypes.byref(h)))
        return Cts(h, self)

    def evaluate_batch(self, model: Model, keys: Keys, queries: Sequence[Cts]) -> List[Cts]:
        n = len(queries)
        arr = (ctypes.c_void_p * n)(*[q.ptr.value for q in queries])
        out = (ctypes.c_void_p * n)()
        check(lib().copse_evaluate_batch(self.ptr, model.ptr, keys.ptr, arr, n, out))
        return [Cts(ctypes.c_void_p(out[i]), self) for i in range(n)]

    def exec_create(self, model: Model, keys: Keys, n_groups: int) -> "Exec":
        h = ctypes.c_void_p()
        check(lib().copse_exec_create(self.ptr, model.ptr, keys.ptr, n_groups, ctypes.byref(h)))
        ex = Exec(h, self)
        ex._keep = (model, keys)
        ex.n_groups = n_groups
        return ex

    def decrypt_labels(self, keys: Keys, meta: Meta, result: Cts, n_queries: int) -> np.ndarray:
        bits = np.zeros(n_queries * meta.m, dtype=np.uint8)
        check(lib().copse_decrypt_labels(self.ptr, keys.ptr, ctypes.byref(meta), result.ptr, n_queries,
                                         _arr(bits, ctypes.c_uint8), bits.size))
        return bits.reshape(n_queries, meta.m)

    # raw ops
    def encrypt_slots(self, keys: Keys, slots: np.ndarray, level: int, seed: bytes, obj: int) -> Cts:
        s = np.ascontiguousarray(np.asarray(slots, dtype=np.uint64).reshape(-1))
        assert s.size == self.N
        h = ctypes.c_void_p()
        check(lib().copse_encrypt_slots(self.ptr, keys.ptr, _arr(s, ctypes.c_uint64), level, _u8(seed), obj,
                                        ctypes.byref(h)))
        return Cts(h, self)

    def decrypt_slots(self, keys: Keys, cts: Cts, i: int = 0) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.uint64)
        check(lib().copse_decrypt_slots(self.ptr, keys.ptr, cts.ptr, i, _arr(out, ctypes.c_uint64)))
        return out.reshape(2, self.N // 2).astype(np.int64)

    def export(self, cts: Cts) -> List[dict]:
        need = ctypes.c_size_t()
        check(lib().copse_cts_export(self.ptr, cts.ptr, None, 0, ctypes.byref(need)))
        buf = np.zeros(need.value, dtype=np.uint64)
        check(lib().copse_cts_export(self.ptr, cts.ptr, _arr(buf, ctypes.c_uint64), buf.size, ctypes.byref(need)))
        out, off = [], 0
        while off < buf.size:
            npolys, level, n = int(buf[off]), int(buf[off + 1]), int(buf[off + 2])
            off += 4
            words = npolys * (level + 1) * n
            out.append(dict(level=level, polys=[buf[off + k * (level + 1) * n: off + (k + 1) * (level + 1) * n]
                                                .reshape(level + 1, n) for k in range(npolys)]))
            off += words
        return out

    def import_(self, polys: Sequence[np.ndarray], level: int) -> Cts:
        parts = [np.array([len(polys), level, self.N, 0], dtype=np.uint64)]
        parts += [np.ascontiguousarray(p, dtype=np.uint64).reshape(-1) for p in polys]
        buf = np.ascontiguousarray(np.concatenate(parts))
        h = ctypes.c_void_p()
        check(lib().copse_cts_import(self.ptr, _arr(buf, ctypes.c_uint64), buf.size, ctypes.byref(h)))
        return Cts(h, self)

    def op(self, keys: Optional[Keys], op: int, a: Cts, b: Optional[Cts] = None, arg: int = 0,
           slots: Optional[np.ndarray] = None, ia: int = 0, ib: int = 0) -> Cts:
        h = ctypes.c_void_p()
        sp = None
        if slots is not None:
            s = np.ascontiguousarray(np.asarray(slots, dtype=np.uint64).reshape(-1))
            sp = _arr(s, ctypes.c_uint64)
        check(lib().copse_ct_op(self.ptr, keys.ptr if keys else None, op, a.ptr, ia, b.ptr if b else None, ib,
                                arg, sp, ctypes.byref(h)))
        return Cts(h, self)

    def rotate_many(self, keys: Keys, a: Cts, rots: Sequence[int], ia: int = 0) -> Cts:
        r = np.ascontiguousarray(np.array(list(rots), dtype=np.int32))
        h = ctypes.c_void_p()
        check(lib().copse_ct_rotate_many(self.ptr, keys.ptr, a.ptr, ia, _arr(r, ctypes.c_int32), len(r),
                                         ctypes.byref(h)))
        return Cts(h, self)

    def poly_mul(self, prime: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.zeros(self.N, dtype=np.uint64)
        check(lib().copse_poly_mul(self.ptr, prime, _arr(a, ctypes.c_uint64), _arr(b, ctypes.c_uint64),
                                   _arr(out, ctypes.c_uint64)))
        return out

    def calib_copy(self, nbytes: int) -> None:
        check(lib().copse_calib_copy(self.ptr, nbytes))

    def profile_enable(self, on: bool = True) -> None:
        check(lib().copse_profile_enable(self.ptr, int(on)))

    def profile_read(self, kind: int, reset: bool = False) -> dict:
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        nbytes = ctypes.c_double()
        check(lib().copse_profile_read(self.ptr, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nbytes),
                                       int(reset)))
        return dict(launches=n.value, ms=ms.value, bytes=nbytes.value)


def forest_compile(text: str, n_features: int, precision: int, log_n: int, fold: bool = False,
                   n1_R: int = 0, n1_L: int = 0):
    raw = text.encode()
    h = ctypes.c_void_p()
    meta = Meta()
    check(lib().copse_forest_compile(raw, len(raw), n_features, precision, log_n, int(fold), n1_R, n1_L,
                                     ctypes.byref(h), ctypes.byref(meta)))
    return Compiled(h), meta


def forest_compile_private(text: str, n_features: int, precision: int, log_n: int, seed: bytes, n_pad: int,
                           fold: bool = False, n1_R: int = 0, n1_L: int = 0):
    raw = text.encode()
    h = ctypes.c_void_p()
    meta = Meta()
    check(lib().copse_forest_compile_private(raw, len(raw), n_features, precision, log_n, int(fold), n1_R, n1_L,
                                             _u8(seed), n_pad, ctypes.byref(h), ctypes.byref(meta)))
    return Compiled(h), meta


def forest_compile_ex(text: str, n_features: int, precision: int, log_n: int, fold: bool = False,
                      n1_R: int = 0, n1_L: int = 0, n1_F: int = 0, server_replication: bool = False,
                      privacy_seed: Optional[bytes] = None, n_pad: int = 0):
    raw = text.encode()
    o = CompileOptions()
    o.fold, o.n1_R, o.n1_L, o.n1_F = int(fold), n1_R, n1_L, n1_F
    o.server_replication = int(server_replication)
    if privacy_seed is not None:
        o.result_privacy = 1
        o.privacy_seed[:] = list(privacy_seed)
        o.n_pad = n_pad
    h = ctypes.c_void_p()
    meta = Meta()
    check(lib().copse_forest_compile_ex(raw, len(raw), n_features, precision, log_n, ctypes.byref(o),
                                        ctypes.byref(h), ctypes.byref(meta)))
    return Compiled(h), meta


def compiled_codebook(compiled: Compiled) -> List[int]:
    n = ctypes.c_size_t()
    check(lib().copse_compiled_codebook(compiled.ptr, None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), dtype=np.uint32)
    check(lib().copse_compiled_codebook(compiled.ptr, _arr(out, ctypes.c_uint32), out.size, ctypes.byref(n)))
    return [int(x) for x in out[:n.value]]


def compiled_rotations(meta: Meta) -> List[int]:
    n = ctypes.c_size_t()
    check(lib().copse_compiled_rotations(ctypes.byref(meta), None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), dtype=np.int32)
    check(lib().copse_compiled_rotations(ctypes.byref(meta), _arr(out, ctypes.c_int32), out.size, ctypes.byref(n)))
    return [int(x) for x in out[:n.value]]


def shake256(msg: bytes, n: int) -> bytes:
    out = (ctypes.c_uint8 * n)()
    m = _u8(msg) if msg else (ctypes.c_uint8 * 1)()
    check(lib().copse_test_shake256(m, len(msg), out, n))
    return bytes(out)


def sample(seed: bytes, domain: str, obj: int, limb: int, kind: int, q: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int64)
    check(lib().copse_test_sample(_u8(seed), domain.encode(), obj, limb, kind, q, n, _arr(out, ctypes.c_int64)))
    return out


def chain_primes(log_n: int, n_data_primes: int, q0_max: int, data_max: int, alpha: int, special_max: int,
                 t: int = 65537) -> List[int]:
    p = Params(log_n, t, n_data_primes, q0_max, data_max, alpha, special_max, 0)
    n = ctypes.c_size_t()
    check(lib().copse_chain_primes(ctypes.byref(p), None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.uint64)
    check(lib().copse_chain_primes(ctypes.byref(p), _arr(out, ctypes.c_uint64), out.size, ctypes.byref(n)))
    return [int(x) for x in out]


def encode(log_n: int, slots: np.ndarray, t: int = 65537) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(slots, dtype=np.uint64).reshape(-1))
    out = np.zeros(1 << log_n, dtype=np.int64)
    check(lib().copse_test_encode(log_n, t, _arr(s, ctypes.c_uint64), _arr(out, ctypes.c_int64)))
    return out


class Exec(_Handle):
    """Captured evaluation of one model over a fixed number of query groups (copse_exec_*)."""
    _destroy = "copse_exec_destroy"

    def run(self, queries: Sequence[Cts]) -> List[Cts]:
        n = len(queries)
        arr = (ctypes.c_void_p * n)(*[q.ptr.value for q in queries])
        out = (ctypes.c_void_p * max(1, n))()
        check(lib().copse_exec_run(self.ptr, arr, n, out))
        return [Cts(ctypes.c_void_p(out[i]), self.owner) for i in range(n)]


class Server(_Handle):
    """Request loop over resident models (copse_server_*)."""
    _destroy = "copse_server_destroy"

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_batch: int = 8):
        h = ctypes.c_void_p()
        check(lib().copse_server_create(ctx.ptr, hbm_budget_bytes, max_batch, ctypes.byref(h)))
        super().__init__(h, ctx)
        self._keep = []

    def add_model(self, model: Model, eval_keys: Keys) -> int:
        mid = ctypes.c_int()
        check(lib().copse_server_add_model(self.ptr, model.ptr, eval_keys.ptr, ctypes.byref(mid)))
        self._keep.append((model, eval_keys))
        return mid.value

    def submit(self, model_id: int, query: Cts) -> int:
        t = ctypes.c_uint64()
        rc = lib().copse_server_submit(self.ptr, model_id, query.ptr, ctypes.byref(t))
        check(rc)
        query.release()   # ownership moved to the server
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> Cts:
        h = ctypes.c_void_p()
        check(lib().copse_server_wait(self.ptr, ticket, timeout_ms, ctypes.byref(h)))
        return Cts(h, self.owner)

    def latency_ms(self, ticket: int) -> float:
        v = ctypes.c_double()
        check(lib().copse_server_latency(self.ptr, ticket, ctypes.byref(v)))
        return v.value
