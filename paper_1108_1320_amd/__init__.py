"""Python binding of the cmm HIP library (libcmm.so).

Argument marshalling only: every step of the sketch product, decoding and
selection runs in the library's HIP kernels.  Functions carry the C names
(``cmm_sketch_product`` ...) and take torch tensors for device buffers; a
small object layer (``Context``, ``Sketch``) frees handles automatically.

The library must have been built (``python -m paper_1108_1320_amd.build``);
``load()`` raises if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmm.so")

CMM_OK, CMM_EINVAL, CMM_ENOMEM, CMM_EHIP, CMM_EUNSUPPORTED, CMM_ESTATE = 0, -1, -2, -3, -4, -5
CMM_F32, CMM_BF16, CMM_FP8_E4M3 = 0, 1, 2
CMM_SUBTRACT_DIAG, CMM_ASYNC, CMM_AUTOTUNE = 1, 2, 4
CMM_TOPK_ALL, CMM_TOPK_UPPER, CMM_TOPK_PER_COLUMN = 0, 1, 2
DTYPES = {"f32": CMM_F32, "bf16": CMM_BF16, "fp8": CMM_FP8_E4M3}
MODES = {"all": CMM_TOPK_ALL, "upper": CMM_TOPK_UPPER, "column": CMM_TOPK_PER_COLUMN}

_lib = None

_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_U32 = C.c_uint32
_U64 = C.c_uint64


class cmm_problem(C.Structure):
    """One product of a batch (the C struct of the same name)."""
    _fields_ = [("A", _P), ("lda", _I64), ("B", _P), ("ldb", _I64), ("n1", _I64), ("m", _I64),
                ("n3", _I64), ("b", _I64), ("d", _I32), ("dtype", _I32), ("scaleA", _P),
                ("scaleB", _P), ("seed", _U64), ("flags", _U32), ("reserved", _U32)]


_PROB = C.POINTER(cmm_problem)
_I32P = C.POINTER(_I32)

_SIGS = {
    "cmm_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "cmm_ctx_set_stream": (C.c_int, [_P, _P]),
    "cmm_ctx_set_workspace_limit": (C.c_int, [_P, _I64]),
    "cmm_ctx_destroy": (C.c_int, [_P]),
    "cmm_strerror": (C.c_char_p, [C.c_int]),
    "cmm_last_error": (C.c_char_p, [_P]),
    "cmm_ctx_profile": (C.c_int, [_P, C.c_int]),
    "cmm_ctx_profile_read": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(_I64)]),
    "cmm_ctx_profile_bytes": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cmm_stream_probe": (C.c_int, [_P, _I64, _I64, _I32, _I32, C.POINTER(C.c_double)]),
    "cmm_sketch_product": (C.c_int, [_P, _P, _P, _I64, _I64, _I32, _U64, C.POINTER(_P)]),
    "cmm_sketch_product_ex": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P,
                                        _I64, _I32, _U64, _P, _U32, C.POINTER(_P)]),
    "cmm_sketch_product_tables": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P,
                                            _I64, _I32, _P, _P, _P, _P, _U32, C.POINTER(_P)]),
    "cmm_sketch_product_noalloc": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P,
                                             _I64, _I32, _U64, _U32, _P]),
    "cmm_sketch_free": (C.c_int, [_P]),
    "cmm_sketch_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64),
                                  C.POINTER(_I64), C.POINTER(_I32)]),
    "cmm_sketch_copy_c": (C.c_int, [_P, _P, _I64, _I32]),
    "cmm_sketch_hash_params": (C.c_int, [_P, _P]),
    "cmm_sketch_hashes": (C.c_int, [_P, _I32, _P, _P, _P, _P]),
    "cmm_sketch_subtract_diagonal": (C.c_int, [_P, _P, _I64]),
    "cmm_sketch_merge": (C.c_int, [_P, _P]),
    "cmm_estimate": (C.c_int, [_P, _I64, _I64, C.POINTER(C.c_double)]),
    "cmm_estimate_batch": (C.c_int, [_P, _P, _P, _I64, _P]),
    "cmm_topk": (C.c_int, [_P, _I32, _I32, _P, _P, _P]),
    "cmm_batch_create": (C.c_int, [_P, _PROB, _I32, _U32, C.POINTER(_P)]),
    "cmm_batch_run": (C.c_int, [_P, _U32]),
    "cmm_batch_sketch": (C.c_int, [_P, _I32, C.POINTER(_P)]),
    "cmm_batch_topk": (C.c_int, [_P, _I32P, _I32, _P, _P, _P]),
    "cmm_batch_free": (C.c_int, [_P]),
    "cmm_sketch_product_batched": (C.c_int, [_P, _PROB, _I32, C.POINTER(_P)]),
    "cmm_autotune": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I32, _I32, _I32P,
                               C.POINTER(C.c_double)]),
    "cmm_tuning_get": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I32, _I32, _I32P]),
    "cmm_tuning_set": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I32, _I32, _I32P]),
    "cmm_tuning_save": (C.c_int, [_P, C.c_char_p]),
    "cmm_tuning_load": (C.c_int, [_P, C.c_char_p]),
    "cmm_frobenius_bound": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P, _I32,
                                      _U64, _U32, _P, C.POINTER(C.c_double)]),
    "cmm_frobenius_signs": (C.c_int, [_P, _I64, _I64, _I32, _U64, _P, _P]),
    "cmm_sketch_product_sparse": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _I64, _I64, _I64, _I64, _I32,
                                            _U64, _U32, C.POINTER(_P)]),
    "cmm_estimate_nnz": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P, _I32, _U64,
                                   _U32, C.c_double, C.POINTER(_I64), _P]),
    "cmm_find_significant": (C.c_int, [_P, _P, _I64, _P, _I64, _I64, _I64, _I64, _I32, _P, _P, _I64,
                                       _I32, _U64, _U32, C.c_double, _I64, _P, _P,
                                       C.POINTER(_I64), C.POINTER(_P)]),
}

EXPORTED = tuple(_SIGS)


class CmmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        super().__init__(f"{where}: {code} ({msg})")
        self.code = code


def load(path: str | None = None):
    """Load libcmm.so (once).  Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1108_1320_amd.build`")
    # torch first: libcmm.so then binds to the HIP runtime torch has loaded,
    # so both share one runtime (device memory and streams pass between them)
    import torch  # noqa: F401
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str, ctx=None):
    if rc != CMM_OK:
        lib = load()
        msg = lib.cmm_last_error(ctx).decode() if ctx else lib.cmm_strerror(rc).decode()
        raise CmmError(rc, where, msg)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ C names

def cmm_ctx_create(device: int = 0, stream=None):
    lib = load()
    out = _P()
    s = stream if stream is not None else _current_stream()
    _check(lib.cmm_ctx_create(device, s, C.byref(out)), "cmm_ctx_create")
    return out


def cmm_ctx_destroy(ctx):
    _check(load().cmm_ctx_destroy(ctx), "cmm_ctx_destroy")


def cmm_ctx_set_stream(ctx, stream):
    _check(load().cmm_ctx_set_stream(ctx, stream), "cmm_ctx_set_stream", ctx)


def cmm_ctx_set_workspace_limit(ctx, nbytes: int):
    _check(load().cmm_ctx_set_workspace_limit(ctx, int(nbytes)), "cmm_ctx_set_workspace_limit", ctx)


def cmm_ctx_profile(ctx, enable: bool):
    _check(load().cmm_ctx_profile(ctx, int(enable)), "cmm_ctx_profile", ctx)


def cmm_ctx_profile_read(ctx, name: str):
    ms = C.c_double(); n = _I64()
    _check(load().cmm_ctx_profile_read(ctx, name.encode(), C.byref(ms), C.byref(n)),
           "cmm_ctx_profile_read", ctx)
    return ms.value, n.value


def cmm_ctx_profile_bytes(ctx, name: str):
    rd = C.c_double(); wr = C.c_double()
    _check(load().cmm_ctx_profile_bytes(ctx, name.encode(), C.byref(rd), C.byref(wr)),
           "cmm_ctx_profile_bytes", ctx)
    return rd.value, wr.value


def cmm_stream_probe(ctx, read_bytes: int, write_bytes: int, nontemporal: bool, reps: int):
    ms = C.c_double()
    _check(load().cmm_stream_probe(ctx, int(read_bytes), int(write_bytes), int(nontemporal), int(reps),
                                   C.byref(ms)), "cmm_stream_probe", ctx)
    return ms.value


def cmm_sketch_product(ctx, A, B, n: int, b: int, d: int, seed: int):
    out = _P()
    _check(load().cmm_sketch_product(ctx, _ptr(A), _ptr(B), n, b, d, seed, C.byref(out)),
           "cmm_sketch_product", ctx)
    return out


def cmm_sketch_product_ex(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, b, d, seed,
                          hash_params=None, flags=0):
    out = _P()
    hp = None
    if hash_params is not None:
        hp = np.ascontiguousarray(hash_params, dtype=np.uint64)
    _check(load().cmm_sketch_product_ex(
        ctx, _ptr(A), lda, _ptr(B), ldb, n1, m, n3, dtype, _ptr(scaleA), _ptr(scaleB), b, d, seed,
        None if hp is None else hp.ctypes.data_as(_P), flags, C.byref(out)),
        "cmm_sketch_product_ex", ctx)
    return out


def cmm_sketch_product_tables(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, b, d,
                              h1, s1, h2, s2, flags=0):
    out = _P()
    h1 = np.ascontiguousarray(h1, dtype=np.int32); s1 = np.ascontiguousarray(s1, dtype=np.int8)
    h2 = np.ascontiguousarray(h2, dtype=np.int32); s2 = np.ascontiguousarray(s2, dtype=np.int8)
    _check(load().cmm_sketch_product_tables(
        ctx, _ptr(A), lda, _ptr(B), ldb, n1, m, n3, dtype, _ptr(scaleA), _ptr(scaleB), b, d,
        h1.ctypes.data_as(_P), s1.ctypes.data_as(_P), h2.ctypes.data_as(_P), s2.ctypes.data_as(_P),
        flags, C.byref(out)), "cmm_sketch_product_tables", ctx)
    return out


def cmm_sketch_free(sk):
    _check(load().cmm_sketch_free(sk), "cmm_sketch_free")


def cmm_sketch_info(sk):
    n1, m, n3, b = _I64(), _I64(), _I64(), _I64(); d = _I32()
    _check(load().cmm_sketch_info(sk, C.byref(n1), C.byref(m), C.byref(n3), C.byref(b), C.byref(d)),
           "cmm_sketch_info")
    return n1.value, m.value, n3.value, b.value, d.value


def cmm_sketch_copy_c(sk, out=None):
    """c[d][b] as a float64 numpy array (or into a device tensor ``out``)."""
    n1, m, n3, b, d = cmm_sketch_info(sk)
    if out is not None:
        _check(load().cmm_sketch_copy_c(sk, _ptr(out), d * b, 1), "cmm_sketch_copy_c")
        return out
    host = np.empty((d, b), dtype=np.float64)
    _check(load().cmm_sketch_copy_c(sk, host.ctypes.data_as(_P), d * b, 0), "cmm_sketch_copy_c")
    return host


def cmm_sketch_hash_params(sk):
    n1, m, n3, b, d = cmm_sketch_info(sk)
    out = np.empty((d, 4, 2), dtype=np.uint64)
    _check(load().cmm_sketch_hash_params(sk, out.ctypes.data_as(_P)), "cmm_sketch_hash_params")
    return out


def cmm_sketch_hashes(sk, t: int):
    n1, m, n3, b, d = cmm_sketch_info(sk)
    h1 = np.empty(n1, np.int32); s1 = np.empty(n1, np.int8)
    h2 = np.empty(n3, np.int32); s2 = np.empty(n3, np.int8)
    _check(load().cmm_sketch_hashes(sk, t, h1.ctypes.data_as(_P), s1.ctypes.data_as(_P),
                                    h2.ctypes.data_as(_P), s2.ctypes.data_as(_P)),
           "cmm_sketch_hashes")
    return h1, s1, h2, s2


def cmm_sketch_subtract_diagonal(sk, diag):
    _check(load().cmm_sketch_subtract_diagonal(sk, _ptr(diag), diag.numel()),
           "cmm_sketch_subtract_diagonal")


def cmm_sketch_merge(dst, src):
    _check(load().cmm_sketch_merge(dst, src), "cmm_sketch_merge")


def cmm_estimate(sk, i: int, j: int) -> float:
    v = C.c_double()
    _check(load().cmm_estimate(sk, i, j, C.byref(v)), "cmm_estimate")
    return v.value


def cmm_estimate_batch(sk, i, j, out):
    _check(load().cmm_estimate_batch(sk, _ptr(i), _ptr(j), i.numel(), _ptr(out)),
           "cmm_estimate_batch")
    return out


def cmm_topk(sk, K: int, mode: int):
    n1, m, n3, b, d = cmm_sketch_info(sk)
    cnt = K * n3 if mode == CMM_TOPK_PER_COLUMN else K
    oi = np.empty(cnt, np.int64); oj = np.empty(cnt, np.int64); ov = np.empty(cnt, np.float32)
    _check(load().cmm_topk(sk, K, mode, oi.ctypes.data_as(_P), oj.ctypes.data_as(_P),
                           ov.ctypes.data_as(_P)), "cmm_topk")
    return oi, oj, ov


def _problems(probs):
    arr = (cmm_problem * len(probs))()
    for q, p in enumerate(probs):
        arr[q] = p
    return arr


def cmm_batch_create(ctx, probs, flags=0):
    out = _P()
    arr = _problems(probs)
    _check(load().cmm_batch_create(ctx, arr, len(probs), flags, C.byref(out)), "cmm_batch_create", ctx)
    return out


def cmm_batch_run(batch, flags=0, ctx=None):
    _check(load().cmm_batch_run(batch, flags), "cmm_batch_run", ctx)


def cmm_batch_sketch(batch, index: int):
    out = _P()
    _check(load().cmm_batch_sketch(batch, index, C.byref(out)), "cmm_batch_sketch")
    return out


def cmm_batch_topk(batch, Ks, mode: int, sizes):
    """cmm_batch_topk with K[q] = Ks[q]; `sizes` are the products' (n1, n3).
    Returns one (i, j, val) triple of host arrays per product."""
    Ks = np.ascontiguousarray(Ks, dtype=np.int32)
    cnt = [int(k) * (n3 if mode == CMM_TOPK_PER_COLUMN else 1) for k, (n1, n3) in zip(Ks, sizes)]
    tot = max(1, sum(cnt))
    oi = np.empty(tot, np.int64); oj = np.empty(tot, np.int64); ov = np.empty(tot, np.float32)
    _check(load().cmm_batch_topk(batch, Ks.ctypes.data_as(_I32P), mode, oi.ctypes.data_as(_P),
                                 oj.ctypes.data_as(_P), ov.ctypes.data_as(_P)), "cmm_batch_topk")
    out, off = [], 0
    for c in cnt:
        out.append((oi[off:off + c], oj[off:off + c], ov[off:off + c]))
        off += c
    return out


def cmm_batch_free(batch):
    _check(load().cmm_batch_free(batch), "cmm_batch_free")


def cmm_sketch_product_batched(ctx, probs):
    outs = (_P * len(probs))()
    arr = _problems(probs)
    _check(load().cmm_sketch_product_batched(ctx, arr, len(probs), outs), "cmm_sketch_product_batched", ctx)
    return [_P(h) for h in outs]


def cmm_autotune(ctx, n1, m, n3, b, d, dtype):
    t = (_I32 * 3)(); ms = C.c_double()
    _check(load().cmm_autotune(ctx, n1, m, n3, b, d, dtype, t, C.byref(ms)), "cmm_autotune", ctx)
    return (t[0], t[1], t[2]), ms.value


def cmm_tuning_get(ctx, n1, m, n3, b, d, dtype):
    t = (_I32 * 3)()
    _check(load().cmm_tuning_get(ctx, n1, m, n3, b, d, dtype, t), "cmm_tuning_get", ctx)
    return (t[0], t[1], t[2])


def cmm_tuning_set(ctx, n1, m, n3, b, d, dtype, tuning):
    t = (_I32 * 3)(*tuning)
    _check(load().cmm_tuning_set(ctx, n1, m, n3, b, d, dtype, t), "cmm_tuning_set", ctx)


def cmm_tuning_save(ctx, path: str):
    _check(load().cmm_tuning_save(ctx, path.encode()), "cmm_tuning_save", ctx)


def cmm_tuning_load(ctx, path: str):
    _check(load().cmm_tuning_load(ctx, path.encode()), "cmm_tuning_load", ctx)


def cmm_frobenius_bound(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, d, seed, flags=0):
    """Returns (X[d] float64, 32 * median X^2)."""
    X = np.empty(d, np.float64); bound = C.c_double()
    _check(load().cmm_frobenius_bound(ctx, _ptr(A), lda, _ptr(B), ldb, n1, m, n3, dtype,
                                      _ptr(scaleA), _ptr(scaleB), d, seed, flags,
                                      X.ctypes.data_as(_P), C.byref(bound)),
           "cmm_frobenius_bound", ctx)
    return X, bound.value


def cmm_frobenius_signs(ctx, n1, n3, d, seed):
    s1 = np.empty((d, n1), np.int8); s2 = np.empty((d, n3), np.int8)
    _check(load().cmm_frobenius_signs(ctx, n1, n3, d, seed, s1.ctypes.data_as(_P),
                                      s2.ctypes.data_as(_P)), "cmm_frobenius_signs", ctx)
    return s1, s2


def cmm_find_significant(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, b, d, seed,
                         flags, delta, cap=1 << 16, want_sketch=False):
    """Returns (i, j, total_count, sketch handle or None)."""
    oi = np.empty(max(cap, 1), np.int64); oj = np.empty(max(cap, 1), np.int64)
    cnt = _I64(); sk = _P()
    _check(load().cmm_find_significant(ctx, _ptr(A), lda, _ptr(B), ldb, n1, m, n3, dtype,
                                       _ptr(scaleA), _ptr(scaleB), b, d, seed, flags, delta, cap,
                                       oi.ctypes.data_as(_P), oj.ctypes.data_as(_P), C.byref(cnt),
                                       C.byref(sk) if want_sketch else None),
           "cmm_find_significant", ctx)
    k = min(cnt.value, cap)
    return oi[:k], oj[:k], cnt.value, (sk if want_sketch else None)


# ------------------------------------------------------------- object layer

class Context:
    """A cmm context on one device, ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        self.handle = cmm_ctx_create(device, stream)

    def close(self):
        if self.handle:
            cmm_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        """Order the context's work on ``stream`` (a torch.cuda.Stream; None:
        torch's current stream) from now on; waits for the old stream first."""
        s = C.c_void_p(stream.cuda_stream) if stream is not None else _current_stream()
        cmm_ctx_set_stream(self.handle, s)

    def set_workspace_limit(self, nbytes: int):
        """Products whose workspace would exceed ``nbytes`` run as k-slabs
        (0 restores the default, half the device memory)."""
        cmm_ctx_set_workspace_limit(self.handle, nbytes)

    def profile(self, enable: bool):
        cmm_ctx_profile(self.handle, enable)

    def profile_read(self, name: str):
        return cmm_ctx_profile_read(self.handle, name)

    def profile_bytes(self, name: str):
        """(read, written) bytes the named kernels moved by design while profiling."""
        return cmm_ctx_profile_bytes(self.handle, name)

    def stream_probe(self, read_bytes: int, write_bytes: int, nontemporal: bool = False, reps: int = 10):
        """HIP-event ms per launch of a plain HBM stream of this shape."""
        return cmm_stream_probe(self.handle, read_bytes, write_bytes, nontemporal, reps)

    def autotune(self, n1, m, n3, b, d, dtype="f32"):
        """Tune the size class of these sizes; returns ((log2c, kmax, cs_blocks), ms)."""
        return cmm_autotune(self.handle, n1, m, n3, b, d, DTYPES[dtype])

    def tuning(self, n1, m, n3, b, d, dtype="f32"):
        return cmm_tuning_get(self.handle, n1, m, n3, b, d, DTYPES[dtype])

    def set_tuning(self, n1, m, n3, b, d, dtype, tuning):
        cmm_tuning_set(self.handle, n1, m, n3, b, d, DTYPES[dtype], tuning)

    def save_tuning(self, path):
        cmm_tuning_save(self.handle, path)

    def load_tuning(self, path):
        cmm_tuning_load(self.handle, path)


class Sketch:
    """Owning wrapper of a cmm_sketch handle."""

    def __init__(self, handle, ctx: Context, owner=None):
        self.handle = handle
        self.ctx = ctx       # keeps the context alive
        self.owner = owner   # a Batch that owns the handle, else None

    def free(self):
        if self.handle and self.owner is None:
            cmm_sketch_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        return cmm_sketch_info(self.handle)

    def c(self):
        return cmm_sketch_copy_c(self.handle)

    def hash_params(self):
        return cmm_sketch_hash_params(self.handle)

    def hashes(self, t):
        return cmm_sketch_hashes(self.handle, t)

    def estimate(self, i, j):
        return cmm_estimate(self.handle, i, j)

    def estimate_batch(self, i, j):
        import torch
        out = torch.empty(i.numel(), dtype=torch.float32, device=i.device)
        return cmm_estimate_batch(self.handle, i, j, out)

    def topk(self, K, mode="all"):
        return cmm_topk(self.handle, K, MODES[mode] if isinstance(mode, str) else mode)

    def subtract_diagonal(self, diag):
        cmm_sketch_subtract_diagonal(self.handle, diag)

    def merge(self, other: "Sketch"):
        cmm_sketch_merge(self.handle, other.handle)


def sketch_product(ctx: Context, At, B, b: int, d: int, seed: int = 0, dtype: str = "f32",
                   scaleA=None, scaleB=None, hash_params=None, subtract_diag: bool = False,
                   n1: int | None = None, n3: int | None = None, m: int | None = None,
                   asynchronous: bool = False) -> Sketch:
    """Sketch of AB from the k-major device arrays At (m x lda, At[k, i] =
    A[i, k]) and B (m x ldb).  Returns a Sketch."""
    m_ = m if m is not None else At.shape[0]
    n1_ = n1 if n1 is not None else At.shape[1]
    n3_ = n3 if n3 is not None else B.shape[1]
    flags = (CMM_SUBTRACT_DIAG if subtract_diag else 0) | (CMM_ASYNC if asynchronous else 0)
    h = cmm_sketch_product_ex(ctx.handle, At, At.stride(0), B, B.stride(0), n1_, m_, n3_,
                              DTYPES[dtype], scaleA, scaleB, b, d, seed, hash_params, flags)
    return Sketch(h, ctx)


def sketch_product_noalloc(ctx: Context, At, B, b: int, d: int, c_out, seed: int = 0, dtype: str = "f32",
                           scaleA=None, scaleB=None, subtract_diag: bool = False,
                           n1: int | None = None, n3: int | None = None, m: int | None = None):
    """cmm_sketch_product_noalloc: the sketch of AB written into the float64
    device tensor ``c_out`` (d x b) with no allocation; stream-ordered."""
    m_ = m if m is not None else At.shape[0]
    n1_ = n1 if n1 is not None else At.shape[1]
    n3_ = n3 if n3 is not None else B.shape[1]
    flags = CMM_SUBTRACT_DIAG if subtract_diag else 0
    _check(load().cmm_sketch_product_noalloc(ctx.handle, _ptr(At), At.stride(0), _ptr(B), B.stride(0), n1_, m_,
                                             n3_, DTYPES[dtype], _ptr(scaleA), _ptr(scaleB), b, d, seed, flags,
                                             _ptr(c_out)), "cmm_sketch_product_noalloc", ctx.handle)


def sketch_product_tables(ctx: Context, At, B, b, h1, s1, h2, s2, dtype="f32") -> Sketch:
    d = np.asarray(h1).shape[0]
    h = cmm_sketch_product_tables(ctx.handle, At, At.stride(0), B, B.stride(0), At.shape[1],
                                  At.shape[0], B.shape[1], DTYPES[dtype], None, None, b, d,
                                  h1, s1, h2, s2)
    return Sketch(h, ctx)


def problem(At, B, b: int, d: int, seed: int = 0, dtype: str = "f32", scaleA=None, scaleB=None,
            subtract_diag: bool = False, n1: int | None = None, n3: int | None = None,
            m: int | None = None) -> cmm_problem:
    """A cmm_problem over the k-major device arrays At (m x lda) and B (m x ldb),
    as in sketch_product.  The tensors must outlive every batch built on it."""
    return cmm_problem(
        A=At.data_ptr(), lda=At.stride(0), B=B.data_ptr(), ldb=B.stride(0),
        n1=n1 if n1 is not None else At.shape[1], m=m if m is not None else At.shape[0],
        n3=n3 if n3 is not None else B.shape[1], b=b, d=d, dtype=DTYPES[dtype],
        scaleA=None if scaleA is None else scaleA.data_ptr(),
        scaleB=None if scaleB is None else scaleB.data_ptr(), seed=seed,
        flags=CMM_SUBTRACT_DIAG if subtract_diag else 0, reserved=0)


class Batch:
    """Owning wrapper of a cmm_batch: products recorded into one HIP graph."""

    def __init__(self, ctx: Context, probs, autotune: bool = False, keep=None):
        self.ctx = ctx
        self.keep = keep   # e.g. the operand tensors, kept alive with the batch
        self.count = len(probs)
        self.handle = cmm_batch_create(ctx.handle, probs, CMM_AUTOTUNE if autotune else 0)

    def run(self, asynchronous: bool = False):
        cmm_batch_run(self.handle, CMM_ASYNC if asynchronous else 0, self.ctx.handle)

    def sketch(self, index: int) -> Sketch:
        return Sketch(cmm_batch_sketch(self.handle, index), self.ctx, owner=self)

    def topk(self, Ks, mode="all"):
        """Top-K of every product (Ks: one K per product, or one int for all);
        the host waits of all products are shared.  Returns a list of
        (i, j, val) per product."""
        if isinstance(Ks, int):
            Ks = [Ks] * self.count
        if len(Ks) != self.count:
            raise ValueError("one K per product")
        sizes = []
        for q in range(self.count):
            n1, m, n3, b, d = cmm_sketch_info(cmm_batch_sketch(self.handle, q))
            sizes.append((n1, n3))
        return cmm_batch_topk(self.handle, Ks, MODES[mode] if isinstance(mode, str) else mode, sizes)

    def free(self):
        if self.handle:
            cmm_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sketch_product_batched(ctx: Context, probs) -> list:
    """Every product of `probs` in one graph launch; returns owned Sketches."""
    return [Sketch(h, ctx) for h in cmm_sketch_product_batched(ctx.handle, probs)]


def frobenius_bound(ctx: Context, At, B, d: int, seed: int = 0, dtype: str = "f32", scaleA=None,
                    scaleB=None, subtract_diag: bool = False, n1: int | None = None,
                    n3: int | None = None, m: int | None = None):
    """(X[d], bound) for the k-major device arrays At (m x lda) and B (m x ldb):
    X_t the AMS sketches of AB, bound = 32 * median X_t^2 >= ||AB||_F^2 whp."""
    m_ = m if m is not None else At.shape[0]
    n1_ = n1 if n1 is not None else At.shape[1]
    n3_ = n3 if n3 is not None else B.shape[1]
    return cmm_frobenius_bound(ctx.handle, At, At.stride(0), B, B.stride(0), n1_, m_, n3_,
                               DTYPES[dtype], scaleA, scaleB, d, seed,
                               CMM_SUBTRACT_DIAG if subtract_diag else 0)


def find_significant(ctx: Context, At, B, b: int, d: int, delta: float, seed: int = 0,
                     dtype: str = "f32", scaleA=None, scaleB=None, subtract_diag: bool = False,
                     cap: int = 1 << 16, want_sketch: bool = False, n1: int | None = None,
                     n3: int | None = None, m: int | None = None):
    """FINDSIGNIFICANTENTRIES(delta) over the k-major device arrays At, B;
    returns (i, j, total_count[, Sketch of AB])."""
    m_ = m if m is not None else At.shape[0]
    n1_ = n1 if n1 is not None else At.shape[1]
    n3_ = n3 if n3 is not None else B.shape[1]
    i, j, total, h = cmm_find_significant(ctx.handle, At, At.stride(0), B, B.stride(0), n1_, m_, n3_,
                                          DTYPES[dtype], scaleA, scaleB, b, d, seed,
                                          CMM_SUBTRACT_DIAG if subtract_diag else 0, delta, cap,
                                          want_sketch)
    if want_sketch:
        return i, j, total, Sketch(h, ctx)
    return i, j, total


def sketch_product_sparse(ctx: Context, a_ptr, a_idx, a_val, b_ptr, b_idx, b_val, n1: int, m: int,
                          n3: int, b: int, d: int, seed: int = 0, subtract_diag: bool = False) -> Sketch:
    """Sketch of AB from sparse device operands: A by columns (CSC: a_ptr
    int64 [m+1], a_idx int32, a_val float32) and B by rows (CSR)."""
    out = _P()
    _check(load().cmm_sketch_product_sparse(ctx.handle, _ptr(a_ptr), _ptr(a_idx), _ptr(a_val),
                                            _ptr(b_ptr), _ptr(b_idx), _ptr(b_val), n1, m, n3, b, d,
                                            seed, CMM_SUBTRACT_DIAG if subtract_diag else 0,
                                            C.byref(out)), "cmm_sketch_product_sparse", ctx.handle)
    return Sketch(out, ctx)


def estimate_nnz(ctx: Context, At, B, d: int, seed: int = 0, dtype: str = "f32", scaleA=None,
                 scaleB=None, subtract_diag: bool = False, zero_rel: float = 1e-5,
                 n1: int | None = None, n3: int | None = None, m: int | None = None):
    """Doubling search of Section 5.1; returns (b, zeros per repetition at the last b)."""
    m_ = m if m is not None else At.shape[0]
    n1_ = n1 if n1 is not None else At.shape[1]
    n3_ = n3 if n3 is not None else B.shape[1]
    bo = _I64(); z = np.empty(d, np.int64)
    _check(load().cmm_estimate_nnz(ctx.handle, _ptr(At), At.stride(0), _ptr(B), B.stride(0), n1_, m_,
                                   n3_, DTYPES[dtype], _ptr(scaleA), _ptr(scaleB), d, seed,
                                   CMM_SUBTRACT_DIAG if subtract_diag else 0, zero_rel, C.byref(bo),
                                   z.ctypes.data_as(_P)), "cmm_estimate_nnz", ctx.handle)
    return bo.value, z
