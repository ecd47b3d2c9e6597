"""ctypes binding of libhafgpu.so: argument marshalling only.

Every computation runs in the HIP library; if the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhafgpu.so")

HAF_OK = 0
KIND_HAF = 0
KIND_LHAF = 1
ERRORS = {
    1: "HAF_E_INVALID_ARG", 2: "HAF_E_TOO_LARGE", 3: "HAF_E_NOT_SYMMETRIC", 4: "HAF_E_NONFINITE",
    5: "HAF_E_DEVICE", 6: "HAF_E_NOMEM", 7: "HAF_E_BUSY", 8: "HAF_E_STATE",
}

# every symbol declared in include/hafgpu.h
EXPORTS = (
    "haf_last_error", "haf_version", "haf_init", "haf_device_info", "haf_c128", "lhaf_c128", "haf_c128x2_host",
    "haf_c128_dev", "lhaf_c128_dev", "haf_c128x2_dev", "haf_terms_dev", "haf_batched_c128",
    "haf_release_workspaces", "haf_set_kernel_path", "haf_server_default_config", "haf_server_create",
    "haf_server_submit", "haf_server_poll", "haf_server_drain", "haf_server_destroy", "haf_now",
    "haf_profile_enable", "haf_profile_read", "haf_batched_get_config", "haf_batched_set_config",
    "haf_batched_tune", "haf_batched_plan", "haf_batched_c128x2", "perm_c128", "perm_c128_dev",
    "haf_c128x2_dev_noalloc", "haf_exact_i64", "haf_modp_c", "haf_dd_c128x2_dev", "haf_dd_c128x2_host",
    "haf_lowrank_c128", "haf_server_debug_fail_ticks", "haf_batched_load_cache",
)


class HafError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(code, str(code)), msg))
        self.code = code


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class c128x2(ctypes.Structure):
    _fields_ = [("re_hi", ctypes.c_double), ("re_lo", ctypes.c_double), ("im_hi", ctypes.c_double),
                ("im_lo", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("arena_bytes", ctypes.c_int64), ("max_active", ctypes.c_int),
                ("max_queue", ctypes.c_int), ("tick_flops", ctypes.c_double), ("tick_coef_bytes", ctypes.c_int64),
                ("continuous", ctypes.c_int)]


class Profile(ctypes.Structure):
    _fields_ = [("coef_launches", ctypes.c_int64), ("coef_ms", ctypes.c_double), ("coef_model_flops", ctypes.c_double),
                ("coef_subsets", ctypes.c_int64), ("series_launches", ctypes.c_int64), ("series_ms", ctypes.c_double),
                ("batched_launches", ctypes.c_int64), ("batched_ms", ctypes.c_double),
                ("batched_model_flops", ctypes.c_double)]


class BatchedConfig(ctypes.Structure):
    _fields_ = [("table", ctypes.c_int), ("span", ctypes.c_int), ("streams", ctypes.c_int), ("grouped", ctypes.c_int),
                ("coef_budget_mb", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int), ("n", ctypes.c_int), ("kind", ctypes.c_int),
                ("value", c128), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libhafgpu.so not built: run `python -m paper_1805_12498_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch first
    # makes the library bind to that one, so device pointers and streams coming
    # from torch belong to the runtime the library uses (one runtime per process).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "haf_last_error": ([], ctypes.c_char_p),
        "haf_version": ([], ctypes.c_char_p),
        "haf_init": ([i], i),
        "haf_device_info": ([ctypes.c_char_p, i], i),
        "haf_c128": ([vp, i, i, vp], i),
        "lhaf_c128": ([vp, i, i, vp], i),
        "haf_c128x2_host": ([vp, i, i, i, vp], i),
        "haf_c128_dev": ([vp, i, i, vp, vp], i),
        "lhaf_c128_dev": ([vp, i, i, vp, vp], i),
        "haf_c128x2_dev": ([vp, i, i, i, vp, vp], i),
        "haf_c128x2_dev_noalloc": ([vp, i, i, i, vp, vp], i),
        "haf_exact_i64": ([vp, i, i, i, vp, ctypes.POINTER(i)], i),
        "haf_dd_c128x2_dev": ([vp, i, i, i, vp, vp], i),
        "haf_dd_c128x2_host": ([vp, i, i, i, vp], i),
        "haf_lowrank_c128": ([vp, i, i, i, vp, ctypes.POINTER(ctypes.c_double)], i),
        "haf_modp_c": ([vp, i, i, i, vp, i, vp], i),
        "haf_terms_dev": ([vp, i, i, i, vp, i, vp, vp], i),
        "haf_batched_c128": ([vp, vp, vp, vp, i, vp, vp], i),
        "haf_batched_c128x2": ([vp, vp, vp, vp, i, vp, vp], i),
        "haf_release_workspaces": ([], i),
        "haf_set_kernel_path": ([i], i),
        "haf_server_default_config": ([vp], None),
        "haf_server_create": ([vp], vp),
        "haf_server_submit": ([vp, vp, i, i, i, ctypes.POINTER(u64)], i),
        "haf_server_poll": ([vp, vp, i, ctypes.POINTER(i)], i),
        "haf_server_drain": ([vp], i),
        "haf_server_debug_fail_ticks": ([vp, i], i),
        "haf_batched_load_cache": ([], i),
        "haf_server_destroy": ([vp], None),
        "haf_now": ([], ctypes.c_double),
        "haf_profile_enable": ([i], i),
        "haf_profile_read": ([vp], i),
        "haf_batched_get_config": ([vp], i),
        "haf_batched_set_config": ([vp], i),
        "haf_batched_tune": ([vp, vp, vp, vp, i, vp, vp, vp, ctypes.POINTER(ctypes.c_double)], i),
        "haf_batched_plan": ([vp, vp, i, vp, i, ctypes.POINTER(i), vp, i, ctypes.POINTER(i)], i),
        "perm_c128": ([vp, i, i, vp], i),
        "perm_c128_dev": ([vp, i, i, vp, vp], i),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(rc: int):
    if rc != HAF_OK:
        raise HafError(rc, load().haf_last_error().decode())


def _host_matrix(A):
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    return np.ascontiguousarray(A, dtype=np.complex128)


def haf_host(A, kind: int = KIND_HAF, x2: bool = False):
    """haf / lhaf of a host matrix (synchronous).  x2 returns (re_hi, re_lo, im_hi, im_lo)."""
    A = _host_matrix(A)
    n = A.shape[0]
    lib = load()
    ptr = A.ctypes.data if n else ctypes.addressof(ctypes.c_double(0.0))
    if x2:
        out = c128x2()
        check(lib.haf_c128x2_host(ctypes.c_void_p(ptr), n, max(n, 1), kind, ctypes.byref(out)))
        return (out.re_hi, out.re_lo, out.im_hi, out.im_lo)
    out = c128()
    fn = lib.haf_c128 if kind == KIND_HAF else lib.lhaf_c128
    check(fn(ctypes.c_void_p(ptr), n, max(n, 1), ctypes.byref(out)))
    return complex(out.re, out.im)


def _int_matrix(A):
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    if A.dtype.kind == "c":
        if np.any(A.imag != 0):
            raise ValueError("exact hafnians take integer matrices")
        A = A.real
    if A.dtype.kind == "f" and np.any(A != np.round(A)):
        raise ValueError("exact hafnians take integer matrices")
    return np.ascontiguousarray(A, dtype=np.int64)


def haf_exact(A, kind: int = KIND_HAF) -> int:
    """Exact haf / lhaf of an integer matrix (GPU sum over prime fields + CRT) as a Python int."""
    A = _int_matrix(A)
    n = A.shape[0]
    mag = np.zeros(8, dtype=np.uint32)
    sign = ctypes.c_int(0)
    ptr = A.ctypes.data if n else ctypes.addressof(ctypes.c_int64(0))
    check(load().haf_exact_i64(ctypes.c_void_p(ptr), n, max(n, 1), kind, ctypes.c_void_p(mag.ctypes.data),
                               ctypes.byref(sign)))
    v = 0
    for limb in mag[::-1]:
        v = (v << 32) | int(limb)
    return sign.value * v


def haf_modp(A, primes, kind: int = KIND_HAF):
    """haf / lhaf of an integer matrix modulo each prime (GPU), as a list of ints."""
    A = _int_matrix(A)
    n = A.shape[0]
    primes = np.ascontiguousarray(primes, dtype=np.uint32)
    res = np.zeros(len(primes), dtype=np.uint32)
    ptr = A.ctypes.data if n else ctypes.addressof(ctypes.c_int64(0))
    check(load().haf_modp_c(ctypes.c_void_p(ptr), n, max(n, 1), kind, ctypes.c_void_p(primes.ctypes.data),
                            len(primes), ctypes.c_void_p(res.ctypes.data)))
    return [int(r) for r in res]


def haf_host_dd(A, kind: int = KIND_HAF):
    """haf / lhaf of a host matrix with every step of each term in double-double
    (synchronous); returns (re_hi, re_lo, im_hi, im_lo)."""
    A = _host_matrix(A)
    n = A.shape[0]
    ptr = A.ctypes.data if n else ctypes.addressof(ctypes.c_double(0.0))
    out = c128x2()
    check(load().haf_dd_c128x2_host(ctypes.c_void_p(ptr), n, max(n, 1), kind, ctypes.byref(out)))
    return (out.re_hi, out.re_lo, out.im_hi, out.im_lo)


def haf_dev_dd(dA_ptr: int, n: int, lda: int, d_out_ptr: int, stream: int = 0, kind: int = KIND_HAF):
    """Enqueue the double-double mode on a device matrix; d_out receives 4 doubles."""
    check(load().haf_dd_c128x2_dev(ctypes.c_void_p(dA_ptr), n, lda, kind, ctypes.c_void_p(d_out_ptr),
                                   ctypes.c_void_p(stream)))


def haf_lowrank(G):
    """haf of the matrix with G G^T above the diagonal, from the n x r factor G (App. C).
    Returns ((re_hi, re_lo, im_hi, im_lo), cond)."""
    G = np.asarray(G)
    if G.ndim != 2:
        raise ValueError("expected an n x r factor")
    G = np.ascontiguousarray(G, dtype=np.complex128)
    n, r = G.shape
    out = c128x2()
    cond = ctypes.c_double(0.0)
    ptr = G.ctypes.data if G.size else ctypes.addressof(ctypes.c_double(0.0))
    check(load().haf_lowrank_c128(ctypes.c_void_p(ptr), n, r, max(r, 1), ctypes.byref(out), ctypes.byref(cond)))
    return (out.re_hi, out.re_lo, out.im_hi, out.im_lo), cond.value


def perm_host(W) -> complex:
    """perm(W) of a host square matrix through the bipartite identity (synchronous)."""
    W = _host_matrix(W)
    n = W.shape[0]
    ptr = W.ctypes.data if n else ctypes.addressof(ctypes.c_double(0.0))
    out = c128()
    check(load().perm_c128(ctypes.c_void_p(ptr), n, max(n, 1), ctypes.byref(out)))
    return complex(out.re, out.im)


def perm_dev(dW_ptr: int, n: int, ldw: int, d_out_ptr: int, stream: int = 0):
    """Enqueue perm(W) of a device matrix; raw device pointers and a hipStream_t value."""
    check(load().perm_c128_dev(ctypes.c_void_p(dW_ptr), n, ldw, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream)))


def haf_dev(dA_ptr: int, n: int, lda: int, d_out_ptr: int, stream: int = 0, kind: int = KIND_HAF, x2: bool = False):
    """Enqueue haf / lhaf of a device matrix; raw device pointers and a hipStream_t value."""
    lib = load()
    if x2:
        rc = lib.haf_c128x2_dev(ctypes.c_void_p(dA_ptr), n, lda, kind, ctypes.c_void_p(d_out_ptr),
                                ctypes.c_void_p(stream))
    else:
        fn = lib.haf_c128_dev if kind == KIND_HAF else lib.lhaf_c128_dev
        rc = fn(ctypes.c_void_p(dA_ptr), n, lda, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream))
    check(rc)


def terms_dev(dA_ptr: int, n: int, lda: int, kind: int, d_masks_ptr: int, count: int, d_terms_ptr: int,
              stream: int = 0):
    check(load().haf_terms_dev(ctypes.c_void_p(dA_ptr), n, lda, kind, ctypes.c_void_p(d_masks_ptr), count,
                               ctypes.c_void_p(d_terms_ptr), ctypes.c_void_p(stream)))


def _batch_arrays(offsets, sizes, kinds):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    kinds = np.ascontiguousarray(kinds, dtype=np.uint8)
    if not (len(offsets) == len(sizes) == len(kinds)):
        raise ValueError("offsets, sizes and kinds differ in length")
    return offsets, sizes, kinds


def batched_dev(dA_ptr: int, offsets, sizes, kinds, d_out_ptr: int, stream: int = 0, x2: bool = False):
    """Enqueue len(sizes) hafnians of matrices packed densely at element offsets of dA
    (x2: double-double results, 4 doubles per matrix)."""
    offsets, sizes, kinds = _batch_arrays(offsets, sizes, kinds)
    lib = load()
    fn = lib.haf_batched_c128x2 if x2 else lib.haf_batched_c128
    check(fn(ctypes.c_void_p(dA_ptr), ctypes.c_void_p(offsets.ctypes.data), ctypes.c_void_p(sizes.ctypes.data),
             ctypes.c_void_p(kinds.ctypes.data), len(sizes), ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream)))


def batched_config() -> dict:
    c = BatchedConfig()
    check(load().haf_batched_get_config(ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in BatchedConfig._fields_}


def set_batched_config(table: int = 0, span: int = 4, streams: int = 4, grouped: int = 1,
                       coef_budget_mb: int = 8192):
    c = BatchedConfig(table, span, streams, grouped, coef_budget_mb)
    check(load().haf_batched_set_config(ctypes.byref(c)))


def batched_tune(dA_ptr: int, offsets, sizes, kinds, d_out_ptr: int, stream: int = 0):
    """Run the autotuner on this batch; returns (chosen config dict, its time in ms)."""
    offsets, sizes, kinds = _batch_arrays(offsets, sizes, kinds)
    c = BatchedConfig()
    ms = ctypes.c_double(0.0)
    check(load().haf_batched_tune(ctypes.c_void_p(dA_ptr), ctypes.c_void_p(offsets.ctypes.data),
                                  ctypes.c_void_p(sizes.ctypes.data), ctypes.c_void_p(kinds.ctypes.data),
                                  len(sizes), ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream),
                                  ctypes.byref(c), ctypes.byref(ms)))
    return {f: getattr(c, f) for f, _ in BatchedConfig._fields_}, ms.value


def batched_load_cache() -> dict:
    """Make this device's entry of the HAF_AUTOTUNE_CACHE file the batched configuration."""
    check(load().haf_batched_load_cache())
    return batched_config()


def batched_plan(sizes, kinds):
    """Host-only plan of the shared batched launches under the current configuration:
    (launches as int64 [n, 8], chunks as int64 [n, 8]); see haf_batched_plan."""
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    kinds = np.ascontiguousarray(kinds, dtype=np.uint8)
    lib = load()
    nl, nc = ctypes.c_int(0), ctypes.c_int(0)
    check(lib.haf_batched_plan(ctypes.c_void_p(sizes.ctypes.data), ctypes.c_void_p(kinds.ctypes.data), len(sizes),
                               None, 0, ctypes.byref(nl), None, 0, ctypes.byref(nc)))
    launches = np.zeros((max(nl.value, 1), 8), dtype=np.int64)
    chunks = np.zeros((max(nc.value, 1), 8), dtype=np.int64)
    check(lib.haf_batched_plan(ctypes.c_void_p(sizes.ctypes.data), ctypes.c_void_p(kinds.ctypes.data), len(sizes),
                               ctypes.c_void_p(launches.ctypes.data), nl.value, ctypes.byref(nl),
                               ctypes.c_void_p(chunks.ctypes.data), nc.value, ctypes.byref(nc)))
    return launches[:nl.value], chunks[:nc.value]


def set_kernel_path(path: int):
    check(load().haf_set_kernel_path(path))


def device_info() -> str:
    buf = ctypes.create_string_buffer(512)
    check(load().haf_device_info(buf, 512))
    return buf.value.decode()


def release_workspaces():
    check(load().haf_release_workspaces())


def profile_enable(on: bool = True):
    check(load().haf_profile_enable(1 if on else 0))


def profile_read() -> dict:
    p = Profile()
    check(load().haf_profile_read(ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in Profile._fields_}


def now() -> float:
    return load().haf_now()


class Server:
    """Continuous-batching request server (see include/hafgpu.h)."""

    def __init__(self, **cfg):
        lib = load()
        c = ServerConfig()
        lib.haf_server_default_config(ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        self._lib = lib
        self._h = lib.haf_server_create(ctypes.byref(c))
        if not self._h:
            raise HafError(8, lib.haf_last_error().decode())

    def submit(self, A, kind: int = KIND_HAF) -> int:
        A = _host_matrix(A)
        t = ctypes.c_uint64(0)
        check(self._lib.haf_server_submit(self._h, ctypes.c_void_p(A.ctypes.data), A.shape[0], A.shape[0], kind,
                                          ctypes.byref(t)))
        return t.value

    def poll(self, max_results: int = 1024):
        buf = (Result * max_results)()
        got = ctypes.c_int(0)
        check(self._lib.haf_server_poll(self._h, buf, max_results, ctypes.byref(got)))
        return [buf[k] for k in range(got.value)]

    def drain(self):
        check(self._lib.haf_server_drain(self._h))

    def debug_fail_ticks(self, count: int):
        """Test hook: handle the next `count` completed ticks as failed launches."""
        check(self._lib.haf_server_debug_fail_ticks(self._h, count))

    def close(self):
        if self._h:
            self._lib.haf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
