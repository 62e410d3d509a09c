"""ctypes binding of libgofmm.so (the C ABI declared in include/gofmm.h).

Argument marshalling only: every step of the compression and of the K~W
evaluation runs inside the library.  PyTorch provides device memory and
streams for W and U.  Importing this module never falls back to anything:
if the library is missing, `lib()` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Callable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgofmm.so")

GRAM_L2, ANGLE = 0, 1
FP32, BF16, BF16X3 = 0, 1, 2
ERRORS = {0: "OK", -1: "EINVAL", -2: "ECALLBACK", -3: "ENOTSPD", -4: "ENOMEM",
          -5: "EHIP", -6: "EIO", -7: "ELIMIT", -8: "ETIMEDOUT"}
KERNEL_KINDS = {"gaussian": 0, "imq": 1, "laplace_like": 2}

SAMPLER = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_int64,
                      C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int64)


class Params(C.Structure):
    _fields_ = [("leaf_size", C.c_int64), ("max_rank", C.c_int64), ("tol", C.c_double),
                ("kappa", C.c_int32), ("budget", C.c_double), ("distance", C.c_int32),
                ("storage", C.c_int32), ("near_storage", C.c_int32), ("seed", C.c_uint64),
                ("threads", C.c_int32), ("ann_max_iters", C.c_int32),
                ("ann_target_recall", C.c_double), ("exact_knn", C.c_int32), ("device_knn", C.c_int32),
                ("device_id", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("depth", C.c_int64), ("n_leaves", C.c_int64),
                ("n_nodes", C.c_int64), ("rank_sum", C.c_int64), ("rank_max", C.c_int64),
                ("near_pairs", C.c_int64), ("far_pairs", C.c_int64),
                ("flops_per_rhs", C.c_double), ("flops_phase", C.c_double * 4),
                ("operator_bytes", C.c_int64), ("operator_bytes_phase", C.c_int64 * 4),
                ("workspace_rows", C.c_int64)]


class GofmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ServerStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("failed", C.c_int64), ("pending", C.c_int64),
                ("inflight", C.c_int64), ("models", C.c_int64), ("admit_queue", C.c_int64),
                ("batches", C.c_int64), ("columns", C.c_int64), ("packed", C.c_int64),
                ("hbm_used", C.c_int64), ("hbm_budget", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double), ("elapsed_ms", C.c_double), ("max_inflight", C.c_int64),
                ("admissions", C.c_int64), ("host_ms_mean", C.c_double), ("admit_ms_mean", C.c_double),
                ("p99_ms_admitting", C.c_double)]


_lib = None

# (name, restype, argtypes) of every function declared in include/gofmm.h
SIGNATURES = [
    ("gofmm_default_params", None, [C.POINTER(Params)]),
    ("gofmm_compress", C.c_int, [C.c_int64, SAMPLER, C.c_void_p, C.POINTER(Params), C.POINTER(C.c_void_p)]),
    ("gofmm_import", C.c_int, [C.c_char_p, SAMPLER, C.c_void_p, C.POINTER(Params), C.POINTER(C.c_void_p)]),
    ("gofmm_use_device_kernel", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    ("gofmm_export", C.c_int, [C.c_void_p, C.c_char_p]),
    ("gofmm_prepare", C.c_int, [C.c_void_p, C.c_int64]),
    ("gofmm_evaluate", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    ("gofmm_evaluate_noalloc", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                         C.c_void_p]),
    ("gofmm_autotune", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    ("gofmm_evaluate_batched", C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_void_p]),
    ("gofmm_autotune_batched", C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_void_p]),
    ("gofmm_batched_status", C.c_int, [C.POINTER(C.c_int32)]),
    ("gofmm_batched_spin_limit", C.c_int, [C.c_int64]),
    ("gofmm_evaluate_status", C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("gofmm_launch_count", C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("gofmm_launch_info", C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int64)]),
    ("gofmm_profile", C.c_int, [C.c_void_p, C.c_int32]),
    ("gofmm_profile_read", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32)]),
    ("gofmm_footprint", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    ("gofmm_stats", C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    ("gofmm_free", None, [C.c_void_p]),
    ("gofmm_last_error", C.c_char_p, []),
    ("gofmm_server_create", C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    ("gofmm_server_add", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]),
    ("gofmm_server_remove", C.c_int, [C.c_void_p, C.c_int32]),
    ("gofmm_server_submit", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    ("gofmm_server_wait", C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double)]),
    ("gofmm_server_test", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("gofmm_server_stats", C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    ("gofmm_server_reset_stats", C.c_int, [C.c_void_p]),
    ("gofmm_server_destroy", None, [C.c_void_p]),
    ("gofmm_kernel_create", C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_double,
                                      C.c_double, C.POINTER(C.c_void_p)]),
    ("gofmm_kernel_sample", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_int64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int64]),
    ("gofmm_kernel_free", None, [C.c_void_p]),
]


def lib() -> C.CDLL:
    """Load libgofmm.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1707_00164_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise GofmmError(rc, lib().gofmm_last_error().decode(errors="replace"))


def params(**kw) -> Params:
    p = Params()
    lib().gofmm_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


class KernelSampler:
    """The library's built-in radial-kernel sampler over a hidden point cloud."""

    def __init__(self, points: np.ndarray, kind: str, h: float, shift: float):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        st = C.c_void_p()
        _check(lib().gofmm_kernel_create(KERNEL_KINDS[kind], pts.shape[0], pts.shape[1],
                                         pts.ctypes.data, float(h), float(shift), C.byref(st)))
        self.state = st
        self.n = pts.shape[0]
        self.fn = C.cast(lib().gofmm_kernel_sample, SAMPLER)

    def sample(self, I, J) -> np.ndarray:
        """K(I, J) in FP64 (original indices), from the library's sampler."""
        I = np.ascontiguousarray(I, dtype=np.int64)
        J = np.ascontiguousarray(J, dtype=np.int64)
        out = np.empty((len(I), len(J)), dtype=np.float64, order="F")   # column-major, ld = |I|
        if len(I) and len(J):
            rc = lib().gofmm_kernel_sample(self.state, len(I), I.ctypes.data_as(C.POINTER(C.c_int64)), len(J),
                                           J.ctypes.data_as(C.POINTER(C.c_int64)),
                                           out.ctypes.data_as(C.POINTER(C.c_double)), len(I))
            if rc != 0:
                raise GofmmError(rc, "kernel sampler failed")
        return np.ascontiguousarray(out)

    def __del__(self):
        if getattr(self, "state", None) and _lib is not None:
            _lib.gofmm_kernel_free(self.state)
            self.state = None


class PySampler:
    """Wraps a Python callable K(I, J) -> (|I|, |J|) array as a sampler."""

    def __init__(self, fn: Callable[[np.ndarray, np.ndarray], np.ndarray], n: int):
        self.n = n
        self.state = None

        def cb(user, nI, I, nJ, J, out, ld):
            try:
                ii = np.ctypeslib.as_array(I, shape=(nI,)).copy()
                jj = np.ctypeslib.as_array(J, shape=(nJ,)).copy()
                blk = np.asarray(fn(ii, jj), dtype=np.float64)
                if blk.shape != (nI, nJ):
                    return 1
                # column-major block: out[i + j * ld] = K(I[i], J[j]); only the
                # cells of the block are written (the last column has nI)
                dst = np.ctypeslib.as_array(out, shape=((nJ - 1) * ld + nI,))
                for j in range(nJ):
                    dst[j * ld:j * ld + nI] = blk[:, j]
                return 0
            except Exception:
                return 1
        self.fn = SAMPLER(cb)


def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(getattr(stream, "cuda_stream", stream))


class Compression:
    """Owner of a gofmm_compression handle."""

    def __init__(self, handle: C.c_void_p, n: int):
        self.h = handle
        self.n = n

    @classmethod
    def compress(cls, sampler, n: Optional[int] = None, **kw) -> "Compression":
        n = sampler.n if n is None else n
        p = params(**kw)
        h = C.c_void_p()
        _check(lib().gofmm_compress(n, sampler.fn, sampler.state, C.byref(p), C.byref(h)))
        return cls(h, n)

    @classmethod
    def load(cls, path: str, sampler, **kw) -> "Compression":
        p = params(**kw)
        h = C.c_void_p()
        _check(lib().gofmm_import(path.encode(), sampler.fn, sampler.state, C.byref(p), C.byref(h)))
        c = cls(h, 0)
        c.n = c.stats().n
        return c

    def export(self, path: str):
        _check(lib().gofmm_export(self.h, path.encode()))

    def use_device_kernel(self, sampler: "KernelSampler", threads: int = 0):
        """Compute the near blocks on the device from the sampler's points
        (the sampler must describe this compression's matrix)."""
        if not isinstance(sampler, KernelSampler):
            raise TypeError("needs the library's KernelSampler")
        _check(lib().gofmm_use_device_kernel(self.h, sampler.state, int(threads)))

    def prepare(self, r_max: int):
        _check(lib().gofmm_prepare(self.h, r_max))

    def stats(self) -> Stats:
        s = Stats()
        _check(lib().gofmm_stats(self.h, C.byref(s)))
        return s

    def footprint(self, r_max: int) -> int:
        b = C.c_int64()
        _check(lib().gofmm_footprint(self.h, r_max, C.byref(b)))
        return int(b.value)

    def launches(self):
        """[(name, flops per rhs, operator bytes)] of the launches of one evaluate."""
        n = C.c_int32()
        _check(lib().gofmm_launch_count(self.h, C.byref(n)))
        out = []
        for i in range(n.value):
            buf = C.create_string_buffer(64)
            f = C.c_double()
            b = C.c_int64()
            _check(lib().gofmm_launch_info(self.h, i, buf, 64, C.byref(f), C.byref(b)))
            out.append((buf.value.decode(), f.value, b.value))
        return out

    def status(self) -> int:
        """1 if a dependency wait of this compression's tree passes gave up (waits for the device)."""
        f = C.c_int32()
        _check(lib().gofmm_evaluate_status(self.h, C.byref(f)))
        return f.value

    def profile(self, enable: bool, launch: int | None = None):
        """Per-launch HIP-event timing: off, every launch, or only `launch`."""
        mode = 0 if not enable else (1 if launch is None else 2 + int(launch))
        _check(lib().gofmm_profile(self.h, mode))

    def profile_read(self):
        """(total ms, record count) per launch since profiling was enabled."""
        n = len(self.launches())
        ms = (C.c_float * n)()
        cnt = (C.c_int32 * n)()
        _check(lib().gofmm_profile_read(self.h, n, ms, cnt))
        return list(ms), list(cnt)

    def evaluate(self, W, U=None, stream=None):
        """U = K~ W for a CUDA float32 tensor W of shape (n, r)."""
        import torch
        if W.dtype != torch.float32 or not W.is_cuda or W.dim() != 2 or W.shape[0] != self.n:
            raise ValueError("W must be a CUDA float32 tensor of shape (n, r)")
        if W.stride(1) != 1:
            raise ValueError("W rows must be contiguous")
        if U is None:
            U = torch.empty_like(W, memory_format=torch.contiguous_format)
        _check(lib().gofmm_evaluate(self.h, W.shape[1], _ptr(W), W.stride(0), _ptr(U), U.stride(0),
                                    _stream(stream)))
        return U

    def evaluate_noalloc(self, W, U, stream=None):
        """U = K~ W with the workspace in the library's fixed scratch array
        (no device allocation; the compression must already be on the device)."""
        _check(lib().gofmm_evaluate_noalloc(self.h, W.shape[1], _ptr(W), W.stride(0), _ptr(U), U.stride(0),
                                            _stream(stream)))
        return U

    def autotune(self, W, U=None, stream=None):
        import torch
        if U is None:
            U = torch.empty_like(W, memory_format=torch.contiguous_format)
        _check(lib().gofmm_autotune(self.h, W.shape[1], _ptr(W), W.stride(0), _ptr(U), U.stride(0),
                                    _stream(stream)))
        return U

    def free(self):
        if self.h:
            lib().gofmm_free(self.h)
            self.h = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.gofmm_free(self.h)
            self.h = None


def evaluate_batched(comps: Sequence[Compression], Ws, Us=None, stream=None, autotune=False):
    """U_i = K~_i W_i for every i in one persistent launch."""
    import torch
    k = len(comps)
    if Us is None:
        Us = [torch.empty_like(w) for w in Ws]
    hs = (C.c_void_p * k)(*[c.h for c in comps])
    rs = (C.c_int64 * k)(*[w.shape[1] for w in Ws])
    wp = (C.c_void_p * k)(*[_ptr(w) for w in Ws])
    lw = (C.c_int64 * k)(*[w.stride(0) for w in Ws])
    up = (C.c_void_p * k)(*[_ptr(u) for u in Us])
    lu = (C.c_int64 * k)(*[u.stride(0) for u in Us])
    fn = lib().gofmm_autotune_batched if autotune else lib().gofmm_evaluate_batched
    _check(fn(k, hs, rs, wp, lw, up, lu, _stream(stream)))
    return Us


def batched_status() -> int:
    """1 if a dependency wait of the last batched launch hit its spin limit."""
    e = C.c_int32()
    _check(lib().gofmm_batched_status(C.byref(e)))
    return int(e.value)


def batched_spin_limit(polls: int):
    _check(lib().gofmm_batched_spin_limit(polls))


class Server:
    """Request loop keeping compressions resident (the library's serving loop)."""

    def __init__(self, hbm_budget_bytes: int, streams: int = 2, max_batch: int = 16):
        h = C.c_void_p()
        _check(lib().gofmm_server_create(int(hbm_budget_bytes), streams, max_batch, C.byref(h)))
        self.h = h
        self.models = {}

    def add(self, comp: Compression, r_max: int) -> int:
        m = C.c_int32()
        _check(lib().gofmm_server_add(self.h, comp.h, int(r_max), C.byref(m)))
        self.models[m.value] = comp
        return m.value

    def remove(self, model: int):
        _check(lib().gofmm_server_remove(self.h, model))
        self.models.pop(model, None)

    def submit(self, model: int, W, U) -> int:
        """Enqueue U = K~ W; W and U (CUDA float32, rows contiguous) must stay alive."""
        q = C.c_int64()
        _check(lib().gofmm_server_submit(self.h, model, W.shape[1], _ptr(W), W.stride(0), _ptr(U),
                                         U.stride(0), C.byref(q)))
        return q.value

    def wait(self, request: int, timeout_ms: int = 0) -> float:
        """Latency (ms) of a finished request; GofmmError ETIMEDOUT after timeout_ms > 0."""
        ms = C.c_double()
        _check(lib().gofmm_server_wait(self.h, request, int(timeout_ms), C.byref(ms)))
        return ms.value

    def test(self, request: int):
        done = C.c_int32()
        ms = C.c_double()
        _check(lib().gofmm_server_test(self.h, request, C.byref(done), C.byref(ms)))
        return bool(done.value), ms.value

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().gofmm_server_stats(self.h, C.byref(st)))
        return st

    def reset_stats(self):
        _check(lib().gofmm_server_reset_stats(self.h))

    def close(self):
        if self.h:
            lib().gofmm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.gofmm_server_destroy(self.h)
            self.h = None
