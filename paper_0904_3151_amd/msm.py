"""Thin ctypes binding of libmsm (C ABI in include/msm.h).

Each ``msm_*`` function here marshals torch tensors into the C call of the
same name: device pointers, sizes and the current HIP stream. Every step of
the computation runs in the library's HIP kernels; PyTorch only provides
device memory and streams.

Importing this module loads ``libmsm.so`` and raises ImportError if it has
not been built (``python -m paper_0904_3151_amd.build``). There is no CPU
fallback.

Tensor conventions: X is float32 (n, d) with unit column stride; R is
float32 (d, ell) contiguous; strings S are int64 (n, W) holding the uint64
words; pair lists are int32 (m, 2) holding uint32 indices (i, j), i < j.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsm.so")

MSM_OK = 0
MSM_E_INVALID = -1
MSM_E_CAPACITY = -2
MSM_E_UNSUPPORTED = -3
MSM_E_NOMEM = -4
MSM_E_HIP = -5

EUCLIDEAN = 0
COSINE = 1
F32 = 0
BF16 = 1
FP8_E4M3 = 2
DTYPES = {"f32": F32, "bf16": BF16, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3}
METRICS = {"euclidean": EUCLIDEAN, "cosine": COSINE}

EXPORTS = ("msm_version", "msm_create", "msm_destroy", "msm_last_error",
           "msm_project", "msm_project_lowp", "msm_enumerate_pairs", "msm_enumerate_pairs_noalloc",
           "msm_enumerate_replicates", "msm_enumerate_groupings",
           "msm_enumerate_last_plan",
           "msm_verify", "msm_bruteforce_eps",
           "msm_project_mlp", "msm_mlp_loss_grad", "msm_mlp_adam", "msm_mlp_train",
           "msm_batch_create", "msm_batch_run", "msm_batch_launch_graph", "msm_batch_tuning",
           "msm_batch_destroy",
           "msm_profile_enable", "msm_profile_only", "msm_profile_reset", "msm_profile_read")


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class Instance(ctypes.Structure):
    """msm_instance: one problem of a batch (device pointers)."""
    _fields_ = [("X", ctypes.c_void_p), ("R", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("pairs", ctypes.c_void_p), ("n", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("cap", ctypes.c_int64), ("d", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("bucket_target", ctypes.c_int32), ("digit_bits", ctypes.c_int32),
                ("buckets_per_group", ctypes.c_int32), ("ms", ctypes.c_float),
                ("n_min", ctypes.c_int64), ("n_max", ctypes.c_int64)]

    def as_dict(self):
        return {"n_min": int(self.n_min), "n_max": int(self.n_max), "bucket_target": self.bucket_target,
                "digit_bits": self.digit_bits, "buckets_per_group": self.buckets_per_group,
                "ms": round(float(self.ms), 4)}


class MSMError(RuntimeError):
    def __init__(self, status: int, message: str, required: int | None = None):
        super().__init__(f"[status {status}] {message}")
        self.status = status
        self.required = required


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_0904_3151_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.msm_version.argtypes = []
    lib.msm_version.restype = i32
    lib.msm_create.argtypes = [i32, ctypes.POINTER(vp)]
    lib.msm_create.restype = i32
    lib.msm_destroy.argtypes = [vp]
    lib.msm_destroy.restype = None
    lib.msm_last_error.argtypes = [vp]
    lib.msm_last_error.restype = ctypes.c_char_p
    lib.msm_project.argtypes = [vp, vp, i64, i32, i64, vp, i32, vp, vp]
    lib.msm_project.restype = i32
    lib.msm_project_lowp.argtypes = [vp, vp, i64, i32, i64, vp, i32, i32, ctypes.c_float, vp,
                                     ctypes.POINTER(i64), vp]
    lib.msm_project_lowp.restype = i32
    lib.msm_enumerate_pairs.argtypes = [vp, vp, i64, i32, i32, i32, vp, i64, ctypes.POINTER(i64), vp]
    lib.msm_enumerate_pairs.restype = i32
    lib.msm_enumerate_pairs_noalloc.argtypes = [vp, vp, i64, i32, i32, i32, vp, i64, ctypes.POINTER(i64), vp]
    lib.msm_enumerate_pairs_noalloc.restype = i32
    lib.msm_enumerate_replicates.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp, i64, ctypes.POINTER(i64), vp]
    lib.msm_enumerate_replicates.restype = i32
    lib.msm_enumerate_groupings.argtypes = [i64, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.msm_enumerate_groupings.restype = i32
    lib.msm_enumerate_last_plan.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.msm_enumerate_last_plan.restype = i32
    lib.msm_verify.argtypes = [vp, vp, i64, i32, i64, vp, i64, i32, ctypes.c_float, vp, i64,
                               ctypes.POINTER(i64), vp]
    lib.msm_verify.restype = i32
    lib.msm_bruteforce_eps.argtypes = [vp, vp, i64, i32, i64, i32, ctypes.c_float, vp, i64,
                                       ctypes.POINTER(i64), vp]
    lib.msm_bruteforce_eps.restype = i32
    f32 = ctypes.c_float
    lib.msm_project_mlp.argtypes = [vp, vp, i64, i32, i64, vp, i32, i32, vp, vp]
    lib.msm_project_mlp.restype = i32
    lib.msm_mlp_loss_grad.argtypes = [vp, vp, i64, i32, i64, vp, i32, i32, vp, vp, i32, f32, f32, vp,
                                      ctypes.POINTER(f32), vp]
    lib.msm_mlp_loss_grad.restype = i32
    lib.msm_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i64, i64, f32, f32, f32, f32, vp]
    lib.msm_mlp_adam.restype = i32
    lib.msm_mlp_train.argtypes = [vp, vp, i64, i32, i64, vp, vp, vp, i32, i32, vp, vp, i64, i32, i64, i64,
                                  f32, f32, f32, ctypes.POINTER(f32), vp]
    lib.msm_mlp_train.restype = i32
    lib.msm_batch_create.argtypes = [vp, ctypes.POINTER(Instance), i32, i32, i32, i32, i32, ctypes.POINTER(vp), vp]
    lib.msm_batch_create.restype = i32
    lib.msm_batch_run.argtypes = [vp, vp, vp]
    lib.msm_batch_run.restype = i32
    lib.msm_batch_launch_graph.argtypes = [vp, vp, vp]
    lib.msm_batch_launch_graph.restype = i32
    lib.msm_batch_tuning.argtypes = [vp, ctypes.POINTER(BatchConfig), i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(BatchConfig), i32, ctypes.POINTER(i32)]
    lib.msm_batch_tuning.restype = i32
    lib.msm_batch_destroy.argtypes = [vp]
    lib.msm_batch_destroy.restype = None
    lib.msm_profile_enable.argtypes = [vp, i32]
    lib.msm_profile_enable.restype = i32
    lib.msm_profile_only.argtypes = [vp, ctypes.c_char_p]
    lib.msm_profile_only.restype = i32
    lib.msm_profile_reset.argtypes = [vp]
    lib.msm_profile_reset.restype = i32
    lib.msm_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32]
    lib.msm_profile_read.restype = i32
    return lib


_lib = _load()


def lib():
    return _lib


def msm_version() -> int:
    return int(_lib.msm_version())


class Context:
    """Owns an msm_ctx (device scratch) on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = _lib.msm_create(int(device), ctypes.byref(h))
        if st != MSM_OK:
            raise MSMError(st, _lib.msm_last_error(None).decode())
        self._h = h
        self.device = int(device)

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return _lib.msm_last_error(self._h).decode()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.msm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _check(ctx: Context, st: int, required: int | None = None):
    if st != MSM_OK:
        raise MSMError(st, ctx.last_error(), required)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _words(ell: int) -> int:
    return (ell + 63) // 64


def msm_project(ctx: Context, X: torch.Tensor, R: torch.Tensor, S: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Sign strings of X @ R (eq. (3)); returns S as int64 (n, W)."""
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    assert R.dtype == torch.float32 and R.dim() == 2 and R.is_contiguous() and R.is_cuda
    n, d = X.shape
    ell = R.shape[1]
    assert R.shape[0] == d
    if S is None:
        S = torch.empty((n, _words(ell)), dtype=torch.int64, device=X.device)
    assert S.dtype == torch.int64 and S.is_contiguous() and S.shape == (n, _words(ell))
    st = _lib.msm_project(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(R), ell,
                          _ptr(S), _stream(stream))
    _check(ctx, st)
    return S


def msm_project_lowp(ctx: Context, X: torch.Tensor, R: torch.Tensor, dtype="bf16", tau: float = 2.0 ** -8,
                     S: torch.Tensor | None = None, count_recomputed: bool = False, stream=None):
    """Sign strings from BF16 / FP8 products with FP32 margin recompute.

    Returns S, or (S, n_recomputed) when ``count_recomputed``.
    """
    if isinstance(dtype, str):
        dtype = DTYPES[dtype]
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    assert R.dtype == torch.float32 and R.dim() == 2 and R.is_contiguous() and R.is_cuda
    n, d = X.shape
    ell = R.shape[1]
    assert R.shape[0] == d
    if S is None:
        S = torch.empty((n, _words(ell)), dtype=torch.int64, device=X.device)
    assert S.dtype == torch.int64 and S.is_contiguous() and S.shape == (n, _words(ell))
    nre = ctypes.c_int64(0)
    st = _lib.msm_project_lowp(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(R), ell, int(dtype),
                               float(tau), _ptr(S), ctypes.byref(nre) if count_recomputed else None,
                               _stream(stream))
    _check(ctx, st)
    return (S, nre.value) if count_recomputed else S


def msm_enumerate_pairs(ctx: Context, S: torch.Tensor, ell: int, k: int, h: int,
                        pairs: torch.Tensor | None = None, cap: int | None = None, stream=None):
    """Pairs within Hamming distance h (Sections 2.1-2.2).

    Writes into ``pairs`` (int32, (cap, 2)) and returns (pairs[:m], m). Raises
    MSMError with status MSM_E_CAPACITY (``.required`` = m) if it did not fit.
    ``pairs=None, cap=0`` is a count-only call returning (None, m).
    """
    assert S.dtype == torch.int64 and S.dim() == 2 and S.is_contiguous() and S.is_cuda
    n = S.shape[0]
    assert S.shape[1] == _words(ell)
    if pairs is None:
        cap = 0 if cap is None else int(cap)
        if cap > 0:
            pairs = torch.empty((cap, 2), dtype=torch.int32, device=S.device)
    else:
        assert pairs.dtype == torch.int32 and pairs.is_contiguous() and pairs.dim() == 2
        cap = pairs.shape[0] if cap is None else int(cap)
    m = ctypes.c_int64(0)
    st = _lib.msm_enumerate_pairs(ctx.handle, _ptr(S), n, int(ell), int(k), int(h), _ptr(pairs), cap,
                                  ctypes.byref(m), _stream(stream))
    _check(ctx, st, m.value)
    return (pairs[: m.value] if pairs is not None else None), m.value


def msm_enumerate_pairs_noalloc(ctx: Context, S: torch.Tensor, ell: int, k: int, h: int,
                                pairs: torch.Tensor | None = None, cap: int | None = None, stream=None):
    """msm_enumerate_pairs computed in the library's fixed per-device buffer
    (no allocation inside the call); same results and conventions."""
    assert S.dtype == torch.int64 and S.dim() == 2 and S.is_contiguous() and S.is_cuda
    n = S.shape[0]
    assert S.shape[1] == _words(ell)
    if pairs is None:
        cap = 0 if cap is None else int(cap)
        assert cap == 0, "pass a preallocated pairs tensor"
    else:
        assert pairs.dtype == torch.int32 and pairs.is_contiguous() and pairs.dim() == 2
        cap = pairs.shape[0] if cap is None else int(cap)
    m = ctypes.c_int64(0)
    st = _lib.msm_enumerate_pairs_noalloc(ctx.handle, _ptr(S), n, int(ell), int(k), int(h), _ptr(pairs), cap,
                                          ctypes.byref(m), _stream(stream))
    _check(ctx, st, m.value)
    return (pairs[: m.value] if pairs is not None else None), m.value


def msm_enumerate_groupings(n: int, ell: int, k: int, h: int):
    """(groupings, j) msm_enumerate_pairs uses for n strings (j = 0: one
    grouping per combination of masked blocks)."""
    g = ctypes.c_int32(0)
    j = ctypes.c_int32(0)
    st = _lib.msm_enumerate_groupings(int(n), int(ell), int(k), int(h), ctypes.byref(g), ctypes.byref(j))
    if st != MSM_OK:
        raise MSMError(st, "msm_enumerate_groupings: invalid arguments")
    return g.value, j.value


def msm_enumerate_last_plan(ctx: Context):
    """(groupings, j) of the last enumeration on ctx (j = 0: per combination)."""
    g = ctypes.c_int32(0)
    j = ctypes.c_int32(0)
    _check(ctx, _lib.msm_enumerate_last_plan(ctx.handle, ctypes.byref(g), ctypes.byref(j)))
    return g.value, j.value


def msm_enumerate_replicates(ctx: Context, S: torch.Tensor, ell: int, k: int, h: int,
                             pairs: torch.Tensor | None = None, cap: int | None = None, stream=None):
    """Union of the Hamming pairs of Q pools (eq. (5)), each pair once.

    S is int64 (Q, n, W). Returns (pairs[:m], m) like msm_enumerate_pairs.
    """
    assert S.dtype == torch.int64 and S.dim() == 3 and S.is_contiguous() and S.is_cuda
    Q, n, Wd = S.shape
    assert Wd == _words(ell)
    if pairs is None:
        cap = 0 if cap is None else int(cap)
        if cap > 0:
            pairs = torch.empty((cap, 2), dtype=torch.int32, device=S.device)
    else:
        assert pairs.dtype == torch.int32 and pairs.is_contiguous() and pairs.dim() == 2
        cap = pairs.shape[0] if cap is None else int(cap)
    m = ctypes.c_int64(0)
    st = _lib.msm_enumerate_replicates(ctx.handle, _ptr(S), n, int(ell), Q, int(k), int(h), _ptr(pairs), cap,
                                       ctypes.byref(m), _stream(stream))
    _check(ctx, st, m.value)
    return (pairs[: m.value] if pairs is not None else None), m.value


def msm_verify(ctx: Context, X: torch.Tensor, pairs: torch.Tensor, metric, eps: float,
               out: torch.Tensor | None = None, cap: int | None = None, stream=None):
    """Pairs of ``pairs`` whose distance is at most eps (Section 4.1).

    Returns (out[:kept], kept); raises MSMError on failure (MSM_E_CAPACITY with
    ``.required`` when ``out`` is too small).
    """
    if isinstance(metric, str):
        metric = METRICS[metric]
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    assert pairs.dtype == torch.int32 and pairs.is_contiguous()
    pairs = pairs.reshape(-1, 2)
    n, d = X.shape
    m = pairs.shape[0]
    if out is None:
        cap = m if cap is None else int(cap)
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=X.device)
    else:
        assert out.dtype == torch.int32 and out.is_contiguous()
        cap = out.shape[0] if cap is None else int(cap)
    kept = ctypes.c_int64(0)
    st = _lib.msm_verify(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(pairs), m,
                         int(metric), float(eps), _ptr(out), cap, ctypes.byref(kept), _stream(stream))
    _check(ctx, st, kept.value)
    return out[: kept.value], kept.value


def msm_bruteforce_eps(ctx: Context, X: torch.Tensor, metric, eps: float, out: torch.Tensor | None = None,
                       cap: int | None = None, stream=None):
    """All pairs with distance <= eps by exhaustive search (Definition 1.1).

    Returns (out[:m], m); ``out=None, cap=0`` counts only.
    """
    if isinstance(metric, str):
        metric = METRICS[metric]
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    n, d = X.shape
    if out is None:
        cap = 0 if cap is None else int(cap)
        if cap > 0:
            out = torch.empty((cap, 2), dtype=torch.int32, device=X.device)
    else:
        assert out.dtype == torch.int32 and out.is_contiguous()
        cap = out.shape[0] if cap is None else int(cap)
    m = ctypes.c_int64(0)
    st = _lib.msm_bruteforce_eps(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, int(metric), float(eps),
                                 _ptr(out), cap, ctypes.byref(m), _stream(stream))
    _check(ctx, st, m.value)
    return (out[: m.value] if out is not None else None), m.value


def bruteforce_eps(ctx: Context, X: torch.Tensor, metric, eps: float, cap_hint: int = 1 << 20, stream=None):
    """msm_bruteforce_eps with an output buffer grown on demand."""
    cap = max(1, int(cap_hint))
    while True:
        try:
            return msm_bruteforce_eps(ctx, X, metric, eps, cap=cap, stream=stream)
        except MSMError as e:
            if e.status != MSM_E_CAPACITY:
                raise
            cap = int(e.required)


def mlp_param_count(d: int, hid: int, ell: int) -> int:
    """Length of the packed parameter vector [W1 | b1 | W2 | b2]."""
    return d * hid + hid + hid * ell + ell


def _check_params(params, d, hid, ell):
    assert params.dtype == torch.float32 and params.is_cuda and params.is_contiguous()
    assert params.numel() == mlp_param_count(d, hid, ell), "params has the wrong length for (d, hid, ell)"


def msm_project_mlp(ctx: Context, X: torch.Tensor, params: torch.Tensor, hid: int, ell: int,
                    S: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sign strings of the learned projection (signs of a2); returns S as int64 (n, W)."""
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    n, d = X.shape
    _check_params(params, d, hid, ell)
    if S is None:
        S = torch.empty((n, _words(ell)), dtype=torch.int64, device=X.device)
    assert S.dtype == torch.int64 and S.is_contiguous() and S.shape == (n, _words(ell))
    st = _lib.msm_project_mlp(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(params), hid, ell,
                              _ptr(S), _stream(stream))
    _check(ctx, st)
    return S


def _check_pairs(pairs, labels):
    assert pairs.dtype == torch.int32 and pairs.is_cuda and pairs.is_contiguous() and pairs.dim() == 2
    assert pairs.shape[1] == 2
    assert labels.dtype == torch.float32 and labels.is_cuda and labels.is_contiguous()
    assert labels.numel() == pairs.shape[0]


def msm_mlp_loss_grad(ctx: Context, X: torch.Tensor, params: torch.Tensor, hid: int, ell: int,
                      pairs: torch.Tensor, labels: torch.Tensor, h: float, lam: float,
                      grad: torch.Tensor | None = None, stream=None):
    """(loss, grad) of the pair loss over pairs (int32 (B, 2)) with labels (float32 (B,))."""
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    n, d = X.shape
    _check_params(params, d, hid, ell)
    _check_pairs(pairs, labels)
    if grad is None:
        grad = torch.empty_like(params)
    assert grad.dtype == torch.float32 and grad.is_contiguous() and grad.numel() == params.numel()
    loss = ctypes.c_float(0.0)
    st = _lib.msm_mlp_loss_grad(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(params), hid, ell,
                                _ptr(pairs), _ptr(labels), pairs.shape[0], float(h), float(lam), _ptr(grad),
                                ctypes.byref(loss), _stream(stream))
    _check(ctx, st)
    return loss.value, grad


def msm_mlp_adam(ctx: Context, params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                 step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
    """One Adam step on params, m, v in place."""
    for t in (params, grad, m, v):
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous() and t.numel() == params.numel()
    st = _lib.msm_mlp_adam(ctx.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(step),
                           float(lr), float(beta1), float(beta2), float(eps), _stream(stream))
    _check(ctx, st)


def msm_mlp_train(ctx: Context, X: torch.Tensor, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                  hid: int, ell: int, pairs: torch.Tensor, labels: torch.Tensor, batch: int, steps: int,
                  first_step: int, lr: float, h: float, lam: float, stream=None):
    """``steps`` loss/gradient + Adam steps over consecutive batches; returns the losses."""
    assert X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1 and X.is_cuda
    n, d = X.shape
    _check_params(params, d, hid, ell)
    _check_pairs(pairs, labels)
    for t in (m, v):
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous() and t.numel() == params.numel()
    losses = (ctypes.c_float * max(1, int(steps)))()
    st = _lib.msm_mlp_train(ctx.handle, _ptr(X), n, d, X.stride(0) if n > 0 else d, _ptr(params), _ptr(m), _ptr(v),
                            hid, ell, _ptr(pairs), _ptr(labels), pairs.shape[0], int(batch), int(steps),
                            int(first_step), float(lr), float(h), float(lam), losses, _stream(stream))
    _check(ctx, st)
    return [float(losses[i]) for i in range(int(steps))]


class Batch:
    """A plan for many independent instances (msm_batch_create): strings by
    eq. (3) and Hamming pairs of every instance in one enqueue.

    ``X_list`` and ``R_list`` hold float32 device tensors (n_i, d_i) and
    (d_i, ell); ``caps`` the pair capacity of each instance. The plan owns
    the output tensors ``S[i]`` (int64 (n_i, W)) and ``pairs[i]`` (int32
    (cap_i, 2)); after a run, instance i's pairs are pairs[i][:m[i]].
    """

    def __init__(self, ctx: Context, X_list, R_list, ell: int, k: int, h: int, caps, autotune: bool = True,
                 stream=None):
        self.ctx = ctx
        self.ell, self.k, self.h = int(ell), int(k), int(h)
        count = len(X_list)
        assert count == len(R_list) == len(caps) and count > 0
        W = _words(ell)
        self.X = list(X_list)
        self.R = list(R_list)
        self.S, self.pairs = [], []
        arr = (Instance * count)()
        for i, (X, R, cap) in enumerate(zip(self.X, self.R, caps)):
            assert X.dtype == torch.float32 and X.dim() == 2 and X.is_cuda
            assert X.shape[0] == 0 or X.stride(1) == 1
            assert R.dtype == torch.float32 and R.is_contiguous() and R.shape == (X.shape[1], ell)
            n, d = X.shape
            S = torch.empty((n, W), dtype=torch.int64, device=X.device)
            P = torch.empty((max(1, int(cap)), 2), dtype=torch.int32, device=X.device)
            self.S.append(S)
            self.pairs.append(P)
            arr[i] = Instance(X.data_ptr() if n else None, R.data_ptr(), S.data_ptr() if n else None, P.data_ptr(),
                              n, X.stride(0) if n > 0 else d, int(cap), d, 0)
        self.count = count
        self._arr = arr
        h_ = ctypes.c_void_p()
        st = _lib.msm_batch_create(ctx.handle, arr, count, self.ell, self.k, self.h, int(bool(autotune)),
                                   ctypes.byref(h_), _stream(stream))
        _check(ctx, st)
        self._h = h_
        self.m = torch.zeros(count, dtype=torch.int64, device=self.X[0].device)

    def run(self, stream=None, graph: bool = False) -> torch.Tensor:
        """Enqueue one run (as one captured graph when ``graph``); returns the
        device tensor of per-instance pair counts."""
        fn = _lib.msm_batch_launch_graph if graph else _lib.msm_batch_run
        _check(self.ctx, fn(self._h, ctypes.c_void_p(self.m.data_ptr()), _stream(stream)))
        return self.m

    def instance_pairs(self, i: int, m: int) -> torch.Tensor:
        return self.pairs[i][: min(int(m), self.pairs[i].shape[0])]

    def tuning(self) -> dict:
        """{"chosen": one configuration per size class present, "tried": every
        candidate timed when the plan was tuned}."""
        nc = ctypes.c_int32(0)
        nt = ctypes.c_int32(0)
        _check(self.ctx, _lib.msm_batch_tuning(self._h, None, 0, ctypes.byref(nc), None, 0, ctypes.byref(nt)))
        chosen = (BatchConfig * max(1, nc.value))()
        tried = (BatchConfig * max(1, nt.value))()
        _check(self.ctx, _lib.msm_batch_tuning(self._h, chosen, nc.value, None, tried, nt.value, None))
        return {"chosen": [chosen[i].as_dict() for i in range(nc.value)],
                "tried": [tried[i].as_dict() for i in range(nt.value)]}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize()
            _lib.msm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def msm_profile_enable(ctx: Context, enable: bool = True):
    _check(ctx, _lib.msm_profile_enable(ctx.handle, int(bool(enable))))


def msm_profile_only(ctx: Context, name: str | None):
    """Time only kernel `name` while timing is on (None: every kernel)."""
    _check(ctx, _lib.msm_profile_only(ctx.handle, None if name is None else name.encode()))


def msm_profile_reset(ctx: Context):
    _check(ctx, _lib.msm_profile_reset(ctx.handle))


def msm_profile_read(ctx: Context) -> dict:
    """{kernel name: (launches, total_ms)} of the event timings so far."""
    cnt = _lib.msm_profile_read(ctx.handle, None, 0)
    if cnt < 0:
        raise MSMError(MSM_E_HIP, ctx.last_error())
    buf = (KernelTime * max(cnt, 1))()
    cnt = _lib.msm_profile_read(ctx.handle, buf, cnt)
    if cnt < 0:
        raise MSMError(MSM_E_HIP, ctx.last_error())
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(cnt)}


def enumerate_pairs(ctx: Context, S: torch.Tensor, ell: int, k: int, h: int, cap_hint: int = 1 << 20,
                    stream=None):
    """msm_enumerate_pairs (S of shape (n, W)) or msm_enumerate_replicates
    (S of shape (Q, n, W)) with an output buffer that is grown on demand."""
    fn = msm_enumerate_replicates if S.dim() == 3 else msm_enumerate_pairs
    cap = max(1, int(cap_hint))
    while True:
        try:
            return fn(ctx, S, ell, k, h, cap=cap, stream=stream)
        except MSMError as e:
            if e.status != MSM_E_CAPACITY:
                raise
            cap = int(e.required)
