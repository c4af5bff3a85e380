"""ctypes binding and numpy helpers for the CPU oracle.

TEST INFRASTRUCTURE ONLY. The oracle is the plain, slow, independent CPU
reference that the HIP library is checked against. Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import it. It
shares no code with the GPU library and the product path never calls it.

All floating point is FP64. See ``msm_oracle.c`` for the data conventions.

Parity pins (tests/test_oracle_*.py) tie every function here to the paper:
closed forms, special cases, printed values, invariants and brute force.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EUCLIDEAN = 0
COSINE = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile msm_oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        i64, i32, vp, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
        L.oracle_project.argtypes = [vp, i64, i32, i64, vp, i32, vp, i64, vp, vp, vp]
        L.oracle_project.restype = None
        L.oracle_hamming_pairs.argtypes = [vp, i64, i32, i32, vp, i64]
        L.oracle_hamming_pairs.restype = i64
        L.oracle_hamming_partners.argtypes = [vp, i64, i32, i32, vp, i64, vp, i64]
        L.oracle_hamming_partners.restype = i64
        L.oracle_msm.argtypes = [vp, i64, i32, i32, i32, vp, i64, vp]
        L.oracle_msm.restype = i64
        L.oracle_verify.argtypes = [vp, i64, i32, i64, vp, i64, i32, dbl, vp, i64, vp]
        L.oracle_verify.restype = i64
        L.oracle_eps_pairs.argtypes = [vp, i64, i32, i64, i32, dbl, vp, i64]
        L.oracle_eps_pairs.restype = i64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(X):
    X = np.asarray(X)
    if X.dtype != np.float32 or X.ndim != 2 or X.strides[1] != 4:
        X = np.ascontiguousarray(X, dtype=np.float32)
    return X


def _ldx(X):
    return X.strides[0] // 4


def project(X, R, rows=None, want_z: bool = False):
    """Sign bits of X @ R in FP64 (Section 3.2, eq. (3)).

    Returns S (nrows x W uint64), plus (Z, xnorm) in FP64 when ``want_z``.
    """
    X = _f32(X)
    R = np.ascontiguousarray(R, dtype=np.float32)
    n, d = X.shape
    assert R.shape[0] == d
    ell = R.shape[1]
    W = (ell + 63) // 64
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cnt = rows.size
    else:
        cnt = n
    S = np.zeros((cnt, W), dtype=np.uint64)
    Z = np.empty((cnt, ell), dtype=np.float64) if want_z else None
    xn = np.empty(cnt, dtype=np.float64) if want_z else None
    lib().oracle_project(_p(X), n, d, _ldx(X), _p(R), ell, _p(rows), cnt, _p(S), _p(Z), _p(xn))
    return (S, Z, xn) if want_z else S


def _pairs_call(fn, *args, cap_hint=1 << 16):
    cap = cap_hint
    while True:
        out = np.empty((max(cap, 1), 2), dtype=np.uint32)
        m = fn(*args, _p(out), cap)
        if m < 0:
            raise RuntimeError("oracle call failed")
        if m <= cap:
            return out[:m].copy()
        cap = m


def hamming_pairs(S, h: int):
    """All (i, j), i < j, with HamDist(s_i, s_j) <= h, exhaustively (eq. (1))."""
    S = np.ascontiguousarray(S, dtype=np.uint64)
    n, W = S.shape
    return _pairs_call(lib().oracle_hamming_pairs, _p(S), n, W, int(h))


def hamming_partners(S, h: int, rows):
    """For each listed row i, every j != i with HamDist <= h, as (min, max)."""
    S = np.ascontiguousarray(S, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n, W = S.shape
    return _pairs_call(lib().oracle_hamming_partners, _p(S), n, W, int(h), _p(rows), rows.size)


def msm(S, ell: int, k: int, h: int, with_stats: bool = False):
    """MSM with blockwise masking (Sections 2.1-2.2); see msm_oracle.c."""
    S = np.ascontiguousarray(S, dtype=np.uint64)
    n, W = S.shape
    assert W == (ell + 63) // 64
    stats = np.zeros(4, dtype=np.int64)
    cap = 1 << 16
    while True:
        buf = np.empty((cap, 2), dtype=np.uint32)
        m = lib().oracle_msm(_p(S), n, int(ell), int(k), int(h), _p(buf), cap, _p(stats))
        if m < 0:
            raise RuntimeError("oracle_msm failed (invalid arguments or out of memory)")
        if m <= cap:
            out = buf[:m].copy()
            break
        cap = m
    if with_stats:
        return out, {"sorts": int(stats[0]), "candidates": int(stats[1]),
                     "rejected": int(stats[2]), "duplicates": int(stats[3])}
    return out


def verify(X, pairs, metric: int, eps: float, want_dist: bool = False):
    """Pairs of ``pairs`` with distance <= eps (Section 4.1), in input order."""
    X = _f32(X)
    n, d = X.shape
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    m = pairs.shape[0]
    out = np.empty((max(m, 1), 2), dtype=np.uint32)
    dist = np.empty(max(m, 1), dtype=np.float64) if want_dist else None
    kept = lib().oracle_verify(_p(X), n, d, _ldx(X), _p(pairs), m, int(metric), float(eps),
                               _p(out), m, _p(dist))
    res = out[:kept].copy()
    return (res, dist[:m].copy()) if want_dist else res


def eps_pairs(X, metric: int, eps: float):
    """All (i, j), i < j, with distance <= eps, exhaustively (Definition 1.1)."""
    X = _f32(X)
    n, d = X.shape
    return _pairs_call(lib().oracle_eps_pairs, _p(X), n, d, _ldx(X), int(metric), float(eps))


def distances(X, pairs, metric: int):
    """FP64 distance of every listed pair (Definition 1.1 / eq. (2))."""
    _, dist = verify(X, pairs, metric, -math.inf, want_dist=True)
    return dist


# --------------------------------------------------------------------------
# Section 4.2: the missing-edge-ratio bound.

def cosine_p(eps: float) -> float:
    """Upper bound p of the per-bit disagreement probability of a neighbour
    pair under cosine LSH: the angle of cosine distance eps over pi
    (Section 4.2, with eq. (4))."""
    return math.acos(1.0 - eps) / math.pi


def missing_edge_bound(ell: int, h: int, p: float, Q: int = 1) -> float:
    """Bound on the expected missing-edge ratio of Section 4.2:

        (1 - sum_{t=0}^{h} C(ell, t) p^t (1-p)^(ell-t))^Q

    the chance that Binomial(ell, p) exceeds h in every one of Q replicates.
    """
    inside = 0.0
    for t in range(0, int(math.floor(h)) + 1):
        if t > ell:
            break
        inside += math.comb(ell, t) * (p ** t) * ((1.0 - p) ** (ell - t))
    miss = max(0.0, 1.0 - inside)
    return miss ** Q


def pair_codes(pairs) -> np.ndarray:
    """Sorted uint64 codes (i << 32 | j) of a pair list, for set comparison."""
    pairs = np.asarray(pairs, dtype=np.uint64).reshape(-1, 2)
    return np.sort((pairs[:, 0] << np.uint64(32)) | pairs[:, 1])
