"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

# Relative sign band of the projection: bits may differ from the FP64
# oracle only where |z| < PROJ_BAND * ||x||.
PROJ_BAND = 1e-5
U32 = 2.0 ** -24   # unit roundoff of FP32


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)


def to_np_strings(S_t):
    return S_t.cpu().numpy().view(np.uint64)


def to_np_pairs(P_t):
    return np.ascontiguousarray(P_t.cpu().numpy()).view(np.uint32).reshape(-1, 2)


def codes(pairs):
    p = np.asarray(pairs, dtype=np.uint64).reshape(-1, 2)
    return np.sort((p[:, 0] << np.uint64(32)) | p[:, 1])


def euclid_band(d, eps):
    """Half-width of the band around eps^2 inside which FP32 and FP64 may
    disagree: d FP32 fused multiply-adds over 16-lane partial sums plus a
    4-level shuffle tree, each adding at most one unit roundoff (all terms
    are non-negative), with margin."""
    return (d + 16) * U32 * eps * eps


def cosine_band(d):
    return (2 * d + 32) * U32
