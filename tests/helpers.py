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
    disagree. The kernel gives each pair to a team of four lanes: a lane
    adds its d/4 squared differences in order with fused multiply-adds and
    two levels of DPP adds sum the four lane totals, so the computed sum
    carries at most d/4 + 2 roundings of non-negative terms, plus 2u from
    each rounded difference before squaring: |error| <= (d/4 + 4) u Delta^2
    to first order. The band (d + 16) u eps^2 contains that bound with
    margin (and also covers teams of other sizes or a serial sum)."""
    return (d + 16) * U32 * eps * eps


def cosine_band(d):
    """Band around eps for the cosine distance 1 - x.y / (|x| |y|): the dot
    product and both squared norms carry at most d/4 + 2 roundings each
    (relative to sum |x_t y_t| <= |x| |y|), the square roots, product,
    quotient and difference one each: |error| <= (d/2 + 8) u to first
    order, inside the band (2d + 32) u."""
    return (2 * d + 32) * U32
