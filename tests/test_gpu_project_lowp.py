"""Parity of msm_project_lowp (eq. (3) with BF16 or row/column-scaled FP8
products, FP32 accumulation and FP32 recompute inside the margin) with the
FP64 oracle.

A bit may differ from the FP64 sign only where the product error can reach
|z|. With A = sum_t |x_t| |r_t|, rounding both operands to BF16 (8-bit
significand, unit roundoff u = 2^-8) moves each product by at most
2u + u^2 = 2^-7 + 2^-16 of its magnitude and the FP32
accumulation adds at most d 2^-24 A. FP8 e4m3 (4-bit significand) moves each
scaled value by at most 2^-4 of itself, or 2^-10 of the scale in the
subnormal range. Entries recomputed in FP32 can differ only inside the FP32
band of the plain projection. Every mismatch must lie inside these bounds."""
import numpy as np
import pytest
import torch

from helpers import PROJ_BAND, announce, to_np_strings
from oracle import oracle as O
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu

TAU = 2.0 ** -8


def error_bound(X, R, dtype):
    X64 = np.abs(X.astype(np.float64))
    R64 = np.abs(R.astype(np.float64))
    A = X64 @ R64
    d = X.shape[1]
    if dtype == "bf16":
        # both operands rounded to 8 significant bits: u = 2^-8, (1+u)^2 - 1
        return (2.0 ** -7 + 2.0 ** -16) * 1.01 * A + d * 2.0 ** -23 * A
    ia = 240.0 / np.maximum(X64.max(axis=1), 1e-300)
    ib = 240.0 / np.maximum(R64.max(axis=0), 1e-300)
    sub_x = (2.0 ** -10 / ia)[:, None] * R64.sum(axis=0)[None, :]
    sub_r = X64.sum(axis=1)[:, None] * (2.0 ** -10 / ib)[None, :]
    return (2 * 2.0 ** -4 + 2.0 ** -8) * 1.01 * A + 1.07 * (sub_x + sub_r) + d * 2.0 ** -23 * A * 1.2


def check(msm, ctx, X, R, dtype, offset=0):
    n, d = X.shape
    ell = R.shape[1]
    announce("project_lowp", dtype, n, d, ell, offset)
    buf = torch.zeros(offset + max(n, 1) * d, dtype=torch.float32, device="cuda")
    Xd = buf[offset: offset + n * d].view(n, d)
    Xd.copy_(torch.from_numpy(X))
    S, nre = msm.msm_project_lowp(ctx, Xd, torch.from_numpy(R).cuda(), dtype, TAU, count_recomputed=True)
    torch.cuda.synchronize()
    So, Z, xn = O.project(X, R, want_z=True)
    bg, bo = I.unpack_bits(to_np_strings(S), ell), I.unpack_bits(So, ell)
    bad = bg != bo
    allowed = (np.abs(Z) <= error_bound(X, R, dtype)) | (np.abs(Z) < PROJ_BAND * xn[:, None])
    assert not (bad & ~allowed).any(), f"{int((bad & ~allowed).sum())} flips outside the error bound"
    full = I.unpack_bits(to_np_strings(S), S.shape[1] * 64)
    assert not full[:, ell:].any()
    in_margin = int((np.abs(Z) < TAU * xn[:, None]).sum())
    flips = float(bad.mean())
    return flips, nre, in_margin


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_lowp_tiny_workload(msm, ctx, dtype):
    X, R = I.workload_inputs(I.TINY)
    flips, nre, in_margin = check(msm, ctx, X, R, dtype)
    # the margin test uses the estimate, so the recomputed count tracks the
    # number of exact values inside the margin
    assert 0.5 * in_margin <= nre <= 2.0 * in_margin + 50
    assert flips < (1e-3 if dtype == "bf16" else 2e-2)


def _sparse(n, d, seed, density=0.05):
    rng = np.random.default_rng(seed)
    X = (rng.random((n, d)) < density) * rng.lognormal(0.0, 1.0, (n, d))
    X[:: max(1, n // 7)] = 0.0
    nrm = np.linalg.norm(X, axis=1, keepdims=True)
    return np.where(nrm > 0, X / np.where(nrm > 0, nrm, 1), 0).astype(np.float32)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_lowp_sparse_cosine_shape(msm, ctx, dtype):
    # the precision workload's shape: d = 256, 240 bits (R does not fit LDS
    # at once for BF16), nonnegative sparse rows, some all-zero
    X = _sparse(3000, 256, seed=17)
    R = I.projection_matrix(256, 240, seed=2003)
    flips, nre, _ = check(msm, ctx, X, R, dtype)
    S = msm.msm_project_lowp(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(R).cuda(), dtype, TAU)
    zero_rows = np.where(~X.any(axis=1))[0]
    assert not to_np_strings(S)[zero_rows].any()


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("n,d,ell,off", [(700, 33, 130, 1), (129, 128, 128, 0), (5, 7, 1, 0)])
def test_lowp_shapes(msm, ctx, dtype, n, d, ell, off):
    X, _ = I.gaussian_mixture(n, d, max(1, n // 10), 0.2, seed=n + d + ell, sigma_mode="coord")
    R = I.projection_matrix(d, ell, seed=ell + 3)
    check(msm, ctx, X, R, dtype, off)


def test_lowp_tau_zero_and_invalid(msm, ctx):
    X, R = I.workload_inputs(I.TINY, n=500)
    Xd, Rd = torch.from_numpy(X).cuda(), torch.from_numpy(R).cuda()
    _, nre = msm.msm_project_lowp(ctx, Xd, Rd, "bf16", 0.0, count_recomputed=True)
    assert nre == 0
    for bad in (dict(dtype=0), dict(dtype=3), dict(tau=-1.0), dict(tau=float("inf"))):
        kw = dict(dtype="bf16", tau=TAU)
        kw.update(bad)
        with pytest.raises(msm.MSMError) as e:
            msm.msm_project_lowp(ctx, Xd, Rd, kw["dtype"], kw["tau"])
        assert e.value.status == msm.MSM_E_INVALID
