"""Parity at the paper-scale workload (n = 1,000,000, d = 128, ell = 128,
k = 8, h = 4, eps = 0.5), in the configuration the benchmark times.

The oracle cannot enumerate 5e11 pairs, so it is checked one output at a
time: projected bits on sampled rows, every Hamming partner of sampled rows
(exhaustive over all n for each), and the verification of sampled candidate
pairs. Global invariants (i < j, indices in range, no duplicates) are checked
on the whole output."""
import numpy as np
import pytest
import torch

from helpers import PROJ_BAND, announce, codes, euclid_band, to_np_pairs, to_np_strings
from oracle import oracle as O
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu

W = I.PAPER_SCALE


@pytest.fixture(scope="module", params=["coord", "radius"])
def run(request, msm, ctx):
    mode = request.param
    announce("fullsize", W.name, mode)
    X, R = I.workload_inputs(W, sigma_mode=mode)
    Xd = torch.from_numpy(X).cuda()
    Rd = torch.from_numpy(R).cuda()
    S = msm.msm_project(ctx, Xd, Rd)
    P, m = msm.enumerate_pairs(ctx, S, W.ell, W.k, W.h, cap_hint=1 << 25)
    V, kept = msm.msm_verify(ctx, Xd, P, W.metric, W.eps)
    torch.cuda.synchronize()
    out = dict(mode=mode, X=X, R=R, S=to_np_strings(S), P_t=P, m=m, V=to_np_pairs(V), kept=kept)
    del Xd, Rd
    yield out
    del S, P, V
    torch.cuda.empty_cache()


def test_fullsize_projection_sampled_rows(run):
    rows = I.subsample_indices(W.n, 3000, seed=W.seed_sub + 11)
    So, Z, xn = O.project(run["X"], run["R"], rows=rows, want_z=True)
    bg = I.unpack_bits(run["S"][rows], W.ell)
    bo = I.unpack_bits(So, W.ell)
    band = np.abs(Z) < PROJ_BAND * xn[:, None]
    assert not ((bg != bo) & ~band).any()


def test_fullsize_pairs_invariants(run):
    P = run["P_t"]
    assert P.shape == (run["m"], 2)
    i = P[:, 0].to(torch.int64)
    j = P[:, 1].to(torch.int64)
    assert bool((i < j).all()) and bool((i >= 0).all()) and bool((j < W.n).all())
    c, _ = torch.sort(i * W.n + j)
    assert not bool((c[1:] == c[:-1]).any()), "duplicate pairs"
    assert run["m"] > 0


def test_fullsize_pairs_sampled_rows(run):
    rows = I.subsample_indices(W.n, 96, seed=W.seed_sub + 12)
    want = codes(O.hamming_partners(run["S"], W.h, rows))
    P = run["P_t"]
    rt = torch.from_numpy(rows).cuda()
    sel = torch.isin(P[:, 0].to(torch.int64), rt) | torch.isin(P[:, 1].to(torch.int64), rt)
    got = codes(to_np_pairs(P[sel].contiguous()))
    assert np.array_equal(got, want), (len(got), len(want))


def test_fullsize_verify_sampled_pairs(run):
    m = run["m"]
    rng = np.random.default_rng(5)
    take = np.sort(rng.choice(m, size=min(m, 200_000), replace=False))
    cand = to_np_pairs(run["P_t"][torch.from_numpy(take).cuda()].contiguous())
    eps64 = float(np.float32(W.eps))
    want_p, dist = O.verify(run["X"], cand, O.EUCLIDEAN, eps64, want_dist=True)
    kept_all = codes(run["V"])
    assert len(kept_all) == run["kept"]
    cc = codes(cand)
    got = cc[np.isin(cc, kept_all)]
    want = codes(want_p)
    diff = np.setxor1d(got, want)
    p64 = cand.astype(np.uint64)
    keyed = (p64[:, 0] << np.uint64(32)) | p64[:, 1]
    band = keyed[np.abs(dist ** 2 - eps64 ** 2) <= euclid_band(W.d, eps64)]
    assert np.isin(diff, band).all()
    assert run["kept"] <= m


def test_fullsize_two_pools_sampled_rows(msm, ctx):
    """The headline configuration: two string pools of the 1M-point
    radius workload, their union with cross-pool dedup (eq. (5)). Every
    pair appears once, and the partners of 64 sampled rows are exactly the
    union over pools of their exhaustive Hamming partners."""
    announce("fullsize two pools", W.name)
    X, _ = I.workload_inputs(W, sigma_mode="radius")
    Xd = torch.from_numpy(X).cuda()
    del X
    Rs = I.projection_matrices(W.d, W.ell, 2, W.seed_r)
    S = torch.empty((2, W.n, 2), dtype=torch.int64, device="cuda")
    for q in range(2):
        msm.msm_project(ctx, Xd, torch.from_numpy(Rs[q]).cuda(), S[q])
    P, m = msm.enumerate_pairs(ctx, S, W.ell, W.k, W.h, cap_hint=1 << 27)
    torch.cuda.synchronize()
    i = P[:, 0].to(torch.int64)
    j = P[:, 1].to(torch.int64)
    assert bool((i < j).all()) and bool((j < W.n).all())
    c, _ = torch.sort(i * W.n + j)
    assert not bool((c[1:] == c[:-1]).any()), "duplicate pairs"
    rows = I.subsample_indices(W.n, 64, seed=W.seed_sub + 13)
    pools = to_np_strings(S.reshape(2 * W.n, 2)).reshape(2, W.n, 2)
    want = np.unique(np.concatenate([codes(O.hamming_partners(pools[q], W.h, rows)) for q in range(2)]))
    rt = torch.from_numpy(rows).cuda()
    sel = torch.isin(i, rt) | torch.isin(j, rt)
    got = codes(to_np_pairs(P[sel].contiguous()))
    assert want.size > 0 and np.array_equal(got, want), (got.size, want.size)
