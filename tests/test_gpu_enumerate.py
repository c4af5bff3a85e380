"""Parity of msm_enumerate_pairs (Sections 2.1-2.2) with the definition:
the GPU pair set must equal {(i, j): i < j, HamDist(s_i, s_j) <= h} exactly
(computed by the oracle's exhaustive search), with every pair once."""
import ctypes
import math

import numpy as np
import pytest
import torch

from helpers import announce, codes, to_np_pairs, to_np_strings
from oracle import oracle as O
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu


def gpu_pairs(msm, ctx, S_np, ell, k, h, cap_hint=1 << 16):
    S = torch.from_numpy(np.ascontiguousarray(S_np).view(np.int64)).cuda()
    P, m = msm.enumerate_pairs(ctx, S, ell, k, h, cap_hint=cap_hint)
    torch.cuda.synchronize()
    return to_np_pairs(P), m


def check(msm, ctx, S_np, ell, k, h, clean=None, cap_hint=1 << 16):
    announce("enumerate", S_np.shape, ell, k, h)
    got, m = gpu_pairs(msm, ctx, S_np, ell, k, h, cap_hint)
    want = O.hamming_pairs(S_np if clean is None else clean, h)
    assert got.shape == (m, 2)
    assert np.all(got[:, 0] < got[:, 1])
    cg = codes(got)
    assert np.all(cg[1:] != cg[:-1]), "duplicate pairs"
    assert np.array_equal(cg, codes(want)), (len(cg), len(want))
    return m


CASES = [
    # (ell, k, h, n, n_seeds, flips)
    (60, 6, 2, 3000, 300, 3),
    (128, 8, 4, 3000, 300, 6),
    (16, 4, 2, 2000, 500, 3),
    (16, 16, 2, 1500, 200, 3),     # k = ell: per-character masking, 120 sorts
    (64, 5, 3, 4000, 400, 5),      # k does not divide ell
    (130, 7, 3, 2500, 250, 4),     # three words
    (256, 8, 3, 2000, 200, 4),     # four words
    (10, 3, 0, 3000, 600, 1),      # h = 0: groups of identical strings
    (40, 2, 1, 3000, 300, 2),
    (200, 10, 8, 2000, 150, 12),
    (33, 11, 1, 2500, 1000, 1),
]


@pytest.mark.parametrize("ell,k,h,n,ns,fl", CASES)
def test_enumerate_matches_definition(msm, ctx, ell, k, h, n, ns, fl):
    S = I.random_strings(n, ell, seed=ell * 131 + k * 7 + h + n, n_seeds=ns, flips=fl)
    assert check(msm, ctx, S, ell, k, h) > 0


def test_enumerate_uniform_strings_ragged(msm, ctx):
    S = I.random_strings(12345, 24, seed=99)
    check(msm, ctx, S, 24, 4, 2)


@pytest.mark.parametrize("mode", ["coord", "radius"])
def test_enumerate_tiny_workload_projection(msm, ctx, mode):
    X, R = I.workload_inputs(I.TINY, sigma_mode=mode)
    S = msm.msm_project(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(R).cuda())
    S_np = to_np_strings(S)
    w = I.TINY
    check(msm, ctx, S_np, w.ell, w.k, w.h, cap_hint=1 << 21)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_enumerate_tiny_n(msm, ctx, n):
    S = np.tile(I.random_strings(1, 50, seed=5), (max(n, 0), 1)) if n else np.zeros((0, 1), np.uint64)
    got, m = gpu_pairs(msm, ctx, S, 50, 5, 2)
    assert m == n * (n - 1) // 2


@pytest.mark.parametrize("n", [300, 1000, 1500, 5000])
def test_enumerate_all_identical(msm, ctx, n):
    # Section 2.3: every pair is a solution; the single group exceeds the
    # LDS bucket and goes through the tile-against-tile path.
    S = np.tile(I.random_strings(1, 60, seed=13), (n, 1))
    m = check(msm, ctx, S, 60, 6, 2, cap_hint=n * (n - 1) // 2)
    assert m == n * (n - 1) // 2


@pytest.mark.parametrize("flips", [0, 1, 2])
def test_enumerate_identical_clusters(msm, ctx, flips):
    # many groups of identical or nearly identical strings: runs where some
    # blocks are constant over the whole run, others vary
    S = I.random_strings(6000, 128, seed=61 + flips, n_seeds=40, flips=flips)
    check(msm, ctx, S, 128, 8, 4, cap_hint=1 << 22)


def test_enumerate_huge_clusters(msm, ctx):
    # a few seeds with thousands of near-copies: runs far above the bucket size
    S = I.random_strings(6000, 64, seed=21, n_seeds=3, flips=1)
    check(msm, ctx, S, 64, 4, 2, cap_hint=1 << 23)


def test_enumerate_ignores_padding_bits(msm, ctx):
    clean = I.random_strings(2000, 70, seed=31, n_seeds=200, flips=3)
    dirty = clean.copy()
    rng = np.random.default_rng(1)
    dirty[:, 1] |= rng.integers(0, 2 ** 62, size=2000, dtype=np.uint64) << np.uint64(6)
    check(msm, ctx, dirty, 70, 7, 3, clean=clean)


def test_enumerate_deterministic_set(msm, ctx):
    S = I.random_strings(5000, 64, seed=41, n_seeds=500, flips=3)
    a, _ = gpu_pairs(msm, ctx, S, 64, 4, 2)
    b, _ = gpu_pairs(msm, ctx, S, 64, 4, 2)
    assert np.array_equal(codes(a), codes(b))


def test_enumerate_capacity_and_count_only(msm, ctx):
    S_np = I.random_strings(3000, 64, seed=51, n_seeds=300, flips=3)
    want = len(O.hamming_pairs(S_np, 3))
    S = torch.from_numpy(S_np.view(np.int64)).cuda()
    P, m = msm.msm_enumerate_pairs(ctx, S, 64, 5, 3, cap=0)
    assert P is None and m == want
    with pytest.raises(msm.MSMError) as e:
        msm.msm_enumerate_pairs(ctx, S, 64, 5, 3, cap=want - 1)
    assert e.value.status == msm.MSM_E_CAPACITY and e.value.required == want
    P, m = msm.msm_enumerate_pairs(ctx, S, 64, 5, 3, cap=want)
    assert m == want


def test_enumerate_invalid_arguments(msm, ctx):
    L = msm.lib()
    S = torch.zeros((10, 2), dtype=torch.int64, device="cuda")
    P = torch.zeros((10, 2), dtype=torch.int32, device="cuda")
    m = ctypes.c_int64(0)

    def call(ell, k, h, pairs=P.data_ptr(), cap=10):
        return L.msm_enumerate_pairs(ctx.handle, S.data_ptr(), 10, ell, k, h, pairs, cap, ctypes.byref(m), None)

    assert call(128, 4, 4) == msm.MSM_E_INVALID        # k <= h
    assert call(128, 4, -1) == msm.MSM_E_INVALID
    assert call(128, 129, 1) == msm.MSM_E_INVALID      # k > ell
    assert call(300, 8, 2) == msm.MSM_E_INVALID        # ell > 256
    assert call(128, 65, 1) == msm.MSM_E_UNSUPPORTED   # k above 64
    assert call(128, 40, 20) == msm.MSM_E_UNSUPPORTED  # too many combinations
    assert call(128, 8, 2, pairs=None, cap=10) == msm.MSM_E_INVALID
    assert call(128, 8, 2, pairs=P.data_ptr() + 4, cap=4) == msm.MSM_E_INVALID  # misaligned


def test_grouping_plan_follows_the_data(msm, ctx):
    """Uniform strings take the hierarchical grouping (15 groupings on pairs
    of blocks at ell = 128, k = 8, h = 4); strings whose blocks carry little
    entropy fall back to one grouping per combination. Both give the exact
    pair set."""
    S = I.random_strings(50_000, 128, seed=71)
    check(msm, ctx, S, 128, 8, 4)
    assert msm.msm_enumerate_last_plan(ctx) == (15, 2)
    # 40 codes repeated: every point shares its string with ~100 others, so
    # two blocks separate far fewer points than four
    codes40 = I.random_strings(40, 128, seed=72)
    rng = np.random.default_rng(73)
    S2 = np.ascontiguousarray(codes40[rng.integers(0, 40, 4000)])
    check(msm, ctx, S2, 128, 8, 4)
    g, j = msm.msm_enumerate_last_plan(ctx)
    assert (g, j) in ((15, 2), (70, 0))


def test_enumerate_mostly_lone_strings(msm, ctx):
    """The precision workload's layout (ell = 240, k = 10, h = 8, 45
    groupings) on 40 000 strings of which 39 000 are uniform and 1 000 are
    near copies: nearly every point is alone in its bucket and in its run,
    and the few runs of two or more sit among many lone points. The set is
    still the exhaustive one."""
    S = I.random_strings(40_000, 240, seed=83, n_seeds=39_000, flips=6)
    assert check(msm, ctx, S, 240, 10, 8) > 0


def test_enumerate_wide_strings_many_buckets(msm, ctx):
    """Four-word strings (ell = 240, k = 10, h = 8) over 64 partition
    buckets per grouping, in clusters of about ten strings within a few
    flips of a seed: the first pass's wide shape takes eight buckets per
    workgroup and merges sibling buckets that fit in LDS together, next to
    buckets that do not fit. The set is the exhaustive one."""
    S = I.random_strings(30_000, 240, seed=97, n_seeds=3000, flips=5)
    assert check(msm, ctx, S, 240, 10, 8, cap_hint=1 << 18) > 0


@pytest.mark.parametrize("ell,k,h,groupings", [
    (128, 8, 4, 15),    # 16-character blocks, family bitmap in LDS
    (96, 12, 3, 20),    # 8-character blocks, 2^12 difference sets
    (128, 16, 3, 20),   # 8-character blocks, bitmap over 2^16 sets read from memory
    (256, 16, 4, 15),   # four words
    (128, 4, 1, 2),     # 32-character blocks
    (60, 6, 2, 10),     # 10-character blocks: the difference set bit by bit
    (130, 7, 3, 10),    # blocks of 19 and 18 characters
])
def test_hierarchical_layouts(msm, ctx, ell, k, h, groupings):
    """The hierarchical grouping on every block layout its pair test
    distinguishes: clusters of strings within a few flips of a seed, so
    that many pairs fall on either side of distance h."""
    S = I.random_strings(6000, ell, seed=ell * 17 + k, n_seeds=600, flips=h + 1)
    assert check(msm, ctx, S, ell, k, h) > 0
    g, j = msm.msm_enumerate_last_plan(ctx)
    assert g == groupings and j > 0


def test_enumerate_rejects_a_group_beyond_the_tile_limit(msm, ctx):
    """17M equal strings form one group of 1.4e14 pairs in every grouping:
    the call returns MSM_E_UNSUPPORTED without testing them, and a normal
    call on the same context works afterwards."""
    n = 17_000_000
    S = torch.zeros((n, 1), dtype=torch.int64, device="cuda")
    announce("enumerate too-big group", n)
    with pytest.raises(msm.MSMError) as e:
        msm.msm_enumerate_pairs(ctx, S, 64, 5, 3, cap=0)
    assert e.value.status == msm.MSM_E_UNSUPPORTED
    del S
    torch.cuda.empty_cache()
    Ssmall = I.random_strings(3000, 64, seed=5, n_seeds=300, flips=4)
    check(msm, ctx, Ssmall, 64, 5, 3)


def two_valued_blocks(n, ell, k, flips, seed):
    """Strings whose every block is one of two fixed values, then up to
    `flips` random flips: j kept blocks split the points into few groups,
    so one grouping per combination is the cheaper plan."""
    rng = np.random.default_rng(seed)
    L = ell // k
    vals = rng.integers(0, 2, size=(k, 2, L), dtype=np.uint8)
    choice = rng.integers(0, 2, size=(n, k))
    bits = np.concatenate([vals[b, choice[:, b]] for b in range(k)], axis=1)
    for r in range(n):
        f = rng.integers(0, flips + 1)
        if f:
            bits[r, rng.choice(ell, size=f, replace=False)] ^= 1
    return I.pack_bits(bits, (ell + 63) // 64)


@pytest.mark.parametrize("ell,k,h", [(128, 16, 3), (128, 8, 2), (128, 4, 1), (64, 8, 2)])
def test_per_combination_field_layouts(msm, ctx, ell, k, h):
    """One grouping per combination on 8-, 16- and 32-character blocks, where
    the pair test works on the difference set of blocks."""
    S = two_valued_blocks(3000, ell, k, h + 1, seed=ell + 7 * k + h)
    assert check(msm, ctx, S, ell, k, h) > 0
    g, j = msm.msm_enumerate_last_plan(ctx)
    assert j == 0 and g == math.comb(k, h)


def clustered_strings_fast(n, ell, n_seeds, flips, seed):
    """Clustered strings for millions of rows: the first n_seeds rows are
    uniform, every other row copies a random seed row and flips up to
    `flips` positions (each of `flips` draws applied with probability 1/2;
    a repeated position flips back). Rows are shuffled."""
    rng = np.random.default_rng(seed)
    W = (ell + 63) // 64
    S = rng.integers(0, np.iinfo(np.uint64).max, size=(n, W), dtype=np.uint64, endpoint=True)
    if ell % 64:
        S[:, -1] &= np.uint64((1 << (ell % 64)) - 1)
    parents = rng.integers(0, n_seeds, size=n - n_seeds)
    S[n_seeds:] = S[parents]
    rows_all = np.arange(n_seeds, n)
    for _ in range(flips):
        pos = rng.integers(0, ell, size=n - n_seeds)
        on = rng.random(n - n_seeds) < 0.5
        r, p = rows_all[on], pos[on]
        S[r, p // 64] ^= np.left_shift(np.uint64(1), (p % 64).astype(np.uint64))
    return S[rng.permutation(n)]


def test_enumerate_most_buckets_sampled_rows(msm, ctx):
    """4.3M clustered strings take the largest partition (8192 buckets, so the
    scatter sorts each tile in several LDS chunks and every thread scans
    several bucket counts). Whole-output invariants, and every Hamming partner
    of sampled rows against the oracle's exhaustive search over all n."""
    n, ell, k, h = 4_300_000, 128, 8, 4
    S_np = clustered_strings_fast(n, ell, n // 8, 6, seed=4301)
    announce("enumerate most buckets", n, ell, k, h)
    S = torch.from_numpy(S_np.view(np.int64)).cuda()
    P, m = msm.enumerate_pairs(ctx, S, ell, k, h, cap_hint=1 << 25)
    torch.cuda.synchronize()
    assert m > 0 and P.shape == (m, 2)
    i = P[:, 0].to(torch.int64)
    j = P[:, 1].to(torch.int64)
    assert bool((i < j).all()) and bool((i >= 0).all()) and bool((j < n).all())
    c, _ = torch.sort(i * n + j)
    assert not bool((c[1:] == c[:-1]).any()), "duplicate pairs"
    del c
    rows = I.subsample_indices(n, 64, seed=4302)
    want = codes(O.hamming_partners(S_np, h, rows))
    rt = torch.from_numpy(rows).cuda()
    sel = torch.isin(i, rt) | torch.isin(j, rt)
    got = codes(to_np_pairs(P[sel].contiguous()))
    assert len(want) > 0
    assert np.array_equal(got, want), (len(got), len(want))
    del S, P, i, j
    torch.cuda.empty_cache()
