"""The hierarchical grouping's emission rule, checked on the CPU against
exhaustive search (host logic; the GPU tests check the library's kernels
that apply it).

Grouping on a set A of j blocks serves every set B of h masked blocks whose
unmasked blocks contain A. A pair whose strings differ in the blocks D
(|D| <= h) has the canonical set B*(D): D plus the smallest blocks not in D,
h in all. The pair is written only in the grouping whose A is the j
smallest blocks outside B*(D). It agrees on those blocks, so it meets in
that grouping; and since A is a function of D, it is written exactly once.
Every D that maps to A leaves the blocks outside the union of those D
unchanged, so the grouping may key on all of those blocks (A among them)
without losing a pair. The number of distinct A is what
msm_enumerate_groupings reports."""
import itertools
import random

import pytest


def block_masks(ell, k):
    L, r = divmod(ell, k)
    out, pos = [], 0
    for b in range(k):
        ln = L + (1 if b < r else 0)
        out.append(((1 << ln) - 1) << pos)
        pos += ln
    return out


def a_of(D, k, h, j):
    B, fill = D, ((1 << k) - 1) & ~D
    for _ in range(bin(D).count("1"), h):
        B |= fill & -fill
        fill &= fill - 1
    U, A = ((1 << k) - 1) & ~B, 0
    for _ in range(j):
        A |= U & -U
        U &= U - 1
    return A


def partitions(k, h, j):
    return sorted({a_of(D, k, h, j) for D in range(1 << k) if bin(D).count("1") <= h})


def key_blocks(A, k, h, j, widen):
    """Blocks a partition groups on: A, or every block no family member touches."""
    if not widen:
        return A
    union = 0
    for D in range(1 << k):
        if bin(D).count("1") <= h and a_of(D, k, h, j) == A:
            union |= D
    return ((1 << k) - 1) & ~union


@pytest.mark.parametrize("widen", [False, True])
@pytest.mark.parametrize("ell,k,h,j", [(16, 4, 2, 1), (16, 4, 2, 2), (60, 6, 2, 3), (64, 5, 3, 1),
                                       (128, 8, 4, 2), (40, 8, 3, 2), (33, 11, 1, 5)])
def test_every_pair_written_once(ell, k, h, j, widen):
    rnd = random.Random(ell * 7 + k * 3 + h + j)
    bm = block_masks(ell, k)
    seeds = [rnd.getrandbits(ell) for _ in range(60)]
    S = []
    for _ in range(300):
        s = rnd.choice(seeds)
        for _ in range(rnd.randint(0, h + 1)):
            s ^= 1 << rnd.randrange(ell)
        S.append(s)
    truth = {(a, b) for a in range(len(S)) for b in range(a + 1, len(S)) if bin(S[a] ^ S[b]).count("1") <= h}
    written = []
    for A in partitions(k, h, j):
        kb = key_blocks(A, k, h, j, widen)
        assert kb & A == A
        keep = 0
        for b in range(k):
            if kb >> b & 1:
                keep |= bm[b]
        groups = {}
        for i, s in enumerate(S):
            groups.setdefault(s & keep, []).append(i)
        for g in groups.values():
            for a, b in itertools.combinations(g, 2):
                x = S[a] ^ S[b]
                if bin(x).count("1") > h:
                    continue
                D = sum(1 << blk for blk in range(k) if x & bm[blk])
                if a_of(D, k, h, j) == A:
                    written.append((a, b))
    assert len(written) == len(set(written)), "a pair was written twice"
    assert set(written) == truth


def test_partition_counts_match_the_library():
    from paper_0904_3151_amd import msm
    assert len(partitions(8, 4, 2)) == msm.msm_enumerate_groupings(1_000_000, 128, 8, 4)[0] == 15
    assert len(partitions(6, 2, 3)) == msm.msm_enumerate_groupings(20_000, 60, 6, 2)[0] == 10
