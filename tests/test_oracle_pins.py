"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows. None of them re-types the oracle's
own formula: they use printed values, hand-worked fixtures, closed forms,
special cases, invariants and exhaustive search on tiny inputs, so that a
dropped term, a wrong sign or index or a transposed operand in the oracle
fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_0904_3151_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _as_set(pairs):
    return set(map(tuple, np.asarray(pairs).reshape(-1, 2).tolist()))


def _strings_from_text(strings):
    bits = np.array([[int(ch) for ch in s] for s in strings], dtype=np.uint8)
    return I.pack_bits(bits)


# --------------------------------------------------------------------------
# Projection, Section 3.2 eq. (3)

def test_project_unit_vectors_read_rows_of_R():
    # x = e_t gives z_c = R[t, c]: bit c of row t must be R[t, c] > 0. A
    # transposed R, a wrong packing word or bit, or a flipped sign fails.
    d, ell = 7, 130
    R = I.projection_matrix(d, ell, seed=11)
    X = np.eye(d, dtype=np.float32)
    S = O.project(X, R)
    assert S.shape == (d, 3)
    bits = I.unpack_bits(S, ell)
    assert np.array_equal(bits, (R > 0).astype(np.uint8))
    # padding bits above ell stay zero
    assert np.all((S[:, 2] >> np.uint64(ell - 128)) == 0)


def test_project_zero_and_ties_give_zero_bit():
    # eq. (3): sign(t) is '1' only if t > 0; t = 0 gives '0'.
    R = np.array([[1.0, 1.0, 1.0], [-1.0, -0.5, -2.0]], dtype=np.float32)
    X = np.array([[0.0, 0.0], [1.0, 1.0]], dtype=np.float32)
    S = O.project(X, R)
    bits = I.unpack_bits(S, 3)
    assert bits[0].tolist() == [0, 0, 0]          # zero vector
    assert bits[1].tolist() == [0, 1, 0]          # z = (0, 0.5, -1)


def test_project_scale_and_negation():
    X, R = I.workload_inputs(I.TINY, n=300)
    S, Z, _ = O.project(X, R, want_z=True)
    S2 = O.project(X * np.float32(4.0), R)        # positive scale keeps signs
    assert np.array_equal(S, S2)
    Sn, Zn, _ = O.project(-X, R, want_z=True)
    b, bn = I.unpack_bits(S, 60), I.unpack_bits(Sn, 60)
    nz = Z != 0
    assert np.array_equal(b[nz], 1 - bn[nz])


@pytest.mark.parametrize("theta_over_pi", [0.05, 0.3, 0.7])
def test_project_bit_collision_law(theta_over_pi):
    # eq. (4): Pr(s_ic != s_jc) = theta_ij / pi for every bit c.
    d, ell = 16, 100_000
    rng = np.random.default_rng(5)
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    v = rng.standard_normal(d)
    v -= v.dot(u) * u
    v /= np.linalg.norm(v)
    th = theta_over_pi * math.pi
    x = np.stack([u, math.cos(th) * u + math.sin(th) * v]).astype(np.float32)
    R = I.projection_matrix(d, ell, seed=77)
    S = O.project(x, R)
    diff = int(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(S[0], S[1])))
    p = theta_over_pi
    sd = math.sqrt(ell * p * (1 - p))
    assert abs(diff - ell * p) < 4 * sd


# --------------------------------------------------------------------------
# Hamming neighbours by definition, Section 2.1 eq. (1)

def test_hamming_hand_fixture():
    g = _load("hamming_hand.json")
    S = _strings_from_text(g["strings"])
    for h, expect in g["pairs_by_h"].items():
        got = O.hamming_pairs(S, int(h))
        assert got.tolist() == expect, h


def test_hamming_partners_match_pairs():
    S = I.random_strings(400, 64, seed=3, n_seeds=60, flips=4)
    P = O.hamming_pairs(S, 3)
    rows = np.array([0, 5, 17, 399])
    got = _as_set(O.hamming_partners(S, 3, rows))
    want = {p for p in _as_set(P) if p[0] in rows or p[1] in rows}
    assert got == want


def test_hamming_full_threshold_gives_all_pairs():
    S = I.random_strings(50, 20, seed=4)
    assert len(O.hamming_pairs(S, 20)) == 50 * 49 // 2


# --------------------------------------------------------------------------
# MSM, Sections 2.1-2.2: exact equality with the definition

MSM_CASES = [
    # (ell, k, h, n, n_seeds, flips)
    (60, 6, 2, 600, 80, 3),
    (128, 8, 4, 500, 60, 6),
    (16, 4, 2, 300, 100, 3),
    (16, 16, 2, 200, 40, 3),     # k = ell: per-character masking
    (64, 5, 3, 500, 60, 5),      # k does not divide ell
    (130, 7, 3, 400, 50, 4),     # three words
    (256, 8, 3, 300, 40, 4),     # four words
    (10, 3, 0, 400, 100, 1),     # h = 0
    (40, 2, 1, 400, 60, 2),
]


@pytest.mark.parametrize("ell,k,h,n,ns,fl", MSM_CASES)
def test_msm_equals_definition(ell, k, h, n, ns, fl):
    S = I.random_strings(n, ell, seed=ell * 131 + k * 7 + h, n_seeds=ns, flips=fl)
    want = O.hamming_pairs(S, h)
    got, st = O.msm(S, ell, k, h, with_stats=True)
    assert got.shape[0] == len(_as_set(got))           # each pair once
    assert np.all(got[:, 0] < got[:, 1])
    assert np.array_equal(O.pair_codes(got), O.pair_codes(want))
    assert st["sorts"] == math.comb(k, h)
    assert len(want) > 0


def test_msm_h0_is_groups_of_identical_strings():
    # Section 2.1, d = 0: sort, cut into equivalence classes, all pairs in each.
    S = I.random_strings(500, 12, seed=9, n_seeds=150, flips=0)
    groups = {}
    for i, row in enumerate(map(tuple, S.tolist())):
        groups.setdefault(row, []).append(i)
    want = {(a, b) for g in groups.values() for x, a in enumerate(g) for b in g[x + 1:]}
    got = O.msm(S, 12, 3, 0)
    assert _as_set(got) == want


def test_msm_per_character_masking_needs_no_filter():
    # Section 2.1: with one character per block, s^C = s'^C for |C| = d is
    # equivalent to HamDist <= d, so no candidate is ever rejected.
    S = I.random_strings(300, 14, seed=10, n_seeds=40, flips=3)
    _, st = O.msm(S, 14, 14, 2, with_stats=True)
    assert st["rejected"] == 0
    assert st["candidates"] > 0
    S = I.random_strings(300, 14, seed=10, n_seeds=40, flips=3)
    _, st2 = O.msm(S, 14, 7, 2, with_stats=True)
    assert st2["rejected"] > 0      # with wider blocks the filter is needed


def test_msm_blockwise_sort_count_fig2c():
    g = _load("blockwise_sorts.json")
    S = I.random_strings(200, g["ell"], seed=12, n_seeds=30, flips=2)
    _, per_char = O.msm(S, g["ell"], g["ell"], g["h"], with_stats=True)
    _, blockwise = O.msm(S, g["ell"], g["k"], g["h"], with_stats=True)
    assert per_char["sorts"] == g["sorts_per_character"]
    assert blockwise["sorts"] == g["sorts_blockwise"]


def test_msm_all_identical_strings():
    # Section 2.3: the worst case, every pair is a solution.
    S = np.tile(I.random_strings(1, 60, seed=13), (300, 1))
    got = O.msm(S, 60, 6, 2)
    assert len(got) == 300 * 299 // 2
    assert len(_as_set(got)) == len(got)


def test_msm_invariant_under_block_count():
    S = I.random_strings(400, 48, seed=14, n_seeds=50, flips=3)
    ref = O.pair_codes(O.msm(S, 48, 4, 2))
    for k in (3, 5, 6, 8, 12, 48):
        assert np.array_equal(O.pair_codes(O.msm(S, 48, k, 2)), ref), k


def test_msm_rejects_invalid():
    S = I.random_strings(10, 16, seed=1)
    with pytest.raises(RuntimeError):
        O.msm(S, 16, 2, 2)          # k must exceed h


# --------------------------------------------------------------------------
# Distances, Definition 1.1 and eq. (2)

def test_cosine_distance_printed_angles():
    g = _load("angle_eps.json")
    for case in g["cases"]:
        th = case["angle_over_pi"] * math.pi
        X = np.array([[1.0, 0.0], [math.cos(th), math.sin(th)]], dtype=np.float32)
        D = O.distances(X, np.array([[0, 1]]), O.COSINE)[0]
        assert float(f"{D:.{case['sig_figs']}g}") == case["eps_printed"]
        # and back: the bit-disagreement bound p of Section 4.2 is the angle / pi
        assert abs(O.cosine_p(D) - case["angle_over_pi"]) < 1e-6


def test_cosine_distance_special_values():
    X = np.array([[1, 2, 3], [2, 4, 6], [-1, -2, -3], [3, 0, -1], [0, 0, 0]], dtype=np.float32)
    P = np.array([[0, 1], [0, 2], [0, 3], [0, 4]])
    D = O.distances(X, P, O.COSINE)
    assert abs(D[0]) < 1e-12          # parallel
    assert abs(D[1] - 2.0) < 1e-12    # opposite
    assert abs(D[2] - 1.0) < 1e-12    # orthogonal
    assert D[3] == 1.0                # zero vector: distance 1 by convention


def test_euclidean_threshold_is_inclusive():
    X = np.array([[0, 0], [3, 4], [6, 8]], dtype=np.float32)
    assert O.eps_pairs(X, O.EUCLIDEAN, 5.0).tolist() == [[0, 1], [1, 2]]
    assert O.eps_pairs(X, O.EUCLIDEAN, 4.999).tolist() == []
    assert O.eps_pairs(X, O.EUCLIDEAN, 10.0).tolist() == [[0, 1], [0, 2], [1, 2]]


def test_unit_vectors_euclidean_is_twice_cosine():
    # Section 5.1: for unit-norm vectors, squared Euclidean distance equals
    # twice the cosine distance.
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 9))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    X = X.astype(np.float32)
    P = np.array([(i, j) for i in range(40) for j in range(i + 1, 40)])
    de = O.distances(X, P, O.EUCLIDEAN)
    dc = O.distances(X, P, O.COSINE)
    x64 = X.astype(np.float64)
    nn = np.linalg.norm(x64, axis=1)
    # the float32 rows are unit only to rounding: correct for their norms
    assert np.allclose(de ** 2, 2 * dc * nn[P[:, 0]] * nn[P[:, 1]]
                       + (nn[P[:, 0]] - nn[P[:, 1]]) ** 2, atol=1e-12)


def test_verify_equals_exhaustive_on_all_pairs():
    X, _ = I.workload_inputs(I.TINY, sigma_mode="radius", n=600)
    allp = np.array([(i, j) for i in range(600) for j in range(i + 1, 600)], dtype=np.uint32)
    eps = float(np.float32(0.4))
    v = O.verify(X, allp, O.EUCLIDEAN, eps)
    e = O.eps_pairs(X, O.EUCLIDEAN, eps)
    assert np.array_equal(O.pair_codes(v), O.pair_codes(e))
    assert len(e) > 0


# --------------------------------------------------------------------------
# Missing-edge-ratio bound, Section 4.2

def test_bound_matches_binomial_tail():
    for ell, h, p, Q in [(50, 0, 0.1, 1), (50, 4, 0.1, 3), (128, 4, 0.02, 1), (240, 8, 0.205, 2)]:
        want = stats.binom.sf(h, ell, p) ** Q
        assert math.isclose(O.missing_edge_bound(ell, h, p, Q), want, rel_tol=1e-9, abs_tol=1e-300)


def test_bound_special_cases_fig3_setting():
    # Figure 3 uses p = 0.1 and length 50. With d = 0 a neighbour is missed
    # unless all 50 bits agree: 1 - 0.9^50 per replicate.
    assert math.isclose(O.missing_edge_bound(50, 0, 0.1, 1), 1 - 0.9 ** 50, rel_tol=1e-12)
    assert math.isclose(O.missing_edge_bound(50, 0, 0.1, 7), (1 - 0.9 ** 50) ** 7, rel_tol=1e-12)
    assert O.missing_edge_bound(50, 50, 0.1, 1) == 0.0
    # more replicates and a larger d both lower the bound (Section 4.2)
    vals = [O.missing_edge_bound(50, h, 0.1, 1) for h in range(0, 9)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert O.missing_edge_bound(50, 4, 0.1, 5) < O.missing_edge_bound(50, 4, 0.1, 4)


def test_bound_is_tight_for_pairs_at_the_radius():
    # A pair at exactly angle theta misses with probability P(Binom(ell, p) > h)
    # where p = theta / pi (eq. (4) and the binomial law of Section 3.2).
    # Project many such pairs with independent R and count misses.
    d, ell, h = 12, 40, 3
    eps = 0.05
    p = O.cosine_p(eps)
    th = math.acos(1 - eps)
    rng = np.random.default_rng(21)
    npairs = 4000
    U = rng.standard_normal((npairs, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    V = rng.standard_normal((npairs, d))
    V -= (V * U).sum(1, keepdims=True) * U
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    Wv = math.cos(th) * U + math.sin(th) * V
    X = np.empty((2 * npairs, d), dtype=np.float32)
    X[0::2], X[1::2] = U, Wv
    misses = 0
    reps = 5
    for r in range(reps):
        R = I.projection_matrix(d, ell, seed=500 + r)
        S = O.project(X, R)
        ham = np.array([sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(S[2 * q], S[2 * q + 1]))
                        for q in range(npairs)])
        misses += int((ham > h).sum())
    tot = reps * npairs
    bound = O.missing_edge_bound(ell, h, p, 1)
    sd = math.sqrt(tot * bound * (1 - bound))
    assert abs(misses - tot * bound) < 4 * sd + 1
