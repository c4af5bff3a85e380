"""Host-side parameter setting (Section 4.3), pinned against the oracle's
independent bound, scipy's binomial tail and the procedure's own rules."""
import math

import pytest
from scipy import stats

from oracle import oracle as O
from paper_0904_3151_amd import params as PR


@pytest.mark.parametrize("ell,h,p", [(50, 0, 0.1), (50, 4, 0.1), (128, 4, 0.02), (240, 8, 0.205), (10, 9, 0.5)])
def test_miss_probability_is_binomial_tail(ell, h, p):
    assert math.isclose(PR.miss_probability(ell, h, p), stats.binom.sf(h, ell, p), rel_tol=1e-9, abs_tol=1e-15)
    assert math.isclose(PR.missing_edge_bound(ell, h, p, 3), O.missing_edge_bound(ell, h, p, 3),
                        rel_tol=1e-9, abs_tol=1e-300)


def test_printed_radii_give_printed_angles():
    # Section 5.2: radii 0.0123 / 0.0489 / 0.109 are angles 0.05 / 0.10 / 0.15 pi
    for eps, ang in [(0.0123, 0.05), (0.0489, 0.10), (0.109, 0.15)]:
        assert abs(PR.flip_probability(eps) - ang) < 5e-4


def test_replicates_needed_is_minimal():
    for ell, h, p, g in [(50, 0, 0.1, 1e-6), (50, 4, 0.1, 1e-6), (50, 8, 0.1, 1e-6), (40, 3, 0.05, 1e-3)]:
        Q = PR.replicates_needed(ell, h, p, g)
        assert PR.missing_edge_bound(ell, h, p, Q) <= g
        if Q > 1:
            assert PR.missing_edge_bound(ell, h, p, Q - 1) > g


def test_fig3_setting_needs_fewer_pools_as_h_grows():
    # Figure 3 (p = 0.1, length 50): many pools at d = 0, few at larger d
    qs = [PR.replicates_needed(50, h, 0.1, 1e-6) for h in range(0, 9)]
    assert all(a >= b for a, b in zip(qs, qs[1:]))
    assert qs[0] > 1000 and qs[8] < 10


@pytest.mark.parametrize("eps,gamma,n", [(0.0123, 1e-6, 1_600_000), (0.0489, 1e-6, 160_000), (0.109, 1e-3, 320_000)])
def test_choose_parameters_follows_the_procedure(eps, gamma, n):
    P = PR.choose_parameters(eps, gamma, n)
    assert P.ell == math.ceil(2 * math.log2(n))
    assert P.Q < 25 and P.bound <= gamma
    if P.h > 0:   # h is the smallest with Q below 25
        assert PR.replicates_needed(P.ell, P.h - 1, P.p, gamma) >= 25
    # the k - h unmasked blocks hold at least log2 n characters
    assert (P.k - P.h) * (P.ell / P.k) >= math.log2(n) - 1e-9 or P.k == P.ell


def test_output_estimate_caps_pools_and_halves_length():
    base = PR.choose_parameters(0.109, 1e-9, 320_000)
    few = PR.choose_parameters(0.109, 1e-9, 320_000, estimated_pairs=0.0)
    assert few.ell == base.ell // 2
    capped = PR.choose_parameters(0.0123, 1e-12, 1_600_000, estimated_pairs=1000.0)
    assert capped.Q <= max(int(30 * 1000 / 1_600_000), 5)
