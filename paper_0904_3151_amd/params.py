"""Parameter setting of Section 4.3: string length, Hamming threshold, number
of string pools and blocks, from the radius and the missing-edge bound.

For cosine LSH the chance that a neighbour pair (cosine distance <= eps)
disagrees on one bit is at most p = arccos(1 - eps) / pi (eq. (4) and
Section 4.2); with strings of ell bits, threshold h and Q independent pools,
the expected missing-edge ratio is at most

    miss(ell, h, p, Q) = P(Binomial(ell, p) > h) ** Q            (Section 4.2)

The procedure (Section 4.3): ell = 2 log2 n; then the smallest h whose
required Q (the least Q with miss <= gamma) stays below 25; then that Q.
With an estimate S of the number of output pairs, Q is capped at
max(30 S / n, 5) and ell is halved when S is close to zero. The number of
blocks k is the smallest that keeps at least log2 n characters in the k - h
unmasked blocks (Section 4.3), i.e. k >= ell h / (ell - log2 n).

This is host-side logic only; it holds none of the GPU path's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


def flip_probability(eps: float) -> float:
    """p = arccos(1 - eps) / pi for cosine distance eps in [0, 2]."""
    if not 0.0 <= eps <= 2.0:
        raise ValueError("cosine radius must lie in [0, 2]")
    return math.acos(1.0 - eps) / math.pi


def miss_probability(ell: int, h: int, p: float) -> float:
    """P(Binomial(ell, p) > h): one pool misses a pair at flip rate p."""
    if h >= ell:
        return 0.0
    # sum the lower tail in log space for stability, then complement
    lower = 0.0
    for t in range(0, h + 1):
        if p <= 0.0:
            term = 1.0 if t == 0 else 0.0
        elif p >= 1.0:
            term = 1.0 if t == ell else 0.0
        else:
            term = math.exp(math.lgamma(ell + 1) - math.lgamma(t + 1) - math.lgamma(ell - t + 1)
                            + t * math.log(p) + (ell - t) * math.log1p(-p))
        lower += term
    return max(0.0, 1.0 - lower)


def missing_edge_bound(ell: int, h: int, p: float, Q: int) -> float:
    return miss_probability(ell, h, p) ** Q


def replicates_needed(ell: int, h: int, p: float, gamma: float, q_max: int = 1 << 20) -> int:
    """Least Q with miss(ell, h, p) ** Q <= gamma (q_max + 1 if none)."""
    m = miss_probability(ell, h, p)
    if m <= gamma:
        return 1
    if m >= 1.0:
        return q_max + 1
    q = max(1, math.ceil(math.log(gamma) / math.log(m)))
    while q > 1 and m ** (q - 1) <= gamma:  # guard the logarithm's rounding
        q -= 1
    while m ** q > gamma:
        q += 1
    return min(q, q_max + 1)


@dataclass(frozen=True)
class Parameters:
    ell: int
    h: int
    Q: int
    k: int
    p: float
    bound: float


def choose_parameters(eps: float, gamma: float, n: int, q_limit: int = 25,
                      estimated_pairs: float | None = None) -> Parameters:
    """(ell, h, Q, k) for cosine radius eps and missing-edge bound gamma."""
    if n < 2:
        raise ValueError("n must be at least 2")
    p = flip_probability(eps)
    ell = max(2, math.ceil(2.0 * math.log2(n)))
    if estimated_pairs is not None and estimated_pairs < 1.0:
        ell = max(2, ell // 2)
    ell = min(ell, 256)
    h = 0
    while h < ell - 1 and replicates_needed(ell, h, p, gamma) >= q_limit:
        h += 1
    Q = replicates_needed(ell, h, p, gamma)
    if estimated_pairs is not None:
        Q = min(Q, max(int(30.0 * estimated_pairs / n), 5))
    need = math.log2(n)
    if h == 0:
        k = 1
    elif ell > need:
        k = max(h + 1, math.ceil(ell * h / (ell - need)))
    else:
        k = h + 1
    k = min(k, ell, 64)
    return Parameters(ell, h, Q, k, p, missing_edge_bound(ell, h, p, Q))
