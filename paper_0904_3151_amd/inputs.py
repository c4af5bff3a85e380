"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays. It holds
none of the method's arithmetic (no projection, no Hamming test, no distance):
both the GPU library and the CPU oracle receive the same arrays from here.

The paper evaluates on a public image collection that is not available here
(Section 5.2). The mixtures below stand in for it with the shapes, sizes and
cluster structure of the benchmark workloads.

Every generator uses numpy's PCG64 with a fixed seed. Seeds follow one scheme:
data = 1000 + N, projection matrix = 2000 + N, subsample = 3000 + N for
workload N.

``sigma_mode`` picks how a cluster's "sigma" is read:

* ``"coord"``: x = c + sigma * g, g ~ N(0, I). sigma is the per-coordinate
  standard deviation (the literal reading of "isotropic Gaussian, sigma").
* ``"radius"``: x = c + (sigma / sqrt(d)) * g. sigma is the cluster's RMS
  radius, so intra-cluster distances are about sigma * sqrt(2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIGMA_MODES = ("coord", "radius")


@dataclass(frozen=True)
class Workload:
    """One named workload: data shape, string parameters and distance test."""

    name: str
    n: int
    d: int
    ell: int
    k: int
    h: int
    eps: float
    metric: str  # "euclidean" or "cosine"
    n_centres: int
    sigma: tuple  # (lo, hi); lo == hi for a fixed sigma
    seed_data: int
    seed_r: int
    seed_sub: int
    subsample: int = 0
    extra: dict = field(default_factory=dict)


# 20k points, d=64, 200 clusters of 100, sigma=0.15; l=60, k=6, h=2, eps=0.4.
TINY = Workload("tiny-n20k-d64-l60", 20_000, 64, 60, 6, 2, 0.4, "euclidean",
                200, (0.15, 0.15), 1001, 2001, 3001)
# 1M points, d=128, 5000 clusters of 200, sigma ~ U[0.05, 0.3]; l=128, k=8, h=4, eps=0.5.
PAPER_SCALE = Workload("mixture-n1M-d128-l128-k8-h4", 1_000_000, 128, 128, 8, 4, 0.5,
                       "euclidean", 5000, (0.05, 0.3), 1002, 2002, 3002, subsample=50_000)
# 2M points as PAPER_SCALE; used by the learned-projection form.
LEARNED_SCALE = Workload("mixture-n2M-d128-l128-k8-h4", 2_000_000, 128, 128, 8, 4, 0.5,
                         "euclidean", 5000, (0.05, 0.3), 1005, 2005, 3005, subsample=50_000)

# 4M L2-normalised nonnegative sparse rows (5% density, lognormal(0, 1)
# values), d=256; l=240, k=10, h=8, cosine eps=0.2. Used by the precision form.
PRECISION = Workload("sparse-n4M-d256-l240-k10-h8", 4_000_000, 256, 240, 10, 8, 0.2, "cosine",
                     0, (0.0, 0.0), 1003, 2003, 3003, subsample=50_000, extra={"density": 0.05})

WORKLOADS = {w.name: w for w in (TINY, PAPER_SCALE, LEARNED_SCALE, PRECISION)}


def gaussian_mixture(n: int, d: int, n_centres: int, sigma, seed: int,
                     sigma_mode: str = "coord", dtype=np.float32):
    """Rows of a Gaussian mixture, already shuffled.

    Centres are N(0, I_d). Each centre gets n // n_centres points (the first
    n % n_centres centres get one more). ``sigma`` is a float or a (lo, hi)
    pair; with a pair, each cluster draws its sigma from U[lo, hi].

    Returns (X float32 n x d row-major, labels int32 n).
    """
    if sigma_mode not in SIGMA_MODES:
        raise ValueError(f"sigma_mode must be one of {SIGMA_MODES}")
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.standard_normal((n_centres, d), dtype=np.float32)
    if isinstance(sigma, (tuple, list)):
        lo, hi = float(sigma[0]), float(sigma[1])
    else:
        lo = hi = float(sigma)
    if lo == hi:
        sig = np.full(n_centres, lo, dtype=np.float32)
    else:
        sig = rng.uniform(lo, hi, size=n_centres).astype(np.float32)
    if sigma_mode == "radius":
        sig = sig / np.float32(np.sqrt(d))
    counts = np.full(n_centres, n // n_centres, dtype=np.int64)
    counts[: n % n_centres] += 1
    labels = np.repeat(np.arange(n_centres, dtype=np.int32), counts)
    labels = rng.permutation(labels)
    X = np.empty((n, d), dtype=dtype)
    chunk = 1 << 18
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        g = rng.standard_normal((b - a, d), dtype=np.float32)
        lab = labels[a:b]
        X[a:b] = centres[lab] + sig[lab, None] * g
    return X, labels


def sparse_lognormal(n: int, d: int, density: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Rows with Bernoulli(density) support and lognormal(0, 1) values,
    scaled to unit L2 norm; rows that draw no support stay all-zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((n, d), dtype=np.float32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        mask = rng.random((b - a, d), dtype=np.float32) < density
        block = np.zeros((b - a, d), dtype=np.float32)
        block[mask] = rng.lognormal(0.0, 1.0, size=int(mask.sum())).astype(np.float32)
        nrm = np.sqrt((block.astype(np.float64) ** 2).sum(axis=1)).astype(np.float32)
        nz = nrm > 0
        block[nz] /= nrm[nz, None]
        X[a:b] = block
    return X


def projection_matrix(d: int, ell: int, seed: int) -> np.ndarray:
    """R in R^{d x ell} with i.i.d. N(0, 1) entries, float32, row-major.

    Column c of R is the random direction r_c of bit c (Section 3.2).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((d, ell), dtype=np.float32)


def projection_matrices(d: int, ell: int, Q: int, seed: int) -> np.ndarray:
    """Q independent projection matrices (Q, d, ell), one per string pool
    (Section 4.1). Pool 0 uses `seed` itself, so it equals
    projection_matrix(d, ell, seed); pool q uses seed + 100 q."""
    return np.stack([projection_matrix(d, ell, seed + 100 * q) for q in range(Q)])


def batched_sizes(count: int, seed: int, n_lo: int = 1000, n_hi: int = 200_000, ds=(32, 64, 128)):
    """Sizes of the batched form's instances: n log-uniform in [n_lo, n_hi]
    and d uniform over ds. Returns (ns int64, ds int64), one entry each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).astype(np.int64)
    dd = rng.choice(np.asarray(ds), count).astype(np.int64)
    return ns, dd


def batched_instances(count: int, seed: int, n_lo: int = 1000, n_hi: int = 200_000,
                      ds=(32, 64, 128), ell: int = 64, sigma: float = 0.2, select=None):
    """Sizes and inputs of independent instances for the batched form:
    n log-uniform in [n_lo, n_hi], d uniform over ds, Gaussian-mixture rows
    with n / 100 clusters (at least one) and per-coordinate sigma, and an
    N(0, 1) projection matrix per instance. Returns a list of (X, R).

    ``select`` draws only the listed instances of the `count`; instance i is
    the same array whichever others are drawn with it."""
    ns, dd = batched_sizes(count, seed, n_lo, n_hi, ds)
    out = []
    for i in (range(count) if select is None else select):
        n, d = int(ns[i]), int(dd[i])
        X, _ = gaussian_mixture(n, d, max(1, n // 100), sigma, seed=seed * 1000 + i)
        out.append((X, projection_matrix(d, ell, seed=seed * 1000 + 500_000 + i)))
    return out


def mlp_initial_parameters(d: int, hid: int, ell: int, seed: int) -> np.ndarray:
    """Initial weights of the learned projection, packed FP32
    [W1 (d x hid) | b1 | W2 (hid x ell) | b2]: W ~ N(0, 2 / fan_in), b = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.standard_normal((d, hid)) * np.sqrt(2.0 / d)
    W2 = rng.standard_normal((hid, ell)) * np.sqrt(2.0 / hid)
    return np.concatenate([W1.ravel(), np.zeros(hid), W2.ravel(), np.zeros(ell)]).astype(np.float32)


def workload_inputs(w: Workload, sigma_mode: str = "coord", n: int | None = None):
    """(X, R) for a named mixture workload; ``n`` truncates to the first rows."""
    n_use = w.n if n is None else int(n)
    if "density" in w.extra:
        X = sparse_lognormal(n_use, w.d, w.extra["density"], w.seed_data)
        return X, projection_matrix(w.d, w.ell, w.seed_r)
    X, _ = gaussian_mixture(w.n, w.d, w.n_centres, w.sigma, w.seed_data, sigma_mode)
    if n_use != w.n:
        X = np.ascontiguousarray(X[:n_use])
    R = projection_matrix(w.d, w.ell, w.seed_r)
    return X, R


def subsample_indices(n: int, size: int, seed: int) -> np.ndarray:
    """Sorted indices of a uniform subsample without replacement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    size = min(int(size), int(n))
    return np.sort(rng.choice(n, size=size, replace=False)).astype(np.int64)


def random_strings(n: int, ell: int, seed: int, n_seeds: int = 0,
                   flips: int = 0, copies: int = 0) -> np.ndarray:
    """Bit strings packed as uint64 words (bit c at word c // 64, bit c % 64).

    With ``n_seeds`` > 0 the first ``n_seeds`` rows are uniform strings and the
    remaining rows are copies of a random seed row with up to ``flips`` bits
    flipped at random positions; otherwise all rows are uniform. Padding bits
    above ``ell`` are zero. Rows are shuffled.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    W = (ell + 63) // 64
    bits = rng.integers(0, 2, size=(n, ell), dtype=np.uint8)
    if n_seeds > 0 and n > n_seeds:
        parents = rng.integers(0, n_seeds, size=n - n_seeds)
        child = bits[parents].copy()
        if flips > 0:
            nf = rng.integers(0, flips + 1, size=n - n_seeds)
            for r in range(n - n_seeds):
                if nf[r]:
                    pos = rng.choice(ell, size=int(nf[r]), replace=False)
                    child[r, pos] ^= 1
        bits[n_seeds:] = child
        bits = bits[rng.permutation(n)]
    return pack_bits(bits, W)


def pack_bits(bits: np.ndarray, W: int | None = None) -> np.ndarray:
    """Pack an (n, ell) 0/1 array into (n, W) uint64 words, little-endian bits."""
    n, ell = bits.shape
    if W is None:
        W = (ell + 63) // 64
    padded = np.zeros((n, W * 64), dtype=np.uint8)
    padded[:, :ell] = bits
    by = np.packbits(padded.reshape(n, W * 8, 8), axis=2, bitorder="little").reshape(n, W * 8)
    return by.view(np.uint64).reshape(n, W).copy()


def unpack_bits(S: np.ndarray, ell: int) -> np.ndarray:
    """Inverse of pack_bits: (n, W) uint64 -> (n, ell) uint8."""
    S = np.ascontiguousarray(S, dtype=np.uint64)
    n, W = S.shape
    by = S.view(np.uint8).reshape(n, W * 8)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :ell].copy()
