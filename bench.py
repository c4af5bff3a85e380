"""Benchmark of the whole path on one GPU: project, enumerate, verify.

One step = msm_project (one call per string pool) + the enumeration
(msm_enumerate_pairs, or msm_enumerate_replicates over Q pools) +
msm_verify, over the paper-scale mixture (n = 1,000,000, d = 128, ell = 128
bits, k = 8 blocks, h = 4, Euclidean eps = 0.5), inputs already resident in
device memory. Prints one JSON line. ``value`` is points per second of whole
steps at the headline reading: clusters of radius sigma (the reading under
which the epsilon graph is not empty), with the least number Q of string
pools whose missing-edge ratio against the exhaustive reference on the
50 000-point subsample is at most 1e-3 (Section 4.1, eq. (5)).

The same line carries the other forms side by side, each with its
missing-edge ratio, points/s, edges/s and the roofline of its dominant
kernel: the single-pool step at the same reading, the per-coordinate
reading of sigma (whose epsilon graph is empty), the precision form (4M
sparse cosine rows with FP32 / BF16 / FP8 projections), the learned
projection (2M mixture points, network trained on the GPU, against random
projection at equal ell) and a summary of the output-sensitivity sweep.

Dedicated runs: ``--workload precision|learned|batched|sweep`` print one
line for that form alone (batched: 512 independent instances in one
captured graph; sweep: n from 125k to 2M and the all-identical worst case).

Usage: python bench.py [--steps K] [--warmup W] [--cpu-sample N | --no-cpu-baseline]
                       [--headline-only] [--reading radius|coord] [--pools Q | --q-max Q]
                       [--workload paper|precision|learned|batched|sweep] [--epochs E]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
METRIC = "points/s + edges/s at n=1M,d=128,ℓ=128,h≤4; missing-edge ratio vs brute"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")

# What the hardware counters show bounds each dominant kernel besides its
# algorithmic roofline (rocprofv3 SQ, TA and TD counters of the same
# workloads, summarised in profiles/).
LIMITERS = {
    "k_verify": "vector-memory path carrying both rows of every candidate (radius: TA 0.91, TD 0.93 busy, VALU 0.40)",
    "k_verify_h": "vector-memory path carrying both FP16 rows of every candidate (radius: TA 0.86, TD 0.92 busy, "
                  "VALU 0.58)",
    "k_bucket": "latency of dependent LDS and string-gather steps (VALU 0.46-0.59, TA 0.24-0.40, TD 0.35-0.61 busy)",
    "k_project_x3": "BF16 matrix cores 0.45 busy (six products per FP32 product)",
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the stored
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, each scaled by the
    same counter's reading for a copy of known size), or None when there is
    no such measurement or one of the kernel's sources has changed since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            entries = json.load(f)["entries"]
    except (OSError, ValueError, KeyError):
        return None
    for e in entries:
        if e.get("kernel") != kernel or e.get("workload") != workload:
            continue
        srcs, shas = e["source"], e["sha256"]
        if isinstance(srcs, str):
            srcs, shas = [srcs], [shas]
        try:
            for src, sha in zip(srcs, shas):
                with open(os.path.join(ROOT, src), "rb") as f:
                    if hashlib.sha256(f.read()).hexdigest() != sha:
                        return None
        except OSError:
            return None
        return e["bytes_per_launch"]
    return None


def copy_calibration(nbytes, reps=3):
    """Device-to-device copies of `nbytes` (the counters' reference)."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "reps": reps}), flush=True)


def algorithmic(kernel, w, n, C, mH, mE, W, launches=1, hid=None):
    """(amount, unit, bound) of algorithmic work per launch of a kernel.

    Units per launch: a launch of the partition and bucket kernels covers n
    points under each of the C groupings (C(k, h) combinations of masked
    blocks, or the hierarchical groupings that replace them) of one string
    pool, and writes its share (1 / `launches`) of the mH pairs; k_verify
    covers the mH candidate pairs and the n rows (k_verify_h the same on
    the rows' FP16 copy, k_half_rows the rounding of X); k_project_f32 the
    n x d x ell products (k_project_x3 makes each of them as six BF16
    products); the low-precision projections read X once; k_mlp_fused makes
    the network's 2 n (d hid + hid ell) products.
    """
    sb = 8 * W  # bytes of one string
    if kernel == "k_project_f32":
        return 2.0 * n * w.d * w.ell / 1e12, "TFLOP/s", "mfma"
    if kernel == "k_project_x3":
        return 6 * 2.0 * n * w.d * w.ell / 1e12, "TFLOP/s", "mfma_bf16"
    if kernel in ("k_project_bf16", "k_project_fp8"):
        return (n * 4 * w.d + n * sb) / 1e9, "GB/s", "hbm"
    if kernel == "k_mlp_fused" and hid:
        return 2.0 * n * (w.d * hid + hid * w.ell) / 1e12, "TFLOP/s", "mfma_bf16"
    if kernel == "k_part_count":
        # the string read and its 4-byte mix written for the scatter
        return n * C * (sb + 4) / 1e9, "GB/s", "hbm"
    if kernel == "k_part_scatter":
        # the mix read and the 8-byte entry written
        return n * C * (4 + 8) / 1e9, "GB/s", "hbm"
    if kernel == "k_bucket":
        # per point and combination: its 8-byte partition entry and its string
        return (n * C * (8 + sb) + mH * 8 / max(launches, 1)) / 1e9, "GB/s", "hbm"
    if kernel == "k_verify":
        # compulsory traffic: candidate pairs in, kept pairs out, each row
        # of X once (the two rows of every candidate are re-read through the
        # caches, not from HBM)
        return (mH * 8 + mE * 8 + n * 4 * w.d) / 1e9, "GB/s", "hbm"
    if kernel == "k_verify_h":
        # the same with the rows' FP16 copy and their 4-byte bounds
        return (mH * 8 + mE * 8 + n * (2 * w.d + 4)) / 1e9, "GB/s", "hbm"
    if kernel == "k_half_rows":
        # X read once, its FP16 copy and the row bounds written
        return n * (4 * w.d + 2 * w.d + 4) / 1e9, "GB/s", "hbm"
    return None


def missing_edge_ratio(msm, ctx, w, Xd, hamming, verified, sub=None):
    """|E* minus E_eps| / |E*| on a seeded subsample (Section 4.2), where E* is
    the exhaustive epsilon graph of the subsample (the exhaustive reference) and E_eps the
    verified pairs with both ends in it. Every MSM decision is per pair, so
    restricting to the subsample is exact."""
    import torch

    from paper_0904_3151_amd import inputs as I
    if sub is None:
        sub = torch.from_numpy(I.subsample_indices(w.n, w.subsample, w.seed_sub)).to(Xd.device)
    t0 = time.perf_counter()
    star, mstar = msm.bruteforce_eps(ctx, Xd[sub].contiguous(), w.metric, w.eps, cap_hint=1 << 22)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    n = Xd.shape[0]
    insub = torch.zeros(n, dtype=torch.bool, device=Xd.device)
    insub[sub] = True

    def codes_in_sub(P):
        i = P[:, 0].to(torch.int64)
        j = P[:, 1].to(torch.int64)
        keep = insub[i] & insub[j]
        return torch.unique(i[keep] * n + j[keep])

    star_codes = sub[star[:, 0].to(torch.int64)] * n + sub[star[:, 1].to(torch.int64)]
    got = codes_in_sub(verified)
    ham = codes_in_sub(hamming)
    missed = int((~torch.isin(star_codes, got)).sum()) if mstar else 0
    false_pos = int((~torch.isin(ham, star_codes)).sum()) if ham.numel() else 0
    return {"subsample": int(sub.numel()), "true_pairs": int(mstar), "missed": missed,
            "ratio": (missed / mstar) if mstar else None,
            "type1_candidates": false_pos, "reference_s": round(t_ref, 3),
            "note": None if mstar else "no pair of the subsample is within eps"}


def host_cpu():
    """Model name of the host CPU (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, X, Rs, sample, Q=1):
    """The oracle (FP64 project, MSM per pool, union, verify) on the first
    `sample` rows: the same step as the GPU's, with Q string pools."""
    import numpy as np

    from oracle import oracle as O
    Xs = np.ascontiguousarray(X[:sample])
    metric = O.EUCLIDEAN if w.metric == "euclidean" else O.COSINE
    t0 = time.perf_counter()
    codes = []
    for q in range(Q):
        S = O.project(Xs, Rs[q])
        codes.append(O.pair_codes(O.msm(S, w.ell, w.k, w.h)))
    u = np.unique(np.concatenate(codes)) if codes else np.zeros(0, np.uint64)
    P = np.stack([(u >> np.uint64(32)).astype(np.uint32), (u & np.uint64(0xFFFFFFFF)).astype(np.uint32)], 1)
    O.verify(Xs, P, metric, float(np.float32(w.eps)))
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    what = "all" if sample == w.n else f"first {sample} of"
    return {"value": sample / t, "unit": "points/s", "cores": threads, "kind": "oracle", "cpu": host_cpu(),
            "sample": f"{what} {w.n} points, one full step (FP64 project of {Q} pool(s) + MSM + union "
                      f"+ verify), {t:.1f} s"}


def flip_rate(X, R, S_dev, rows):
    """Fraction of sign bits on sampled rows that differ from the FP64
    projection (oracle), and the fraction outside the 1e-5 |x| band."""
    import numpy as np

    from oracle import oracle as O
    from paper_0904_3151_amd import inputs as I
    So, Z, xn = O.project(X, R, rows=rows, want_z=True)
    ell = R.shape[1]
    bg = I.unpack_bits(S_dev[rows].cpu().numpy().view(np.uint64), ell)
    bo = I.unpack_bits(So, ell)
    bad = bg != bo
    band = np.abs(Z) < 1e-5 * xn[:, None]
    return float(bad.mean()), float((bad & ~band).mean())


def _grow(fn, *args, cap_hint=1 << 20):
    """Call a pair-producing binding with a buffer grown on capacity errors."""
    cap = max(1, int(cap_hint))
    while True:
        try:
            return fn(*args, cap=cap)
        except Exception as e:  # MSMError with the required count
            if getattr(e, "required", None) is None or getattr(e, "status", 0) != -2:
                raise
            cap = int(e.required) + 1


def run_mixture(msm, ctx, w, Xd, project, steps, warmup, ref_sub=None, Q=1, keep_S=False):
    """Time `steps` whole steps (project, enumerate, verify) over a workload
    already on the device, then measure the missing-edge ratio.
    `project(S)` writes the strings: S is (n, W), or (Q, n, W) for Q pools,
    enumerated by msm_enumerate_replicates. Returns a dict of results."""
    import torch

    n, W = Xd.shape[0], (w.ell + 63) // 64
    S = torch.empty((Q, n, W) if Q > 1 else (n, W), dtype=torch.int64, device=Xd.device)
    enum = msm.msm_enumerate_replicates if Q > 1 else msm.msm_enumerate_pairs

    # size the output buffers with a count-only pass
    project(S)
    _, mH = enum(ctx, S, w.ell, w.k, w.h, cap=0)
    # groupings the enumeration made (C(k, h), or fewer hierarchical ones)
    C, jblk = msm.msm_enumerate_last_plan(ctx)
    pairs = torch.empty((max(1, int(mH * 1.05) + 1024), 2), dtype=torch.int32, device=Xd.device)
    verified = torch.empty_like(pairs)
    log(f"{w.name} Q={Q}: hamming pairs {mH}, groupings {C}, j {jblk}")

    def step():
        project(S)
        P, m = enum(ctx, S, w.ell, w.k, w.h, pairs=pairs)
        V, kept = msm.msm_verify(ctx, Xd, P, w.metric, w.eps, out=verified)
        return m, kept

    for _ in range(warmup):
        step()
    # Per-kernel breakdown from a profiled pass of `steps` steps before the
    # timed region (every launch then carries two HIP events, which cost
    # some microseconds each); in the timed region only the kernel with the
    # most time carries events, and its figures replace the breakdown's.
    torch.cuda.synchronize()
    msm.msm_profile_reset(ctx)
    msm.msm_profile_enable(ctx, True)
    for _ in range(steps):
        step()
    msm.msm_profile_enable(ctx, False)
    prof = msm.msm_profile_read(ctx)
    dom = max(prof, key=lambda k: prof[k][1])
    msm.msm_profile_reset(ctx)
    msm.msm_profile_only(ctx, dom)
    msm.msm_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mH, mE = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    msm.msm_profile_enable(ctx, False)
    prof_live = msm.msm_profile_read(ctx)
    msm.msm_profile_only(ctx, None)
    prof[dom] = prof_live[dom]
    ms_step = (t1 - t0) * 1e3 / steps
    phase = {}
    for name, (launches, total) in prof.items():
        phase[name] = {"launches": launches, "avg_ms": total / max(launches, 1), "ms_per_step": total / steps,
                       "timed_region": name == dom}
    t_enum = sum(v["ms_per_step"] for k, v in phase.items()
                 if k in ("k_part_count", "k_part_scan", "k_part_scatter", "k_bucket", "k_bucket_large", "k_big"))
    missing = missing_edge_ratio(msm, ctx, w, Xd, pairs[:mH], verified[:mE], sub=ref_sub)
    res = {"ms_per_step": ms_step, "points_per_s": n / (ms_step / 1e3), "steps": steps, "pools": Q,
           "combinations": C,
           "hier_j": jblk, "hamming_pairs": int(mH), "eps_pairs": int(mE), "phase": phase,
           "hamming_pairs_per_s_enumerate": (mH / (t_enum / 1e3)) if t_enum else None,
           "eps_pairs_per_s_total": mE / (ms_step / 1e3), "missing_edge_ratio": missing}
    if keep_S:
        res["S"] = S
    del pairs, verified
    return res


def roofline_of(res, w, n, W, tag, hid=None):
    """Roofline object of the kernel with the most time per step; `tag`
    names the workload variant for the stored traffic measurement."""
    phase = res["phase"]
    dom = max(phase, key=lambda k: phase[k]["ms_per_step"])
    per_step = max(1, round(phase[dom]["launches"] / max(res.get("steps", 1), 1)))
    alg = algorithmic(dom, w, n, res["combinations"], res["hamming_pairs"], res["eps_pairs"], W,
                      launches=per_step, hid=hid)
    if alg is None:
        return {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}
    amount, unit, bound = alg
    achieved = amount / (phase[dom]["avg_ms"] / 1e3)
    peak = {"mfma": FP32_MFMA_PEAK_TFLOPS, "mfma_bf16": BF16_MFMA_PEAK_TFLOPS}.get(bound, HBM_PEAK_GBS)
    traffic = measured_traffic(dom, tag) if bound == "hbm" else None
    out = {"kernel": dom, "bound": "mfma" if bound.startswith("mfma") else bound, "achieved": round(achieved, 2),
           "peak": peak, "unit": unit, "frac": round(achieved / peak, 4),
           "traffic": round(traffic / 1e9, 4) if traffic is not None else None,
           "traffic_unit": "GB per launch", "algorithmic_per_launch": round(amount, 4)}
    if dom in LIMITERS:
        out["limiter"] = LIMITERS[dom]
    return out


def compact(res, full_kernels=True):
    out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items() if k not in ("phase", "S")}
    if full_kernels:
        out["kernels"] = {k: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                          for k, v in sorted(res["phase"].items())}
    else:
        out["kernels_ms_per_step"] = {k: round(v["ms_per_step"], 4) for k, v in sorted(res["phase"].items())}
    return out


def form_summary(res, roof):
    """The fields every form reports side by side."""
    mr = res["missing_edge_ratio"]
    return {"ms_per_step": round(res["ms_per_step"], 4), "points_per_s": round(res["points_per_s"], 1),
            "pools": res.get("pools", 1), "groupings": res["combinations"],
            "hamming_pairs": res["hamming_pairs"], "eps_pairs": res["eps_pairs"],
            "edges_per_s": {"hamming_pairs_per_s_enumerate": round(res["hamming_pairs_per_s_enumerate"] or 0, 1),
                            "eps_pairs_per_s_total": round(res["eps_pairs_per_s_total"], 1)},
            "missing_edge_ratio": mr["ratio"], "missing": {k: mr[k] for k in ("subsample", "true_pairs", "missed")},
            "roofline": roof,
            "kernels_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in sorted(res["phase"].items())}}


def choose_pools(msm, ctx, w, Xd, Rs, q_max, target):
    """Least number of string pools Q (each projected by its own R) whose
    missing-edge ratio on the reference subsample is at most `target`:
    one untimed pass per Q = 1, 2, ... (Section 4.1, eq. (5); for
    Euclidean radii on data that are not normalised the bound of Section
    4.2 does not apply, so Q is measured rather than computed)."""
    import torch

    n, W = Xd.shape[0], (w.ell + 63) // 64
    table = []
    chosen = None
    for Q in range(1, q_max + 1):
        S = torch.empty((Q, n, W) if Q > 1 else (n, W), dtype=torch.int64, device=Xd.device)
        for q in range(Q):
            msm.msm_project(ctx, Xd, Rs[q], S[q] if Q > 1 else S)
        P, mH = msm.enumerate_pairs(ctx, S, w.ell, w.k, w.h, cap_hint=1 << 27)
        V, mE = msm.msm_verify(ctx, Xd, P, w.metric, w.eps)
        mr = missing_edge_ratio(msm, ctx, w, Xd, P, V)
        table.append({"Q": Q, "hamming_pairs": int(mH), "eps_pairs": int(mE), "ratio": mr["ratio"],
                      "missed": mr["missed"], "true_pairs": mr["true_pairs"]})
        log(f"pools Q={Q}: {table[-1]}")
        del S, P, V
        torch.cuda.empty_cache()
        if mr["ratio"] is not None and mr["ratio"] <= target:
            chosen = Q
            break
    return (chosen or q_max), table


def form_precision(args, steps, warmup):
    """The precision form: 4M sparse cosine rows projected in FP32, BF16 and
    row-scaled FP8 (FP32 recompute inside |z| < 2^-8 |x|), then the same
    enumeration and verification; per dtype: flip rate against the FP64
    projection on sampled rows, recomputed fraction, missing-edge ratio."""
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm
    from paper_0904_3151_amd import params as PR

    w = I.PRECISION
    log(f"generating {w.name}")
    X, R = I.workload_inputs(w)
    n, W = w.n, (w.ell + 63) // 64
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Rd = torch.from_numpy(R).to(dev)
    ctx = msm.Context(0)
    tau = 2.0 ** -8
    sub = torch.from_numpy(I.subsample_indices(n, w.subsample, w.seed_sub)).to(dev)
    rows = I.subsample_indices(n, 20_000, w.seed_sub + 1)
    per = {}
    for dt in ("f32", "bf16", "fp8"):
        def project(S, dt=dt):
            if dt == "f32":
                msm.msm_project(ctx, Xd, Rd, S)
            else:
                msm.msm_project_lowp(ctx, Xd, Rd, dt, tau, S)

        res = run_mixture(msm, ctx, w, Xd, project, steps, warmup, ref_sub=sub, keep_S=True)
        fr, fr_out = flip_rate(X, R, res["S"], rows)
        nre = msm.msm_project_lowp(ctx, Xd, Rd, dt, tau, res["S"], count_recomputed=True)[1] if dt != "f32" else 0
        per[dt] = form_summary(res, roofline_of(res, w, n, W, f"{w.name}:{dt}"))
        per[dt].update({"flip_rate_vs_fp64": fr, "flip_rate_outside_1e-5_band": fr_out,
                        "recomputed_fraction": nre / (n * w.ell)})
        log(f"precision {dt}: {per[dt]}")
        del res
        torch.cuda.empty_cache()
    p = PR.flip_probability(w.eps)
    out = {"config": {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                      "metric": w.metric, "tau": tau, "reference_subsample": int(sub.numel())},
           "per_dtype": per,
           "bound_section_4_2": {"p": p, "miss_per_pool": PR.miss_probability(w.ell, w.h, p),
                                 "pools_for_1e-3": PR.replicates_needed(w.ell, w.h, p, 1e-3)},
           "note": ("at ell = 240 and h = 8 the Hamming threshold lies far below the angle that cosine "
                    "eps = 0.2 allows, so nearly every epsilon-pair is missed whatever the projection's "
                    "precision; no number of pools within reach meets 1e-3 (the bound above), and the form "
                    "compares the precisions' flip rates and speed")}
    ctx.close()
    del Xd, Rd, X
    torch.cuda.empty_cache()
    return out


def form_learned(args, steps, warmup):
    """The learned-projection form: 2M mixture points (cluster radius reading
    of sigma), a 128-512-128 network trained on the GPU on epsilon-pairs and
    non-pairs mined by the exhaustive search from a 100k-point sample, then
    whole steps with learned and with random strings at equal ell, each
    measured on a 50k subsample disjoint from the training sample."""
    import numpy as np
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import learned as L
    from paper_0904_3151_amd import msm

    w = I.LEARNED_SCALE
    log(f"generating {w.name} (radius)")
    X, R = I.workload_inputs(w, sigma_mode="radius")
    n, W = w.n, (w.ell + 63) // 64
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Rd = torch.from_numpy(R).to(dev)
    del X
    ctx = msm.Context(0)
    train_idx = I.subsample_indices(n, 100_000, w.seed_sub + 7)
    held = np.setdiff1d(np.arange(n, dtype=np.int64), train_idx)
    ref_sub = torch.from_numpy(held[I.subsample_indices(held.size, w.subsample, w.seed_sub)]).to(dev)
    Xt = Xd[torch.from_numpy(train_idx).to(dev)].contiguous()
    t0 = time.perf_counter()
    tp, tl, stats = L.mine_pairs(ctx, Xt, w.eps, n_pos=200_000, n_neg=200_000, seed=w.seed_sub + 8)
    torch.cuda.synchronize()
    t_mine = time.perf_counter() - t0
    # the loss's h is twice the MSM threshold: epsilon-pairs are pulled to
    # Hamming distance h_MSM, other pairs pushed beyond 6 h_MSM
    cfg = L.TrainConfig(hid=512, ell=w.ell, h=args.train_h or 2 * w.h, lam=0.05, lr=1e-3, batch=4096,
                        epochs=args.epochs, seed=11)
    t0 = time.perf_counter()
    params, _, _, losses, nsteps = L.train(ctx, Xt, tp, tl, cfg, I.mlp_initial_parameters(w.d, cfg.hid, w.ell, 12))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"mined {stats} in {t_mine:.1f} s; trained {nsteps - 1} steps in {t_train:.1f} s, "
        f"loss {losses[0]:.3f} -> {np.mean(losses[-20:]):.3f}")
    learned = run_mixture(msm, ctx, w, Xd, lambda S: msm.msm_project_mlp(ctx, Xd, params, cfg.hid, w.ell, S),
                          steps, warmup, ref_sub)
    rand = run_mixture(msm, ctx, w, Xd, lambda S: msm.msm_project(ctx, Xd, Rd, S), steps, warmup, ref_sub)
    ph = learned["phase"].get("k_mlp_fused")
    mlp_roof = None
    if ph:
        amount, unit, _ = algorithmic("k_mlp_fused", w, n, 0, 0, 0, W, hid=cfg.hid)
        ach = amount / (ph["avg_ms"] / 1e3)
        mlp_roof = {"kernel": "k_mlp_fused", "bound": "mfma", "achieved": round(ach, 2),
                    "peak": BF16_MFMA_PEAK_TFLOPS, "unit": unit, "frac": round(ach / BF16_MFMA_PEAK_TFLOPS, 4),
                    "traffic": None}
    out = {"config": {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                      "metric": w.metric, "hidden": cfg.hid, "train_sample": int(train_idx.size),
                      "reference_subsample": int(ref_sub.numel()), "sigma_mode": "radius"},
           "training": {"mining": stats, "mining_s": round(t_mine, 2), "steps": nsteps - 1,
                        "train_s": round(t_train, 2), "loss_first": losses[0],
                        "loss_last20": float(np.mean(losses[-20:])), "config": vars(cfg)},
           "learned": form_summary(learned, roofline_of(learned, w, n, W, f"{w.name}:radius:learned")),
           "random_lsh": form_summary(rand, roofline_of(rand, w, n, W, f"{w.name}:radius")),
           "roofline_projection": mlp_roof}
    ctx.close()
    del Xd, Rd, Xt
    torch.cuda.empty_cache()
    return out


def form_sweep(args, steps, warmup, cpu_n=0):
    """Output sensitivity (Sections 2.3 and 5.4): whole steps on the
    paper-scale mixture (radius reading, 5000 clusters) at n = 125k ... 2M,
    with time per 10k output pairs and the dominant kernel's roofline at
    each n, the oracle's step at the smallest n on the host, and the worst
    case of Section 2.3 where all strings are identical and every pair is
    output."""
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    w0 = I.PAPER_SCALE
    dev = torch.device("cuda:0")
    ctx = msm.Context(0)
    R = I.projection_matrix(w0.d, w0.ell, w0.seed_r)
    Rd = torch.from_numpy(R).to(dev)
    rows = []
    cpu = None
    for n in (125_000, 250_000, 500_000, 1_000_000, 2_000_000):
        X, _ = I.gaussian_mixture(n, w0.d, w0.n_centres, w0.sigma, w0.seed_data, "radius")
        w = I.Workload(f"sweep-mixture-n{n}", n, w0.d, w0.ell, w0.k, w0.h, w0.eps, w0.metric, w0.n_centres,
                       w0.sigma, w0.seed_data, w0.seed_r, w0.seed_sub, subsample=min(n, 50_000))
        Xd = torch.from_numpy(X).to(dev)
        res = run_mixture(msm, ctx, w, Xd, lambda S: msm.msm_project(ctx, Xd, Rd, S), steps, warmup)
        roof = roofline_of(res, w, n, 2, f"{w.name}:radius")
        mr = res["missing_edge_ratio"]
        rows.append({"n": n, "ms_per_step": round(res["ms_per_step"], 4), "points_per_s": round(res["points_per_s"], 1),
                     "hamming_pairs": res["hamming_pairs"], "eps_pairs": res["eps_pairs"],
                     "ms_per_10k_eps_pairs": round(res["ms_per_step"] / max(res["eps_pairs"], 1) * 1e4, 6),
                     "missing_edge_ratio": mr["ratio"], "groupings": res["combinations"],
                     "dominant": roof["kernel"], "dominant_frac": roof["frac"], "dominant_unit": roof["unit"]})
        log(rows[-1])
        if cpu_n and n == 125_000:
            cpu = cpu_baseline(w, X, [R], n)
            cpu["sample"] = f"n = {n} of the sweep, " + cpu["sample"]
        del Xd, X, res
        torch.cuda.empty_cache()
    # worst case: n identical strings, all n (n - 1) / 2 pairs are output
    n = 20_000
    S = torch.zeros((n, 2), dtype=torch.int64, device=dev)
    _, m = msm.msm_enumerate_pairs(ctx, S, w0.ell, w0.k, w0.h, cap=0)
    pairs = torch.empty((m, 2), dtype=torch.int32, device=dev)
    msm.msm_enumerate_pairs(ctx, S, w0.ell, w0.k, w0.h, pairs=pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        msm.msm_enumerate_pairs(ctx, S, w0.ell, w0.k, w0.h, pairs=pairs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    worst = {"n": n, "pairs": int(m), "expected": n * (n - 1) // 2, "ms": round(ms, 3),
             "pairs_per_s": round(m / ms * 1e3, 1),
             "write_GB_per_s": round(m * 8 / (ms / 1e3) / 1e9, 1)}
    log(worst)
    ratios = [round(rows[i + 1]["ms_per_step"] / rows[i]["ms_per_step"], 3) for i in range(len(rows) - 1)]
    pair_ratios = [round(rows[i + 1]["eps_pairs"] / max(rows[i]["eps_pairs"], 1), 3) for i in range(len(rows) - 1)]
    ctx.close()
    return {"config": {"workload": "sweep-mixture-d128-l128-k8-h4-radius", "k": w0.k, "h": w0.h, "ell": w0.ell,
                       "eps": w0.eps},
            "sweep": rows, "time_ratio_when_n_doubles": ratios, "eps_pairs_ratio_when_n_doubles": pair_ratios,
            "all_identical": worst, "cpu_baseline": cpu}


def line(metric_value, ms, args, dtype, data, config, **extra):
    out = {"metric": METRIC, "value": round(metric_value, 1), "unit": "points/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": data, "config": config}
    out.update(extra)
    return out


def run_precision(args):
    f = form_precision(args, args.steps, args.warmup)
    bf = f["per_dtype"]["bf16"]
    print(json.dumps(line(bf["points_per_s"], bf["ms_per_step"], args, "bf16", "synthetic sparse lognormal rows",
                          f["config"], **{k: v for k, v in f.items() if k != "config"},
                          roofline=bf["roofline"], cpu_baseline=None)), flush=True)


def run_learned(args):
    f = form_learned(args, args.steps, args.warmup)
    le = f["learned"]
    print(json.dumps(line(le["points_per_s"], le["ms_per_step"], args, "bf16",
                          "synthetic Gaussian mixture, sigma_mode=radius", f["config"],
                          **{k: v for k, v in f.items() if k != "config"}, roofline=le["roofline"],
                          cpu_baseline=None)), flush=True)


def run_sweep(args):
    f = form_sweep(args, args.steps, args.warmup, cpu_n=0 if args.no_cpu_baseline else 1)
    last = f["sweep"][-2]
    print(json.dumps(line(last["points_per_s"], last["ms_per_step"], args, "f32",
                          "synthetic Gaussian mixture, sigma_mode=radius", f["config"],
                          **{k: v for k, v in f.items() if k not in ("config", "cpu_baseline")},
                          roofline=None, cpu_baseline=f["cpu_baseline"])), flush=True)


def run_batched(args):
    """The batched form: 512 independent instances (n log-uniform in
    [1000, 200000], d in {32, 64, 128}, Gaussian mixtures with n / 100
    clusters and sigma 0.2, ell = 64, k = 5, h = 3), projected and enumerated
    by one captured graph per step. Also timed: the same run enqueued
    eagerly (with per-kernel times) and the instances one by one through
    msm_project + msm_enumerate_pairs."""
    import numpy as np
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    ell, k, h, count = 64, 5, 3, 512
    log("generating 512 instances")
    inst = I.batched_instances(count, seed=1004, ell=ell)
    dev = torch.device("cuda:0")
    Xs = [torch.from_numpy(X).to(dev) for X, _ in inst]
    Rs = [torch.from_numpy(R).to(dev) for _, R in inst]
    ns = np.array([X.shape[0] for X, _ in inst], dtype=np.int64)
    ds = np.array([X.shape[1] for X, _ in inst], dtype=np.int64)
    N = int(ns.sum())
    del inst
    ctx = msm.Context(0)
    caps = [int(40 * n) for n in ns]
    t0 = time.perf_counter()
    b = msm.Batch(ctx, Xs, Rs, ell, k, h, caps, autotune=True)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    tuning = b.tuning()
    log(f"plan + autotune {t_plan:.2f} s, chosen {tuning['chosen']}")
    for _ in range(args.warmup):
        b.run(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m = b.run(graph=True)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / args.steps
    m = m.cpu().numpy()
    overflow = int((m > np.array(caps)).sum())
    # eager runs with per-kernel event timing
    msm.msm_profile_reset(ctx)
    msm.msm_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / args.steps
    msm.msm_profile_enable(ctx, False)
    prof = msm.msm_profile_read(ctx)
    phase = {name: {"launches": l, "avg_ms": t / max(l, 1), "ms_per_step": t / args.steps}
             for name, (l, t) in prof.items()}
    # the instances one at a time through the single-problem entry points
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(count):
        S = msm.msm_project(ctx, Xs[i], Rs[i])
        msm.msm_enumerate_pairs(ctx, S, ell, k, h, cap=0)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    # untimed: the single-problem enumeration of the batch's own strings
    # gives each instance's count (the two projections may differ in bits
    # within their rounding band, so their strings are not compared)
    same = True
    for i in range(count):
        _, mi = msm.msm_enumerate_pairs(ctx, b.S[i], ell, k, h, cap=0)
        same &= (mi == m[i])
    C = 10
    dom = max(phase, key=lambda q: phase[q]["ms_per_step"]) if phase else None
    roof = None
    if dom:
        mH = int(m.sum())
        per = {"k_bpart_count": N * C * 8, "k_bpart_scatter": N * C * 16, "k_bucket_batch": N * C * 16 + mH * 8,
               "k_project_batch": int((ns * ds).sum()) * 4 + N * 16}
        if dom in per:
            ach = per[dom] / 1e9 / (phase[dom]["avg_ms"] / 1e3)
            roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    out = {"metric": METRIC, "value": round(N / (ms_graph / 1e3), 1), "unit": "points/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_graph, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic Gaussian mixtures, one per instance",
           "config": {"workload": "batched-512-instances-l64-k5-h3", "instances": count, "total_points": N,
                      "n_range": [int(ns.min()), int(ns.max())], "ell": ell, "k": k, "h": h},
           "hamming_pairs": int(m.sum()), "hamming_pairs_per_s": round(float(m.sum()) / (ms_graph / 1e3), 1),
           "instances_over_capacity": overflow,
           "ms_per_step_eager": round(ms_eager, 4), "ms_one_by_one": round(ms_seq, 2),
           # time the kernels themselves take per step (events around each
           # launch in the eager runs): the graph's time beyond it is launch
           # gaps that one persistent kernel could remove
           "kernel_sum_ms": round(sum(v["ms_per_step"] for v in phase.values()), 4),
           "one_by_one_counts_match": bool(same), "plan_and_tune_s": round(t_plan, 2), "autotune": tuning,
           "kernels": {q: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                       for q, v in sorted(phase.items())},
           "roofline": roof, "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    b.close()
    ctx.close()




def run_paper(args):
    """The default line: the headline step (radius reading, Q pools chosen
    for a missing-edge ratio of at most 1e-3) and the other forms."""
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    w = I.PAPER_SCALE
    target = 1e-3
    reading = args.reading
    log(f"generating {w.name} ({reading})")
    X, _ = I.workload_inputs(w, sigma_mode=reading)
    n, W = w.n, (w.ell + 63) // 64
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    q_top = max(args.q_max, args.pools)
    Rs_np = I.projection_matrices(w.d, w.ell, q_top, w.seed_r)
    Rs = [torch.from_numpy(Rs_np[q]).to(dev) for q in range(q_top)]
    ctx = msm.Context(0)
    if args.pools > 0 or reading == "coord":
        # a fixed number of pools (the per-coordinate reading has no
        # epsilon-pairs, so no ratio to choose it by)
        Q, q_table = max(1, args.pools), None
    else:
        Q, q_table = choose_pools(msm, ctx, w, Xd, Rs, args.q_max, target)

    def project_pools(S, Q=Q):
        if Q == 1:
            msm.msm_project(ctx, Xd, Rs[0], S)
        else:
            for q in range(Q):
                msm.msm_project(ctx, Xd, Rs[q], S[q])

    res = run_mixture(msm, ctx, w, Xd, project_pools, args.steps, args.warmup, Q=Q)
    tag = f"{w.name}:{reading}" + (f":q{Q}" if Q > 1 else "")
    roof = roofline_of(res, w, n, W, tag)
    forms = {}
    errors = {}

    def attempt(name, fn):
        try:
            forms[name] = fn()
        except Exception as e:  # a form that fails is reported, the headline stands
            errors[name] = f"{type(e).__name__}: {e}"
            log(f"form {name} failed: {errors[name]}")
        torch.cuda.empty_cache()

    small = max(1, min(args.steps, 5))
    if not args.headline_only:
        def single_pool():
            r1 = run_mixture(msm, ctx, w, Xd, lambda S: msm.msm_project(ctx, Xd, Rs[0], S), small,
                             min(args.warmup, 2))
            return form_summary(r1, roofline_of(r1, w, n, W, f"{w.name}:radius"))

        if Q > 1 and reading == "radius":
            attempt("single_pool_radius", single_pool)

        def coord():
            Xc, _ = I.workload_inputs(w, sigma_mode="coord")
            Xcd = torch.from_numpy(Xc).to(dev)
            del Xc
            rc = run_mixture(msm, ctx, w, Xcd, lambda S: msm.msm_project(ctx, Xcd, Rs[0], S), small,
                             min(args.warmup, 2))
            out = form_summary(rc, roofline_of(rc, w, n, W, f"{w.name}:coord"))
            out["note"] = "per-coordinate reading of sigma: no pair lies within eps, the ratio is undefined"
            return out

        if reading == "radius":
            attempt("coord_reading", coord)
    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample if 0 < args.cpu_sample < n else n
        log(f"cpu baseline on {sample} points, {Q} pool(s)")
        cpu = cpu_baseline(w, X, Rs_np, sample, Q=Q)
    del X
    if not args.headline_only:
        attempt("learned", lambda: form_learned(args, small, min(args.warmup, 2)))
        attempt("precision", lambda: form_precision(args, small, min(args.warmup, 2)))
        attempt("sweep", lambda: form_sweep(args, small, min(args.warmup, 2)))

    c = compact(res)
    mr = res["missing_edge_ratio"]
    mr["target"] = target
    out = line(res["points_per_s"], res["ms_per_step"], args, "f32",
               f"synthetic Gaussian mixture, sigma_mode={reading}",
               {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                "metric": w.metric, "sigma_mode": reading, "pools": Q, "groupings": res["combinations"],
                "hier_j": res["hier_j"],
                "projection_arith": ("fp32 as three bf16 parts, six products, fp32 accumulation"
                                     if w.ell <= 128 and w.d <= 256 else "fp32 products")},
               edges_per_s={"hamming_pairs_per_s_enumerate": c["hamming_pairs_per_s_enumerate"],
                            "eps_pairs_per_s_total": c["eps_pairs_per_s_total"]},
               counts={"hamming_pairs": res["hamming_pairs"], "eps_pairs": res["eps_pairs"]},
               kernels=c["kernels"], missing_edge_ratio=mr, pools_search=q_table, roofline=roof,
               cpu_baseline=cpu, forms=forms, form_errors=errors or None)
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=500_000,
                    help="rows for the CPU oracle (0: all); the default keeps the oracle's step near 10 s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline step (no other forms in the line)")
    ap.add_argument("--q-max", type=int, default=6, help="most string pools the headline may use")
    ap.add_argument("--pools", type=int, default=0,
                    help="string pools of the headline step (0: the least whose missing-edge ratio is <= 1e-3)")
    ap.add_argument("--reading", default="radius", choices=["radius", "coord"],
                    help="reading of the mixture's sigma for the headline step (cluster radius, or per coordinate)")
    ap.add_argument("--epochs", type=int, default=20, help="training epochs of the learned form")
    ap.add_argument("--train-h", type=int, default=0,
                    help="h of the training loss of the learned form (0: twice the workload's h)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES on the device a few times (reference for the HBM counters)")
    ap.add_argument("--workload", default="paper", choices=["paper", "precision", "learned", "batched", "sweep"],
                    help="paper: the 1M mixture with every form (default); precision: 4M sparse rows, "
                         "FP32/BF16/FP8; learned: 2M mixture, trained network vs random projection; "
                         "batched: 512 instances in one captured graph; "
                         "sweep: n from 125k to 2M and the all-identical worst case")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the MSM path here is built and measured on a single "
              "MI355X (see the design notes for how it would shard).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    {"paper": run_paper, "precision": run_precision, "learned": run_learned, "batched": run_batched,
     "sweep": run_sweep}[args.workload](args)


if __name__ == "__main__":
    main()
