"""Benchmark of the whole path on one GPU: project, enumerate, verify.

One step = msm_project + msm_enumerate_pairs + msm_verify over the paper-scale
mixture (n = 1,000,000, d = 128, ell = 128 bits, k = 8 blocks, h = 4,
Euclidean eps = 0.5), inputs already resident in device memory. Prints one
JSON line. ``value`` is points per second of whole steps. The run is repeated
under the other reading of the mixture's sigma (per-coordinate standard
deviation, or cluster radius), under which the epsilon graph is not empty
and the missing-edge ratio is defined.

Other workloads: ``--workload precision`` (4M sparse cosine rows, FP32 /
BF16 / FP8 projections) and ``--workload learned`` (2M mixture points, the
learned projection trained on the GPU against random projection) and
``--workload batched`` (512 independent instances in one captured graph)
and ``--workload sweep`` (output sensitivity: n from 125k to 2M, and the
all-identical worst case).

Usage: python bench.py [--steps K] [--warmup W] [--sigma-mode coord|radius]
                       [--cpu-sample N | --no-cpu-baseline] [--no-second-reading]
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


def algorithmic(kernel, w, n, C, mH, mE, W):
    """(amount, unit, bound) of algorithmic work per launch of a kernel.

    Units per launch: a launch of the partition and bucket kernels covers n
    points under each of the C groupings (C(k, h) combinations of masked
    blocks, or the hierarchical groupings that replace them); k_verify covers the mH
    candidate pairs and the n rows; k_project_f32 the n x d x ell products
    (k_project_x3 makes each of them as six BF16 products).
    """
    sb = 8 * W  # bytes of one string
    if kernel == "k_project_f32":
        return 2.0 * n * w.d * w.ell / 1e12, "TFLOP/s", "mfma"
    if kernel == "k_project_x3":
        return 6 * 2.0 * n * w.d * w.ell / 1e12, "TFLOP/s", "mfma_bf16"
    if kernel == "k_part_count":
        return n * C * sb / 1e9, "GB/s", "hbm"
    if kernel == "k_part_scatter":
        return n * C * (sb + 8) / 1e9, "GB/s", "hbm"
    if kernel == "k_bucket":
        # per point and combination: its 8-byte partition entry and its string
        return (n * C * (8 + sb) + mH * 8) / 1e9, "GB/s", "hbm"
    if kernel == "k_verify":
        # compulsory traffic: candidate pairs in, kept pairs out, each row
        # of X once (the two rows of every candidate are re-read through the
        # caches, not from HBM)
        return (mH * 8 + mE * 8 + n * 4 * w.d) / 1e9, "GB/s", "hbm"
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


def cpu_baseline(w, X, R, sample):
    """The oracle (FP64 project, MSM, verify) on the first `sample` rows."""
    import numpy as np

    from oracle import oracle as O
    Xs = np.ascontiguousarray(X[:sample])
    t0 = time.perf_counter()
    S = O.project(Xs, R)
    P = O.msm(S, w.ell, w.k, w.h)
    O.verify(Xs, P, O.EUCLIDEAN, float(np.float32(w.eps)))
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    what = "all" if sample == w.n else f"first {sample} of"
    return {"value": sample / t, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"{what} {w.n} points, one full step (FP64 project + MSM + verify), {t:.1f} s"}


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


def run_precision(args):
    """The precision form: 4M sparse cosine rows projected in FP32, BF16 and
    row-scaled FP8 (FP32 recompute inside |z| < 2^-8 |x|), then the same
    enumeration and verification. One JSON line with every dtype."""
    import numpy as np
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    w = I.PRECISION
    log(f"generating {w.name}")
    X, R = I.workload_inputs(w)
    n, W = w.n, (w.ell + 63) // 64
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Rd = torch.from_numpy(R).to(dev)
    S = torch.empty((n, W), dtype=torch.int64, device=dev)
    ctx = msm.Context(0)
    tau = 2.0 ** -8
    sub = torch.from_numpy(I.subsample_indices(n, w.subsample, w.seed_sub)).to(dev)
    star, mstar = msm.bruteforce_eps(ctx, Xd[sub].contiguous(), w.metric, w.eps, cap_hint=1 << 22)
    insub = torch.zeros(n, dtype=torch.bool, device=dev)
    insub[sub] = True
    star_codes = sub[star[:, 0].to(torch.int64)] * n + sub[star[:, 1].to(torch.int64)]
    rows = I.subsample_indices(n, 20_000, w.seed_sub + 1)
    per = {}
    for dt in ("f32", "bf16", "fp8"):
        def project():
            if dt == "f32":
                msm.msm_project(ctx, Xd, Rd, S)
            else:
                msm.msm_project_lowp(ctx, Xd, Rd, dt, tau, S)

        project()
        _, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, cap=0)
        pairs = torch.empty((max(1, int(mH * 1.05) + 1024), 2), dtype=torch.int32, device=dev)
        verified = torch.empty_like(pairs)
        for _ in range(args.warmup):
            project()
            P, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
            msm.msm_verify(ctx, Xd, P, w.metric, w.eps, out=verified)
        msm.msm_profile_reset(ctx)
        msm.msm_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            project()
            P, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
            V, mE = msm.msm_verify(ctx, Xd, P, w.metric, w.eps, out=verified)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        msm.msm_profile_enable(ctx, False)
        prof = msm.msm_profile_read(ctx)
        _, nre = (msm.msm_project_lowp(ctx, Xd, Rd, dt, tau, S, count_recomputed=True) if dt != "f32"
                  else (None, 0))
        fr, fr_out = flip_rate(X, R, S, rows)
        i = V[:, 0].to(torch.int64)
        j = V[:, 1].to(torch.int64)
        keep = insub[i] & insub[j]
        got = torch.unique(i[keep] * n + j[keep])
        missed = int((~torch.isin(star_codes, got)).sum()) if mstar else 0
        per[dt] = {"ms_per_step": round(ms, 4), "points_per_s": round(n / (ms / 1e3), 1),
                   "hamming_pairs": int(mH), "eps_pairs": int(mE),
                   "flip_rate_vs_fp64": fr, "flip_rate_outside_1e-5_band": fr_out,
                   "recomputed_fraction": nre / (n * w.ell),
                   "missing_edge_ratio": (missed / mstar) if mstar else None,
                   "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in sorted(prof.items())}}
        log(f"{dt}: {per[dt]}")
        del pairs, verified
    out = {"metric": METRIC, "value": per["bf16"]["points_per_s"], "unit": "points/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": per["bf16"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic sparse lognormal rows",
           "config": {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                      "metric": w.metric, "tau": tau, "reference_subsample": int(sub.numel()),
                      "reference_true_pairs": int(mstar)},
           "per_dtype": per}
    print(json.dumps(out), flush=True)
    ctx.close()


def run_mixture(msm, ctx, w, X, Xd, project, steps, warmup, ref_sub=None):
    """Time `steps` whole steps (project, enumerate, verify) over a mixture
    workload already on the device, then measure the missing-edge ratio.
    `project(S)` writes the strings. Returns a dict of results."""
    import torch

    n, W = Xd.shape[0], (w.ell + 63) // 64
    S = torch.empty((n, W), dtype=torch.int64, device=Xd.device)

    # size the output buffers with a count-only pass
    project(S)
    _, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, cap=0)
    # groupings the enumeration made (C(k, h), or fewer hierarchical ones)
    C, jblk = msm.msm_enumerate_last_plan(ctx)
    pairs = torch.empty((max(1, int(mH * 1.05) + 1024), 2), dtype=torch.int32, device=Xd.device)
    verified = torch.empty_like(pairs)
    log(f"hamming pairs {mH}, groupings {C}, j {jblk}")

    def step():
        project(S)
        P, m = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
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
                 if k in ("k_part_count", "k_part_scan", "k_part_scatter", "k_bucket", "k_big"))
    missing = missing_edge_ratio(msm, ctx, w, Xd, pairs[:mH], verified[:mE], sub=ref_sub)
    res = {"ms_per_step": ms_step, "points_per_s": n / (ms_step / 1e3), "combinations": C, "hier_j": jblk,
           "hamming_pairs": int(mH), "eps_pairs": int(mE), "phase": phase,
           "hamming_pairs_per_s_enumerate": (mH / (t_enum / 1e3)) if t_enum else None,
           "eps_pairs_per_s_total": mE / (ms_step / 1e3), "missing_edge_ratio": missing}
    del pairs, verified, S
    return res


def roofline_of(res, w, n, W, tag):
    """Roofline object of the kernel with the most time per step; `tag`
    names the workload variant for the stored traffic measurement."""
    phase = res["phase"]
    dom = max(phase, key=lambda k: phase[k]["ms_per_step"])
    alg = algorithmic(dom, w, n, res["combinations"], res["hamming_pairs"], res["eps_pairs"], W)
    if alg is None:
        return {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}
    amount, unit, bound = alg
    achieved = amount / (phase[dom]["avg_ms"] / 1e3)
    peak = {"mfma": FP32_MFMA_PEAK_TFLOPS, "mfma_bf16": BF16_MFMA_PEAK_TFLOPS}.get(bound, HBM_PEAK_GBS)
    traffic = measured_traffic(dom, tag) if bound == "hbm" else None
    return {"kernel": dom, "bound": "mfma" if bound.startswith("mfma") else bound, "achieved": round(achieved, 2),
            "peak": peak, "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": round(traffic / 1e9, 4) if traffic is not None else None,
            "traffic_unit": "GB per launch", "algorithmic_per_launch": round(amount, 4)}


def compact(res):
    out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items() if k != "phase"}
    out["kernels"] = {k: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                      for k, v in sorted(res["phase"].items())}
    return out


def run_learned(args):
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

    learned = run_mixture(msm, ctx, w, X, Xd, lambda S: msm.msm_project_mlp(ctx, Xd, params, cfg.hid, w.ell, S),
                          args.steps, args.warmup, ref_sub)
    log(f"learned: {compact(learned)}")
    rand = run_mixture(msm, ctx, w, X, Xd, lambda S: msm.msm_project(ctx, Xd, Rd, S), args.steps, args.warmup,
                       ref_sub)
    log(f"random: {compact(rand)}")
    flops = 2.0 * n * (w.d * cfg.hid + cfg.hid * w.ell)
    ph = learned["phase"].get("k_mlp_fused")
    mlp_roof = None
    if ph:
        ach = flops / (ph["avg_ms"] / 1e3) / 1e12
        mlp_roof = {"kernel": "k_mlp_fused", "bound": "mfma", "achieved": round(ach, 2),
                    "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / BF16_MFMA_PEAK_TFLOPS, 4),
                    "traffic": None}
    out = {"metric": METRIC, "value": round(learned["points_per_s"], 1), "unit": "points/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(learned["ms_per_step"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic Gaussian mixture, sigma_mode=radius",
           "config": {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                      "metric": w.metric, "hidden": cfg.hid, "train_sample": int(train_idx.size),
                      "reference_subsample": int(ref_sub.numel())},
           "training": {"mining": stats, "mining_s": round(t_mine, 2), "steps": nsteps - 1,
                        "train_s": round(t_train, 2), "loss_first": losses[0],
                        "loss_last20": float(np.mean(losses[-20:])), "config": vars(cfg)},
           "learned": compact(learned), "random_lsh": compact(rand),
           "roofline": roofline_of(learned, w, n, W, f"{w.name}:radius:learned"), "roofline_projection": mlp_roof,
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    ctx.close()


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
    same = True
    for i in range(count):
        S = msm.msm_project(ctx, Xs[i], Rs[i])
        _, mi = msm.msm_enumerate_pairs(ctx, S, ell, k, h, cap=0)
        same &= (mi == m[i])
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
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
           "one_by_one_counts_match": bool(same), "plan_and_tune_s": round(t_plan, 2), "autotune": tuning,
           "kernels": {q: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                       for q, v in sorted(phase.items())},
           "roofline": roof, "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    b.close()
    ctx.close()


def run_sweep(args):
    """Output sensitivity (Sections 2.3 and 5.4): whole steps on the
    paper-scale mixture (radius reading, 5000 clusters) at n = 125k ... 2M,
    with time per 10k output pairs, and the worst case of Section 2.3 where
    all strings are identical and every pair is output."""
    import numpy as np
    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    w = I.PAPER_SCALE
    dev = torch.device("cuda:0")
    ctx = msm.Context(0)
    R = torch.from_numpy(I.projection_matrix(w.d, w.ell, w.seed_r)).to(dev)
    rows = []
    for n in (125_000, 250_000, 500_000, 1_000_000, 2_000_000):
        X, _ = I.gaussian_mixture(n, w.d, w.n_centres, w.sigma, w.seed_data, "radius")
        Xd = torch.from_numpy(X).to(dev)
        del X
        S = torch.empty((n, 2), dtype=torch.int64, device=dev)
        msm.msm_project(ctx, Xd, R, S)
        _, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, cap=0)
        pairs = torch.empty((int(mH * 1.05) + 1024, 2), dtype=torch.int32, device=dev)
        out = torch.empty_like(pairs)
        for _ in range(args.warmup):
            msm.msm_project(ctx, Xd, R, S)
            P, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
            msm.msm_verify(ctx, Xd, P, w.metric, w.eps, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            msm.msm_project(ctx, Xd, R, S)
            P, mH = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
            _, mE = msm.msm_verify(ctx, Xd, P, w.metric, w.eps, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        rows.append({"n": n, "ms_per_step": round(ms, 4), "hamming_pairs": int(mH), "eps_pairs": int(mE),
                     "ms_per_10k_pairs": round(ms / max(mE, 1) * 1e4, 6), "points_per_s": round(n / ms * 1e3, 1)})
        log(rows[-1])
        del Xd, S, pairs, out, P
        torch.cuda.empty_cache()
    # worst case: n identical strings, all n (n - 1) / 2 pairs are output
    n = 20_000
    S = torch.zeros((n, 2), dtype=torch.int64, device=dev)
    _, m = msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, cap=0)
    pairs = torch.empty((m, 2), dtype=torch.int32, device=dev)
    msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        msm.msm_enumerate_pairs(ctx, S, w.ell, w.k, w.h, pairs=pairs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    worst = {"n": n, "pairs": int(m), "expected": n * (n - 1) // 2, "ms": round(ms, 3),
             "pairs_per_s": round(m / ms * 1e3, 1)}
    log(worst)
    ratios = [round(rows[i + 1]["ms_per_step"] / rows[i]["ms_per_step"], 3) for i in range(len(rows) - 1)]
    last = rows[-2]
    out = {"metric": METRIC, "value": last["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": last["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic Gaussian mixture, sigma_mode=radius",
           "config": {"workload": "sweep-mixture-d128-l128-k8-h4-radius", "k": w.k, "h": w.h, "ell": w.ell},
           "sweep": rows, "time_ratio_when_n_doubles": ratios, "all_identical": worst,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sigma-mode", default="coord", choices=["coord", "radius"])
    ap.add_argument("--cpu-sample", type=int, default=0, help="rows for the CPU oracle (0: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-second-reading", action="store_true",
                    help="skip the run under the other reading of sigma")
    ap.add_argument("--epochs", type=int, default=20, help="training epochs of the learned form")
    ap.add_argument("--train-h", type=int, default=0,
                    help="h of the training loss of the learned form (0: twice the workload's h)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES on the device a few times (reference for the HBM counters)")
    ap.add_argument("--workload", default="paper", choices=["paper", "precision", "learned", "batched", "sweep"],
                    help="paper: the 1M mixture (default); precision: 4M sparse rows, FP32/BF16/FP8; "
                         "learned: 2M mixture, trained network vs random projection; "
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
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "learned":
        run_learned(args)
        return
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "sweep":
        run_sweep(args)
        return

    import torch

    from paper_0904_3151_amd import inputs as I
    from paper_0904_3151_amd import msm

    w = I.PAPER_SCALE
    log(f"generating {w.name} ({args.sigma_mode})")
    X, R = I.workload_inputs(w, sigma_mode=args.sigma_mode)
    n, W = w.n, (w.ell + 63) // 64
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Rd = torch.from_numpy(R).to(dev)
    ctx = msm.Context(0)
    res = run_mixture(msm, ctx, w, X, Xd, lambda S: msm.msm_project(ctx, Xd, Rd, S), args.steps, args.warmup)
    roof = roofline_of(res, w, n, W, f"{w.name}:{args.sigma_mode}")
    second = None
    if not args.no_second_reading:
        other = "radius" if args.sigma_mode == "coord" else "coord"
        log(f"generating {w.name} ({other})")
        X2, _ = I.workload_inputs(w, sigma_mode=other)
        X2d = torch.from_numpy(X2).to(dev)
        del X2
        r2 = run_mixture(msm, ctx, w, None, X2d, lambda S: msm.msm_project(ctx, X2d, Rd, S), args.steps,
                         args.warmup)
        second = compact(r2)
        second["sigma_mode"] = other
        second["roofline"] = roofline_of(r2, w, n, W, f"{w.name}:{other}")
        del X2d
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample if 0 < args.cpu_sample < n else n
        log(f"cpu baseline on {sample} points")
        cpu = cpu_baseline(w, X, R, sample)

    c = compact(res)
    out = {
        "metric": METRIC,
        "value": round(res["points_per_s"], 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic Gaussian mixture, sigma_mode={args.sigma_mode}",
        "config": {"workload": w.name, "n": n, "d": w.d, "ell": w.ell, "k": w.k, "h": w.h, "eps": w.eps,
                   "metric": w.metric, "groupings": res["combinations"], "hier_j": res["hier_j"],
                   "sigma_mode": args.sigma_mode,
                   "projection_arith": ("fp32 as three bf16 parts, six products, fp32 accumulation"
                                        if w.ell <= 128 and w.d <= 256 else "fp32 products")},
        "edges_per_s": {"hamming_pairs_per_s_enumerate": c["hamming_pairs_per_s_enumerate"],
                        "eps_pairs_per_s_total": c["eps_pairs_per_s_total"]},
        "counts": {"hamming_pairs": res["hamming_pairs"], "eps_pairs": res["eps_pairs"]},
        "kernels": c["kernels"],
        "missing_edge_ratio": res["missing_edge_ratio"],
        "roofline": roof,
        "second_reading": second,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
