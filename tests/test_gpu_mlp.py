"""Learned projection on the GPU: forward bits, loss and gradients, Adam and
training, checked against the FP64 oracle of oracle/mlp.py.

Bits. The GPU rounds every matrix operand to BF16 (unit roundoff u = 2^-8)
and accumulates in FP32, so a product carries relative error at most
2u + u^2, and a K-term FP32 sum adds at most (K + 2) 2^-24 of the sum of the
magnitudes (bias add included). With A1 = |x| |W1| + |b1|, the first layer
is off by at most e1 = (2u + u^2 + (d + 2) 2^-24) A1; GELU is 1.13-Lipschitz,
and its FP32 evaluation adds at most 2^-20 (|a1| + 1); the second layer then
is off by at most eg |W2| + (2u + u^2 + (hid + 2) 2^-24)((|g| + eg) |W2| +
|b2|). A bit may differ from the FP64 sign only where |a2| is within that.

Gradients. The same rounding reaches the gradient through the loss; its
normwise relative error is a small multiple of 2u. The tests bound it per
parameter block (W1, b1, W2, b2) by 3e-2 and ask for a cosine of at least
0.999, which a transposed operand, a dropped term or a wrong sign fails by
far."""
import math

import numpy as np
import pytest
import torch

from helpers import announce, codes, to_np_pairs, to_np_strings
from oracle import mlp as OM
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu

UB = 2.0 ** -8
U32 = 2.0 ** -24


def bit_error_bound(X, params, d, hid, ell):
    W1, b1, W2, b2 = OM.unpack(params, d, hid, ell)
    x = np.asarray(X, np.float64)
    c = 2 * UB + UB * UB
    a1 = x @ W1 + b1
    e1 = 1.01 * (c + (d + 2) * U32) * (np.abs(x) @ np.abs(W1) + np.abs(b1))
    g = OM.gelu(a1)
    eg = 1.13 * e1 + 2.0 ** -20 * (np.abs(a1) + 1.0)
    return 1.01 * (eg @ np.abs(W2) + (c + (hid + 2) * U32) * ((np.abs(g) + eg) @ np.abs(W2) + np.abs(b2)))


def params_with_biases(d, hid, ell, seed):
    p = I.mlp_initial_parameters(d, hid, ell, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    o1 = d * hid
    p[o1:o1 + hid] = rng.normal(0.0, 0.2, hid)
    o2 = o1 + hid + hid * ell
    p[o2:o2 + ell] = rng.normal(0.0, 0.2, ell)
    return p.astype(np.float32)


def check_bits(msm, ctx, X, params, hid, ell, offset=0):
    n, d = X.shape
    announce("project_mlp", n, d, hid, ell, offset)
    buf = torch.zeros(offset + max(n, 1) * d, dtype=torch.float32, device="cuda")
    Xd = buf[offset: offset + n * d].view(n, d)
    Xd.copy_(torch.from_numpy(X))
    S = msm.msm_project_mlp(ctx, Xd, torch.from_numpy(params).cuda(), hid, ell)
    torch.cuda.synchronize()
    So, a2 = OM.bits(X, params, d, hid, ell)
    Sg = to_np_strings(S)
    bg, bo = I.unpack_bits(Sg, ell), I.unpack_bits(So, ell)
    bad = bg != bo
    allowed = np.abs(a2) <= bit_error_bound(X, params, d, hid, ell)
    assert not (bad & ~allowed).any(), f"{int((bad & ~allowed).sum())} bits differ outside the error bound"
    full = I.unpack_bits(Sg, Sg.shape[1] * 64)
    assert not full[:, ell:].any(), "padding bits must be 0"
    return float(bad.mean()) if bad.size else 0.0


@pytest.mark.parametrize("n,d,hid,ell,off", [
    (3000, 128, 512, 128, 0),   # the learned workload's network shape, fused kernel, vector loads
    (3000, 128, 512, 128, 1),   # same, X not 16-byte aligned
    (700, 33, 100, 60, 0),      # ragged d and hid, one word
    (1029, 200, 96, 100, 0),    # d > 128, seven column blocks
    (513, 128, 64, 130, 0),     # ell > 128: separate GEMMs, three words
    (300, 300, 70, 64, 0),      # d > 256: separate GEMMs
    (5, 7, 3, 1, 0),            # tiny everything
])
def test_project_mlp_bits(msm, ctx, n, d, hid, ell, off):
    X, _ = I.gaussian_mixture(n, d, max(1, n // 50), 0.2, seed=n + d, sigma_mode="coord")
    params = params_with_biases(d, hid, ell, seed=hid + ell)
    flips = check_bits(msm, ctx, X, params, hid, ell, off)
    assert flips < 1e-2


def test_project_mlp_empty_and_invalid(msm, ctx):
    d, hid, ell = 16, 8, 20
    p = torch.from_numpy(params_with_biases(d, hid, ell, 3)).cuda()
    S = msm.msm_project_mlp(ctx, torch.zeros((0, d), device="cuda"), p, hid, ell)
    assert S.shape == (0, 1)
    X = torch.zeros((10, d), device="cuda")
    Sz = torch.empty((10, 1), dtype=torch.int64, device="cuda")
    st = msm.lib().msm_project_mlp(ctx.handle, msm._ptr(X), 10, d, d, msm._ptr(p), hid, 257, msm._ptr(Sz), None)
    assert st == msm.MSM_E_INVALID
    st = msm.lib().msm_project_mlp(ctx.handle, msm._ptr(X), 10, d, d - 1, msm._ptr(p), hid, ell, msm._ptr(Sz), None)
    assert st == msm.MSM_E_INVALID
    st = msm.lib().msm_project_mlp(ctx.handle, None, 10, d, d, msm._ptr(p), hid, ell, msm._ptr(Sz), None)
    assert st == msm.MSM_E_INVALID


def _pair_batch(n, B, seed, same_frac=0.25):
    rng = np.random.default_rng(seed)
    pairs = rng.integers(0, n, (B, 2)).astype(np.uint32)
    same = rng.random(B) < same_frac  # identical points make the non-pair hinge active
    pairs[same, 1] = pairs[same, 0]
    labels = (rng.random(B) < 0.5).astype(np.float32)
    return pairs, labels


def _blocks(v, d, hid, ell):
    o = np.cumsum([0] + OM.sizes(d, hid, ell))
    return [v[o[i]:o[i + 1]] for i in range(4)]


@pytest.mark.parametrize("n,d,hid,ell,B,h,lam", [
    (2000, 32, 64, 40, 300, 8, 0.1),
    (4000, 128, 512, 128, 2048, 16, 0.05),   # the learned workload's shape, split-K weight gradients
    (500, 7, 33, 70, 5, 12, 0.0),            # ragged everything, a tiny batch
])
def test_loss_grad_vs_oracle(msm, ctx, n, d, hid, ell, B, h, lam):
    announce("mlp_loss_grad", n, d, hid, ell, B)
    X, _ = I.gaussian_mixture(n, d, max(1, n // 40), 0.3, seed=n + B, sigma_mode="coord")
    params = params_with_biases(d, hid, ell, seed=d + hid)
    pairs, labels = _pair_batch(n, B, seed=B)
    loss, grad = msm.msm_mlp_loss_grad(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(params).cuda(), hid, ell,
                                       torch.from_numpy(pairs.view(np.int32)).cuda(),
                                       torch.from_numpy(labels).cuda(), h, lam)
    lo, go = OM.loss_and_grad(X, pairs, labels, params, d, hid, ell, h, lam)
    assert abs(loss - lo) <= 2e-2 * abs(lo) + 1e-6, (loss, lo)
    gg = grad.cpu().numpy().astype(np.float64)
    for name, a, b in zip(("W1", "b1", "W2", "b2"), _blocks(gg, d, hid, ell), _blocks(go, d, hid, ell)):
        nb = np.linalg.norm(b)
        if nb == 0:
            assert np.linalg.norm(a) <= 1e-6, name
            continue
        rel = np.linalg.norm(a - b) / nb
        cos = float(a @ b / (np.linalg.norm(a) * nb))
        print(f"[grad] {name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel <= 3e-2 and cos >= 0.999, (name, rel, cos)


def test_loss_grad_rejects_bad_indices(msm, ctx):
    d, hid, ell = 8, 16, 12
    X = torch.randn(100, d, device="cuda")
    p = torch.from_numpy(params_with_biases(d, hid, ell, 5)).cuda()
    pairs = torch.tensor([[0, 1], [5, 100]], dtype=torch.int32, device="cuda")
    labels = torch.ones(2, device="cuda")
    with pytest.raises(msm.MSMError) as e:
        msm.msm_mlp_loss_grad(ctx, X, p, hid, ell, pairs, labels, 2, 0.1)
    assert e.value.status == msm.MSM_E_INVALID
    with pytest.raises(msm.MSMError) as e:
        msm.msm_mlp_loss_grad(ctx, X, p, hid, ell, pairs[:1], labels[:1], -1.0, 0.1)
    assert e.value.status == msm.MSM_E_INVALID


def test_adam_vs_oracle(msm, ctx):
    rng = np.random.default_rng(11)
    n = 100_003
    p, g, m = (rng.normal(0, 1, n) for _ in range(3))
    v = rng.random(n) * 1e-2
    tp, tg, tm, tv = (torch.from_numpy(a.astype(np.float32)).cuda() for a in (p, g, m, v))
    lr = 1e-3
    for step in (1, 7):
        announce("mlp_adam", step)
        p32, g32, m32, v32 = (t.cpu().numpy().astype(np.float64) for t in (tp, tg, tm, tv))
        msm.msm_mlp_adam(ctx, tp, tg, tm, tv, step, lr)
        # the library receives the hyperparameters as FP32; the oracle takes
        # those same values
        f32 = lambda x: float(np.float32(x))  # noqa: E731
        pr, mr, vr = OM.adam(p32, g32, m32, v32, step, f32(lr), f32(0.9), f32(0.999), f32(1e-8))
        np.testing.assert_allclose(tm.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(tv.cpu().numpy(), vr, rtol=1e-6, atol=1e-10)
        # FP32 update: the step lr m^/(sqrt v^ + eps) carries a few units of
        # FP32 rounding relative to itself; params carry one more rounding
        np.testing.assert_allclose(tp.cpu().numpy(), pr, rtol=2e-7, atol=lr * 1e-5)
    with pytest.raises(msm.MSMError):
        msm.msm_mlp_adam(ctx, tp, tg, tm, tv, 0, lr)


def test_train_matches_single_steps_and_lowers_loss(msm, ctx):
    n, d, hid, ell, B, h, lam = 3000, 32, 64, 32, 256, 4, 0.05
    announce("mlp_train", n, d, hid, ell, B)
    X, _ = I.gaussian_mixture(n, d, 30, 0.3, seed=77, sigma_mode="coord")
    Xd = torch.from_numpy(X).cuda()
    p0 = params_with_biases(d, hid, ell, 9)
    pairs, labels = _pair_batch(n, 8 * B, seed=5)
    pt = torch.from_numpy(pairs.view(np.int32)).cuda()
    lt = torch.from_numpy(labels).cuda()
    # two steps through the single-step entry points
    pa = torch.from_numpy(p0).cuda()
    ma, va = torch.zeros_like(pa), torch.zeros_like(pa)
    la = []
    for t in range(2):
        loss, grad = msm.msm_mlp_loss_grad(ctx, Xd, pa, hid, ell, pt[t * B:(t + 1) * B].contiguous(),
                                           lt[t * B:(t + 1) * B].contiguous(), h, lam)
        msm.msm_mlp_adam(ctx, pa, grad, ma, va, t + 1, 1e-3)
        la.append(loss)
    pb = torch.from_numpy(p0).cuda()
    mb, vb = torch.zeros_like(pb), torch.zeros_like(pb)
    lb = msm.msm_mlp_train(ctx, Xd, pb, mb, vb, hid, ell, pt, lt, B, 2, 1, 1e-3, h, lam)
    # same kernels on the same batches; only the order of atomic additions differs
    np.testing.assert_allclose(lb, la, rtol=1e-4)
    np.testing.assert_allclose(mb.cpu().numpy(), ma.cpu().numpy(), rtol=1e-3, atol=1e-6)
    # training continues from step 3 and lowers the loss
    more = msm.msm_mlp_train(ctx, Xd, pb, mb, vb, hid, ell, pt, lt, B, 200, 3, 3e-3, h, lam)
    assert all(math.isfinite(x) for x in more)
    assert np.mean(more[-16:]) < 0.7 * np.mean(lb)


def test_checkpoint_roundtrip(msm, ctx, tmp_path):
    from paper_0904_3151_amd import learned as L
    d, hid, ell = 24, 40, 48
    cfg = L.TrainConfig(hid=hid, ell=ell, h=3, epochs=1)
    p = torch.from_numpy(params_with_biases(d, hid, ell, 21)).cuda()
    m, v = torch.randn_like(p), torch.rand_like(p)
    path = str(tmp_path / "mlp")
    L.save(path, p, m, v, 17, d, cfg)
    p2, m2, v2, step, d2, cfg2 = L.load(path)
    assert step == 17 and d2 == d and cfg2 == cfg
    for a, b in ((p, p2), (m, m2), (v, v2)):
        assert torch.equal(a, b)
    X = torch.randn(500, d, device="cuda")
    assert torch.equal(msm.msm_project_mlp(ctx, X, p, hid, ell), msm.msm_project_mlp(ctx, X, p2, hid, ell))


def _missing(msm, ctx, Xe, S, ell, k, h, eps, truth_codes):
    cand, m_h = msm.enumerate_pairs(ctx, S, ell, k, h)
    kept, m_e = msm.msm_verify(ctx, Xe, cand, "euclidean", eps)
    found = codes(to_np_pairs(kept))
    missing = np.setdiff1d(truth_codes, found).size / max(1, truth_codes.size)
    return missing, m_h, m_e


def test_learned_projection_gain_over_random_lsh(msm, ctx):
    """Trained on pairs mined from one sample of a Gaussian mixture, the
    learned strings miss fewer epsilon-pairs of held-out points from the same
    mixture than random-projection strings of the same length, with MSM at the
    same (ell, k, h), without a blow-up of the Hamming candidates."""
    from paper_0904_3151_amd import learned as L
    d, ell, k, h, eps = 64, 64, 5, 3, 0.5
    X, _ = I.gaussian_mixture(30_000, d, 300, (0.05, 0.3), seed=4242, sigma_mode="radius")
    Xt = torch.from_numpy(X[:10_000]).cuda()
    Xe = torch.from_numpy(np.ascontiguousarray(X[10_000:])).cuda()
    announce("mlp_gain: mining")
    pairs, labels, stats = L.mine_pairs(ctx, Xt, eps, n_pos=60_000, n_neg=60_000, seed=1)
    print("[gain] mined", stats)
    cfg = L.TrainConfig(hid=256, ell=ell, h=h, lam=0.05, lr=2e-3, batch=2048, epochs=12, seed=3)
    announce("mlp_gain: training")
    params, _, _, losses, _ = L.train(ctx, Xt, pairs, labels, cfg, I.mlp_initial_parameters(d, cfg.hid, ell, 8))
    print(f"[gain] loss first {losses[0]:.4f} last {np.mean(losses[-10:]):.4f}")
    announce("mlp_gain: evaluation")
    truth, m_true = msm.bruteforce_eps(ctx, Xe, "euclidean", eps)
    tc = codes(to_np_pairs(truth))
    R = torch.from_numpy(I.projection_matrix(d, ell, seed=99)).cuda()
    miss_r, cand_r, _ = _missing(msm, ctx, Xe, msm.msm_project(ctx, Xe, R), ell, k, h, eps, tc)
    miss_l, cand_l, _ = _missing(msm, ctx, Xe, msm.msm_project_mlp(ctx, Xe, params, cfg.hid, ell), ell, k, h, eps,
                                 tc)
    print(f"[gain] true pairs {m_true}; random: missing {miss_r:.4e}, candidates {cand_r}; "
          f"learned: missing {miss_l:.4e}, candidates {cand_l}")
    assert m_true > 10_000
    assert miss_l <= 0.5 * miss_r
    assert cand_l <= 3 * max(cand_r, m_true)
