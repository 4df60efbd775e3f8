"""GPU parity of the learned Gaussian selection: network forward (BF16
MFMA), proposals, fallback decisions, restricted posteriors, training
gradients (FP32) and the Adam step.

Tolerances:
  * Network forward vs the oracle's emulation of the same arithmetic (BF16
    weights and activations, FP32 sums): the two differ only in the order of
    FP32 summation, so hidden activations agree exactly except where a sum
    lands within a few FP32 ulps of a BF16 rounding boundary; then they differ
    by one BF16 ulp (2^-7 relative).  Such flips move a logit by about
    |W3| 2^-7 |h2| ~ 5e-4 each: max |dz| <= 1e-2.
  * Proposals: exactly the top-k of the GPU's own logits (ties to the lower
    index); against the oracle's top-k, identical whenever the oracle's gap
    between the k-th and (k+1)-th logit exceeds twice the frame's logit
    discrepancy, and within that discrepancy otherwise.
  * Restricted posteriors vs the oracle on the frames whose proposals and
    fallback decision are unambiguous: <= 1e-4 abs (the plain form's bound).
  * Training gradients, FP32 on MFMA vs FP64: relative Frobenius <= 1e-4 per
    parameter block (sums over up to 2048 terms), loss relative <= 1e-6; at
    the full network shape, where gradient blocks cancel strongly, the error
    is measured relative to the magnitude of the summed terms (<= 1e-5), on a
    batch without pre-activations within FP32 rounding of a ReLU kink.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu

H1 = H2 = 512
K = 20


def _sparse_from_dense(gamma, kp=16):
    idx = np.argsort(-gamma, axis=1, kind="stable")[:, :kp]
    val = np.take_along_axis(gamma, idx, axis=1)
    idx = np.where(val > 0, idx, -1).astype(np.int32)
    return idx, val.astype(np.float32)


def _dense_from_lists(idx, val, C):
    g = np.zeros((idx.shape[0], C))
    rows = np.repeat(np.arange(idx.shape[0]), idx.shape[1])
    m = idx.ravel() >= 0
    np.add.at(g, (rows[m], idx.ravel()[m]), val.ravel()[m])
    return g


@pytest.fixture(scope="module")
def cfg4():
    wl = synth.make(4, n_utts=6)
    C, D = wl.shape.C, wl.shape.D
    ctx = make_ctx(wl)
    params = synth.mlp_init(D, H1, H2, C, seed=0)
    mean, std = oracle.feature_stats(wl.X)
    mean, std = mean.astype(np.float32), std.astype(np.float32)
    ctx.selector_set(dev(params), dev(mean), dev(std), H1=H1, H2=H2, k=K, min_mass=0.99,
                     max_train_batch=512)
    X = dev(wl.X)
    F = wl.F
    h1 = torch.empty((F, H1), dtype=torch.bfloat16, device="cuda")
    h2 = torch.empty((F, H2), dtype=torch.bfloat16, device="cuda")
    z = torch.empty((F, C), dtype=torch.float32, device="cuda")
    prop = torch.empty((F, K), dtype=torch.int32, device="cuda")
    mass = torch.empty(F, dtype=torch.float32, device="cuda")
    fb = torch.empty(F, dtype=torch.int32, device="cuda")
    ctx.selector_forward(X, h1, h2, z, prop, mass, fb)
    ctx.sync_status()
    gpu = dict(h1=h1.float().cpu().numpy(), h2=h2.float().cpu().numpy(), z=z.cpu().numpy(),
               prop=prop.cpu().numpy(), mass=mass.cpu().numpy(), fb=fb.cpu().numpy())
    pw = synth.mlp_split(params, D, H1, H2, C)
    z_o, h1_o, h2_o = oracle.mlp_forward_bf16(pw, wl.X, mean, std)
    return dict(wl=wl, ctx=ctx, params=params, pw=pw, mean=mean, std=std, X=X, gpu=gpu,
                z_o=z_o, h1_o=h1_o, h2_o=h2_o)


def test_feature_stats_kernel_matches_numpy(cfg4):
    wl, ctx = cfg4["wl"], cfg4["ctx"]
    m, s = ctx.feature_stats(cfg4["X"])
    m_ref, s_ref = oracle.feature_stats(wl.X)
    np.testing.assert_allclose(m.cpu().numpy(), m_ref, rtol=1e-6, atol=1e-6 * s_ref.max())
    np.testing.assert_allclose(s.cpu().numpy(), s_ref, rtol=1e-6)


def test_network_forward_matches_the_bf16_oracle(cfg4):
    g = cfg4["gpu"]
    for name, ref in (("h1", cfg4["h1_o"]), ("h2", cfg4["h2_o"])):
        same = np.mean(g[name] == ref)
        rel = np.abs(g[name] - ref) / np.maximum(np.abs(ref), 1e-30)
        print(f"{name}: exactly equal {same:.5f}, max rel diff {rel[g[name] != ref].max(initial=0):.3e}")
        assert same >= 0.99
    dz = np.abs(g["z"] - cfg4["z_o"])
    print(f"z: max |dz| {dz.max():.3e}, 99.9th pct {np.quantile(dz, 0.999):.3e}, "
          f"|z| max {np.abs(cfg4['z_o']).max():.2f}")
    assert dz.max() <= 1e-2


def test_proposals_are_the_exact_top_k_of_the_logits(cfg4):
    g = cfg4["gpu"]
    z = g["z"]
    ref = np.argsort(-z, axis=1, kind="stable")[:, :K]
    np.testing.assert_array_equal(g["prop"], ref)
    q = np.exp(z.astype(np.float64) - z.max(axis=1, keepdims=True))
    q /= q.sum(axis=1, keepdims=True)
    mass = np.take_along_axis(q, ref, axis=1).sum(axis=1)
    assert np.abs(g["mass"] - mass).max() <= 2e-5
    np.testing.assert_array_equal(g["fb"], (g["mass"] < np.float32(0.99)).astype(np.int32))


def test_proposals_agree_with_the_oracle_within_the_logit_discrepancy(cfg4):
    g, z_o = cfg4["gpu"], cfg4["z_o"]
    delta = np.abs(g["z"] - z_o).max(axis=1)
    order = oracle.topk(z_o, K + 1)
    kth = np.take_along_axis(z_o, order[:, K - 1:K], axis=1)[:, 0]
    nxt = np.take_along_axis(z_o, order[:, K:K + 1], axis=1)[:, 0]
    clear = (kth - nxt) > 2 * delta
    for t in range(z_o.shape[0]):
        if clear[t]:
            assert set(g["prop"][t]) == set(order[t, :K]), t
        else:
            assert np.all(z_o[t, g["prop"][t]] >= kth[t] - 2 * delta[t]), t
    mass_o = oracle.proposed_mass(z_o, order[:, :K])
    bound = np.expm1(2 * delta) + 2e-5
    assert np.all(np.abs(g["mass"] - mass_o) <= bound)
    print(f"frames {len(clear)}, ambiguous top-k {np.sum(~clear)}, "
          f"fallback fraction {g['fb'].mean():.3f}")


@pytest.mark.parametrize("mode", ["none", "half", "all"])
def test_learned_posteriors_match_the_oracle(cfg4, mode):
    """No fallback (min_mass 0), about half the frames falling back (min_mass
    at the median proposal mass) and every frame falling back (min_mass 1)."""
    from paper_1906_08556_amd import ivx
    wl, ctx, g = cfg4["wl"], cfg4["ctx"], cfg4["gpu"]
    C, F = wl.shape.C, wl.F
    min_mass = {"none": 0.0, "half": float(np.median(g["mass"])), "all": 1.0}[mode]
    ctx.selector_set(dev(cfg4["params"]), dev(cfg4["mean"]), dev(cfg4["std"]), H1=H1, H2=H2,
                     k=K, min_mass=min_mass, max_train_batch=512)
    pi = torch.empty((F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((F, 16), dtype=torch.float32, device="cuda")
    fll = torch.empty(F, dtype=torch.float64, device="cuda")
    ctx.ubm_posteriors(cfg4["X"], post_idx=pi, post_val=pv, frame_ll=fll, sel=ivx.IVX_SEL_LEARNED)
    ctx.sync_status()
    nfb, pairs = ctx.selector_counts()
    fb_g = g["mass"] < np.float32(min_mass)
    assert nfb == int(fb_g.sum())
    assert pairs == int((~fb_g).sum()) * K
    gam_g = _dense_from_lists(pi.cpu().numpy(), pv.cpu().numpy(), C)
    z_o = cfg4["z_o"]
    idx_o = oracle.topk(z_o, K)
    mass_o = oracle.proposed_mass(z_o, idx_o)
    gam_o, fb_o, lse_o = oracle.learned_posteriors(wl.X, wl.w, wl.mu, wl.cov, idx_o, mass_o,
                                                   min_mass)
    # frames whose proposals or fallback decision depend on the last BF16 bits
    delta = np.abs(g["z"] - z_o).max(axis=1)
    order = oracle.topk(z_o, K + 1)
    kth = np.take_along_axis(z_o, order[:, K - 1:K], axis=1)[:, 0]
    nxt = np.take_along_axis(z_o, order[:, K:K + 1], axis=1)[:, 0]
    near = np.abs(mass_o - min_mass) <= np.expm1(2 * delta) + 2e-5
    ok = ((kth - nxt) > 2 * delta) & ~near
    print(f"min_mass {min_mass}: fallback {fb_o.mean():.3f}, compared frames {ok.sum()} of {F}")
    assert ok.mean() >= 0.95
    assert np.array_equal(fb_o[ok], fb_g[ok])
    err = np.abs(gam_g[ok] - gam_o[ok]).max()
    lerr = np.abs(fll.cpu().numpy()[ok] - lse_o[ok]).max()
    print(f"  max |dgamma| {err:.2e}, max |dll| {lerr:.2e}")
    assert err <= 1e-4
    assert lerr <= 1e-6


def _train_ctx():
    wl = synth.make(1)
    C, D = wl.shape.C, wl.shape.D
    ctx = make_ctx(wl)
    params = synth.mlp_init(D, 128, 128, C, seed=1)
    mean, std = oracle.feature_stats(wl.X)
    ctx.selector_set(dev(params), dev(mean.astype(np.float32)), dev(std.astype(np.float32)),
                     H1=128, H2=128, k=8, min_mass=0.99, max_train_batch=256)
    gam, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    idx, val = _sparse_from_dense(gam)
    return wl, ctx, params, mean, std, idx, val


def test_training_gradients_match_the_oracle():
    wl, ctx, params, mean, std, idx, val = _train_ctx()
    C, D = wl.shape.C, wl.shape.D
    fidx = synth.sample_frames(wl.F, 256, seed=3)
    grad = torch.empty(ctx.selector_param_count(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.selector_grad(dev(wl.X), dev(fidx), dev(idx), dev(val), grad=grad, loss=loss)
    ctx.sync_status()
    pw = [p.astype(np.float64) for p in synth.mlp_split(params, D, 128, 128, C)]
    Xh = oracle.standardise(wl.X[fidx], mean.astype(np.float32).astype(np.float64),
                            std.astype(np.float32).astype(np.float64))
    z, cache = oracle.mlp_forward(pw, Xh)
    gam = _dense_from_lists(idx[fidx], val[fidx], C)
    l_ref = oracle.ce_loss(z, gam)
    g_ref = oracle.mlp_backward(pw, cache, z, gam)
    g_gpu = synth.mlp_split(grad.cpu().numpy(), D, 128, 128, C)
    print(f"loss gpu {loss.item():.9f} oracle {l_ref:.9f}")
    assert abs(loss.item() - l_ref) <= 1e-6 * abs(l_ref)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), g_gpu, g_ref):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"  d{name}: rel {rel:.2e}")
        assert rel <= 1e-4


def _abs_backward(pw, cache, z, gam):
    """The backward pass with every quantity replaced by its absolute value:
    the scale of the sums each gradient entry is made of (forward error
    bounds of FP32 sums are relative to it)."""
    W1, b1, W2, b2, W3, b3 = [np.abs(p) for p in pw]
    Xh, a1, h1, a2, h2 = cache
    q = oracle.softmax(z)
    dz = (q * gam.sum(1, keepdims=True) + gam) / z.shape[0]
    da2 = (dz @ W3) * (a2 > 0)
    da1 = (da2 @ W2) * (a1 > 0)
    return (da1.T @ np.abs(Xh), da1.sum(0), da2.T @ np.abs(h1), da2.sum(0), dz.T @ np.abs(h2),
            dz.sum(0))


def test_training_gradients_match_the_oracle_at_full_shape():
    """Config-5 network shape.  A pre-activation within FP32 rounding of zero
    can take the other ReLU branch on the GPU; the batch is therefore drawn
    from frames whose hidden pre-activations (oracle, FP64) all lie further
    than 1e-3 from zero, and each gradient block is compared relative to the
    magnitude of its terms (the absolute-value backward pass)."""
    wl = synth.make(4, n_utts=4)
    C, D = wl.shape.C, wl.shape.D
    ctx = make_ctx(wl)
    params = synth.mlp_init(D, H1, H2, C, seed=2)
    mean, std = [a.astype(np.float32) for a in oracle.feature_stats(wl.X)]
    ctx.selector_set(dev(params), dev(mean), dev(std), H1=H1, H2=H2, k=K, min_mass=0.99,
                     max_train_batch=512)
    pw = [p.astype(np.float64) for p in synth.mlp_split(params, D, H1, H2, C)]
    cand = synth.sample_frames(wl.F, 2048, seed=4)
    _, cc = oracle.mlp_forward(pw, oracle.standardise(wl.X[cand], mean.astype(np.float64),
                                                      std.astype(np.float64)))
    clear = (np.abs(cc[1]).min(1) > 1e-3) & (np.abs(cc[3]).min(1) > 1e-3)
    fidx = cand[clear][:512]
    assert len(fidx) == 512
    gam, _ = oracle.posteriors(oracle.frame_loglik(wl.X[fidx], wl.w, wl.mu, wl.cov))
    idx_b, val_b = _sparse_from_dense(gam)
    idx = np.full((wl.F, 16), -1, np.int32)
    val = np.zeros((wl.F, 16), np.float32)
    idx[fidx], val[fidx] = idx_b, val_b
    grad = torch.empty(ctx.selector_param_count(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.selector_grad(dev(wl.X), dev(fidx), dev(idx), dev(val), grad=grad, loss=loss)
    ctx.sync_status()
    Xh = oracle.standardise(wl.X[fidx], mean.astype(np.float64), std.astype(np.float64))
    z, cache = oracle.mlp_forward(pw, Xh)
    gd = _dense_from_lists(idx_b, val_b, C)
    g_ref = oracle.mlp_backward(pw, cache, z, gd)
    g_abs = _abs_backward(pw, cache, z, gd)
    l_ref = oracle.ce_loss(z, gd)
    print(f"loss gpu {loss.item():.9f} oracle {l_ref:.9f}")
    assert abs(loss.item() - l_ref) <= 1e-6 * abs(l_ref)
    worst = 0.0
    for name, a, b, m in zip(("W1", "b1", "W2", "b2", "W3", "b3"),
                             synth.mlp_split(grad.cpu().numpy(), D, H1, H2, C), g_ref, g_abs):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        rel_abs = np.linalg.norm(a - b) / np.linalg.norm(m)
        print(f"  d{name}: rel {rel:.2e}, relative to the term magnitudes {rel_abs:.2e}")
        worst = max(worst, rel_abs)
    assert worst <= 1e-5


def test_adam_step_matches_the_oracle():
    wl, ctx, params, mean, std, idx, val = _train_ctx()
    C, D = wl.shape.C, wl.shape.D
    fidx = synth.sample_frames(wl.F, 256, seed=5)
    X, fi, pi, pv = dev(wl.X), dev(fidx), dev(idx), dev(val)
    grad = torch.empty(ctx.selector_param_count(), dtype=torch.float32, device="cuda")
    ctx.selector_grad(X, fi, pi, pv, grad=grad)
    lr = 1e-3
    ctx.selector_train_step(X, fi, pi, pv, lr)
    new = ctx.selector_get().cpu().numpy().astype(np.float64)
    ctx.sync_status()
    g_gpu = grad.cpu().numpy().astype(np.float64)
    pw = [p.astype(np.float64) for p in synth.mlp_split(params, D, 128, 128, C)]
    Xh = oracle.standardise(wl.X[fidx], mean.astype(np.float32).astype(np.float64),
                            std.astype(np.float32).astype(np.float64))
    z, cache = oracle.mlp_forward(pw, Xh)
    g_ref = np.concatenate([a.ravel() for a in oracle.mlp_backward(
        pw, cache, z, _dense_from_lists(idx[fidx], val[fidx], C))])
    p0 = params.astype(np.float64)
    p_ref, _, _ = oracle.adam_update(p0, g_ref, np.zeros_like(p0), np.zeros_like(p0), 1, lr=lr)
    tol = lr * (1e-5 + 2 * np.abs(g_gpu - g_ref) / (np.abs(g_ref) + 1e-8)) + 1e-7 * np.abs(p0)
    assert np.all(np.abs((new - p0) - (p_ref - p0)) <= tol)


def test_out_of_range_training_frame_is_reported():
    from paper_1906_08556_amd import ivx
    wl, ctx, params, mean, std, idx, val = _train_ctx()
    fidx = np.array([0, 1, wl.F + 5], dtype=np.int64)
    ctx.selector_grad(dev(wl.X), dev(fidx), dev(idx), dev(val))
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.sync_status()



def test_trained_selector_gains_over_the_untrained_one():
    """Trains the selector on the GPU, by the library's own forward and
    backward kernels, on exact all-component posteriors of 500 utterances of
    the shape-6 workload (frames near their components), and evaluates it on
    100 held-out utterances against the untrained network and against the
    plain all-component form: how many frames leave the all-component path,
    how much exact-posterior mass the kept frames' proposals miss, how much
    scoring work remains, and how far the i-vectors move.  Correctness never
    depends on the network (fallback frames are exact, kept frames are exact
    over their proposals); the gain does."""
    from paper_1906_08556_amd import ivx
    wl = synth.make(6, n_utts=600)
    C, D, R = wl.shape.C, wl.shape.D, wl.shape.R
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init))
    X = dev(wl.X)
    F = wl.F
    Utr = 500
    Ftr = int(wl.utt_off[Utr])
    Fe = F - Ftr
    pi = torch.empty((F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((F, 16), dtype=torch.float32, device="cuda")
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv)
    mean, std = ctx.feature_stats(X[:Ftr])
    B = 4096
    ctx.selector_set(dev(synth.mlp_init(D, H1, H2, C, seed=0)), mean, std, H1=H1, H2=H2, k=K,
                     min_mass=0.99, max_train_batch=B)
    Xe, off_e = X[Ftr:], dev(wl.utt_off[Utr:] - wl.utt_off[Utr])
    g_all = _dense_from_lists(pi[Ftr:].cpu().numpy(), pv[Ftr:].cpu().numpy(), C)

    def evaluate():
        mass = torch.empty(Fe, dtype=torch.float32, device="cuda")
        prop = torch.empty((Fe, K), dtype=torch.int32, device="cuda")
        ctx.selector_forward(Xe, prop=prop, mass=mass)
        miss = 1.0 - np.take_along_axis(g_all, prop.cpu().numpy().astype(np.int64), 1).sum(1)
        fb = mass.cpu().numpy() < 0.99
        return fb, miss

    fb0, _ = evaluate()
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    losses = []
    steps = 3000
    for step in range(steps):
        fidx = dev(synth.sample_frames(Ftr, B, seed=step))
        ctx.selector_train_step(X, fidx, pi, pv, 1e-3 if step < 0.7 * steps else 3e-4, loss=loss)
        if step % 500 == 0 or step == steps - 1:
            losses.append(loss.item())
    ctx.sync_status()
    fb1, miss = evaluate()
    ctx.extract_ivectors(Xe, off_e, torch.empty((wl.U - Utr, R), dtype=torch.float32,
                                                device="cuda"), sel=ivx.IVX_SEL_LEARNED)
    nfb, pairs = ctx.selector_counts()
    phi_a = torch.empty((wl.U - Utr, R), dtype=torch.float32, device="cuda")
    phi_l = torch.empty_like(phi_a)
    ctx.extract_ivectors(Xe, off_e, phi_a)
    ctx.extract_ivectors(Xe, off_e, phi_l, sel=ivx.IVX_SEL_LEARNED)
    ctx.sync_status()
    a, b = phi_a.cpu().numpy().astype(np.float64), phi_l.cpu().numpy().astype(np.float64)
    cos = np.sum(a * b, 1) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
    # scoring work per frame relative to all components: network + proposals
    # of kept frames + all components for fallback frames (FLOP counts)
    work = (Fe * 2.683e6 + pairs * 3.7e3 + nfb * 7.746e6) / (Fe * 7.746e6)
    kept = ~fb1
    print(f"losses {['%.3f' % v for v in losses]}")
    print(f"fallback untrained {fb0.mean():.3f} trained {fb1.mean():.3f}; kept-frame missed "
          f"mass mean {miss[kept].mean():.3e}, median {np.median(miss[kept]):.2e}; "
          f"work vs all components {work:.3f}; i-vector cosine min {cos.min():.6f} "
          f"median {np.median(cos):.8f}")
    assert losses[-1] < 0.25 * losses[0]
    assert fb0.mean() >= 0.99
    assert fb1.mean() <= 0.8
    assert work < 1.0
