"""GPU parity of the pruned alignment (Sec. 4.2: diagonal-UBM top-20
preselection, full-covariance posteriors on the preselected components,
posteriors below 0.025 dropped and the rest renormalised).

The preselection is an integer decision taken from FP32 diagonal scores.
Their error is bounded by the FP32 rounding of a 128-term sum: |dl| <=
2 * 128 * 2^-24 * sum_k |w_ck x~_k| (the term magnitudes, computed here from
the oracle's coefficients).  Frames whose oracle gap between the 20th and
21st diagonal score is within twice that bound, or whose restricted
posteriors come within 1e-5 of the pruning threshold, are ambiguous (they
must be rare); on all other frames the posteriors must match the oracle to
1e-4 absolute (the plain form's bound).  On an ambiguous frame several
results are correct: the GPU's must equal the oracle's pruned posteriors
(1e-4) over some preselection that is a valid top 20 within the FP32 bound
(every component more than 2 eps above the 21st score in it, every one more
than 2 eps below the 20th out, the rest chosen from the band between), with
the pruning decision of a posterior within 1e-5 of the threshold taken
either way.
"""
import itertools
import numpy as np
import pytest
import torch

import oracle
import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu
K, PRUNE = 20, 0.025


def _dense(idx, val, C):
    g = np.zeros((idx.shape[0], C))
    rows = np.repeat(np.arange(idx.shape[0]), idx.shape[1])
    m = idx.ravel() >= 0
    np.add.at(g, (rows[m], idx.ravel()[m]), val.ravel()[m])
    return g


def _term_magnitude(wl):
    """sum_k |w_ck x~_k| of the diagonal quadratic form, per (frame, c)."""
    X = wl.X.astype(np.float64)
    shift = (wl.w[:, None] * wl.mu).sum(0) / wl.w.sum()
    var = np.stack([np.diag(c) for c in wl.cov])
    xs = X - shift
    mus = wl.mu - shift
    D = X.shape[1]
    g = (np.log(wl.w) - 0.5 * D * np.log(2 * np.pi) - 0.5 * np.log(var).sum(1)
         - 0.5 * (mus ** 2 / var).sum(1))
    return (np.abs(g)[None, :] + np.abs(xs) @ np.abs(mus / var).T
            + (xs ** 2) @ (0.5 / var).T)


@pytest.mark.parametrize("shape", [1, 2])
def test_pruned_posteriors_match_the_oracle(shape):
    from paper_1906_08556_amd import ivx
    wl = synth.make(shape, n_utts=40 if shape == 1 else 6)
    C = wl.shape.C
    k = min(K, C)
    ctx = make_ctx(wl)
    ctx.pruned_set(k, PRUNE)
    X = dev(wl.X)
    F = wl.F
    pi = torch.empty((F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((F, 16), dtype=torch.float32, device="cuda")
    fll = torch.empty(F, dtype=torch.float64, device="cuda")
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv, frame_ll=fll, sel=ivx.IVX_SEL_PRUNED)
    ctx.sync_status()
    g_gpu = _dense(pi.cpu().numpy(), pv.cpu().numpy(), C)
    lld = oracle.diag_frame_loglik(wl.X, wl.w, wl.mu, wl.cov)
    order = oracle.preselect(lld, min(k + 1, C))
    idx = order[:, :k]
    g_o, lse_o = oracle.pruned_posteriors(wl.X, wl.w, wl.mu, wl.cov, idx, PRUNE)
    # ambiguity of the preselection and of the pruning decision
    eps = 2 * 128 * 2.0 ** -24 * _term_magnitude(wl).max(axis=1)
    if k < C:
        kth = np.take_along_axis(lld, order[:, k - 1:k], 1)[:, 0]
        nxt = np.take_along_axis(lld, order[:, k:k + 1], 1)[:, 0]
        clear = (kth - nxt) > 2 * eps
    else:
        clear = np.ones(F, bool)
    ll = oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov)
    g_sub, _ = oracle.posteriors(np.take_along_axis(ll, idx, 1))
    near = (np.abs(g_sub - PRUNE) < 1e-5).any(axis=1)
    ok = clear & ~near
    err = np.abs(g_gpu[ok] - g_o[ok]).max()
    lerr = np.abs(fll.cpu().numpy()[ok] - lse_o[ok]).max()
    kept = (g_gpu > 0).sum(1)
    # ambiguous frames: some valid top-k preselection must give the GPU's result
    amb = np.nonzero(~ok)[0]
    n_enum, worst_amb = 0, 0.0
    for t in amb:
        v = lld[t]
        kth = v[order[t, k - 1]]
        nxt = v[order[t, k]] if k < C else -np.inf
        must = np.nonzero(v > nxt + 2 * eps[t])[0]
        band = np.nonzero((v >= kth - 2 * eps[t]) & (v <= nxt + 2 * eps[t]))[0]
        need = k - len(must)
        assert 0 <= need <= len(band)
        # every component the GPU kept lies in a valid preselection
        assert np.isin(np.nonzero(g_gpu[t] > 0)[0], np.concatenate([must, band])).all()
        best = np.inf
        for pick in itertools.islice(itertools.combinations(band, need), 2000):
            sel = np.concatenate([must, np.asarray(pick, dtype=must.dtype)])[None, :]
            for thr in (PRUNE - 1e-5, PRUNE, PRUNE + 1e-5):
                g_alt, _ = oracle.pruned_posteriors(wl.X[t:t + 1], wl.w, wl.mu, wl.cov, sel, thr,
                                                    ll=ll[t:t + 1])
                best = min(best, np.abs(g_gpu[t] - g_alt[0]).max())
            n_enum += 1
        worst_amb = max(worst_amb, best)
    print(f"shape {shape}: frames {F}, compared {ok.sum()}, max |dgamma| {err:.2e}, "
          f"max |dll| {lerr:.2e}, kept per frame mean {kept.mean():.2f} max {kept.max()}; "
          f"ambiguous {len(amb)}: closest valid preselection max |dgamma| {worst_amb:.2e} "
          f"({n_enum} preselections tried)")
    assert worst_amb <= 1e-4
    assert ok.mean() >= 0.95
    assert err <= 1e-4
    assert lerr <= 1e-6
    np.testing.assert_allclose(g_gpu.sum(1), 1.0, atol=1e-5)
    assert (g_gpu[g_gpu > 0] >= PRUNE * (1 - 1e-5)).all()


def test_pruned_statistics_and_extraction_follow_the_lists():
    """n from bw_stats with the pruned alignment equals the per-utterance sums
    of the pruned posterior lists; extraction runs on the same alignment."""
    from paper_1906_08556_amd import ivx
    wl = synth.make(2, n_utts=8)
    C, D, R = wl.shape.C, wl.shape.D, wl.shape.R
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init))
    ctx.pruned_set(K, PRUNE)
    X, off = dev(wl.X), dev(wl.utt_off)
    pi = torch.empty((wl.F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((wl.F, 16), dtype=torch.float32, device="cuda")
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv, sel=ivx.IVX_SEL_PRUNED)
    n = torch.empty((wl.U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((wl.U, C, D), dtype=torch.float32, device="cuda")
    ctx.bw_stats(X, off, n, f, sel=ivx.IVX_SEL_PRUNED)
    phi_p = torch.empty((wl.U, R), dtype=torch.float32, device="cuda")
    phi_a = torch.empty((wl.U, R), dtype=torch.float32, device="cuda")
    ctx.extract_ivectors(X, off, phi_p, sel=ivx.IVX_SEL_PRUNED)
    ctx.extract_ivectors(X, off, phi_a)
    ctx.sync_status()
    g = _dense(pi.cpu().numpy(), pv.cpu().numpy(), C)
    n_ref = np.stack([g[wl.utt_off[u]:wl.utt_off[u + 1]].sum(0) for u in range(wl.U)])
    np.testing.assert_allclose(n.cpu().numpy(), n_ref, rtol=1e-5, atol=1e-5)
    a, b = phi_a.cpu().numpy().astype(np.float64), phi_p.cpu().numpy().astype(np.float64)
    cos = (a * b).sum(1) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
    print(f"i-vector cosine pruned vs all components: min {cos.min():.7f}")
    assert np.isfinite(b).all()


def test_pruned_set_rejects_bad_arguments():
    from paper_1906_08556_amd import ivx
    wl = synth.make(1, n_utts=2)
    ctx = make_ctx(wl)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.pruned_set(0, PRUNE)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.pruned_set(20, 0.6)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.ubm_posteriors(dev(wl.X), sel=ivx.IVX_SEL_PRUNED,
                           post_idx=torch.empty((wl.F, 16), dtype=torch.int32, device="cuda"))
