"""Pins of the oracle's standard formulation (Sec. 2.1: mu_c(u) = m_c + T_c omega,
omega ~ N(0, I)) against brute force and invariants: centring against the
explicit scatter around m_c, the E-step against Gaussian conditioning of the
stacked joint with means m_c, the objective against the stacked marginal, the
minimum-divergence re-parametrisation against the supervector distribution it
must preserve, and monotone EM at fixed statistics."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
import synth


def _tiny(D=3, C=4, R=2, U=3, lo=4, hi=7, seed=0):
    return synth.tiny(D=D, C=C, R=R, U=U, lo=lo, hi=hi, seed=seed)


def _hard_gamma(wl):
    g = np.zeros((wl.F, wl.shape.C))
    g[np.arange(wl.F), wl.comp] = 1.0
    return g


def _random_std(wl, seed=3, scale=0.7):
    g = np.random.default_rng(seed)
    C, D, R = wl.shape.C, wl.shape.D, wl.shape.R
    T = scale * g.standard_normal((C, D, R))
    A = g.standard_normal((C, D + 3, D)) / np.sqrt(D + 3)
    Sigma = np.einsum("cki,ckj->cij", A, A) + 0.1 * np.eye(D)
    m = wl.mu + 0.5 * g.standard_normal((C, D))
    return T, Sigma, m


def test_centring_equals_the_explicit_scatter_around_m():
    wl = _tiny(D=3, C=4, R=2, U=3)
    X = wl.X.astype(np.float64)
    rng = np.random.default_rng(7)
    gamma = rng.dirichlet(np.ones(4), size=wl.F)          # soft alignments
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    _, _, m = _random_std(wl)
    fc, Sc = oracle.center_stats(n, f, S, m)
    for u in range(wl.U):
        for c in range(4):
            acc = np.zeros(3)
            for t in range(int(wl.utt_off[u]), int(wl.utt_off[u + 1])):
                acc += gamma[t, c] * (X[t] - m[c])
            np.testing.assert_allclose(fc[u, c], acc, rtol=1e-12, atol=1e-12)
    for c in range(4):
        ref = np.zeros((3, 3))
        for t in range(wl.F):
            d = X[t] - m[c]
            ref += gamma[t, c] * np.outer(d, d)
        np.testing.assert_allclose(Sc[c], ref, rtol=1e-10, atol=1e-10)


def test_standard_estep_equals_conditioning_of_the_joint_with_means_m():
    wl = _tiny(D=3, C=4, R=2, U=3)
    T, Sigma, m = _random_std(wl)
    X = wl.X.astype(np.float64)
    n, f, S = oracle.bw_stats(X, wl.utt_off, _hard_gamma(wl))
    fc, _ = oracle.center_stats(n, f, S, m)
    e = oracle.estep(n, fc, T, Sigma, np.zeros(wl.shape.R))
    D, R = wl.shape.D, wl.shape.R
    for u in range(wl.U):
        a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
        comps = wl.comp[a:b]
        A = np.concatenate([T[c] for c in comps], axis=0)
        mm = np.concatenate([m[c] for c in comps])
        Sxx = A @ A.T
        for i, c in enumerate(comps):
            Sxx[i * D:(i + 1) * D, i * D:(i + 1) * D] += Sigma[c]
        K = np.linalg.solve(Sxx, A).T
        np.testing.assert_allclose(e["phi"][u], K @ (X[a:b].reshape(-1) - mm), rtol=1e-9,
                                   atol=1e-11)
        np.testing.assert_allclose(e["Phi"][u], np.eye(R) - K @ A, rtol=1e-9, atol=1e-11)


def test_standard_objective_equals_the_stacked_marginal_with_means_m():
    wl = _tiny(D=3, C=4, R=2, U=3)
    T, Sigma, m = _random_std(wl)
    X = wl.X.astype(np.float64)
    n, f, S = oracle.bw_stats(X, wl.utt_off, _hard_gamma(wl))
    fc, Sc = oracle.center_stats(n, f, S, m)
    e = oracle.estep(n, fc, T, Sigma, np.zeros(wl.shape.R))
    acc = oracle.accumulate(n, fc, e["phi"], e["Phi"])
    obj = oracle.objective(acc["N"], Sc, Sigma, e["ll_u"].sum())
    ref = 0.0
    for u in range(wl.U):
        a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
        comps = wl.comp[a:b]
        A = np.concatenate([T[c] for c in comps], axis=0)
        cov = A @ A.T
        for i, c in enumerate(comps):
            cov[i * 3:(i + 1) * 3, i * 3:(i + 1) * 3] += Sigma[c]
        mean = np.concatenate([m[c] for c in comps])
        ref += multivariate_normal.logpdf(X[a:b].reshape(-1), mean, cov)
    assert np.isclose(obj, ref, rtol=1e-11, atol=1e-9)


def test_mindiv_standard_preserves_the_supervector_distribution():
    """With omega ~ N(h, G) under the old model and omega' ~ N(0, I) under the
    new one, the stacked supervector has the same mean and covariance."""
    rng = np.random.default_rng(11)
    C, D, R = 3, 4, 5
    T = rng.standard_normal((C, D, R))
    m = rng.standard_normal((C, D))
    h = rng.standard_normal(R)
    B = rng.standard_normal((R, R + 2))
    G = B @ B.T / (R + 2) + 0.2 * np.eye(R)
    H = G + np.outer(h, h)
    T1, m1 = oracle.mindiv_standard(h, H, T, m, update_mean=True)
    Ts, Ts1 = T.reshape(C * D, R), T1.reshape(C * D, R)
    np.testing.assert_allclose(m1.reshape(-1), m.reshape(-1) + Ts @ h, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Ts1 @ Ts1.T, Ts @ G @ Ts.T, rtol=1e-11, atol=1e-11)
    # the new loading is a triangular re-mix: T1 = T L with L lower-triangular
    L = np.linalg.lstsq(Ts, Ts1, rcond=None)[0]
    np.testing.assert_allclose(np.triu(L, 1), 0.0, atol=1e-10)
    assert np.all(np.diag(L) > 0)
    # samples: m + T (h + L w') == m1 + T1 w'
    for _ in range(3):
        wp = rng.standard_normal(R)
        np.testing.assert_allclose(m + T @ (h + L @ wp), m1 + T1 @ wp, rtol=1e-11, atol=1e-11)


def test_mindiv_standard_at_the_prior_is_the_identity():
    rng = np.random.default_rng(12)
    T = rng.standard_normal((2, 3, 4))
    m = rng.standard_normal((2, 3))
    for method in ("chol", "eig"):
        T1, m1 = oracle.mindiv_standard(np.zeros(4), np.eye(4), T, m, method=method,
                                        update_mean=True)
        np.testing.assert_allclose(np.einsum("cdr,cer->cde", T1, T1),
                                   np.einsum("cdr,cer->cde", T, T), atol=1e-13)
        np.testing.assert_allclose(m1, m, atol=1e-15)
    T1, _ = oracle.mindiv_standard(np.zeros(4), np.eye(4), T, m)
    np.testing.assert_allclose(T1, T, atol=1e-15)


@pytest.mark.parametrize("method", ["chol", "eig"])
def test_mindiv_standard_without_mean_update_whitens_with_G_and_keeps_m(method):
    """The P1-only update (the standard form's re-estimation): the bias is
    kept and the loading covariance becomes T G T^T for either whitening."""
    rng = np.random.default_rng(13)
    C, D, R = 2, 5, 4
    T = rng.standard_normal((C, D, R))
    m = rng.standard_normal((C, D))
    h = rng.standard_normal(R)
    B = rng.standard_normal((R, R + 3))
    G = B @ B.T / (R + 3) + 0.1 * np.eye(R)
    T1, m1 = oracle.mindiv_standard(h, G + np.outer(h, h), T, m, method=method)
    np.testing.assert_array_equal(m1, m)
    Ts, Ts1 = T.reshape(C * D, R), T1.reshape(C * D, R)
    np.testing.assert_allclose(Ts1 @ Ts1.T, Ts @ G @ Ts.T, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("update_sigma,mindiv", [(True, True), (True, False), (False, True),
                                                 (False, False)])
def test_standard_em_is_monotone_at_fixed_statistics(update_sigma, mindiv):
    """Each iteration maximises the EM auxiliary function (in T, Sigma and,
    with minimum divergence and the bias update, the prior's mean and
    covariance), so the objective at fixed alignments cannot decrease.  The
    P1-only update drops h and is not such a step, so it is not asserted."""
    wl = synth.make(1, n_utts=12, D=6, C=8, R=4, U=12, lengths="uniform:20:40")
    X = wl.X.astype(np.float64)
    ubm = (wl.w, wl.mu, wl.cov)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(X, *ubm))
    stats = oracle.bw_stats(X, wl.utt_off, gamma)
    T, Sigma, p, m = oracle.init_tv_standard(wl.mu, wl.cov, 0.3 * wl.T_init)
    objs = []
    for _ in range(6):
        r = oracle.em_iteration_standard(X, wl.utt_off, ubm, (T, Sigma, p, m),
                                         update_sigma=update_sigma, mindiv=mindiv,
                                         update_mean=True, stats=stats)
        objs.append(r["objective"])
        T, Sigma, m = r["T"], r["Sigma"], r["m"]
    d = np.diff(objs)
    assert np.all(d >= -1e-9 * np.abs(objs[0])), objs
    assert objs[-1] > objs[0]


def test_standard_mindiv_whitens_the_posterior_moments_of_a_recentred_model():
    """After m <- m + T h and T <- T L_G, mapping the old posterior moments
    through omega' = L_G^{-1} (omega - h) gives mean 0 and second moment I."""
    wl = synth.make(1, n_utts=10, D=5, C=6, R=3, U=10, lengths="uniform:15:30")
    X = wl.X.astype(np.float64)
    ubm = (wl.w, wl.mu, wl.cov)
    T, Sigma, p, m = oracle.init_tv_standard(wl.mu, wl.cov, 0.4 * wl.T_init)
    r = oracle.em_iteration_standard(X, wl.utt_off, ubm, (T, Sigma, p, m), mindiv=True,
                                     update_mean=True)
    acc = r["acc"]
    h = acc["hsum"] / acc["count"]
    H = acc["Hsum"] / acc["count"]
    Tnew_nomd = oracle.em_iteration_standard(X, wl.utt_off, ubm, (T, Sigma, p, m),
                                             mindiv=False)["T"]
    L = np.linalg.lstsq(Tnew_nomd.reshape(-1, 3), r["T"].reshape(-1, 3), rcond=None)[0]
    phi = r["estep"]["phi"]
    Phi = r["estep"]["Phi"]
    Li = np.linalg.inv(L)
    mp = (phi - h) @ Li.T
    second = np.mean([Li @ (Phi[u] + np.outer(phi[u] - h, phi[u] - h)) @ Li.T
                      for u in range(len(phi))], axis=0)
    np.testing.assert_allclose(mp.mean(axis=0), 0.0, atol=1e-10)
    np.testing.assert_allclose(second, np.eye(3), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(r["m"], m + np.einsum("cdr,r->cd", Tnew_nomd, h), rtol=1e-12,
                               atol=1e-12)
    np.testing.assert_allclose(H - np.outer(h, h), L @ L.T, rtol=1e-9, atol=1e-11)
