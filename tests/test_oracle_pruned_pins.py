"""Pins of the pruned-alignment oracle (diagonal-UBM preselection, Sec. 4.2)."""
import numpy as np
import scipy.stats

import oracle
import synth


def test_diagonal_loglik_matches_scipy_with_diagonal_covariances():
    wl = synth.tiny(D=4, C=5, U=4)
    X = wl.X[:12].astype(np.float64)
    ll = oracle.diag_frame_loglik(X, wl.w, wl.mu, wl.cov)
    for c in range(5):
        ref = np.log(wl.w[c]) + scipy.stats.multivariate_normal.logpdf(
            X, wl.mu[c], np.diag(np.diag(wl.cov[c])))
        np.testing.assert_allclose(ll[:, c], ref, rtol=1e-12, atol=1e-10)


def test_preselection_orders_by_score_then_index():
    ll = np.array([[0.0, 2.0, 2.0, 1.0, 2.0]])
    assert oracle.preselect(ll, 3).tolist() == [[1, 2, 4]]
    rng = np.random.default_rng(0)
    z = rng.integers(0, 3, size=(15, 9)).astype(float)
    for t in range(15):
        ref = sorted(range(9), key=lambda c: (-z[t, c], c))[:4]
        assert oracle.preselect(z[t:t + 1], 4)[0].tolist() == ref


def test_no_pruning_and_all_components_gives_the_full_posteriors():
    wl = synth.tiny(C=6, U=10)
    X = wl.X
    idx = oracle.preselect(oracle.diag_frame_loglik(X, wl.w, wl.mu, wl.cov), 6)
    g, lse = oracle.pruned_posteriors(X, wl.w, wl.mu, wl.cov, idx, prune=0.0)
    ref, ref_lse = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    np.testing.assert_allclose(g, ref, atol=1e-14)
    np.testing.assert_allclose(lse, ref_lse, rtol=1e-13)


def test_pruning_drops_small_posteriors_and_renormalises():
    """Hand-built case: a frame whose restricted posteriors are (0.9, 0.08,
    0.015, 0.005) keeps 0.9 and 0.08, renormalised to 0.9/0.98, 0.08/0.98."""
    D = 1
    w = np.array([0.25, 0.25, 0.25, 0.25])
    cov = np.ones((4, 1, 1))
    target = np.array([0.9, 0.08, 0.015, 0.005])
    # equal weights and variances: posteriors ~ exp(-(x - mu_c)^2 / 2); with
    # x = 0 choose mu_c = sqrt(-2 log p_c + const)
    mu = np.sqrt(-2.0 * np.log(target / target.max()))[:, None]
    X = np.zeros((1, D))
    idx = np.array([[0, 1, 2, 3]])
    g, _ = oracle.pruned_posteriors(X, w, mu, cov, idx, prune=0.025)
    np.testing.assert_allclose(g[0], [0.9 / 0.98, 0.08 / 0.98, 0.0, 0.0], rtol=1e-12)


def test_pruned_posteriors_sum_to_one_and_respect_the_threshold():
    wl = synth.tiny(C=8, U=20)
    X = wl.X
    idx = oracle.preselect(oracle.diag_frame_loglik(X, wl.w, wl.mu, wl.cov), 3)
    g, _ = oracle.pruned_posteriors(X, wl.w, wl.mu, wl.cov, idx, prune=0.025)
    np.testing.assert_allclose(g.sum(axis=1), 1.0, atol=1e-12)
    nz = g[g > 0]
    assert nz.min() >= 0.025
    # only preselected components carry mass
    mask = np.zeros_like(g, dtype=bool)
    np.put_along_axis(mask, idx, True, axis=1)
    assert np.all(g[~mask] == 0)
