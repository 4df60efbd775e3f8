"""Pins of the back-end oracle (whitening, length normalisation, class
scatter, LDA, two-covariance PLDA scores, EER) against closed forms,
brute force and invariants that hold whatever the implementation."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import backend as be


def _classes(K=6, per=9, R=5, seed=0, spread=2.0):
    rng = np.random.default_rng(seed)
    centres = spread * rng.standard_normal((K, R))
    A = rng.standard_normal((R, R)) / np.sqrt(R)
    X = np.concatenate([centres[k] + rng.standard_normal((per, R)) @ A for k in range(K)])
    return X, np.repeat(np.arange(K), per)


def test_whitening_gives_identity_covariance():
    X, _ = _classes()
    mu, W = be.whitening(X)
    Y = (X - mu) @ W.T
    np.testing.assert_allclose(Y.T @ Y / len(Y), np.eye(X.shape[1]), atol=1e-10)


def test_length_norm_keeps_direction_and_unit_length():
    X, _ = _classes()
    mu = X.mean(0)
    Y = be.center_lnorm(X, mu)
    np.testing.assert_allclose(np.linalg.norm(Y, axis=1), 1.0, atol=1e-13)
    cos = np.sum(Y * (X - mu), 1) / np.linalg.norm(X - mu, axis=1)
    np.testing.assert_allclose(cos, 1.0, atol=1e-13)


def test_scatter_explicit_loops_and_total_covariance():
    X, lab = _classes(K=4, per=5, R=3)
    m, Sw, Sb = be.class_scatter(X, lab)
    N, R = X.shape
    Sw_ref = np.zeros((R, R))
    Sb_ref = np.zeros((R, R))
    for k in range(4):
        idx = [i for i in range(N) if lab[i] == k]
        mk = sum(X[i] for i in idx) / len(idx)
        for i in idx:
            Sw_ref += np.outer(X[i] - mk, X[i] - mk)
        Sb_ref += len(idx) * np.outer(mk - m, mk - m)
    np.testing.assert_allclose(Sw, Sw_ref / N, atol=1e-12)
    np.testing.assert_allclose(Sb, Sb_ref / N, atol=1e-12)
    # law of total covariance: Sw + Sb = total scatter
    Xc = X - X.mean(0)
    np.testing.assert_allclose(Sw + Sb, Xc.T @ Xc / N, atol=1e-12)


def test_lda_two_classes_is_fishers_direction():
    X, lab = _classes(K=2, per=40, R=4, seed=3)
    V, lam = be.lda(X, lab, 1)
    _, Sw, _ = be.class_scatter(X, lab)
    m0, m1 = X[lab == 0].mean(0), X[lab == 1].mean(0)
    fisher = np.linalg.solve(Sw, m1 - m0)
    cos = abs(V[:, 0] @ fisher) / (np.linalg.norm(V[:, 0]) * np.linalg.norm(fisher))
    assert cos > 1 - 1e-12


def test_lda_columns_are_sw_orthonormal_and_maximise_the_fisher_ratio():
    X, lab = _classes(K=7, per=12, R=6, seed=4)
    V, lam = be.lda(X, lab, 3)
    _, Sw, Sb = be.class_scatter(X, lab)
    np.testing.assert_allclose(V.T @ Sw @ V, np.eye(3), atol=1e-10)
    np.testing.assert_allclose(np.diag(V.T @ Sb @ V), lam, atol=1e-10)
    assert np.all(np.diff(lam) <= 0)
    rng = np.random.default_rng(9)
    dirs = rng.standard_normal((5000, 6))
    ratio = np.einsum("ij,jk,ik->i", dirs, Sb, dirs) / np.einsum("ij,jk,ik->i", dirs, Sw, dirs)
    assert ratio.max() <= lam[0] * (1 + 1e-12)


def test_plda_llr_one_dimension_by_quadrature():
    """p(y1, y2 | same) = int N(y1; mu+s, W) N(y2; mu+s, W) N(s; 0, B) ds."""
    mu, B, W = 0.3, 1.7, 0.6
    s = np.linspace(-30, 30, 600001)
    ds = s[1] - s[0]
    for y1, y2 in [(0.1, 0.4), (2.0, -1.5), (-3.0, -2.5)]:
        same = np.sum(norm.pdf(y1, mu + s, np.sqrt(W)) * norm.pdf(y2, mu + s, np.sqrt(W))
                      * norm.pdf(s, 0, np.sqrt(B))) * ds
        diff = norm.pdf(y1, mu, np.sqrt(B + W)) * norm.pdf(y2, mu, np.sqrt(B + W))
        llr = be.plda_llr([[y1]], [[y2]], np.array([mu]), np.array([[B]]), np.array([[W]]))[0]
        assert np.isclose(llr, np.log(same / diff), rtol=1e-9, atol=1e-9)


def test_plda_llr_symmetry_no_speaker_variability_and_mean_identity():
    rng = np.random.default_rng(2)
    d = 3
    A = rng.standard_normal((d, d))
    B = A @ A.T / d + 0.2 * np.eye(d)
    C = rng.standard_normal((d, d))
    W = C @ C.T / d + 0.3 * np.eye(d)
    mu = rng.standard_normal(d)
    y1, y2 = rng.standard_normal((5, d)), rng.standard_normal((5, d))
    np.testing.assert_allclose(be.plda_llr(y1, y2, mu, B, W), be.plda_llr(y2, y1, mu, B, W),
                               atol=1e-12)
    np.testing.assert_allclose(be.plda_llr(y1, y2, mu, 1e-12 * np.eye(d), W), 0.0, atol=1e-9)
    # E_same[exp(-llr)] = E_same[p_diff / p_same] = 1 (Monte Carlo)
    n = 200000
    L = np.linalg.cholesky(B)
    Lw = np.linalg.cholesky(W)
    spk = rng.standard_normal((n, d)) @ L.T
    a = mu + spk + rng.standard_normal((n, d)) @ Lw.T
    b = mu + spk + rng.standard_normal((n, d)) @ Lw.T
    r = np.exp(-be.plda_llr(a, b, mu, B, W))
    assert abs(r.mean() - 1.0) < 5 * r.std() / np.sqrt(n)


def _eer_bruteforce(s, t):
    """Operating points by direct counting at every candidate threshold, then
    the crossing of the straight segments between consecutive points."""
    ths = sorted(set(s)) + [float("inf")]
    nt, nn = sum(t), len(t) - sum(t)
    pts = [(sum(1 for x, y in zip(s, t) if y and x < th) / nt,
            sum(1 for x, y in zip(s, t) if not y and x >= th) / nn) for th in ths]
    for (a, b), (c, d) in zip(pts, pts[1:]):
        if a <= b and c >= d:
            return a + (b - a) / ((b - a) - (d - c)) * (c - a) if (b - a) != (d - c) else a
    raise AssertionError


def test_eer_bruteforce_and_special_cases():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = int(rng.integers(4, 30))
        s = np.round(rng.standard_normal(n), 1)              # ties included
        t = rng.random(n) < 0.4
        if t.all() or not t.any():
            continue
        assert abs(be.eer(s, t) - _eer_bruteforce(list(s), list(t))) < 1e-12
    assert be.eer([3, 4, 5, 0, 1, 2], [1, 1, 1, 0, 0, 0]) == 0.0       # separable
    assert be.eer([0, 1, 2, 3, 4, 5], [1, 1, 1, 0, 0, 0]) == 1.0       # reversed
    assert be.eer([1, 1, 1, 1], [1, 0, 1, 0]) == 0.5                   # a constant score
    n = 100000
    d = 1.5
    s = np.concatenate([d + rng.standard_normal(n), rng.standard_normal(n)])
    t = np.concatenate([np.ones(n, bool), np.zeros(n, bool)])
    assert abs(be.eer(s, t) - norm.cdf(-d / 2)) < 0.005
