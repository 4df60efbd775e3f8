"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test checks one oracle function against an independent route to the
same quantity: brute-force Gaussian densities, Gaussian conditioning of the
joint (latent vector, frames), brute-force marginal likelihoods of the
stacked frames, 1-D quadrature over the latent variable, finite differences
of the EM auxiliary function, explicit loops, and the invariants that the
paper states for minimum-divergence re-estimation (Sec. 3.1).
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
import synth


def _tiny(D=3, C=4, R=2, U=3, lo=4, hi=7, seed=0):
    return synth.tiny(D=D, C=C, R=R, U=U, lo=lo, hi=hi, seed=seed)


def _hard_stats(wl):
    """One-hot alignments from the generating components."""
    F = wl.F
    C = wl.shape.C
    gamma = np.zeros((F, C))
    gamma[np.arange(F), wl.comp] = 1.0
    return gamma


def _random_tv(wl, seed=1, scale=0.7):
    g = np.random.default_rng(seed)
    C, D, R = wl.shape.C, wl.shape.D, wl.shape.R
    T = scale * g.standard_normal((C, D, R))
    A = g.standard_normal((C, D + 3, D)) / np.sqrt(D + 3)
    Sigma = np.einsum("cki,ckj->cij", A, A) + 0.1 * np.eye(D)
    p = np.zeros(R)
    p[0] = 1.5
    p[1:] = 0.3 * g.standard_normal(R - 1)
    return T, Sigma, p


def _stacked_marginal(X, comps, T, Sigma, prior_mean, prior_cov):
    """log N(vec x; A m, A P A^T + blockdiag Sigma) for frames x_t aligned to comps."""
    A = np.concatenate([T[c] for c in comps], axis=0)
    D = T.shape[1]
    n = len(comps)
    cov = A @ prior_cov @ A.T
    for i, c in enumerate(comps):
        cov[i * D:(i + 1) * D, i * D:(i + 1) * D] += Sigma[c]
    return multivariate_normal.logpdf(np.asarray(X, np.float64).reshape(-1), A @ prior_mean, cov)


# ---------------------------------------------------------------- O2 / O3
def test_frame_loglik_matches_bruteforce_density():
    wl = _tiny(D=3, C=4)
    X = wl.X.astype(np.float64)
    ll = oracle.frame_loglik(X, wl.w, wl.mu, wl.cov)
    D = X.shape[1]
    for c in range(wl.shape.C):
        Pinv = np.linalg.inv(wl.cov[c])
        det = np.linalg.det(wl.cov[c])
        for t in range(X.shape[0]):
            d = X[t] - wl.mu[c]
            dens = (2 * np.pi) ** (-D / 2) * det ** -0.5 * np.exp(-0.5 * d @ Pinv @ d)
            assert np.isclose(ll[t, c], np.log(wl.w[c] * dens), rtol=0, atol=1e-10)


def test_frame_loglik_matches_scipy_at_config1_shape():
    wl = synth.make(1, n_utts=2)
    X = wl.X[:50].astype(np.float64)
    ll = oracle.frame_loglik(X, wl.w, wl.mu, wl.cov)
    for c in range(0, wl.shape.C, 7):
        ref = np.log(wl.w[c]) + multivariate_normal.logpdf(X, wl.mu[c], wl.cov[c])
        np.testing.assert_allclose(ll[:, c], ref, rtol=1e-11, atol=1e-9)


def test_posteriors_normalised_and_match_linear_space():
    wl = _tiny(D=2, C=5)
    X = wl.X.astype(np.float64)
    ll = oracle.frame_loglik(X, wl.w, wl.mu, wl.cov)
    gamma, lse = oracle.posteriors(ll)
    np.testing.assert_allclose(gamma.sum(axis=1), 1.0, atol=1e-14)
    # linear-space brute force (values are moderate at D=2)
    dens = np.stack([wl.w[c] * multivariate_normal.pdf(X, wl.mu[c], wl.cov[c])
                     for c in range(wl.shape.C)], axis=1)
    np.testing.assert_allclose(gamma, dens / dens.sum(axis=1, keepdims=True), atol=1e-12)
    np.testing.assert_allclose(lse, np.log(dens.sum(axis=1)), atol=1e-10)


def test_single_component_posterior_is_one():
    wl = _tiny(D=3, C=1)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    np.testing.assert_array_equal(gamma, 1.0)


# ---------------------------------------------------------------- O4
def test_bw_stats_explicit_loops():
    wl = _tiny(D=3, C=4, U=3)
    X = wl.X.astype(np.float64)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    U, C, D = wl.U, wl.shape.C, wl.shape.D
    for u in range(U):
        for c in range(C):
            nn, ff = 0.0, np.zeros(D)
            for t in range(int(wl.utt_off[u]), int(wl.utt_off[u + 1])):
                nn += gamma[t, c]
                ff += gamma[t, c] * X[t]
            assert np.isclose(n[u, c], nn, atol=1e-13)
            np.testing.assert_allclose(f[u, c], ff, atol=1e-12)
        assert np.isclose(n[u].sum(), wl.utt_off[u + 1] - wl.utt_off[u])
    for c in range(C):
        SS = np.zeros((D, D))
        for t in range(X.shape[0]):
            for i in range(D):
                for j in range(D):
                    SS[i, j] += gamma[t, c] * X[t, i] * X[t, j]
        np.testing.assert_allclose(S[c], SS, atol=1e-11)
        assert np.all(np.linalg.eigvalsh(S[c]) > -1e-10)


# ---------------------------------------------------------------- O1
def test_init_tv_follows_augmented_initialisation():
    wl = _tiny(D=3, C=4, R=3)
    T, Sigma, p = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    assert p[0] == 100.0 and np.all(p[1:] == 0)
    np.testing.assert_array_equal(T[:, :, 0], wl.mu / 100.0)
    np.testing.assert_array_equal(T[:, :, 1:], wl.T_init[:, :, 1:])
    np.testing.assert_array_equal(Sigma, wl.cov)
    # realigning with the initial model reproduces the UBM means (a no-op)
    np.testing.assert_allclose(oracle.realign_means(T, p), wl.mu, rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------- O5 / O6
def test_estep_equals_gaussian_conditioning_of_the_joint():
    wl = _tiny(D=3, C=4, R=2, U=3)
    T, Sigma, p = _random_tv(wl)
    gamma = _hard_stats(wl)
    X = wl.X.astype(np.float64)
    n, f, _ = oracle.bw_stats(X, wl.utt_off, gamma)
    e = oracle.estep(n, f, T, Sigma, p)
    R, D = wl.shape.R, wl.shape.D
    for u in range(wl.U):
        a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
        comps = wl.comp[a:b]
        A = np.concatenate([T[c] for c in comps], axis=0)
        Sxx = A @ A.T
        for i, c in enumerate(comps):
            Sxx[i * D:(i + 1) * D, i * D:(i + 1) * D] += Sigma[c]
        x = X[a:b].reshape(-1)
        K = np.linalg.solve(Sxx, A).T       # Cov(w, x) Sxx^{-1}
        mean = p + K @ (x - A @ p)
        cov = np.eye(R) - K @ A
        np.testing.assert_allclose(e["phi"][u], mean, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(e["Phi"][u], cov, rtol=1e-9, atol=1e-11)


def test_estep_phi_is_the_closed_form_linear_solve():
    wl = synth.make(1, n_utts=6)
    T, Sigma, p = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    n, f, _ = oracle.bw_stats(wl.X, wl.utt_off, gamma, second_order=False)
    e = oracle.estep(n, f, T, Sigma, p)
    for u in range(wl.U):
        np.testing.assert_allclose(np.linalg.solve(e["L"][u], e["b"][u]), e["phi"][u], rtol=1e-8)
        np.testing.assert_allclose(np.linalg.inv(e["L"][u]), e["Phi"][u], rtol=1e-7, atol=1e-12)


def test_estep_without_data_returns_the_prior():
    wl = _tiny(D=3, C=4, R=3)
    T, Sigma, p = _random_tv(wl)
    n = np.zeros((2, 4))
    f = np.zeros((2, 4, 3))
    e = oracle.estep(n, f, T, Sigma, p)
    np.testing.assert_allclose(e["phi"], np.tile(p, (2, 1)), atol=1e-15)
    np.testing.assert_allclose(e["Phi"], np.tile(np.eye(3), (2, 1, 1)), atol=1e-15)
    np.testing.assert_allclose(e["ll_u"], 0.0, atol=1e-13)


# ---------------------------------------------------------------- O7
def test_objective_equals_bruteforce_marginal_hard_alignments():
    wl = _tiny(D=3, C=4, R=2, U=3)
    T, Sigma, p = _random_tv(wl)
    gamma = _hard_stats(wl)
    X = wl.X.astype(np.float64)
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    e = oracle.estep(n, f, T, Sigma, p)
    acc = oracle.accumulate(n, f, e["phi"], e["Phi"])
    obj = oracle.objective(acc["N"], S, Sigma, e["ll_u"].sum())
    ref = 0.0
    for u in range(wl.U):
        a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
        ref += _stacked_marginal(X[a:b], wl.comp[a:b], T, Sigma, p, np.eye(wl.shape.R))
    assert np.isclose(obj, ref, rtol=1e-11, atol=1e-9)


def test_objective_soft_alignments_matches_quadrature_R1():
    wl = _tiny(D=2, C=3, R=1, U=2, lo=3, hi=5)
    X = wl.X.astype(np.float64)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    T, Sigma, p = _random_tv(wl, scale=0.5)
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    e = oracle.estep(n, f, T, Sigma, p)
    acc = oracle.accumulate(n, f, e["phi"], e["Phi"])
    obj = oracle.objective(acc["N"], S, Sigma, e["ll_u"].sum())
    grid = np.linspace(-40, 40, 400001)
    dw = grid[1] - grid[0]
    ref = 0.0
    for u in range(wl.U):
        a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
        lg = -0.5 * np.log(2 * np.pi) - 0.5 * (grid - p[0]) ** 2
        for t in range(a, b):
            for c in range(3):
                mean = T[c][:, 0][None, :] * grid[:, None]
                lg += gamma[t, c] * multivariate_normal.logpdf(X[t] - mean, np.zeros(2), Sigma[c])
        m = lg.max()
        ref += m + np.log(np.exp(lg - m).sum() * dw)
    assert np.isclose(obj, ref, rtol=1e-9, atol=1e-7)


def test_accumulate_explicit_loops():
    g = np.random.default_rng(3)
    U, C, D, R = 3, 2, 2, 3
    n = g.random((U, C))
    f = g.standard_normal((U, C, D))
    phi = g.standard_normal((U, R))
    M = g.standard_normal((U, R, R))
    Phi = np.einsum("uij,ukj->uik", M, M)
    acc = oracle.accumulate(n, f, phi, Phi)
    for c in range(C):
        A = np.zeros((R, R))
        Cc = np.zeros((D, R))
        for u in range(U):
            for i in range(R):
                for j in range(R):
                    A[i, j] += n[u, c] * (Phi[u, i, j] + phi[u, i] * phi[u, j])
            for d in range(D):
                for r in range(R):
                    Cc[d, r] += f[u, c, d] * phi[u, r]
        np.testing.assert_allclose(acc["A"][c], A, atol=1e-13)
        np.testing.assert_allclose(acc["Cc"][c], Cc, atol=1e-13)
        assert np.isclose(acc["N"][c], sum(n[u, c] for u in range(U)))
    np.testing.assert_allclose(acc["hsum"], sum(phi[u] for u in range(U)))
    np.testing.assert_allclose(acc["Hsum"], sum(Phi[u] + np.outer(phi[u], phi[u]) for u in range(U)))


# ---------------------------------------------------------------- O8
def _Q(T, Sigma, acc, S):
    """EM auxiliary function (T, Sigma part) from the expected sufficient statistics."""
    q = 0.0
    for c in range(T.shape[0]):
        Tc, Cc, A = T[c], acc["Cc"][c], acc["A"][c]
        M = S[c] - Cc @ Tc.T - Tc @ Cc.T + Tc @ A @ Tc.T
        sign, logdet = np.linalg.slogdet(Sigma[c])
        q += -0.5 * acc["N"][c] * logdet - 0.5 * np.trace(np.linalg.solve(Sigma[c], M))
    return q


def test_mstep_is_a_stationary_point_of_the_em_auxiliary_function():
    wl = _tiny(D=3, C=4, R=2, U=4, lo=15, hi=25)
    X = wl.X.astype(np.float64)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    T, Sigma, p = _random_tv(wl)
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    e = oracle.estep(n, f, T, Sigma, p)
    acc = oracle.accumulate(n, f, e["phi"], e["Phi"])
    T1, S1, info = oracle.mstep(acc, S, T, Sigma, update_sigma=True, min_count=0.0)
    assert not info["notpd"]
    eps = 1e-6
    for c in range(4):
        for (i, j) in [(0, 0), (1, 1), (2, 0)]:
            Tp, Tm = T1.copy(), T1.copy()
            Tp[c, i, j] += eps
            Tm[c, i, j] -= eps
            grad = (_Q(Tp, S1, acc, S) - _Q(Tm, S1, acc, S)) / (2 * eps)
            assert abs(grad) < 1e-5 * max(1.0, acc["N"][c])
        for (i, j) in [(0, 0), (1, 0), (2, 1)]:
            Sp, Sm = S1.copy(), S1.copy()
            Sp[c, i, j] += eps
            Sp[c, j, i] = Sp[c, i, j]
            Sm[c, i, j] -= eps
            Sm[c, j, i] = Sm[c, i, j]
            grad = (_Q(T1, Sp, acc, S) - _Q(T1, Sm, acc, S)) / (2 * eps)
            assert abs(grad) < 1e-4 * max(1.0, acc["N"][c])
    # the two algebraic forms of the residual-covariance update agree
    for c in range(4):
        Tc, Cc, A = T1[c], acc["Cc"][c], acc["A"][c]
        long_form = (S[c] - Cc @ Tc.T - Tc @ Cc.T + Tc @ A @ Tc.T) / acc["N"][c]
        np.testing.assert_allclose(S1[c], 0.5 * (long_form + long_form.T), rtol=1e-9, atol=1e-10)


def test_mstep_skips_components_without_data():
    wl = _tiny(D=3, C=4, R=2)
    T, Sigma, p = _random_tv(wl)
    acc = dict(N=np.array([0.4, 2.0, 0.0, 3.0]), A=np.tile(2 * np.eye(2), (4, 1, 1)),
               Cc=np.ones((4, 3, 2)))
    S = np.tile(10 * np.eye(3), (4, 1, 1))
    T1, S1, info = oracle.mstep(acc, S, T, Sigma)
    assert info["skipped"] == [0, 2]
    np.testing.assert_array_equal(T1[0], T[0])
    np.testing.assert_array_equal(S1[2], Sigma[2])


@pytest.mark.parametrize("update_sigma,md", [(True, "chol"), (False, "chol"), (True, None),
                                             (True, "eig")])
def test_em_objective_never_decreases(update_sigma, md):
    wl = synth.make(1, D=6, C=8, R=5, U=25, lengths="uniform:20:40")
    ubm = (wl.w, wl.mu, wl.cov)
    X = wl.X.astype(np.float64)
    gamma, lse = oracle.posteriors(oracle.frame_loglik(X, *ubm))
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    tv = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    objs = []
    for _ in range(6):
        r = oracle.em_iteration(X, wl.utt_off, ubm, tv, update_sigma=update_sigma,
                                mindiv_method=md, realign=False, stats=(n, f, S, gamma, lse))
        objs.append(r["objective"])
        tv = (r["T"], r["Sigma"], r["p"])
    d = np.diff(objs)
    assert np.all(d >= -1e-8 * np.abs(objs[1:])), objs
    assert objs[-1] > objs[0]


# ---------------------------------------------------------------- O9
def _em_stats(seed=0):
    wl = _tiny(D=3, C=4, R=3, U=5, lo=6, hi=10, seed=seed)
    X = wl.X.astype(np.float64)
    gamma = _hard_stats(wl)
    T, Sigma, p = _random_tv(wl)
    n, f, S = oracle.bw_stats(X, wl.utt_off, gamma)
    e = oracle.estep(n, f, T, Sigma, p)
    acc = oracle.accumulate(n, f, e["phi"], e["Phi"])
    return wl, X, T, Sigma, p, acc, S


@pytest.mark.parametrize("method", ["chol", "eig"])
def test_mindiv_transform_invariants(method):
    wl, X, T, Sigma, p, acc, S = _em_stats()
    h = acc["hsum"] / acc["count"]
    H = acc["Hsum"] / acc["count"]
    T1, p1, aux = oracle.mindiv(h, H, T, method=method)
    R = len(h)
    P1, P2, G = aux["P1"], aux["P2"], aux["G"]
    np.testing.assert_allclose(P1 @ G @ P1.T, np.eye(R), atol=1e-10)          # whitening
    np.testing.assert_allclose(P2, P2.T, atol=1e-15)                          # symmetric
    np.testing.assert_allclose(P2 @ P2, np.eye(R), atol=1e-13)                # involution
    g = P1 @ h
    np.testing.assert_allclose(P2 @ g, np.linalg.norm(g) * np.eye(R)[0], atol=1e-12)  # eq. (9)
    np.testing.assert_allclose(p1, np.linalg.norm(g) * np.eye(R)[0], atol=1e-12)     # eq. (12)
    # transformed accumulators: centred second moment is I, uncentred is I + p p^T
    M = P2 @ P1
    np.testing.assert_allclose(M @ G @ M.T, np.eye(R), atol=1e-10)
    np.testing.assert_allclose(M @ H @ M.T, np.eye(R) + np.outer(p1, p1), atol=1e-9)
    if method == "chol":
        np.testing.assert_allclose(aux["P1inv"] @ aux["P1"], np.eye(R), atol=1e-12)


def test_mindiv_reparameterisation_preserves_the_marginal_likelihood():
    """T' = T P1^{-1} P2^{-1} with prior N(p', I) describes the same data
    distribution as T with the re-estimated prior N(h, G)."""
    wl, X, T, Sigma, p, acc, S = _em_stats(seed=2)
    h = acc["hsum"] / acc["count"]
    H = acc["Hsum"] / acc["count"]
    G = H - np.outer(h, h)
    for method in ["chol", "eig"]:
        T1, p1, _ = oracle.mindiv(h, H, T, method=method)
        for u in range(wl.U):
            a, b = int(wl.utt_off[u]), int(wl.utt_off[u + 1])
            comps = wl.comp[a:b]
            l0 = _stacked_marginal(X[a:b], comps, T, Sigma, h, G)
            l1 = _stacked_marginal(X[a:b], comps, T1, Sigma, p1, np.eye(len(h)))
            assert np.isclose(l0, l1, rtol=1e-11, atol=1e-9)


def test_mindiv_identity_reflection_when_mean_is_on_e1():
    R = 4
    h = np.array([3.0, 0, 0, 0])
    H = np.eye(R) * 2 + np.outer(h, h)
    T = np.random.default_rng(0).standard_normal((2, 3, R))
    T1, p1, aux = oracle.mindiv(h, H, T)
    np.testing.assert_array_equal(aux["P2"], np.eye(R))
    np.testing.assert_allclose(p1, [3 / np.sqrt(2), 0, 0, 0], atol=1e-14)


# ---------------------------------------------------------------- O10 / O11
def test_extract_equals_estep_mean():
    wl = synth.make(1, n_utts=5)
    T, Sigma, p = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    phi = oracle.extract(wl.X, wl.utt_off, wl.w, wl.mu, wl.cov, T, Sigma, p)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    n, f, _ = oracle.bw_stats(wl.X, wl.utt_off, gamma, second_order=False)
    np.testing.assert_array_equal(phi, oracle.estep(n, f, T, Sigma, p)["phi"])


def test_realignment_uses_first_column_times_offset():
    wl = synth.make(1, n_utts=20)
    ubm = (wl.w, wl.mu, wl.cov)
    tv = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    r = oracle.em_iteration(wl.X, wl.utt_off, ubm, tv)
    np.testing.assert_allclose(r["mu"], r["p"][0] * r["T"][:, :, 0])
    assert r["p"][0] > 0 and np.all(np.abs(r["p"][1:]) <= 1e-12 * r["p"][0])
