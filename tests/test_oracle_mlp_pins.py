"""Pins of the learned-selection oracle (oracle.mlp) against finite
differences, closed forms, library routines and special cases."""
import numpy as np
import pytest
import scipy.special
import scipy.stats

import oracle
import synth


def _tiny_net(rng, D=5, H1=7, H2=6, C=9):
    return (rng.normal(size=(H1, D)), rng.normal(size=H1) * 0.1,
            rng.normal(size=(H2, H1)) * 0.5, rng.normal(size=H2) * 0.1,
            rng.normal(size=(C, H2)) * 0.5, rng.normal(size=C) * 0.1)


def _targets(rng, F, C):
    g = rng.random((F, C)) ** 4
    return g / g.sum(axis=1, keepdims=True)


def test_softmax_and_loss_match_library_routines():
    rng = np.random.default_rng(1)
    z = rng.normal(size=(11, 9)) * 30.0
    g = _targets(rng, 11, 9)
    np.testing.assert_allclose(oracle.softmax(z), scipy.special.softmax(z, axis=1), rtol=1e-12,
                               atol=1e-300)
    np.testing.assert_allclose(oracle.log_softmax(z), scipy.special.log_softmax(z, axis=1),
                               rtol=1e-12, atol=1e-12)
    # cross-entropy = H(gamma) + KL(gamma || q), frame by frame
    q = scipy.special.softmax(z, axis=1)
    ref = np.mean([scipy.stats.entropy(g[t]) + scipy.stats.entropy(g[t], q[t]) for t in range(11)])
    assert abs(oracle.ce_loss(z, g) - ref) <= 1e-10 * abs(ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    params = _tiny_net(rng)
    X = rng.normal(size=(13, 5))
    g = _targets(rng, 13, 9)
    z, cache = oracle.mlp_forward(params, X)
    grads = oracle.mlp_backward(params, cache, z, g)
    eps = 1e-6
    for pi, (P, G) in enumerate(zip(params, grads)):
        assert G.shape == P.shape
        flat = np.arange(P.size)
        for e in rng.choice(flat, size=min(12, P.size), replace=False):
            idx = np.unravel_index(e, P.shape)
            plus = [p.copy() for p in params]
            minus = [p.copy() for p in params]
            plus[pi][idx] += eps
            minus[pi][idx] -= eps
            fd = (oracle.ce_loss(oracle.mlp_forward(plus, X)[0], g)
                  - oracle.ce_loss(oracle.mlp_forward(minus, X)[0], g)) / (2 * eps)
            assert abs(fd - G[idx]) <= 1e-7 + 1e-5 * abs(fd), (pi, idx, fd, G[idx])


def test_logit_gradient_is_q_minus_gamma():
    """With targets summing to one, d loss / d b3 = mean_t (q_t - gamma_t)."""
    rng = np.random.default_rng(3)
    params = _tiny_net(rng)
    X = rng.normal(size=(8, 5))
    g = _targets(rng, 8, 9)
    z, cache = oracle.mlp_forward(params, X)
    db3 = oracle.mlp_backward(params, cache, z, g)[5]
    q = scipy.special.softmax(z, axis=1)
    np.testing.assert_allclose(db3, (q - g).mean(axis=0), rtol=1e-10, atol=1e-14)


def test_adam_with_a_constant_gradient_moves_lr_per_step():
    """Bias correction makes m_hat = g and v_hat = g^2 at every step for a
    constant gradient, so each step moves by lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.02, 1e-3, -40.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 8):
        p, m, v = oracle.adam_update(p, g, m, v, t, lr=1e-2)
    np.testing.assert_allclose(p, -7 * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(4)
    target = rng.normal(size=6)
    p, m, v = np.zeros(6), np.zeros(6), np.zeros(6)
    for t in range(1, 4001):
        p, m, v = oracle.adam_update(p, 2 * (p - target), m, v, t, lr=1e-2)
    np.testing.assert_allclose(p, target, atol=1e-3)


def test_training_lowers_the_loss():
    rng = np.random.default_rng(5)
    params = list(_tiny_net(rng))
    X = rng.normal(size=(64, 5))
    g = _targets(rng, 64, 9)
    state = [(np.zeros_like(p), np.zeros_like(p)) for p in params]
    l0 = oracle.ce_loss(oracle.mlp_forward(params, X)[0], g)
    for t in range(1, 301):
        z, cache = oracle.mlp_forward(params, X)
        grads = oracle.mlp_backward(params, cache, z, g)
        for i in range(6):
            params[i], m, v = oracle.adam_update(params[i], grads[i], *state[i], t, lr=1e-2)
            state[i] = (m, v)
    l1 = oracle.ce_loss(oracle.mlp_forward(params, X)[0], g)
    assert l1 < 0.8 * l0


def test_topk_orders_ties_by_lower_index():
    z = np.array([[1.0, 3.0, 3.0, 2.0, 3.0, -1.0]])
    assert oracle.topk(z, 2).tolist() == [[1, 2]]
    assert oracle.topk(z, 5).tolist() == [[1, 2, 4, 3, 0]]
    rng = np.random.default_rng(6)
    zz = rng.integers(0, 4, size=(20, 12)).astype(float)  # many ties
    for t in range(20):
        ref = sorted(range(12), key=lambda c: (-zz[t, c], c))[:7]
        assert oracle.topk(zz[t:t + 1], 7)[0].tolist() == ref


def test_all_components_proposed_reproduces_all_c_posteriors():
    wl = synth.tiny(C=6, U=60)
    X = wl.X
    C = wl.shape.C
    z = np.random.default_rng(7).normal(size=(X.shape[0], C))
    idx = oracle.topk(z, C)
    mass = oracle.proposed_mass(z, idx)
    np.testing.assert_allclose(mass, 1.0, atol=1e-12)
    gam, fb, lse = oracle.learned_posteriors(X, wl.w, wl.mu, wl.cov, idx, mass)
    ref, ref_lse = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    assert not fb.any()
    np.testing.assert_allclose(gam, ref, atol=1e-14)
    np.testing.assert_allclose(lse, ref_lse, rtol=1e-13)
    np.testing.assert_allclose(oracle.missed_mass(ref, idx), 0.0, atol=1e-12)


def test_restricted_posteriors_are_bayes_over_the_proposed_set():
    """Against brute-force densities (determinant and inverse, no Cholesky) of
    a mixture made of the proposed components only."""
    wl = synth.tiny(C=6, U=10)
    X = wl.X[:40].astype(np.float64)
    C, D = wl.shape.C, wl.shape.D
    rng = np.random.default_rng(8)
    idx = np.stack([rng.permutation(C)[:3] for _ in range(40)])
    mass = np.ones(40)
    mass[5] = 0.5  # falls back to all C
    gam, fb, _ = oracle.learned_posteriors(X, wl.w, wl.mu, wl.cov, idx, mass)
    assert fb.tolist() == [t == 5 for t in range(40)]
    for t in range(40):
        comps = range(C) if t == 5 else idx[t]
        logp = []
        for c in comps:
            d = X[t] - wl.mu[c]
            logp.append(np.log(wl.w[c]) - 0.5 * D * np.log(2 * np.pi)
                        - 0.5 * np.log(np.linalg.det(wl.cov[c]))
                        - 0.5 * d @ np.linalg.inv(wl.cov[c]) @ d)
        logp = np.array(logp)
        post = np.exp(logp - logp.max())
        post /= post.sum()
        ref = np.zeros(C)
        ref[list(comps)] = post
        np.testing.assert_allclose(gam[t], ref, atol=1e-10)
        assert abs(gam[t].sum() - 1.0) <= 1e-12


def test_everything_falls_back_when_min_mass_exceeds_one():
    wl = synth.tiny(C=6, U=10)
    X = wl.X[:50]
    z = np.random.default_rng(9).normal(size=(50, wl.shape.C))
    idx = oracle.topk(z, 4)
    mass = oracle.proposed_mass(z, idx)
    gam, fb, _ = oracle.learned_posteriors(X, wl.w, wl.mu, wl.cov, idx, mass, min_mass=1.5)
    assert fb.all()
    ref, _ = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    np.testing.assert_allclose(gam, ref, atol=1e-14)


def test_bf16_rounding_matches_torch_and_hand_cases():
    import torch
    rng = np.random.default_rng(10)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, size=5000),
                        [0.0, -0.0, 1.0, -2.5, 3.4e38]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(oracle.round_bf16(a), ref)
    # ties go to the even mantissa: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert oracle.round_bf16(np.float32(1 + 2.0 ** -8)) == np.float32(1.0)
    assert oracle.round_bf16(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)
    assert oracle.round_bf16(np.float32(1 + 2.0 ** -9)) == np.float32(1.0)


def test_bf16_forward_is_close_to_the_exact_network_and_exact_on_representable_values():
    rng = np.random.default_rng(11)
    params = _tiny_net(rng)
    X = rng.normal(size=(50, 5))
    mean, std = np.zeros(5), np.ones(5)
    z64, _ = oracle.mlp_forward(params, X)
    z16, h1, h2 = oracle.mlp_forward_bf16(params, X, mean, std)
    assert np.abs(z16 - z64).max() <= 0.05 * np.abs(z64).max()
    # small integers: every weight, input and hidden value lies on the BF16
    # grid (|h| < 256) and every sum is exact in FP32, so the BF16 network
    # equals integer arithmetic
    W1 = rng.integers(-1, 2, size=(7, 5)).astype(float)
    W2 = rng.integers(-1, 2, size=(6, 7)).astype(float)
    W3 = rng.integers(-1, 2, size=(9, 6)).astype(float)
    b = [rng.integers(-1, 2, size=n).astype(float) for n in (7, 6, 9)]
    Xi = rng.integers(-2, 3, size=(40, 5)).astype(float)
    z16, h1, h2 = oracle.mlp_forward_bf16((W1, b[0], W2, b[1], W3, b[2]), Xi, mean, std)
    e1 = np.maximum(Xi @ W1.T + b[0], 0)
    e2 = np.maximum(e1 @ W2.T + b[1], 0)
    assert e2.max() < 256
    np.testing.assert_array_equal(h1, e1)
    np.testing.assert_array_equal(h2, e2)
    np.testing.assert_array_equal(z16, e2 @ W3.T + b[2])


def test_feature_stats_and_standardise_on_a_hand_example():
    """Population (not sample) standard deviation, per feature column; the
    standardised columns have mean 0 and population variance 1."""
    X = np.array([[1.0, 2.0, -4.0], [3.0, 6.0, -4.0 + 1e-3], [5.0, 10.0, -4.0 - 1e-3]])
    mean, std = oracle.feature_stats(X)
    np.testing.assert_allclose(mean, [3.0, 6.0, -4.0], rtol=0, atol=1e-15)
    # column 1: deviations -2, 0, 2 -> population variance 8/3 (the sample
    # variance would be 4); column 2 is column 1 doubled; column 3: 0, +-1e-3
    np.testing.assert_allclose(std, [np.sqrt(8.0 / 3.0), 2.0 * np.sqrt(8.0 / 3.0),
                                     np.sqrt(2e-6 / 3.0)], rtol=1e-9)
    Z = oracle.standardise(X, mean, std)
    np.testing.assert_allclose(Z[:, 0], [-np.sqrt(1.5), 0.0, np.sqrt(1.5)], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(Z[:, 0], Z[:, 1], rtol=1e-12, atol=1e-15)  # scale-free
    np.testing.assert_allclose(Z.mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose((Z ** 2).mean(axis=0), 1.0, rtol=1e-9)
