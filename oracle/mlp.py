"""FP64 oracle of the learned Gaussian selection (test infrastructure only).

The selector is a small network that proposes, for every frame, k components
whose exact full-covariance posteriors are then computed; it stands where the
paper's Kaldi-style preselection (a diagonal-covariance UBM picking the 20
best components before full-covariance scoring, Sec. 4.2) stands.  The
network and its training are additions that the paper does not describe:

  x_hat = (x - m) / s                      global standardisation
  z     = W3 relu(W2 relu(W1 x_hat + b1) + b2) + b3,   q = softmax(z)
  loss  = -(1/F) sum_t sum_c gamma_tc log q_tc          (soft targets: the
                                                         exact posteriors)
  top-k = the k largest z_tc, ties to the lower component index
  mass  = sum_{c in top-k} q_tc             (computable without scoring all C)

A frame whose mass is below min_mass takes the all-C posteriors (Sec. 4.2
posteriors over every component); every other frame takes the exact
posteriors restricted to its k proposals and renormalised over them.
"""
from __future__ import annotations

import numpy as np

from .tv import frame_loglik, posteriors


def feature_stats(X):
    """Global mean and (population) standard deviation of the features."""
    X = np.asarray(X, dtype=np.float64)
    return X.mean(axis=0), X.std(axis=0)


def standardise(X, mean, std):
    return (np.asarray(X, dtype=np.float64) - mean) / std


def mlp_forward(params, Xh):
    """params = (W1 [H1,D], b1, W2 [H2,H1], b2, W3 [C,H2], b3).  Returns the
    logits z [F,C] and the cache (Xh, a1, h1, a2, h2) of the backward pass."""
    W1, b1, W2, b2, W3, b3 = params
    a1 = Xh @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (Xh, a1, h1, a2, h2)


def round_bf16(a):
    """Round to the nearest BF16 value (ties to even) and return float32.
    BF16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of
    an IEEE float32 (finite inputs)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def mlp_forward_bf16(params, X, mean, std):
    """The deployed network's arithmetic, used where its output decides an
    integer (the proposals, the fallback): x_hat = (x - mean) * (1 / std) in
    FP32; weights and x_hat rounded to BF16; each layer's products summed in
    FP32 with the bias added after the sum; ReLU, then rounding to BF16, for
    the hidden layers.  Returns (z, h1, h2) as float32."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float32) for p in params]
    mean = np.asarray(mean, dtype=np.float32)
    istd = (np.float32(1.0) / np.asarray(std, dtype=np.float32)).astype(np.float32)
    xh = round_bf16((np.asarray(X, dtype=np.float32) - mean) * istd)
    h1 = round_bf16(np.maximum(xh @ round_bf16(W1).T + b1, np.float32(0.0)))
    h2 = round_bf16(np.maximum(h1 @ round_bf16(W2).T + b2, np.float32(0.0)))
    z = (h2 @ round_bf16(W3).T + b3).astype(np.float32)
    return z, h1, h2


def log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    return z - (m + np.log(np.exp(z - m).sum(axis=1, keepdims=True)))


def softmax(z):
    return np.exp(log_softmax(z))


def ce_loss(z, gamma):
    """Soft-target cross-entropy, averaged over frames."""
    return float(-(gamma * log_softmax(z)).sum() / z.shape[0])


def mlp_backward(params, cache, z, gamma):
    """Gradients of ce_loss with respect to (W1, b1, W2, b2, W3, b3).

    d loss / d z_tc = (q_tc * sum_c' gamma_tc' - gamma_tc) / F, which is
    (q - gamma) / F when the targets of a frame sum to one; the rest is the
    chain rule through the two ReLU layers."""
    W1, b1, W2, b2, W3, b3 = params
    Xh, a1, h1, a2, h2 = cache
    F = z.shape[0]
    dz = (softmax(z) * gamma.sum(axis=1, keepdims=True) - gamma) / F
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    da2 = (dz @ W3) * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    dW1 = da1.T @ Xh
    db1 = da1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def adam_update(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) at step count t >= 1; returns the
    new (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def topk(z, k):
    """Indices of the k largest logits per frame, largest first; equal values
    are ordered by the lower component index."""
    order = np.argsort(-np.asarray(z, dtype=np.float64), axis=1, kind="stable")
    return order[:, :k]


def proposed_mass(z, idx):
    """The network's own softmax mass on the proposed components."""
    q = softmax(np.asarray(z, dtype=np.float64))
    return np.take_along_axis(q, idx, axis=1).sum(axis=1)


def learned_posteriors(X, w, mu, cov, idx, mass, min_mass=0.99):
    """Posteriors of the learned selection as a dense [F,C] array.

    Frames with mass < min_mass get the all-C posteriors; the others get the
    exact posteriors of their proposed components, renormalised over them.
    Returns (gamma, fallback mask [F] bool, per-frame log-likelihood over the
    set that was scored)."""
    ll = frame_loglik(X, w, mu, cov)
    F, C = ll.shape
    fb = np.asarray(mass) < min_mass
    gamma_all, lse_all = posteriors(ll)
    gamma = np.zeros((F, C))
    lse = np.empty(F)
    gamma[fb] = gamma_all[fb]
    lse[fb] = lse_all[fb]
    rows = np.nonzero(~fb)[0]
    if rows.size:
        sub = np.take_along_axis(ll[rows], idx[rows], axis=1)
        g_sub, l_sub = posteriors(sub)
        gamma[rows[:, None], idx[rows]] = g_sub
        lse[rows] = l_sub
    return gamma, fb, lse


def missed_mass(gamma_all, idx):
    """1 - sum of the exact all-C posteriors on the proposed components."""
    return 1.0 - np.take_along_axis(gamma_all, idx, axis=1).sum(axis=1)
