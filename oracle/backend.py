"""Scoring back-end of Sec. 4.1 (the paragraph after extraction), FP64 -- test
infrastructure only.

After extraction the i-vectors are centred, whitened when minimum divergence
was not used, length-normalised, reduced from 400 to 200 dimensions by LDA
and scored with a Gaussian PLDA; accuracy is the equal error rate over
target and non-target trials.  The paper names these steps and cites the
Gaussian PLDA analysis for the last two; the readings taken here where it
gives no formulas:
  * whitening: the eigendecomposition of the covariance, W = Lambda^{-1/2} Q^T;
  * LDA: maximise the ratio of between- to within-class scatter,
    Sb v = lambda Sw v, eigenvectors normalised so that V^T Sw V = I, sorted
    by decreasing eigenvalue;
  * PLDA: the two-covariance model y = mu + s + e, s ~ N(0, B) per speaker,
    e ~ N(0, W) per utterance, with moment estimates (B, W = the LDA
    between- and within-class scatter of the training i-vectors) and the
    verification score the log-likelihood ratio of "same speaker" against
    "different speakers";
  * EER: the crossing of P_miss = P_fa on the operating points of all
    score thresholds (misses: targets below the threshold; false alarms:
    non-targets at or above it) joined by straight segments, so that tied
    target and non-target scores share the error evenly.
"""
from __future__ import annotations

import numpy as np
from scipy.stats import multivariate_normal


def whitening(X):
    """Mean and whitening matrix of the rows of X: W = Lambda^{-1/2} Q^T with
    the covariance Q Lambda Q^T (divisor N)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    Xc = X - mu
    cov = Xc.T @ Xc / len(X)
    lam, Q = np.linalg.eigh(cov)
    return mu, (lam ** -0.5)[:, None] * Q.T


def center_lnorm(X, mean, W=None):
    """Rows centred on `mean`, optionally whitened (y = W (x - mean)), then
    scaled to unit Euclidean length."""
    Y = np.asarray(X, dtype=np.float64) - mean
    if W is not None:
        Y = Y @ np.asarray(W, dtype=np.float64).T
    return Y / np.linalg.norm(Y, axis=1, keepdims=True)


def class_scatter(X, labels):
    """Global mean, within-class and between-class scatter (divisor N):
    Sw = 1/N sum_k sum_{i in k} (x_i - m_k)(x_i - m_k)^T,
    Sb = 1/N sum_k n_k (m_k - m)(m_k - m)^T."""
    X = np.asarray(X, dtype=np.float64)
    labels = np.asarray(labels)
    N, R = X.shape
    m = X.mean(axis=0)
    Sw = np.zeros((R, R))
    Sb = np.zeros((R, R))
    for k in np.unique(labels):
        Xk = X[labels == k]
        mk = Xk.mean(axis=0)
        D = Xk - mk
        Sw += D.T @ D
        Sb += len(Xk) * np.outer(mk - m, mk - m)
    return m, Sw / N, Sb / N


def lda(X, labels, dim):
    """LDA projection V [R][dim] (columns Sw-orthonormal, by decreasing
    eigenvalue of Sb v = lambda Sw v) and the eigenvalues."""
    _, Sw, Sb = class_scatter(X, labels)
    L = np.linalg.cholesky(Sw)
    Li = np.linalg.inv(L)
    lam, U = np.linalg.eigh(Li @ Sb @ Li.T)
    order = np.argsort(-lam, kind="stable")[:dim]
    return Li.T @ U[:, order], lam[order]


def plda_fit(Y, labels):
    """Two-covariance PLDA by moment estimates: (mu, B, W)."""
    mu, W, B = class_scatter(Y, labels)
    return mu, B, W


def plda_llr(Y1, Y2, mu, B, W):
    """Log-likelihood ratios of the pairs (Y1[i], Y2[i]):
    log N([y1; y2]; [mu; mu], [[B+W, B], [B, B+W]])
      - log N(y1; mu, B+W) - log N(y2; mu, B+W)."""
    Y1 = np.atleast_2d(np.asarray(Y1, dtype=np.float64))
    Y2 = np.atleast_2d(np.asarray(Y2, dtype=np.float64))
    d = Y1.shape[1]
    T = B + W
    joint = np.block([[T, B], [B, T]])
    same = multivariate_normal(np.concatenate([mu, mu]), joint).logpdf(np.hstack([Y1, Y2]))
    one = multivariate_normal(mu, T)
    return np.atleast_1d(same - one.logpdf(Y1) - one.logpdf(Y2))


def eer(scores, is_target):
    """Equal error rate: the operating points (P_miss(t), P_fa(t)) at every
    threshold t among the scores and above them, with
    P_miss(t) = #(targets < t) / #targets and
    P_fa(t) = #(non-targets >= t) / #non-targets, joined by straight
    segments; the EER is where that polyline crosses P_miss = P_fa."""
    s = np.asarray(scores, dtype=np.float64)
    tgt = np.asarray(is_target, dtype=bool)
    st, sn = np.sort(s[tgt]), np.sort(s[~tgt])
    pts = []
    for t in list(np.unique(s)) + [np.inf]:
        pm = np.searchsorted(st, t, side="left") / len(st)
        pf = (len(sn) - np.searchsorted(sn, t, side="left")) / len(sn)
        pts.append((pm, pf))
    for (pm0, pf0), (pm1, pf1) in zip(pts[:-1], pts[1:]):
        if pm0 <= pf0 and pm1 >= pf1:
            d0, d1 = pf0 - pm0, pf1 - pm1
            lam = d0 / (d0 - d1) if d0 != d1 else 0.0
            return pm0 + lam * (pm1 - pm0)
    raise AssertionError("the operating points always cross")
