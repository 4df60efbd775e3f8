"""FP64 oracle of the augmented TV-model EM iteration (test infrastructure only).

Notation follows the paper: n_c(u), f_c(u), S_c are the Baum-Welch statistics
(Sec. 2), T_c the per-component blocks of the total variability matrix, Sigma_c
the residual covariances, p the prior offset, phi(u) / Phi(u) the posterior
mean / covariance of the latent vector (eqs. (3)-(4)), h / H the
minimum-divergence sums (eqs. (6)-(7)), P1 / P2 the whitening and Householder
transforms (eqs. (8)-(11)).  Element 1 of the paper's latent vector (the prior
offset dimension) is index 0 here.  Statistics are NOT centred (augmented
formulation, Sec. 2.2).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

LOG2PI = float(np.log(2.0 * np.pi))


# --------------------------------------------------------------------------
# Frame alignment (Sec. 3.2 step 1; Sec. 4.2): full-covariance UBM posteriors
# --------------------------------------------------------------------------
def frame_loglik(X, w, mu, cov):
    """log( w_c N(x_t; mu_c, cov_c) ) for every frame t and component c.

    Direct form through the Cholesky factor L_c of cov_c:
      log w_c - D/2 log 2pi - sum_i log L_c[i,i] - 1/2 || L_c^{-1}(x_t - mu_c) ||^2
    Returns [F, C] float64.
    """
    X = np.asarray(X, dtype=np.float64)
    F, D = X.shape
    C = len(w)
    ll = np.empty((F, C))
    for c in range(C):
        L = np.linalg.cholesky(cov[c])
        y = solve_triangular(L, (X - mu[c]).T, lower=True)
        ll[:, c] = (np.log(w[c]) - 0.5 * D * LOG2PI - np.sum(np.log(np.diag(L)))
                    - 0.5 * np.sum(y * y, axis=0))
    return ll


def posteriors(ll):
    """Frame posteriors gamma_tc = exp(ll_tc - lse_t) and the per-frame
    log-likelihood lse_t = log sum_c exp(ll_tc)."""
    m = ll.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(ll - m).sum(axis=1))
    return np.exp(ll - lse[:, None]), lse


def bw_stats(X, utt_off, gamma, second_order=True):
    """Uncentred Baum-Welch statistics (Sec. 2, augmented formulation).

    n[u, c] = sum_t gamma_tc, f[u, c] = sum_t gamma_tc x_t (frames t of u),
    S[c] = sum_u sum_t gamma_tc x_t x_t^T (totals over all utterances).
    """
    X = np.asarray(X, dtype=np.float64)
    U = len(utt_off) - 1
    F, D = X.shape
    C = gamma.shape[1]
    n = np.zeros((U, C))
    f = np.zeros((U, C, D))
    for u in range(U):
        a, b = int(utt_off[u]), int(utt_off[u + 1])
        g = gamma[a:b]
        n[u] = g.sum(axis=0)
        f[u] = g.T @ X[a:b]
    S = None
    if second_order:
        S = np.empty((C, D, D))
        for c in range(C):
            S[c] = (gamma[:, c:c + 1] * X).T @ X
    return n, f, S


# --------------------------------------------------------------------------
# Model initialisation (Sec. 2.1 and 2.2)
# --------------------------------------------------------------------------
def init_tv(mu, cov, T_rand, p0=100.0):
    """Augmented initialisation: T_c from the supplied N(0,1) draws with its
    first column replaced by mu_c / p0, Sigma_c = UBM covariance, p = p0 e_1."""
    T = np.array(T_rand, dtype=np.float64, copy=True)
    T[:, :, 0] = mu / p0
    Sigma = np.array(cov, dtype=np.float64, copy=True)
    p = np.zeros(T.shape[2])
    p[0] = p0
    return T, Sigma, p


# --------------------------------------------------------------------------
# E-step (eqs. (3)-(4))
# --------------------------------------------------------------------------
def tv_precompute(T, Sigma):
    """V_c = Sigma_c^{-1} T_c and U_c = T_c^T Sigma_c^{-1} T_c (the terms of eqs. (3)-(4))."""
    C, D, R = T.shape
    V = np.empty_like(T)
    Uc = np.empty((C, R, R))
    for c in range(C):
        V[c] = cho_solve(cho_factor(Sigma[c], lower=True), T[c])
        Uc[c] = T[c].T @ V[c]
    return V, Uc


def estep(n, f, T, Sigma, p, want_cov=True, pre=None):
    """Posterior precision / covariance / mean of the latent vector per utterance.

    L(u)   = I + sum_c n_c(u) T_c^T Sigma_c^{-1} T_c      (inverse of eq. (3))
    b(u)   = p + sum_c T_c^T Sigma_c^{-1} f_c(u)
    phi(u) = L(u)^{-1} b(u)                                (eq. (4))
    Phi(u) = L(u)^{-1}                                     (eq. (3))
    ll(u)  = -1/2 log|L(u)| + 1/2 b(u)^T phi(u) - 1/2 p^T p
    ll(u) is the utterance's share of the marginal log-likelihood of the
    alignment-weighted statistics (the latent vector integrated out).
    ``pre`` may pass (V, U) from tv_precompute(T, Sigma) when they are
    already at hand.
    """
    C, D, R = T.shape
    U = n.shape[0]
    V, Uc = pre if pre is not None else tv_precompute(T, Sigma)
    Lu = np.eye(R)[None] + (n @ Uc.reshape(C, R * R)).reshape(U, R, R)
    b = p[None, :] + f.reshape(U, C * D) @ V.reshape(C * D, R)
    phi = np.empty((U, R))
    Phi = np.empty((U, R, R)) if want_cov else None
    llu = np.empty(U)
    logdet = np.empty(U)
    for u in range(U):
        cf = cho_factor(Lu[u], lower=True)
        phi[u] = cho_solve(cf, b[u])
        if want_cov:
            Phi[u] = cho_solve(cf, np.eye(R))
        logdet[u] = 2.0 * np.sum(np.log(np.diag(cf[0])))
        llu[u] = -0.5 * logdet[u] + 0.5 * b[u] @ phi[u] - 0.5 * p @ p
    return dict(phi=phi, Phi=Phi, b=b, L=Lu, ll_u=llu, logdet=logdet)


# --------------------------------------------------------------------------
# M-step accumulators (eqs. (6)-(7) plus the cited EM's sufficient statistics)
# --------------------------------------------------------------------------
def accumulate(n, f, phi, Phi):
    """Sums over utterances of the batch:
    N_c = sum_u n_c(u)
    A_c = sum_u n_c(u) (Phi(u) + phi(u) phi(u)^T)
    Cc_c = sum_u f_c(u) phi(u)^T
    hsum = sum_u phi(u),  Hsum = sum_u (Phi(u) + phi(u) phi(u)^T)
    (h = hsum / U and H = Hsum / U are eqs. (6)-(7)).
    """
    U, C = n.shape
    D = f.shape[2]
    R = phi.shape[1]
    Psi = Phi + phi[:, :, None] * phi[:, None, :]
    N = n.sum(axis=0)
    A = (n.T @ Psi.reshape(U, R * R)).reshape(C, R, R)
    Cc = (f.reshape(U, C * D).T @ phi).reshape(C, D, R)
    return dict(N=N, A=A, Cc=Cc, hsum=phi.sum(axis=0), Hsum=Psi.sum(axis=0), count=U)


def objective(N, S, Sigma, ll_u_sum):
    """Marginal log-likelihood of the alignment-weighted statistics under the
    TV model at fixed alignments (the EM objective):
      sum_c N_c (-D/2 log 2pi - 1/2 log|Sigma_c|) - 1/2 sum_c tr(Sigma_c^{-1} S_c) + sum_u ll(u)
    """
    C, D, _ = Sigma.shape
    tot = 0.0
    for c in range(C):
        cf = cho_factor(Sigma[c], lower=True)
        logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
        tot += N[c] * (-0.5 * D * LOG2PI - 0.5 * logdet)
        tot -= 0.5 * np.trace(cho_solve(cf, S[c]))
    return tot + ll_u_sum


# --------------------------------------------------------------------------
# M-step (Sec. 3.2 step 3: T_c, then Sigma_c; factor-analysis EM cited there)
# --------------------------------------------------------------------------
def mstep(acc, S, T, Sigma, update_sigma=True, min_count=0.5):
    """T_c <- Cc_c A_c^{-1};  Sigma_c <- sym((S_c - T_c^new Cc_c^T) / N_c).

    A component without data (N_c < min_count = 0.5) keeps its T_c and
    Sigma_c.  The paper is silent on empty components; soft counts cluster at
    integer frame counts when posteriors are near one-hot, so the threshold
    sits between 0 and 1 frame rather than on an integer.  A new Sigma_c
    that is not positive definite is rejected (old one kept).
    Returns (T_new, Sigma_new, info) with info = dict(skipped=[...], notpd=[...]).
    """
    N, A, Cc = acc["N"], acc["A"], acc["Cc"]
    T_new = np.array(T, copy=True)
    S_new = np.array(Sigma, copy=True)
    skipped, notpd = [], []
    for c in range(len(N)):
        if N[c] < min_count:
            skipped.append(c)
            continue
        T_new[c] = cho_solve(cho_factor(A[c], lower=True), Cc[c].T).T
        if update_sigma:
            M = (S[c] - T_new[c] @ Cc[c].T) / N[c]
            M = 0.5 * (M + M.T)
            try:
                np.linalg.cholesky(M)
                S_new[c] = M
            except np.linalg.LinAlgError:
                notpd.append(c)
    return T_new, S_new, dict(skipped=skipped, notpd=notpd)


# --------------------------------------------------------------------------
# Minimum-divergence re-estimation, augmented formulation (eqs. (6)-(12))
# --------------------------------------------------------------------------
def mindiv(h, H, T, method="chol", tiny=1e-12):
    """Returns (T_upd, p_upd, aux).

    G = H - h h^T; P1 whitens G (Cholesky: P1 = L_G^{-1} with G = L_G L_G^T;
    eig: P1 = Lambda^{-1/2} Q^T with G = Q Lambda Q^T).  h~ = P1 h / ||P1 h||;
    a = alpha h~ + beta e_1 with alpha = 1/sqrt(2(1 - h~[1])), beta = -alpha;
    P2 = I - 2 a a^T (a Householder reflection, eqs. (8)-(11)).
    T_c <- T_c P1^{-1} P2^{-1};  p <- P2 P1 h (eq. (12)).

    1 - h~[1] is formed as ||g_{2:}||^2 / (||g|| (||g|| + g_1)) when g_1 > 0
    (g = P1 h) to avoid cancellation; when ||g_{2:}|| <= tiny ||g|| the
    reflection is the identity.
    """
    R = len(h)
    G = H - np.outer(h, h)
    if method == "chol":
        LG = np.linalg.cholesky(G)
        P1 = solve_triangular(LG, np.eye(R), lower=True)
        P1inv = LG
    elif method == "eig":
        lam, Q = np.linalg.eigh(G)
        P1 = (lam ** -0.5)[:, None] * Q.T
        P1inv = Q * np.sqrt(lam)[None, :]
    else:
        raise ValueError(method)
    g = P1 @ h
    gn = np.linalg.norm(g)
    htil = g / gn
    tail = np.linalg.norm(g[1:])
    if tail <= tiny * gn:
        P2 = np.eye(R)
    else:
        one_minus = tail * tail / (gn * (gn + g[0])) if g[0] > 0 else 1.0 - htil[0]
        alpha = 1.0 / np.sqrt(2.0 * one_minus)
        beta = -alpha
        e1 = np.zeros(R)
        e1[0] = 1.0
        a = alpha * htil + beta * e1
        P2 = np.eye(R) - 2.0 * np.outer(a, a)
    P2inv = P2.T  # a reflection is orthogonal
    T_upd = np.einsum("cdr,rs->cds", T, P1inv @ P2inv)
    p_upd = P2 @ (P1 @ h)
    return T_upd, p_upd, dict(G=G, P1=P1, P2=P2, P1inv=P1inv)


# --------------------------------------------------------------------------
# Realignment (Sec. 3.2 and step 5 of the training loop)
# --------------------------------------------------------------------------
def realign_means(T, p):
    """Updated UBM means: the first columns of T_c multiplied by the prior offset p."""
    return p[0] * T[:, :, 0]


def extract(X, utt_off, w, mu, cov, T, Sigma, p):
    """i-vectors (eq. (4) posterior means) with the trained model and the UBM."""
    gamma, _ = posteriors(frame_loglik(X, w, mu, cov))
    n, f, _ = bw_stats(X, utt_off, gamma, second_order=False)
    return estep(n, f, T, Sigma, p, want_cov=False)["phi"]


def em_iteration(X, utt_off, ubm, tv, update_sigma=True, mindiv_method="chol",
                 realign=True, stats=None):
    """One iteration of the five-step training loop (Sec. 3.2).

    ubm = (w, mu, cov); tv = (T, Sigma, p).  Returns a dict with every
    intermediate: gamma, lse, n, f, S, E-step outputs, accumulators, the
    objective at the incoming parameters, and the updated model (T, Sigma, p,
    mu).  ``mindiv_method=None`` skips minimum divergence; ``stats`` reuses
    fixed alignments (n, f, S, gamma, lse).
    """
    w, mu, cov = ubm
    T, Sigma, p = tv
    if stats is None:
        ll = frame_loglik(X, w, mu, cov)
        gamma, lse = posteriors(ll)
        n, f, S = bw_stats(X, utt_off, gamma)
    else:
        n, f, S, gamma, lse = stats
    e = estep(n, f, T, Sigma, p)
    acc = accumulate(n, f, e["phi"], e["Phi"])
    obj = objective(acc["N"], S, Sigma, e["ll_u"].sum())
    T1, S1, info = mstep(acc, S, T, Sigma, update_sigma=update_sigma)
    p1 = p.copy()
    aux = None
    if mindiv_method is not None:
        h = acc["hsum"] / acc["count"]
        H = acc["Hsum"] / acc["count"]
        T1, p1, aux = mindiv(h, H, T1, method=mindiv_method)
    mu1 = realign_means(T1, p1) if realign else mu.copy()
    return dict(gamma=gamma, lse=lse, n=n, f=f, S=S, estep=e, acc=acc, objective=obj,
                T=T1, Sigma=S1, p=p1, mu=mu1, mstep_info=info, mindiv=aux)


# --------------------------------------------------------------------------
# Kaldi-style pruned alignment (Sec. 4.2): a diagonal-covariance UBM picks
# the 20 best components per frame, the full-covariance UBM scores only
# those, and posteriors below 0.025 are dropped before renormalising.
# --------------------------------------------------------------------------
def diag_frame_loglik(X, w, mu, cov):
    """log( w_c N(x_t; mu_c, diag(cov_c)) ) for every frame and component, the
    diagonal UBM taken as the diagonal of the full-covariance one."""
    X = np.asarray(X, dtype=np.float64)
    var = np.stack([np.diag(c) for c in cov])               # [C, D]
    D = X.shape[1]
    ll = np.empty((X.shape[0], len(w)))
    for c in range(len(w)):
        d = X - mu[c]
        ll[:, c] = (np.log(w[c]) - 0.5 * D * LOG2PI - 0.5 * np.sum(np.log(var[c]))
                    - 0.5 * np.sum(d * d / var[c], axis=1))
    return ll


def preselect(ll_diag, k):
    """The k best components of every frame by the diagonal UBM, best first,
    equal scores ordered by the lower component index."""
    order = np.argsort(-ll_diag, axis=1, kind="stable")
    return order[:, :k]


def pruned_posteriors(X, w, mu, cov, idx, prune=0.025, ll=None):
    """Full-covariance posteriors restricted to the preselected components
    idx [F, k] and renormalised over them; entries below `prune` are then
    dropped and the rest renormalised.  Returns the dense [F, C] posteriors
    and the per-frame log-likelihood over the preselected set.  ``ll`` may
    pass the frames' full-covariance log-likelihoods (frame_loglik) when
    they are already at hand."""
    if ll is None:
        ll = frame_loglik(X, w, mu, cov)
    sub = np.take_along_axis(ll, idx, axis=1)
    g_sub, lse = posteriors(sub)
    g_sub = np.where(g_sub < prune, 0.0, g_sub)
    g_sub = g_sub / g_sub.sum(axis=1, keepdims=True)
    gamma = np.zeros_like(ll)
    np.put_along_axis(gamma, idx, g_sub, axis=1)
    return gamma, lse


# --------------------------------------------------------------------------
# Standard formulation (Sec. 2.1): mu_c(u) = m_c + T_c omega(u), omega ~ N(0, I),
# first- and second-order statistics centred on the bias m_c, prior offset 0.
# --------------------------------------------------------------------------
def init_tv_standard(mu, cov, T_rand):
    """T_c <- N(0, 1) draws, m_c <- UBM means, Sigma_c <- UBM covariances,
    p = 0 (Sec. 2.1)."""
    R = T_rand.shape[2]
    return (np.array(T_rand, dtype=np.float64), np.array(cov, dtype=np.float64), np.zeros(R),
            np.array(mu, dtype=np.float64))


def center_stats(n, f, S, m):
    """Centred statistics: f~_c(u) = f_c(u) - n_c(u) m_c and
    S~_c = sum_u sum_t gamma_tc (x_t - m_c)(x_t - m_c)^T
         = S_c - F_c m_c^T - m_c F_c^T + N_c m_c m_c^T,
    with F_c = sum_u f_c(u), N_c = sum_u n_c(u)."""
    fc = f - n[:, :, None] * m[None, :, :]
    F = f.sum(axis=0)
    N = n.sum(axis=0)
    Sc = (S - np.einsum("cd,ce->cde", F, m) - np.einsum("cd,ce->cde", m, F)
          + N[:, None, None] * np.einsum("cd,ce->cde", m, m))
    return fc, Sc


def mindiv_standard(h, H, T, m, method="chol", update_mean=False):
    """Minimum divergence in the standard formulation (Sec. 3.1): G = H - h h^T
    is whitened by P1 (Cholesky: P1^{-1} = L_G with G = L_G L_G^T; eig:
    P1^{-1} = Q Lambda^{1/2} with G = Q Lambda Q^T) and T_c <- T_c P1^{-1};
    that update alone is the standard form's re-estimation.  With
    update_mean, the bias also absorbs the i-vector mean first (Sec. 5):
    m_c <- m_c + T_c h, so that m_c + T_c omega is kept for omega = h + P1^{-1} omega'.
    Returns (T_upd, m_upd)."""
    G = H - np.outer(h, h)
    if method == "chol":
        P1inv = np.linalg.cholesky(G)
    elif method == "eig":
        lam, Q = np.linalg.eigh(G)
        P1inv = Q * np.sqrt(lam)[None, :]
    else:
        raise ValueError(method)
    m1 = m + np.einsum("cdr,r->cd", T, h) if update_mean else np.array(m, copy=True)
    T1 = np.einsum("cdr,rs->cds", T, P1inv)
    return T1, m1


def em_iteration_standard(X, utt_off, ubm, tv, update_sigma=True, mindiv=True,
                          update_mean=False, method="chol", stats=None):
    """One training iteration of the standard formulation: posteriors from
    the UBM, statistics centred on m, E-step with p = 0, accumulators, the
    objective at the incoming parameters, M-step (T, optionally Sigma) and
    optionally minimum divergence (with the bias update if update_mean).
    tv = (T, Sigma, p, m) with p = 0; returns the updated (T, Sigma, m) and
    the intermediates."""
    w, mu, cov = ubm
    T, Sigma, p, m = tv
    if stats is None:
        gamma, lse = posteriors(frame_loglik(X, w, mu, cov))
        n, f, S = bw_stats(X, utt_off, gamma)
    else:
        n, f, S = stats
    fc, Sc = center_stats(n, f, S, m)
    e = estep(n, fc, T, Sigma, p)
    acc = accumulate(n, fc, e["phi"], e["Phi"])
    obj = objective(acc["N"], Sc, Sigma, e["ll_u"].sum())
    T1, S1, info = mstep(acc, Sc, T, Sigma, update_sigma=update_sigma)
    m1 = np.array(m, copy=True)
    if mindiv:
        h = acc["hsum"] / acc["count"]
        H = acc["Hsum"] / acc["count"]
        T1, m1 = mindiv_standard(h, H, T1, m, method=method, update_mean=update_mean)
    return dict(n=n, f=f, S=S, fc=fc, Sc=Sc, estep=e, acc=acc, objective=obj, T=T1, Sigma=S1,
                m=m1, mstep_info=info)
