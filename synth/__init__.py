"""Seeded synthetic workloads shaped like the paper's TV-model training data.

This module only draws random inputs: a full-covariance UBM, a "true" total
variability matrix used to shift component means per utterance, per-utterance
feature frames, and the standard-normal matrix that the training
initialisation consumes (Sec. 2.1: T_c entries drawn from N(0, 1)).  It holds
none of the method's arithmetic (no log-likelihoods, statistics, E-step or
M-step); both the FP64 oracle and the GPU path read what it returns.

Generator recipe (all draws PCG64, seeded from SeedSequence([config, seed])):
  * weights  w ~ Dirichlet(1_C)
  * means    mu_c ~ N(0, 4 I)
  * covs     Sigma_c = A^T A, A in R^{(D+5) x D}, A_ij ~ N(0, 1/(D+5))
  * T_true   entries ~ N(0, 0.05)   (0.05 is a variance); shape 6 reads the
             same text with 0.05 as the standard deviation (variance 0.0025)
  * utterance u: w_u ~ N(0, I_R); c_t ~ Cat(w);
               x_t = mu_{c_t} + T_true_{c_t} w_u + chol(Sigma_{c_t}) z_t,
               z_t ~ N(0, I_D)
  * features are produced in float64 and stored as float32; both sides read
    the float32 values.
  * every utterance draws from its own child seed, so any utterance subset is
    reproducible; the float64 arithmetic runs in fixed chunks of
    ``CHUNK`` utterances aligned to absolute utterance indices.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

CHUNK = 100


@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    D: int
    C: int
    R: int
    U: int
    lengths: str  # "uniform:lo:hi" or "loguniform:lo:hi"
    iters: int
    t_var: float = 0.05  # variance of the T_true entries


# Workload shapes.  Shape 3 shares shape 2's data, shape 5 shares shape 4's.
SHAPES = {
    1: Shape("tiny-fp64-oracle", 20, 64, 32, 200, "uniform:100:300", 3),
    2: Shape("full-fp32-plain", 60, 2048, 400, 4000, "uniform:500:1500", 5),
    3: Shape("full-bf16-precision", 60, 2048, 400, 4000, "uniform:500:1500", 5),
    4: Shape("batching-loguniform", 60, 2048, 400, 20000, "loguniform:200:3000", 5),
    5: Shape("learned-selection", 60, 2048, 400, 20000, "loguniform:200:3000", 5),
    6: Shape("batching-loguniform-tstd", 60, 2048, 400, 20000, "loguniform:200:3000", 5,
             t_var=0.0025),
}
DATA_OF = {1: 1, 2: 2, 3: 2, 4: 4, 5: 4, 6: 6}


@dataclasses.dataclass
class Workload:
    shape: Shape
    seed: int
    w: np.ndarray          # [C] f64
    mu: np.ndarray         # [C, D] f64
    cov: np.ndarray        # [C, D, D] f64
    T_true: np.ndarray     # [C, D, R] f64
    T_init: np.ndarray     # [C, D, R] f64, N(0, 1) draws for the TV initialisation
    X: np.ndarray          # [F, D] f32, utterances concatenated
    utt_off: np.ndarray    # [U+1] int64
    comp: np.ndarray       # [F] int32, generating component (diagnostics only)

    @property
    def F(self) -> int:
        return int(self.utt_off[-1])

    @property
    def U(self) -> int:
        return len(self.utt_off) - 1


def _children(shape_id: int, seed: int):
    ss = np.random.SeedSequence([DATA_OF[shape_id], seed])
    ubm, ttrue, lens, tinit, utts = ss.spawn(5)
    return ubm, ttrue, lens, tinit, utts


def _lengths(spec: str, U: int, rng: np.random.Generator) -> np.ndarray:
    kind, lo, hi = spec.split(":")
    lo, hi = int(lo), int(hi)
    if kind == "uniform":
        return rng.integers(lo, hi + 1, size=U).astype(np.int64)
    if kind == "loguniform":
        return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=U))).astype(np.int64)
    raise ValueError(spec)


def make_ubm(D: int, C: int, rng: np.random.Generator):
    """Full-covariance UBM draws: Dirichlet weights, N(0,4I) means, Wishart covariances."""
    w = rng.dirichlet(np.ones(C))
    mu = 2.0 * rng.standard_normal((C, D))
    A = rng.standard_normal((C, D + 5, D)) / np.sqrt(D + 5)
    cov = np.matmul(np.transpose(A, (0, 2, 1)), A)
    cov = 0.5 * (cov + np.transpose(cov, (0, 2, 1)))
    return w, mu, cov


def make(shape_id: int, seed: int = 0, n_utts: Optional[int] = None,
         D: Optional[int] = None, C: Optional[int] = None, R: Optional[int] = None,
         U: Optional[int] = None, lengths: Optional[str] = None) -> Workload:
    """Generate workload ``shape_id`` (1..6).

    ``n_utts`` keeps only the first n utterances (they are identical to the
    first n of the full workload).  D/C/R/U/lengths override the shape for
    small custom cases (tests); overriding any of them changes the data.
    """
    base = SHAPES[shape_id]
    sh = dataclasses.replace(
        base,
        D=D if D is not None else base.D,
        C=C if C is not None else base.C,
        R=R if R is not None else base.R,
        U=U if U is not None else base.U,
        lengths=lengths if lengths is not None else base.lengths,
    )
    s_ubm, s_ttrue, s_lens, s_tinit, s_utts = _children(shape_id, seed)
    if (D, C, R, U, lengths) != (None,) * 5:
        # custom shapes get their own stream so they never alias a named workload
        extra = np.random.SeedSequence([DATA_OF[shape_id], seed, sh.D, sh.C, sh.R, sh.U])
        s_ubm, s_ttrue, s_lens, s_tinit, s_utts = extra.spawn(5)
    Dd, Cc, Rr = sh.D, sh.C, sh.R
    w, mu, cov = make_ubm(Dd, Cc, np.random.Generator(np.random.PCG64(s_ubm)))
    T_true = np.sqrt(sh.t_var) * np.random.Generator(np.random.PCG64(s_ttrue)).standard_normal((Cc, Dd, Rr))
    T_init = np.random.Generator(np.random.PCG64(s_tinit)).standard_normal((Cc, Dd, Rr))
    lens = _lengths(sh.lengths, sh.U, np.random.Generator(np.random.PCG64(s_lens)))
    nU = sh.U if n_utts is None else min(n_utts, sh.U)
    lens = lens[:nU]
    utt_off = np.zeros(nU + 1, dtype=np.int64)
    utt_off[1:] = np.cumsum(lens)
    F = int(utt_off[-1])

    chol = np.linalg.cholesky(cov)  # sampling transform for z -> N(0, Sigma_c)
    cw = np.cumsum(w)
    cw[-1] = 1.0
    X = np.empty((F, Dd), dtype=np.float32)
    comp = np.empty(F, dtype=np.int32)
    utt_seeds = s_utts.spawn(sh.U)[:nU]
    for c0 in range(0, nU, CHUNK):
        c1 = min(nU, c0 + CHUNK)
        zs, cs, ws, uidx = [], [], [], []
        for u in range(c0, c1):
            g = np.random.Generator(np.random.PCG64(utt_seeds[u]))
            wu = g.standard_normal(Rr)
            ct = np.searchsorted(cw, g.random(int(lens[u])), side="right").astype(np.int64)
            ct = np.minimum(ct, Cc - 1)
            zt = g.standard_normal((int(lens[u]), Dd))
            ws.append(wu)
            cs.append(ct)
            zs.append(zt)
            uidx.append(np.full(int(lens[u]), u - c0, dtype=np.int64))
        ct = np.concatenate(cs)
        zt = np.concatenate(zs)
        ut = np.concatenate(uidx)
        Wc = np.stack(ws, axis=1)  # [R, n_chunk]
        xt = np.empty_like(zt)
        order = np.argsort(ct, kind="stable")
        bounds = np.searchsorted(ct[order], np.arange(Cc + 1))
        for c in range(Cc):
            sel = order[bounds[c]:bounds[c + 1]]
            if sel.size == 0:
                continue
            shift = (T_true[c] @ Wc[:, ut[sel]]).T
            xt[sel] = mu[c] + shift + zt[sel] @ chol[c].T
        f0, f1 = int(utt_off[c0]), int(utt_off[c1])
        X[f0:f1] = xt.astype(np.float32)
        comp[f0:f1] = ct.astype(np.int32)
    return Workload(sh, seed, w, mu, cov, T_true, T_init, X, utt_off, comp)


def tiny(D=3, C=4, R=2, U=3, lo=4, hi=7, seed=0) -> Workload:
    """A very small custom workload for brute-force pins."""
    return make(1, seed=seed, D=D, C=C, R=R, U=U, lengths=f"uniform:{lo}:{hi}")


def mlp_init(D, H1, H2, C, seed=0):
    """Initial selector parameters, flat FP32 in the order W1 [H1][D], b1,
    W2 [H2][H1], b2, W3 [C][H2], b3: weights N(0, 2 / fan_in), biases 0."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([9001, seed])))
    parts = [rng.normal(0.0, np.sqrt(2.0 / D), size=(H1, D)), np.zeros(H1),
             rng.normal(0.0, np.sqrt(2.0 / H1), size=(H2, H1)), np.zeros(H2),
             rng.normal(0.0, np.sqrt(2.0 / H2), size=(C, H2)), np.zeros(C)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def mlp_split(flat, D, H1, H2, C):
    """Views of a flat parameter vector as (W1, b1, W2, b2, W3, b3)."""
    shapes = [(H1, D), (H1,), (H2, H1), (H2,), (C, H2), (C,)]
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(np.asarray(flat[o:o + n]).reshape(sh))
        o += n
    return tuple(out)


def sample_frames(F, B, seed):
    """B distinct frame indices in [0, F), drawn without replacement."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([9002, seed])))
    return np.sort(rng.choice(F, size=B, replace=False)).astype(np.int64)


def speakers(shape_id: int = 2, n_spk: int = 400, per_spk: int = 8, lengths: str = "uniform:200:600",
             rho: float = 0.5, seed: int = 0):
    """Speaker-labelled utterances under the model of workload ``shape_id``
    (same UBM and T_true): every speaker draws y_s ~ N(0, I_R) and each of its
    utterances w_u = sqrt(rho) y_s + sqrt(1 - rho) z_u, z_u ~ N(0, I_R), so
    w_u ~ N(0, I_R) overall and rho is the between-speaker share of its
    variance.  Frames as in ``make``.  Returns (Workload, labels [U] int32)."""
    base = make(shape_id, seed=seed, n_utts=1)
    sh = dataclasses.replace(base.shape, U=n_spk * per_spk, lengths=lengths)
    C, D, R = sh.C, sh.D, sh.R
    ss = np.random.SeedSequence([7001, shape_id, seed, n_spk, per_spk])
    s_spk, s_lens, s_utts = ss.spawn(3)
    Y = np.random.Generator(np.random.PCG64(s_spk)).standard_normal((n_spk, R))
    U = n_spk * per_spk
    lens = _lengths(lengths, U, np.random.Generator(np.random.PCG64(s_lens)))
    labels = np.repeat(np.arange(n_spk, dtype=np.int32), per_spk)
    utt_off = np.zeros(U + 1, dtype=np.int64)
    utt_off[1:] = np.cumsum(lens)
    chol = np.linalg.cholesky(base.cov)
    cw = np.cumsum(base.w)
    cw[-1] = 1.0
    X = np.empty((int(utt_off[-1]), D), dtype=np.float32)
    comp = np.empty(int(utt_off[-1]), dtype=np.int32)
    T2 = base.T_true.reshape(C * D, R)
    useeds = s_utts.spawn(U)
    for c0 in range(0, U, 64):
        c1 = min(U, c0 + 64)
        draws = []
        for u in range(c0, c1):
            g = np.random.Generator(np.random.PCG64(useeds[u]))
            wu = np.sqrt(rho) * Y[labels[u]] + np.sqrt(1.0 - rho) * g.standard_normal(R)
            n = int(lens[u])
            ct = np.minimum(np.searchsorted(cw, g.random(n), side="right"), C - 1)
            draws.append((wu, ct, g.standard_normal((n, D))))
        M = (T2 @ np.stack([d[0] for d in draws], axis=1)).reshape(C, D, c1 - c0)
        for j, (wu, ct, zt) in enumerate(draws):
            u = c0 + j
            xt = base.mu[ct] + M[ct, :, j] + np.einsum("tde,te->td", chol[ct], zt)
            X[utt_off[u]:utt_off[u + 1]] = xt.astype(np.float32)
            comp[utt_off[u]:utt_off[u + 1]] = ct
    wl = Workload(sh, seed, base.w, base.mu, base.cov, base.T_true, base.T_init, X, utt_off, comp)
    return wl, labels
