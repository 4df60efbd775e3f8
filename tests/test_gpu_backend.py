"""GPU parity of the scoring back-end (Sec. 4.1) against the FP64 oracle:
whitening, length normalisation, LDA, two-covariance PLDA and trial scores,
and the EER of the GPU scores.

Tolerances (from the arithmetic): the scatter matrices are FP64 sums of the
FP32 inputs (the oracle reads the same FP32 values), the eigenproblems are
solved by FP64 Jacobi to an off-diagonal norm of 1e-13 of the matrix norm,
so whitening and LDA agree with the oracle to ~1e-9 relative, or
1e-14 cond(Sw) for an ill-conditioned within-class scatter, where the
eigenvalues are separated; eigenvectors are compared up to sign, and where
eigenvalues lie close together only the invariant subspace checks are used.
Length-normalised vectors and PLDA scores are stored in FP32: |dy| <= 1e-6,
|d score| <= 2e-5 (1 + |score|).
"""
import numpy as np
import pytest
import torch

from oracle import backend as be

pytestmark = pytest.mark.gpu


def _classes(K, per, R, seed, spread=1.0, noise_rank=None):
    rng = np.random.default_rng(seed)
    centres = spread * rng.standard_normal((K, R))
    A = rng.standard_normal((R, R)) / np.sqrt(R) + 0.3 * np.eye(R)
    X = np.concatenate([centres[k] + rng.standard_normal((per, R)) @ A for k in range(K)])
    return X.astype(np.float32), np.repeat(np.arange(K, dtype=np.int32), per)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def backend():
    from paper_1906_08556_amd import ivx
    b = ivx.Backend(512, 8000, 600)
    yield b
    b.close()


@pytest.mark.parametrize("dim", [37, 400])
def test_whitening_matches_the_oracle(backend, dim):
    X, _ = _classes(50, 60, dim, seed=dim)
    mean, W = backend.whitening(_dev(X))
    mean, W = mean.cpu().numpy(), W.cpu().numpy()
    mo, Wo = be.whitening(X)
    np.testing.assert_allclose(mean, mo, rtol=0, atol=1e-12 * np.abs(mo).max())
    Xc = X.astype(np.float64) - mo
    cov = Xc.T @ Xc / len(X)
    err = np.abs(W @ cov @ W.T - np.eye(dim)).max()
    print(f"dim {dim}: |W cov W^T - I| max {err:.2e}")
    assert err <= 1e-9
    # W^T W = cov^{-1} is unique whatever the eigenvector order and signs
    rel = np.linalg.norm(W.T @ W - Wo.T @ Wo) / np.linalg.norm(Wo.T @ Wo)
    assert rel <= 1e-9


def test_length_norm_matches_the_oracle(backend):
    X, _ = _classes(20, 30, 400, seed=1)
    mo, Wo = be.whitening(X)
    for W in (None, Wo):
        Y = backend.lnorm(_dev(X), _dev(mo), None if W is None else _dev(W)).cpu().numpy()
        Yo = be.center_lnorm(X, mo, W)
        err = np.abs(Y - Yo).max()
        print("lnorm max |dy|", err, "whitened" if W is not None else "")
        assert err <= 1e-6


def _align_signs(V, Vo):
    s = np.sign(np.sum(V * Vo, axis=0))
    return V * s


def test_lda_small_matches_the_oracle(backend):
    X, lab = _classes(12, 40, 9, seed=5, spread=2.0)
    V, ev = backend.lda(_dev(X), _dev(lab), 12, 5)
    V, ev = V.cpu().numpy(), ev.cpu().numpy()
    Vo, evo = be.lda(X, lab, 5)
    np.testing.assert_allclose(ev, evo, rtol=1e-10, atol=1e-12)
    V = _align_signs(V, Vo)
    np.testing.assert_allclose(V, Vo, rtol=1e-8, atol=1e-9 * np.abs(Vo).max())


def test_lda_full_size_invariants(backend):
    """400 -> 200 with 300 classes (the paper's dimensions)."""
    X, lab = _classes(300, 20, 400, seed=6, spread=0.5)
    V, ev = backend.lda(_dev(X), _dev(lab), 300, 200)
    V, ev = V.cpu().numpy(), ev.cpu().numpy()
    Vo, evo = be.lda(X, lab, 200)
    _, Sw, Sb = be.class_scatter(X, lab)
    # FP64 on both sides: errors grow with the conditioning of Sw (4.6e5 here)
    ew = np.linalg.eigvalsh(Sw)
    tol = max(1e-10, 1e-14 * ew.max() / ew.min())
    print(f"cond(Sw) {ew.max() / ew.min():.2e}, tolerance {tol:.1e}")
    np.testing.assert_allclose(ev, evo, rtol=tol, atol=1e-12 * evo[0])
    np.testing.assert_allclose(V.T @ Sw @ V, np.eye(200), atol=tol)
    np.testing.assert_allclose(V.T @ Sb @ V, np.diag(evo), atol=tol * evo[0])
    # columns with well separated eigenvalues agree with the oracle's up to sign
    gap = np.minimum(np.abs(np.diff(np.r_[np.inf, evo])), np.abs(np.diff(np.r_[evo, -np.inf])))
    sep = gap > 1e-3 * evo[0]
    Va = _align_signs(V, Vo)
    err = np.abs(Va[:, sep] - Vo[:, sep]).max() / np.abs(Vo).max()
    print(f"LDA 400->200: {sep.sum()} separated columns, max rel diff {err:.2e}")
    assert err <= 1e-6


def test_plda_scores_match_the_oracle(backend):
    d = 200
    Y, lab = _classes(150, 12, d, seed=7, spread=0.8)
    mu, A, psi = backend.plda_fit(_dev(Y), _dev(lab), 150)
    mu, A, psi = [t.cpu().numpy() for t in (mu, A, psi)]
    muo, Bo, Wo = be.plda_fit(Y, lab)
    np.testing.assert_allclose(mu, muo, atol=1e-12)
    np.testing.assert_allclose(A.T @ Wo @ A, np.eye(d), atol=1e-9)
    np.testing.assert_allclose(A.T @ Bo @ A, np.diag(psi), atol=1e-9 * psi.max())
    # trials between held-out vectors: same-class and different-class pairs
    E, elab = _classes(150, 4, d, seed=7, spread=0.8)
    rng = np.random.default_rng(8)
    n = len(E)
    tr = np.stack([rng.integers(0, n, 3000), rng.integers(0, n, 3000)], axis=1).astype(np.int32)
    same = np.stack([np.arange(0, n, 4), np.arange(1, n, 4)], axis=1).astype(np.int32)
    tr = np.concatenate([tr, same])
    s = backend.plda_score((_dev(mu), _dev(A), _dev(psi)), _dev(E), _dev(E), _dev(tr)).cpu().numpy()
    backend.status()
    so = be.plda_llr(E[tr[:, 0]], E[tr[:, 1]], muo, Bo, Wo)
    err = np.max(np.abs(s - so) / (1 + np.abs(so)))
    print(f"PLDA scores: max |ds| / (1 + |s|) = {err:.2e}, score range {so.min():.1f}..{so.max():.1f}")
    assert err <= 2e-5
    # EER from the GPU scores: the library and the oracle agree on the same
    # scores, and the GPU scores give the oracle scores' EER
    from paper_1906_08556_amd import ivx
    tgt = (elab[tr[:, 0]] == elab[tr[:, 1]])
    e_lib = ivx.eer(s, tgt)
    assert abs(e_lib - be.eer(s.astype(np.float64), tgt)) < 1e-12
    assert abs(e_lib - be.eer(so, tgt)) <= 2.0 / tgt.sum()
    print(f"EER {e_lib:.4f} over {tgt.sum()} target / {(~tgt).sum()} non-target trials")


def test_backend_errors(backend):
    from paper_1906_08556_amd import ivx
    X, lab = _classes(5, 10, 8, seed=9)
    bad = lab.copy()
    bad[3] = 7
    with pytest.raises(ivx.IvxError):
        backend.lda(_dev(X), _dev(bad), 5, 2)
    with pytest.raises(ivx.IvxError):          # fewer vectors than dimensions: Sw singular
        backend.lda(_dev(X[:6]), _dev(lab[:6]), 5, 2)
    mu, A, psi = backend.plda_fit(_dev(X), _dev(lab), 5)
    tr = np.array([[0, 1], [2, 99]], np.int32)
    s = backend.plda_score((mu, A, psi), _dev(X), _dev(X), _dev(tr))
    with pytest.raises(ivx.IvxError):
        backend.status()
    assert np.isnan(s.cpu().numpy()[1]) and np.isfinite(s.cpu().numpy()[0])


def _pairs(labels):
    i, j = np.triu_indices(len(labels), k=1)
    return np.stack([i, j], axis=1).astype(np.int32), labels[i] == labels[j]


def test_chain_on_synthetic_speakers_matches_the_oracle_chain(backend):
    """Speaker-labelled utterances drawn from the shape-1 model; i-vectors
    extracted with that model in the standard formulation (T_true, bias mu,
    Sigma = UBM covariances, p = 0) by each side; then centring, whitening
    and length norm with training-speaker statistics, LDA 32 -> 16 and PLDA
    trained on 40 speakers, all pairs of the other 40 speakers scored.  The
    oracle runs the whole chain on its own i-vectors.  Bounds follow the
    extraction tolerance (i-vector cosine >= 0.9999): scores within
    1e-3 (1 + |s|), EER within 3 target trials."""
    import oracle
    import synth
    from _gpu_helpers import dev, make_ctx
    from paper_1906_08556_amd import ivx
    wl, lab = synth.speakers(1, n_spk=80, per_spk=6, lengths="uniform:100:300", rho=0.5)
    R = wl.shape.R
    ctx = make_ctx(wl)
    ctx.set_tv(dev(wl.T_true), dev(wl.cov), dev(np.zeros(R)))
    ctx.set_bias(dev(wl.mu))
    phi = torch.empty((wl.U, R), dtype=torch.float32, device="cuda")
    ctx.extract_ivectors(dev(wl.X), dev(wl.utt_off), phi)
    ctx.sync_status()
    # oracle i-vectors from its own posteriors and centred statistics
    gamma, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    n, f, _ = oracle.bw_stats(wl.X, wl.utt_off, gamma, second_order=False)
    fc = f - n[:, :, None] * wl.mu[None]
    phio = oracle.estep(n, fc, wl.T_true, wl.cov, np.zeros(R), want_cov=False)["phi"]
    g = phi.cpu().numpy()
    cos = np.sum(g * phio, 1) / (np.linalg.norm(g, axis=1) * np.linalg.norm(phio, axis=1))
    assert cos.min() >= 0.9999

    train = lab < 40
    test = ~train
    # GPU chain
    Xtr, Xte = phi[torch.from_numpy(train).cuda()], phi[torch.from_numpy(test).cuda()]
    mean, W = backend.whitening(Xtr.contiguous())
    Ytr = backend.lnorm(Xtr.contiguous(), mean, W)
    Yte = backend.lnorm(Xte.contiguous(), mean, W)
    V, _ = backend.lda(Ytr, _dev(lab[train]), 40, 16)
    Ptr, Pte = backend.project(Ytr, V), backend.project(Yte, V)
    model = backend.plda_fit(Ptr, _dev(lab[train]), 40)
    tr, tgt = _pairs(lab[test])
    s = backend.plda_score(model, Pte, Pte, _dev(tr)).cpu().numpy()
    backend.status()
    # oracle chain
    mo, Wo = be.whitening(phio[train])
    Yo_tr = be.center_lnorm(phio[train], mo, Wo)
    Yo_te = be.center_lnorm(phio[test], mo, Wo)
    Vo, _ = be.lda(Yo_tr, lab[train], 16)
    muo, Bo, Wpo = be.plda_fit(Yo_tr @ Vo, lab[train])
    Pte_o = Yo_te @ Vo
    so = be.plda_llr(Pte_o[tr[:, 0]], Pte_o[tr[:, 1]], muo, Bo, Wpo)
    err = np.max(np.abs(s - so) / (1 + np.abs(so)))
    e_gpu, e_o = ivx.eer(s, tgt), be.eer(so, tgt)
    print(f"chain: max |ds| / (1 + |s|) {err:.2e}; EER gpu {e_gpu:.4f} oracle {e_o:.4f} "
          f"({tgt.sum()} target / {(~tgt).sum()} non-target trials)")
    assert err <= 1e-3
    assert abs(e_gpu - e_o) <= 3.0 / tgt.sum()
    assert e_gpu < 0.25
