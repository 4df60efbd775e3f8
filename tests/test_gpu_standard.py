"""GPU parity of the standard formulation (Sec. 2.1: mu_c(u) = m_c + T_c omega,
omega ~ N(0, I), statistics centred on m_c, p = 0) against the FP64 oracle:
initialisation, centred statistics, standard minimum divergence with and
without the bias update, extraction, and one full iteration of each of the
four training variants (minimum divergence on/off x Sigma update on/off)
plus the bias-updating one, each iteration seeded with the oracle's state.

Tolerances (derived from the arithmetic of each GPU step):
  * centred f: the terms gamma (x - m_c) are summed in FP32 from FP32
    posteriors; the same bounds as the uncentred statistics (rtol 1e-5,
    atol 1e-4).  Centred S: FP64 sums of FP32 posteriors times exact FP64
    products; |error| <= 2e-7 sum_t gamma |x - m|_i |x - m|_j.
  * minimum divergence: FP64 on both sides from the same accumulators,
    relative <= 1e-9.
  * a full iteration: as for the augmented form, T, Sigma, m relative
    Frobenius <= 1e-4 and the objective relative <= 1e-6.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _gpu_helpers import dev, make_ctx, packed_upper

pytestmark = pytest.mark.gpu


def relfro(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def pack_tp(M, tb=16):
    R = M.shape[-1]
    nb = (R + tb - 1) // tb
    P = np.zeros(M.shape[:-2] + (nb * tb, nb * tb))
    P[..., :R, :R] = M
    tiles = [P[..., bi * tb:(bi + 1) * tb, bj * tb:(bj + 1) * tb].reshape(M.shape[:-2] + (tb * tb,))
             for bi in range(nb) for bj in range(bi + 1)]
    return np.concatenate(tiles, axis=-1)


@pytest.fixture(scope="module")
def std1():
    wl = synth.make(1)
    gamma, _ = oracle.posteriors(oracle.frame_loglik(wl.X, wl.w, wl.mu, wl.cov))
    n, f, S = oracle.bw_stats(wl.X, wl.utt_off, gamma)
    tv = oracle.init_tv_standard(wl.mu, wl.cov, wl.T_init)
    return wl, gamma, (n, f, S), tv


def _std_ctx(wl, T, Sigma, m):
    ctx = make_ctx(wl)
    ctx.set_tv(dev(T), dev(Sigma), dev(np.zeros(wl.shape.R)))
    ctx.set_bias(dev(m))
    return ctx


def test_init_tv_standard_matches_oracle():
    wl = synth.make(1, n_utts=4)
    ctx = make_ctx(wl)
    ctx.init_tv_standard(dev(wl.T_init))
    Tg, Sg, pg, _ = [t.cpu().numpy() for t in ctx.get_tv()]
    mg = ctx.get_bias().cpu().numpy()
    T0, S0, p0, m0 = oracle.init_tv_standard(wl.mu, wl.cov, wl.T_init)
    np.testing.assert_array_equal(Tg, T0)
    np.testing.assert_array_equal(Sg, S0)
    np.testing.assert_array_equal(pg, p0)
    np.testing.assert_array_equal(mg, m0)


def test_centred_statistics_match_oracle(std1):
    wl, gamma, (n_ref, f_ref, S_ref), tv = std1
    rng = np.random.default_rng(5)
    m = wl.mu + 0.3 * rng.standard_normal(wl.mu.shape)   # a bias other than the UBM means
    ctx = _std_ctx(wl, tv[0], tv[1], m)
    U, C, D = wl.U, wl.shape.C, wl.shape.D
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    S = torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device="cuda")
    ctx.bw_stats(dev(wl.X), dev(wl.utt_off), n, f, S_acc=S)
    ctx.sync_status()
    fc_ref, Sc_ref = oracle.center_stats(n_ref, f_ref, S_ref, m)
    n, f, S = n.cpu().numpy(), f.cpu().numpy(), S.cpu().numpy()
    np.testing.assert_allclose(n, n_ref, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(f, fc_ref, rtol=1e-5, atol=1e-4)
    X = wl.X.astype(np.float64)
    S_abs = np.stack([(gamma[:, c:c + 1] * np.abs(X - m[c])).T @ np.abs(X - m[c])
                      for c in range(C)])
    ratio = np.max(np.abs(S - packed_upper(Sc_ref)) / (2e-7 * packed_upper(S_abs) + 1e-9))
    print("centred S error / bound", ratio)
    assert ratio <= 1.0
    # the same context returns to uncentred statistics without a bias
    ctx.set_bias(None)
    S2 = torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device="cuda")
    f2 = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    n2 = torch.empty((U, C), dtype=torch.float32, device="cuda")
    ctx.bw_stats(dev(wl.X), dev(wl.utt_off), n2, f2, S_acc=S2)
    ctx.sync_status()
    np.testing.assert_allclose(f2.cpu().numpy(), f_ref, rtol=1e-5, atol=1e-4)


@pytest.mark.parametrize("update_mean", [False, True])
def test_standard_mindiv_matches_oracle(std1, update_mean):
    wl, gamma, (n, f, S), tv = std1
    T, Sigma, p, m = tv
    fc, _ = oracle.center_stats(n, f, S, m)
    e = oracle.estep(n, fc, T, Sigma, p)
    ref = oracle.accumulate(n, fc, e["phi"], e["Phi"])
    ctx = _std_ctx(wl, T, Sigma, m)
    acc = ctx.new_accum()
    acc.h.copy_(dev(ref["hsum"]))
    acc.H.copy_(dev(pack_tp(ref["Hsum"])))
    acc.count.fill_(float(ref["count"]))
    if update_mean:
        ctx.tv_mindiv_standard(acc, update_mean=True)
    else:
        ctx.tv_mindiv(acc)       # the standard context's re-estimation: P1 only
    ctx.sync_status()
    T1, m1 = oracle.mindiv_standard(ref["hsum"] / ref["count"], ref["Hsum"] / ref["count"], T, m,
                                    update_mean=update_mean)
    Tg, _, pg, _ = [t.cpu().numpy() for t in ctx.get_tv()]
    mg = ctx.get_bias().cpu().numpy()
    assert relfro(Tg, T1) <= 1e-9
    assert relfro(mg, m1) <= 1e-9
    assert np.all(pg == 0.0)


def _gpu_iteration(ctx, wl, X, off, update_sigma, mindiv, update_mean):
    U, C, D, R = wl.U, wl.shape.C, wl.shape.D, wl.shape.R
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    S = torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device="cuda")
    ctx.bw_stats(X, off, n, f, S_acc=S)
    phi = torch.empty((U, R), dtype=torch.float32, device="cuda")
    Phi = torch.empty((U, R * (R + 1) // 2), dtype=torch.float32, device="cuda")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tv_estep(n, f, phi, Phi=Phi, ll_acc=ll)
    acc = ctx.new_accum()
    ctx.tv_mstep_accumulate(n, f, phi, Phi, acc)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tv_mstep_solve(acc, S, update_sigma=update_sigma, ll_sum=ll, objective=obj)
    if mindiv:
        ctx.tv_mindiv_standard(acc, update_mean=update_mean)
    ctx.sync_status()
    return obj.item()


VARIANTS = [(True, True, False), (True, False, False), (False, True, False),
            (False, False, False), (True, True, True)]


@pytest.mark.parametrize("update_sigma,mindiv,update_mean", VARIANTS,
                         ids=["sigma-mindiv", "sigma", "mindiv", "plain", "sigma-mindiv-mean"])
def test_standard_iterations_match_oracle(std1, update_sigma, mindiv, update_mean):
    """Each GPU iteration starts from the oracle's state (T, Sigma, m) and is
    compared with the oracle's iteration from that state."""
    wl, gamma, stats, tv = std1
    ubm = (wl.w, wl.mu, wl.cov)
    X, off = dev(wl.X), dev(wl.utt_off)
    T, Sigma, p, m = tv
    ctx = make_ctx(wl)
    for it in range(2):
        ctx.set_tv(dev(T), dev(Sigma), dev(p))
        ctx.set_bias(dev(m))
        obj = _gpu_iteration(ctx, wl, X, off, update_sigma, mindiv, update_mean)
        r = oracle.em_iteration_standard(wl.X, wl.utt_off, ubm, (T, Sigma, p, m),
                                         update_sigma=update_sigma, mindiv=mindiv,
                                         update_mean=update_mean, stats=stats)
        Tg, Sg, pg, _ = [t.cpu().numpy() for t in ctx.get_tv()]
        mg = ctx.get_bias().cpu().numpy()
        print(f"iter {it}: obj gpu {obj:.6f} oracle {r['objective']:.6f}  T relfro "
              f"{relfro(Tg, r['T']):.2e}  Sigma relfro {relfro(Sg, r['Sigma']):.2e}  "
              f"m relfro {relfro(mg, r['m']):.2e}")
        assert abs(obj - r["objective"]) <= 1e-6 * abs(r["objective"])
        assert relfro(Tg, r["T"]) <= 1e-4
        assert relfro(Sg, r["Sigma"]) <= 1e-4
        assert relfro(mg, r["m"]) <= 1e-4
        assert np.all(pg == 0.0)
        T, Sigma, m = r["T"], r["Sigma"], r["m"]


def test_standard_extract_matches_oracle(std1):
    wl, gamma, (n, f, S), tv = std1
    T, Sigma, p, m = tv
    ctx = _std_ctx(wl, T, Sigma, m)
    phi = torch.empty((wl.U, wl.shape.R), dtype=torch.float32, device="cuda")
    ctx.extract_ivectors(dev(wl.X), dev(wl.utt_off), phi)
    ctx.sync_status()
    fc, _ = oracle.center_stats(n, f, S, m)
    ref = oracle.estep(n, fc, T, Sigma, p, want_cov=False)["phi"]
    a = phi.cpu().numpy()
    cos = np.sum(a * ref, 1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(ref, axis=1))
    print("extract min cosine", cos.min())
    assert cos.min() >= 0.9999


def test_formulation_guards():
    from paper_1906_08556_amd import ivx
    wl = synth.make(1, n_utts=4)
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init), 100.0)               # augmented
    with pytest.raises(ivx.IvxError):
        ctx.get_bias()
    with pytest.raises(ivx.IvxError):
        ctx.tv_mindiv_standard(ctx.new_accum())
    ctx.init_tv_standard(dev(wl.T_init))              # standard
    with pytest.raises(ivx.IvxError):
        ctx.ubm_update_means()
    with pytest.raises(ivx.IvxError):
        ctx.tv_mindiv_standard(ctx.new_accum(), method=1)
    ctx.init_tv(dev(wl.T_init), 100.0)               # back to augmented
    with pytest.raises(ivx.IvxError):
        ctx.get_bias()


def test_graph_replays_the_standard_iteration():
    """A graph captured on a standard context centres the statistics and
    applies the standard re-estimation; each replay matches the eager
    iteration from the same state (bounds as for the augmented graph)."""
    from paper_1906_08556_amd import ivx
    wl = synth.make(1)
    U, C, D, R = wl.U, wl.shape.C, wl.shape.D, wl.shape.R
    X, off = dev(wl.X), dev(wl.utt_off)
    cg, ce = make_ctx(wl), make_ctx(wl)
    cg.init_tv_standard(dev(wl.T_init))
    z = lambda *s, dt=torch.float32: torch.full(s, float("nan"), dtype=dt, device="cuda")
    b = dict(n=z(U, C), f=z(U, C, D), S=z(C, D * (D + 1) // 2, dt=torch.float64), phi=z(U, R),
             Phi=z(U, R * (R + 1) // 2), llf=z(1, dt=torch.float64), llu=z(1, dt=torch.float64),
             obj=z(1, dt=torch.float64))
    acc = cg.new_accum()
    with pytest.raises(ivx.IvxError):
        cg.graph_create_em(X, off, b["n"], b["f"], b["S"], b["phi"], b["Phi"], acc, b["llf"],
                           b["llu"], b["obj"], update_sigma=True, realign=True)
    g = cg.graph_create_em(X, off, b["n"], b["f"], b["S"], b["phi"], b["Phi"], acc, b["llf"],
                           b["llu"], b["obj"], update_sigma=True, realign=False)
    for it in range(3):
        T, Sigma, p, _ = cg.get_tv()
        ce.set_tv(T, Sigma, p)
        ce.set_bias(cg.get_bias())
        obj_e = _gpu_iteration(ce, wl, X, off, True, True, False)
        g.launch()
        cg.sync_status()
        Te, Se, _, _ = [t.cpu().numpy() for t in ce.get_tv()]
        Tg, Sg, pg, _ = [t.cpu().numpy() for t in cg.get_tv()]
        obj_g = b["obj"].item()
        print(f"replay {it}: obj graph {obj_g:.9f} eager {obj_e:.9f}  T {relfro(Tg, Te):.2e}  "
              f"Sigma {relfro(Sg, Se):.2e}")
        assert abs(obj_g - obj_e) <= 1e-7 * abs(obj_e)
        assert relfro(Tg, Te) <= 1e-5
        assert relfro(Sg, Se) <= 1e-5
        assert np.all(pg == 0.0)
        np.testing.assert_array_equal(cg.get_bias().cpu().numpy(), wl.mu)
    g.close()
