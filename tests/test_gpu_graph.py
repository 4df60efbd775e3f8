"""The captured EM iteration (one HIP graph per iteration) against the eager
sequence of calls.

Each replay starts from a state that the eager side copies first (T, Sigma,
p, UBM means), so the two run the same kernels on the same inputs.  The only
difference between them is the order of LDS float atomics in the n/f
accumulation, which perturbs n and f at FP32 rounding; through the E-step
(cond(L) up to ~2e4) and the M-step this gives T, Sigma and mu relative
differences far below 1e-5 and objective differences below 1e-7 relative.
Between replays the program does its own eager work and synchronises, and
every replay is checked.
"""
import numpy as np
import pytest
import torch

import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu


def relfro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _eager_iteration(ctx, wl, X, off, realign):
    U, C, D, R = wl.U, wl.shape.C, wl.shape.D, wl.shape.R
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    S = torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device="cuda")
    llf = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.bw_stats(X, off, n, f, S_acc=S, ll_acc=llf)
    phi = torch.empty((U, R), dtype=torch.float32, device="cuda")
    Phi = torch.empty((U, R * (R + 1) // 2), dtype=torch.float32, device="cuda")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tv_estep(n, f, phi, Phi=Phi, ll_acc=ll)
    acc = ctx.new_accum()
    ctx.tv_mstep_accumulate(n, f, phi, Phi, acc)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tv_mstep_solve(acc, S, update_sigma=True, ll_sum=ll, objective=obj)
    ctx.tv_mindiv(acc)
    if realign:
        ctx.ubm_update_means()
    ctx.sync_status()
    return obj.item(), llf.item(), phi


def _graph_buffers(wl):
    U, C, D, R = wl.U, wl.shape.C, wl.shape.D, wl.shape.R
    z = lambda *s, dt=torch.float32: torch.full(s, float("nan"), dtype=dt, device="cuda")
    return dict(n=z(U, C), f=z(U, C, D), S=z(C, D * (D + 1) // 2, dt=torch.float64),
                phi=z(U, R), Phi=z(U, R * (R + 1) // 2), ll_frames=z(1, dt=torch.float64),
                ll_utts=z(1, dt=torch.float64), objective=z(1, dt=torch.float64))


@pytest.mark.parametrize("realign", [True, False])
def test_graph_replays_match_the_eager_iteration(realign):
    wl = synth.make(1)
    X, off = dev(wl.X), dev(wl.utt_off)
    cg, ce = make_ctx(wl), make_ctx(wl)
    cg.init_tv(dev(wl.T_init))
    acc = cg.new_accum()
    # stale values everywhere: the graph must clear what it accumulates
    for t in (acc.A, acc.Cc, acc.N, acc.h, acc.H, acc.count):
        t.fill_(1e30)
    b = _graph_buffers(wl)
    g = cg.graph_create_em(X, off, b["n"], b["f"], b["S"], b["phi"], b["Phi"], acc,
                           b["ll_frames"], b["ll_utts"], b["objective"], update_sigma=True,
                           realign=realign)
    torch.cuda.synchronize()
    # capture executes nothing
    assert torch.isnan(b["objective"]).all()
    for it in range(4):
        T, Sigma, p, mu = cg.get_tv()
        ce.set_ubm(dev(wl.w), mu, dev(wl.cov))
        ce.set_tv(T, Sigma, p)
        obj_e, llf_e, phi_e = _eager_iteration(ce, wl, X, off, realign)
        _ = (phi_e * 2.0).sum().item()  # unrelated eager work between replays
        g.launch()
        cg.sync_status()
        torch.cuda.synchronize()
        Te, Se, pe, mue = [t.cpu().numpy() for t in ce.get_tv()]
        Tg, Sg, pg, mug = [t.cpu().numpy() for t in cg.get_tv()]
        obj_g, llf_g = b["objective"].item(), b["ll_frames"].item()
        phi_g = b["phi"].cpu().numpy()
        print(f"replay {it}: obj graph {obj_g:.9f} eager {obj_e:.9f}  T {relfro(Tg, Te):.2e}  "
              f"Sigma {relfro(Sg, Se):.2e}  mu {relfro(mug, mue):.2e}  "
              f"phi {relfro(phi_g, phi_e.cpu().numpy()):.2e}")
        assert abs(obj_g - obj_e) <= 1e-7 * abs(obj_e)
        assert abs(llf_g - llf_e) <= 1e-9 * abs(llf_e)
        assert relfro(Tg, Te) <= 1e-5
        assert relfro(Sg, Se) <= 1e-5
        assert abs(pg[0] - pe[0]) <= 1e-6 * abs(pe[0])
        assert relfro(mug, mue) <= 1e-5
        assert relfro(phi_g, phi_e.cpu().numpy()) <= 1e-4
        if not realign:
            assert np.array_equal(mug, wl.mu)
    g.close()


def test_graph_on_bf16_path_matches_eager_bf16():
    from paper_1906_08556_amd import ivx
    wl = synth.make(1)
    X, off = dev(wl.X), dev(wl.utt_off)
    cg = make_ctx(wl)
    cg.init_tv(dev(wl.T_init))
    acc = cg.new_accum()
    b = _graph_buffers(wl)
    g = cg.graph_create_em(X, off, b["n"], b["f"], b["S"], b["phi"], b["Phi"], acc,
                           b["ll_frames"], b["ll_utts"], b["objective"], prec=ivx.IVX_BF16)
    ce = make_ctx(wl)
    T, Sigma, p, _ = cg.get_tv()
    ce.set_tv(T, Sigma, p)
    U, C, D = wl.U, wl.shape.C, wl.shape.D
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    ce.bw_stats(X, off, n, f, prec=ivx.IVX_BF16)
    g.launch()
    cg.sync_status()
    ce.sync_status()
    dn = (b["n"] - n).abs().max().item()
    print("bf16 graph vs eager max |dn|", dn)
    assert dn <= 1e-5
    g.close()
