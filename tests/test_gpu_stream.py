"""The streaming host pipeline (Sec. 4.2, Fig. 1) on the GPU: a pass over
host-resident utterances in ragged fixed-size batches against the same calls
on the whole set resident in HBM, and an iteration from the streamed
accumulators against the FP64 oracle.

Tolerances: each batch runs the very kernels of the resident pass on the
same utterances, so per-utterance n, f and i-vectors agree to FP32 rounding
(LDS atomics and split-K sums reorder; relative <= 1e-5); accumulators and S
are FP64 sums over the same terms in another order (relative <= 1e-9 for S,
which sums exact products of the same FP32 posteriors; <= 1e-7 for N, whose
terms n_c(u) come from LDS float atomics in a run-dependent order; <= 1e-6
for A, Cc, h, H, which sum FP32 products of the reordered E-step).  The
M-step from the streamed accumulators is held to the full-iteration bounds
of the resident path: T, Sigma relative Frobenius <= 1e-4, objective <= 1e-6.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu


def relfro(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def wl1():
    return synth.make(1)


def _buffers(ctx, U):
    C, D, R = ctx.C, ctx.D, ctx.R
    return dict(S=torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device="cuda"),
                llf=torch.zeros(1, dtype=torch.float64, device="cuda"),
                llu=torch.zeros(1, dtype=torch.float64, device="cuda"),
                phi=torch.zeros((U, R), dtype=torch.float32, device="cuda"),
                acc=ctx.new_accum())


def _resident_pass(ctx, wl):
    from paper_1906_08556_amd import ivx  # noqa: F401
    U, C, D, R = wl.U, ctx.C, ctx.D, ctx.R
    b = _buffers(ctx, U)
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    Phi = torch.empty((U, R * (R + 1) // 2), dtype=torch.float32, device="cuda")
    ctx.bw_stats(dev(wl.X), dev(wl.utt_off), n, f, S_acc=b["S"], ll_acc=b["llf"])
    ctx.tv_estep(n, f, b["phi"], Phi=Phi, ll_acc=b["llu"])
    ctx.tv_mstep_accumulate(n, f, b["phi"], Phi, b["acc"])
    ctx.sync_status()
    return b


def _compare(bs, br):
    assert relfro(bs["S"].cpu(), br["S"].cpu()) <= 1e-9
    assert abs(bs["llf"].item() - br["llf"].item()) <= 1e-9 * abs(br["llf"].item())
    assert abs(bs["llu"].item() - br["llu"].item()) <= 1e-6 * abs(br["llu"].item())
    a, r = bs["acc"], br["acc"]
    assert relfro(a.N.cpu(), r.N.cpu()) <= 1e-7
    assert a.count.item() == r.count.item()
    for name in ("A", "Cc", "h", "H"):
        e = relfro(getattr(a, name).cpu(), getattr(r, name).cpu())
        print(f"  {name} relfro {e:.2e}")
        assert e <= 1e-6
    e = relfro(bs["phi"].cpu(), br["phi"].cpu())
    print(f"  phi relfro {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("max_utts,max_frames,loaders,slots",
                         [(37, 6000, 3, 2), (200, 10_000, 1, 4), (1, 300, 6, 3)])
def test_streamed_pass_equals_the_resident_pass(wl1, max_utts, max_frames, loaders, slots):
    from paper_1906_08556_amd import ivx
    wl = wl1
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init), 100.0)
    br = _resident_pass(ctx, wl)
    starts = ivx.plan_batches(wl.utt_off, max_utts, max_frames)
    print(f"batches {len(starts) - 1} (max {max_utts} utterances / {max_frames} frames)")
    st = ivx.Stream(ctx, max_utts, max_frames, loaders=loaders, slots=slots)
    bs = _buffers(ctx, wl.U)
    st.em_pass(wl.utt_off, bs["acc"], X=wl.X, S_acc=bs["S"], ll_frames=bs["llf"],
               ll_utts=bs["llu"], phi_out=bs["phi"])
    ctx.sync_status()
    _compare(bs, br)
    st.close()


def test_back_to_back_passes_wait_for_the_previous_pass(wl1):
    """A pass returns while the GPU still computes its last batches; passes
    issued back to back (and on another stream) must not overwrite device
    buffers those batches still read."""
    from paper_1906_08556_amd import ivx
    wl = wl1
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init), 100.0)
    br = _resident_pass(ctx, wl)
    st = ivx.Stream(ctx, 37, 6000, loaders=3, slots=2)
    outs = [_buffers(ctx, wl.U) for _ in range(3)]
    side = torch.cuda.Stream()
    for i, b in enumerate(outs):
        s = side if i == 1 else None
        st.em_pass(wl.utt_off, b["acc"], X=wl.X, S_acc=b["S"], ll_frames=b["llf"],
                   ll_utts=b["llu"], phi_out=b["phi"], stream=s)
    phi_x = torch.zeros((wl.U, ctx.R), dtype=torch.float32, device="cuda")
    st.extract(wl.utt_off, phi_x, X=wl.X, stream=side)
    torch.cuda.synchronize()
    ctx.sync_status()
    for b in outs:
        _compare(b, br)
    assert relfro(phi_x.cpu(), br["phi"].cpu()) <= 1e-5
    st.close()


def test_streamed_iteration_matches_the_oracle(wl1):
    """A context sized for 50 utterances / 12k frames trains on all 200
    utterances (~40k frames) through the stream; the M-step, minimum
    divergence and realignment then run on the streamed accumulators."""
    from paper_1906_08556_amd import ivx
    wl = wl1
    ctx = make_ctx(wl, max_utts=50, max_frames=12_000)
    tv = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    ubm = (wl.w, wl.mu, wl.cov)
    st = ivx.Stream(ctx, 50, 12_000, loaders=4, slots=3)
    for it in range(2):
        ctx.set_ubm(dev(ubm[0]), dev(ubm[1]), dev(ubm[2]))
        ctx.set_tv(dev(tv[0]), dev(tv[1]), dev(tv[2]))
        b = _buffers(ctx, wl.U)
        st.em_pass(wl.utt_off, b["acc"], X=wl.X, S_acc=b["S"], ll_frames=b["llf"],
                   ll_utts=b["llu"])
        obj = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.tv_mstep_solve(b["acc"], b["S"], update_sigma=True, ll_sum=b["llu"], objective=obj)
        ctx.tv_mindiv(b["acc"])
        ctx.ubm_update_means()
        ctx.sync_status()
        r = oracle.em_iteration(wl.X, wl.utt_off, ubm, tv, realign=True)
        Tg, Sg, pg, mug = [t.cpu().numpy() for t in ctx.get_tv()]
        print(f"iter {it}: obj {obj.item():.6f} oracle {r['objective']:.6f} T {relfro(Tg, r['T']):.2e} "
              f"Sigma {relfro(Sg, r['Sigma']):.2e} mu {relfro(mug, r['mu']):.2e}")
        assert abs(obj.item() - r["objective"]) <= 1e-6 * abs(r["objective"])
        assert relfro(Tg, r["T"]) <= 1e-4
        assert relfro(Sg, r["Sigma"]) <= 1e-4
        assert relfro(mug, r["mu"]) <= 1e-4
        tv = (r["T"], r["Sigma"], r["p"])
        ubm = (wl.w, r["mu"], wl.cov)
    st.close()


def test_streamed_extraction_and_frame_source(wl1):
    """Extraction through the stream equals extract_ivectors on the resident
    set; a frame source that generates the same frames on demand gives the
    same accumulators as the host array."""
    from paper_1906_08556_amd import ivx
    wl = wl1
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init), 100.0)
    phi_r = torch.zeros((wl.U, ctx.R), dtype=torch.float32, device="cuda")
    ctx.extract_ivectors(dev(wl.X), dev(wl.utt_off), phi_r)
    st = ivx.Stream(ctx, 23, 5000, loaders=4, slots=4)
    phi_s = torch.zeros_like(phi_r)
    st.extract(wl.utt_off, phi_s, X=wl.X)
    ctx.sync_status()
    e = relfro(phi_s.cpu(), phi_r.cpu())
    print("extract relfro", e)
    assert e <= 1e-5

    def source(u0, u1, out):
        out[:] = wl.X[wl.utt_off[u0]:wl.utt_off[u1]]

    ba, bb = _buffers(ctx, wl.U), _buffers(ctx, wl.U)
    st.em_pass(wl.utt_off, ba["acc"], X=wl.X, S_acc=ba["S"], ll_frames=ba["llf"],
               ll_utts=ba["llu"], phi_out=ba["phi"])
    st.em_pass(wl.utt_off, bb["acc"], source=source, S_acc=bb["S"], ll_frames=bb["llf"],
               ll_utts=bb["llu"], phi_out=bb["phi"])
    ctx.sync_status()
    _compare(bb, ba)
    st.close()


def test_stream_errors_are_reported():
    from paper_1906_08556_amd import ivx
    wl = synth.make(1, n_utts=20)
    ctx = make_ctx(wl, max_utts=10, max_frames=2000)
    ctx.init_tv(dev(wl.T_init), 100.0)
    with pytest.raises(ivx.IvxError):            # beyond the context's limits
        ivx.Stream(ctx, 11, 2000)
    with pytest.raises(ivx.IvxError):
        ivx.Stream(ctx, 10, 2000, slots=1)
    st = ivx.Stream(ctx, 10, 250, loaders=2, slots=2)
    acc = ctx.new_accum()
    too_long = int(np.max(np.diff(wl.utt_off))) > 250
    assert too_long
    with pytest.raises(ivx.IvxError):            # an utterance longer than a batch
        st.em_pass(wl.utt_off, acc, X=wl.X)
    st.close()
    st = ivx.Stream(ctx, 10, 2000, loaders=3, slots=2)
    calls = []

    def failing(u0, u1, out):
        calls.append(u0)
        if u0 > 0:
            raise RuntimeError("source failure")
        out[:] = wl.X[wl.utt_off[u0]:wl.utt_off[u1]]

    with pytest.raises(ivx.IvxError):
        st.em_pass(wl.utt_off, acc, source=failing)
    with pytest.raises(ivx.IvxError):            # both X and a source
        st.em_pass(wl.utt_off, acc, X=wl.X, source=failing)
    ctx.sync_status()
    st.close()
