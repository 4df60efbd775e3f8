"""The autotuner and the launch shapes it chooses between.

Every launch shape computes the same posteriors: the candidate lists keep
every component within the margin of the frame's final best score whatever
the number of components per launch, and the exact FP64 rescoring is shared,
so the posterior lists agree exactly, and n and f (exact fixed-point sums of
the same posteriors) are identical; the split linear-term GEMM changes
the FP32 summation order of b(u) (i-vectors <= 1e-4 relative, cond(L) ~1e4).
"""
import numpy as np
import pytest
import torch

import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_1906_08556_amd import ivx
    wl = synth.make(2, n_utts=30)
    ctx = make_ctx(wl)
    ctx.init_tv(dev(wl.T_init))
    X, off = dev(wl.X), dev(wl.utt_off)
    return ivx, wl, ctx, X, off


def _run(ctx, wl, X, off, prec):
    U, C, D, R = wl.U, wl.shape.C, wl.shape.D, wl.shape.R
    pi = torch.empty((wl.F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((wl.F, 16), dtype=torch.float32, device="cuda")
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv, prec=prec)
    n = torch.empty((U, C), dtype=torch.float32, device="cuda")
    f = torch.empty((U, C, D), dtype=torch.float32, device="cuda")
    ctx.bw_stats(X, off, n, f, prec=prec)
    phi = torch.empty((U, R), dtype=torch.float32, device="cuda")
    ctx.tv_estep(n, f, phi, prec=prec)
    ctx.sync_status()
    return [t.cpu().numpy() for t in (pi, pv, n, f, phi)]


def test_autotune_returns_a_valid_tuning(setup):
    ivx, wl, ctx, X, off = setup
    t = ctx.autotune(X, off)
    print("tuning", t)
    assert t["frame_ncb"] in (2, 4, 8) and t["frame_ncb_bf16"] in (2, 4, 8)
    assert t["b_split"] >= 1
    assert ctx.tuning_get() == t


@pytest.mark.parametrize("prec", [0, 1])
def test_every_launch_shape_gives_the_same_results(setup, prec):
    ivx, wl, ctx, X, off = setup
    ctx.tuning_set(frame_ncb=8, frame_ncb_bf16=8, b_split=0, frame_direct=0, mstep_left=0)
    ref = _run(ctx, wl, X, off, prec)
    for kw in (dict(frame_ncb=4, frame_ncb_bf16=4), dict(frame_ncb=2, frame_ncb_bf16=2),
               dict(frame_ncb=8, frame_direct=1), dict(frame_ncb=4, frame_direct=1),
               dict(b_split=1), dict(b_split=16)):
        ctx.tuning_set(**kw)
        out = _run(ctx, wl, X, off, prec)
        np.testing.assert_array_equal(out[0], ref[0])
        np.testing.assert_array_equal(out[1], ref[1])
        np.testing.assert_array_equal(out[2], ref[2])
        np.testing.assert_array_equal(out[3], ref[3])
        rel = np.linalg.norm(out[4] - ref[4]) / np.linalg.norm(ref[4])
        print(kw, "phi rel", rel)
        assert rel <= 1e-4
        ctx.tuning_set(frame_ncb=8, frame_ncb_bf16=8, b_split=0, frame_direct=0, mstep_left=0)


def test_tuning_set_rejects_unknown_shapes(setup):
    ivx, wl, ctx, X, off = setup
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.tuning_set(frame_ncb=6)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.tuning_set(b_split=4096)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.tuning_set(frame_direct=2)
    with pytest.raises(ivx.IvxError, match="EINVAL"):
        ctx.tuning_set(mstep_left=2)

