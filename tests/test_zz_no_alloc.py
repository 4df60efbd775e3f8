"""ubm_posteriors_static (the frame-posterior entry point whose workspace is
the library's fixed per-device array) against ubm_posteriors on the same
context and inputs: two calls in a row, the second on fewer frames, so the
second call runs on the array as the first left it.  Posterior lists are
integer decisions taken by the same kernels in the same precision and must be
identical; posterior values and frame log-likelihoods come from the same
FP64 arithmetic and must agree to 1e-12."""
import numpy as np
import pytest
import torch

import synth
from _gpu_helpers import dev, make_ctx

pytestmark = pytest.mark.gpu


def _lists(F):
    return (torch.full((F, 16), -7, dtype=torch.int32, device="cuda"),
            torch.full((F, 16), float("nan"), dtype=torch.float32, device="cuda"),
            torch.full((F,), float("nan"), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_static_workspace_posteriors_match_the_context_entry_point(prec):
    wl = synth.make(2, n_utts=24)
    ctx = make_ctx(wl)
    # two calls in a row: the full batch, then a smaller one (ragged tail)
    for F in (wl.F, wl.F // 3 + 17):
        X = dev(wl.X[:F])
        pa, va, la = _lists(F)
        pb, vb, lb = _lists(F)
        ctx.ubm_posteriors(X, post_idx=pa, post_val=va, frame_ll=la, prec=prec)
        ctx.ubm_posteriors_static(X, pb, vb, frame_ll=lb, prec=prec)
        ctx.sync_status()
        pa, va, la = pa.cpu().numpy(), va.cpu().numpy(), la.cpu().numpy()
        pb, vb, lb = pb.cpu().numpy(), vb.cpu().numpy(), lb.cpu().numpy()
        print(f"F={F}: lists equal {np.array_equal(pa, pb)}, max |dval| "
              f"{np.abs(va - vb).max():.2e}, max |dll| {np.abs(la - lb).max():.2e}")
        np.testing.assert_array_equal(pa, pb)
        np.testing.assert_allclose(vb, va, rtol=0, atol=1e-12)
        np.testing.assert_allclose(lb, la, rtol=1e-12, atol=0)
        assert np.isfinite(vb).all() and (pb >= -1).all()


def test_static_workspace_refuses_batches_beyond_the_array():
    from paper_1906_08556_amd import ivx
    wl = synth.make(1, n_utts=2)
    ctx = make_ctx(wl)
    limit = ivx.load().ivx_static_bytes()
    F = limit // 392 + 1024     # more frames than the array holds
    X = torch.empty((F, wl.shape.D), dtype=torch.float32, device="cuda")
    pi = torch.empty((F, 16), dtype=torch.int32, device="cuda")
    pv = torch.empty((F, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(ivx.IvxError, match="static workspace"):
        ctx.ubm_posteriors_static(X, pi, pv)
