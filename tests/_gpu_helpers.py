"""Shared helpers of the GPU parity tests (upload, context set-up, unpacking)."""
import numpy as np
import torch

from paper_1906_08556_amd import ivx


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def make_ctx(wl, max_utts=None, max_frames=None):
    C, D, R = wl.shape.C, wl.shape.D, wl.shape.R
    ctx = ivx.Context(C, D, R, max_utts or max(1, wl.U), max_frames or max(1, wl.F))
    ctx.set_ubm(dev(wl.w), dev(wl.mu), dev(wl.cov))
    return ctx


def packed_upper(M):
    """Row-by-row upper triangle of a symmetric matrix (the ABI's packed layout)."""
    iu = np.triu_indices(M.shape[-1])
    return M[..., iu[0], iu[1]]


def unpack_upper(P, R):
    iu = np.triu_indices(R)
    M = np.zeros(P.shape[:-1] + (R, R), dtype=np.float64)
    M[..., iu[0], iu[1]] = P
    M[..., iu[1], iu[0]] = P
    return M


def unpack_tp(P, R, tb=16):
    """Tile-packed symmetric storage (lower tiles, row-major inside a tile) to full."""
    nb = (R + tb - 1) // tb
    Rp = nb * tb
    M = np.zeros(P.shape[:-1] + (Rp, Rp), dtype=np.float64)
    k = 0
    for bi in range(nb):
        for bj in range(bi + 1):
            blk = P[..., k:k + tb * tb].reshape(P.shape[:-1] + (tb, tb))
            M[..., bi * tb:(bi + 1) * tb, bj * tb:(bj + 1) * tb] = blk
            if bi != bj:
                M[..., bj * tb:(bj + 1) * tb, bi * tb:(bi + 1) * tb] = np.swapaxes(blk, -1, -2)
            k += tb * tb
    return M[..., :R, :R]
