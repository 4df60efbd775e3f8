"""ctypes binding of libivx.so (argument marshalling only).

Every entry point of include/ivx.h has a method of the same name here.
Tensors are torch tensors on the context's device; the binding checks dtype,
device and contiguity, passes raw pointers and the current HIP stream, and
raises IvxError on a non-zero status.  No arithmetic of the method happens
here: if libivx.so is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libivx.so")

IVX_FP32, IVX_BF16 = 0, 1
IVX_SEL_ALL, IVX_SEL_LEARNED, IVX_SEL_PRUNED = 0, 1, 2
KP = 16  # posterior list capacity per frame

STATUS = {0: "IVX_OK", -1: "IVX_EINVAL", -2: "IVX_ENOMEM", -3: "IVX_ENOTPD", -4: "IVX_EDEVICE",
          -5: "IVX_ENUMERIC", -6: "IVX_ECAPACITY"}


class IvxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("D", ctypes.c_int32), ("R", ctypes.c_int32),
                ("max_batch_utts", ctypes.c_int32), ("max_batch_frames", ctypes.c_int64)]


class SelectorDims(ctypes.Structure):
    _fields_ = [("H1", ctypes.c_int32), ("H2", ctypes.c_int32), ("k", ctypes.c_int32),
                ("min_mass", ctypes.c_float), ("max_train_batch", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("frame_ncb", ctypes.c_int32), ("frame_ncb_bf16", ctypes.c_int32),
                ("b_split", ctypes.c_int32), ("frame_direct", ctypes.c_int32),
                ("mstep_left", ctypes.c_int32),
                ("estep_global", ctypes.c_int32), ("mstep_global", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Accum(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("Cc", ctypes.c_void_p), ("N", ctypes.c_void_p),
                ("h", ctypes.c_void_p), ("H", ctypes.c_void_p), ("count", ctypes.c_void_p)]


class StreamConfig(ctypes.Structure):
    _fields_ = [("max_batch_utts", ctypes.c_int32), ("max_batch_frames", ctypes.c_int64),
                ("loaders", ctypes.c_int32), ("slots", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32, _I64, _F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
# int32 (void* user, int64 u0, int64 u1, const int64* utt_off, float* X_dst)
FrameSource = ctypes.CFUNCTYPE(ctypes.c_int32, _P, _I64, _I64, ctypes.POINTER(_I64), _P)

# name -> (restype, argtypes)
PROTOTYPES = {
    "ivx_create": (_I32, [ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(_P)]),
    "ivx_destroy": (None, [_P]),
    "ivx_last_error": (ctypes.c_char_p, []),
    "ivx_sync_status": (_I32, [_P, _P]),
    "ivx_tp_size": (_I64, [_I32]),
    "ivx_set_ubm": (_I32, [_P, _P, _P, _P, _P]),
    "ivx_init_tv": (_I32, [_P, _P, _F64, _P]),
    "ivx_init_tv_standard": (_I32, [_P, _P, _P]),
    "ivx_set_bias": (_I32, [_P, _P, _P]),
    "ivx_get_bias": (_I32, [_P, _P, _P]),
    "ivx_set_tv": (_I32, [_P, _P, _P, _P, _P]),
    "ivx_get_tv": (_I32, [_P, _P, _P, _P, _P, _P]),
    "ubm_posteriors": (_I32, [_P, _P, _I64, _I32, _I32, _P, _P, _P, _I32, _P, _P]),
    "ubm_posteriors_static": (_I32, [_P, _P, _I64, _I32, _P, _P, _I32, _P, _P]),
    "ivx_static_bytes": (_I64, []),
    "bw_stats": (_I32, [_P, _P, _P, _I64, _I64, _I32, _I32, _P, _P, _P, _P, _P]),
    "tv_estep": (_I32, [_P, _P, _P, _I64, _I32, _P, _P, _P, _P, _P]),
    "tv_mstep_accumulate": (_I32, [_P, _P, _P, _P, _P, _I64, ctypes.POINTER(Accum), _P]),
    "extract_ivectors": (_I32, [_P, _P, _P, _I64, _I64, _I32, _I32, _P, _P]),
    "tv_mstep_solve": (_I32, [_P, ctypes.POINTER(Accum), _P, ctypes.c_int, _P, _P, _P, _P]),
    "tv_mindiv": (_I32, [_P, ctypes.POINTER(Accum), ctypes.c_int, _P]),
    "tv_mindiv_standard": (_I32, [_P, ctypes.POINTER(Accum), ctypes.c_int, ctypes.c_int, _P]),
    "ubm_update_means": (_I32, [_P, _P]),
    "ivx_graph_create_em": (_I32, [_P, _P, _P, _I64, _I64, _I32, _P, _P, _P, _P, _P,
                                   ctypes.POINTER(Accum), _P, _P, _P, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(_P)]),
    "ivx_graph_launch": (_I32, [_P, _P]),
    "ivx_graph_destroy": (None, [_P]),
    "ivx_feature_stats": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "ivx_selector_set": (_I32, [_P, ctypes.POINTER(SelectorDims), _P, _P, _P, _P]),
    "ivx_selector_param_count": (_I64, [_P]),
    "ivx_pruned_set": (_I32, [_P, _I32, ctypes.c_float, _P]),
    "ivx_selector_get": (_I32, [_P, _P, _P]),
    "ivx_selector_forward": (_I32, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "ivx_selector_grad": (_I32, [_P, _P, _I64, _P, _I32, _P, _P, _P, _P, _P]),
    "ivx_selector_train_step": (_I32, [_P, _P, _I64, _P, _I32, _P, _P, ctypes.c_float, _P, _P]),
    "ivx_selector_counts": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P]),
    "ivx_autotune": (_I32, [_P, _P, _P, _I64, _I64, ctypes.POINTER(Tuning), _P]),
    "ivx_tuning_get": (_I32, [_P, ctypes.POINTER(Tuning)]),
    "ivx_tuning_set": (_I32, [_P, ctypes.POINTER(Tuning)]),
    "ivx_plan_batches": (_I32, [_P, _I64, _I32, _I64, _P, _I64, ctypes.POINTER(_I64)]),
    "ivx_stream_create": (_I32, [_P, ctypes.POINTER(StreamConfig), ctypes.POINTER(_P)]),
    "ivx_stream_destroy": (None, [_P]),
    "ivx_stream_em_pass": (_I32, [_P, _P, FrameSource, _P, _P, _I64, _I32, _I32, _P, _P, _P,
                                  ctypes.POINTER(Accum), _P, _P]),
    "ivx_stream_extract": (_I32, [_P, _P, FrameSource, _P, _P, _I64, _I32, _I32, _P, _P]),
    "ivx_backend_create": (_I32, [_I32, _I64, _I32, ctypes.c_int, ctypes.POINTER(_P)]),
    "ivx_backend_destroy": (None, [_P]),
    "ivx_backend_whitening": (_I32, [_P, _P, _I64, _I32, _P, _P, _P]),
    "ivx_backend_lnorm": (_I32, [_P, _P, _I64, _I32, _P, _P, _P, _P]),
    "ivx_backend_lda": (_I32, [_P, _P, _I64, _I32, _P, _I32, _I32, _P, _P, _P]),
    "ivx_backend_project": (_I32, [_P, _P, _I64, _I32, _P, _I32, _P, _P]),
    "ivx_backend_plda_fit": (_I32, [_P, _P, _I64, _I32, _P, _I32, _P, _P, _P, _P]),
    "ivx_backend_plda_score": (_I32, [_P, _P, _P, _P, _I32, _P, _I64, _P, _I64, _P, _I64, _P,
                                      _P]),
    "ivx_backend_status": (_I32, [_P, _P]),
    "ivx_eer": (_I32, [_P, _P, _I64, ctypes.POINTER(ctypes.c_double)]),
    "ivx_profile_enable": (_I32, [_P, _I32]),
    "ivx_profile_read": (_I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), _I32]),
}

PROFILE_GROUPS = ["frame_select", "rescore", "stats_nf", "stats_S", "tv_prep", "estep_gemm",
                  "estep_chol", "accumulate", "mstep_solve", "mindiv", "ubm_prepare", "sel_mlp",
                  "sel_score", "sel_train"]

_lib = None


def load() -> ctypes.CDLL:
    """Loads libivx.so and binds every prototype; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1906_08556_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, name: str, device=None):
    if t is None:
        return None
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: expected device {device}, got {t.device}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One ivx_ctx: model storage and workspace for fixed (C, D, R) and batch limits."""

    def __init__(self, C: int, D: int, R: int, max_batch_utts: int, max_batch_frames: int,
                 device: int = 0):
        self.lib = load()
        self.C, self.D, self.R = C, D, R
        self.max_batch_utts, self.max_batch_frames = max_batch_utts, max_batch_frames
        self.device = torch.device("cuda", device)
        dims = Dims(C, D, R, max_batch_utts, max_batch_frames)
        h = ctypes.c_void_p()
        self._check(self.lib.ivx_create(ctypes.byref(dims), device, ctypes.byref(h)))
        self.h = h
        self.TP = int(self.lib.ivx_tp_size(R))

    def close(self):
        if getattr(self, "h", None):
            self.lib.ivx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, status: int):
        if status != 0:
            msg = self.lib.ivx_last_error().decode(errors="replace")
            raise IvxError(status, msg)

    def _p(self, t, dtype, name):
        return _ptr(t, dtype, name, self.device)

    # ------------------------------------------------------------------ model
    def sync_status(self, stream=None):
        self._check(self.lib.ivx_sync_status(self.h, _stream(stream)))

    def set_ubm(self, w, mu, cov, stream=None):
        f = torch.float64
        self._check(self.lib.ivx_set_ubm(self.h, self._p(w, f, "w"), self._p(mu, f, "mu"),
                                         self._p(cov, f, "cov"), _stream(stream)))

    def init_tv(self, T_rand, p0=100.0, stream=None):
        self._check(self.lib.ivx_init_tv(self.h, self._p(T_rand, torch.float64, "T_rand"),
                                         float(p0), _stream(stream)))

    def init_tv_standard(self, T_rand, stream=None):
        self._check(self.lib.ivx_init_tv_standard(
            self.h, self._p(T_rand, torch.float64, "T_rand"), _stream(stream)))

    def set_bias(self, m, stream=None):
        """m [C][D] FP64 device tensor (standard formulation), or None (augmented)."""
        self._check(self.lib.ivx_set_bias(self.h, self._p(m, torch.float64, "m"),
                                          _stream(stream)))

    def get_bias(self, stream=None):
        m = torch.empty((self.C, self.D), dtype=torch.float64, device=self.device)
        self._check(self.lib.ivx_get_bias(self.h, self._p(m, torch.float64, "m"),
                                          _stream(stream)))
        return m

    def set_tv(self, T, Sigma, p, stream=None):
        f = torch.float64
        self._check(self.lib.ivx_set_tv(self.h, self._p(T, f, "T"), self._p(Sigma, f, "Sigma"),
                                        self._p(p, f, "p"), _stream(stream)))

    def get_tv(self, stream=None):
        f = torch.float64
        dev = self.device
        T = torch.empty((self.C, self.D, self.R), dtype=f, device=dev)
        Sigma = torch.empty((self.C, self.D, self.D), dtype=f, device=dev)
        p = torch.empty(self.R, dtype=f, device=dev)
        mu = torch.empty((self.C, self.D), dtype=f, device=dev)
        self._check(self.lib.ivx_get_tv(self.h, self._p(T, f, "T"), self._p(Sigma, f, "Sigma"),
                                        self._p(p, f, "p"), self._p(mu, f, "mu"), _stream(stream)))
        return T, Sigma, p, mu

    # --------------------------------------------------------------- hot path
    def ubm_posteriors(self, X, gamma=None, post_idx=None, post_val=None, frame_ll=None,
                       prec=IVX_FP32, sel=IVX_SEL_ALL, stream=None):
        F = X.shape[0]
        self._check(self.lib.ubm_posteriors(
            self.h, self._p(X, torch.float32, "X"), F, prec, sel,
            self._p(gamma, torch.float32, "gamma"), self._p(post_idx, torch.int32, "post_idx"),
            self._p(post_val, torch.float32, "post_val"), KP,
            self._p(frame_ll, torch.float64, "frame_ll"), _stream(stream)))

    def ubm_posteriors_static(self, X, post_idx, post_val, frame_ll=None, prec=IVX_FP32,
                              stream=None):
        F = X.shape[0]
        self._check(self.lib.ubm_posteriors_static(
            self.h, self._p(X, torch.float32, "X"), F, prec,
            self._p(post_idx, torch.int32, "post_idx"), self._p(post_val, torch.float32, "post_val"),
            KP, self._p(frame_ll, torch.float64, "frame_ll"), _stream(stream)))

    def bw_stats(self, X, utt_off, n, f, S_acc=None, ll_acc=None, prec=IVX_FP32,
                 sel=IVX_SEL_ALL, stream=None):
        U = utt_off.shape[0] - 1
        self._check(self.lib.bw_stats(
            self.h, self._p(X, torch.float32, "X"), self._p(utt_off, torch.int64, "utt_off"), U,
            X.shape[0], prec, sel, self._p(n, torch.float32, "n"), self._p(f, torch.float32, "f"),
            self._p(S_acc, torch.float64, "S_acc"), self._p(ll_acc, torch.float64, "ll_acc"),
            _stream(stream)))

    def tv_estep(self, n, f, phi, Phi=None, ll_acc=None, info=None, prec=IVX_FP32, stream=None):
        U = n.shape[0]
        self._check(self.lib.tv_estep(
            self.h, self._p(n, torch.float32, "n"), self._p(f, torch.float32, "f"), U, prec,
            self._p(phi, torch.float32, "phi"), self._p(Phi, torch.float32, "Phi"),
            self._p(ll_acc, torch.float64, "ll_acc"), self._p(info, torch.int32, "info"),
            _stream(stream)))

    def new_accum(self) -> "Accumulators":
        return Accumulators(self)

    def tv_mstep_accumulate(self, n, f, phi, Phi, acc: "Accumulators", stream=None):
        U = n.shape[0]
        s = acc.struct()
        self._check(self.lib.tv_mstep_accumulate(
            self.h, self._p(n, torch.float32, "n"), self._p(f, torch.float32, "f"),
            self._p(phi, torch.float32, "phi"), self._p(Phi, torch.float32, "Phi"), U,
            ctypes.byref(s), _stream(stream)))

    def extract_ivectors(self, X, utt_off, phi, prec=IVX_FP32, sel=IVX_SEL_ALL, stream=None):
        U = utt_off.shape[0] - 1
        self._check(self.lib.extract_ivectors(
            self.h, self._p(X, torch.float32, "X"), self._p(utt_off, torch.int64, "utt_off"), U,
            X.shape[0], prec, sel, self._p(phi, torch.float32, "phi"), _stream(stream)))

    def tv_mstep_solve(self, acc: "Accumulators", S, update_sigma=True, ll_sum=None,
                       objective=None, status=None, stream=None):
        s = acc.struct()
        self._check(self.lib.tv_mstep_solve(
            self.h, ctypes.byref(s), self._p(S, torch.float64, "S"), int(bool(update_sigma)),
            self._p(ll_sum, torch.float64, "ll_sum"), self._p(objective, torch.float64, "objective"),
            self._p(status, torch.int32, "status"), _stream(stream)))

    def tv_mindiv(self, acc: "Accumulators", method=0, stream=None):
        s = acc.struct()
        self._check(self.lib.tv_mindiv(self.h, ctypes.byref(s), int(method), _stream(stream)))

    def tv_mindiv_standard(self, acc: "Accumulators", update_mean=False, method=0, stream=None):
        s = acc.struct()
        self._check(self.lib.tv_mindiv_standard(self.h, ctypes.byref(s), int(method),
                                                int(bool(update_mean)), _stream(stream)))

    def ubm_update_means(self, stream=None):
        self._check(self.lib.ubm_update_means(self.h, _stream(stream)))

    # ------------------------------------------------------- iteration graph
    def graph_create_em(self, X, utt_off, n, f, S, phi, Phi, acc: "Accumulators", ll_frames,
                        ll_utts, objective, update_sigma=True, realign=True, prec=IVX_FP32):
        """Captures one full EM iteration; returns an EMGraph (keeps the buffers alive)."""
        U = utt_off.shape[0] - 1
        h = ctypes.c_void_p()
        acc_s = acc.struct()
        f32, f64 = torch.float32, torch.float64
        self._check(self.lib.ivx_graph_create_em(
            self.h, self._p(X, f32, "X"), self._p(utt_off, torch.int64, "utt_off"), U, X.shape[0],
            prec, self._p(n, f32, "n"), self._p(f, f32, "f"), self._p(S, f64, "S"),
            self._p(phi, f32, "phi"), self._p(Phi, f32, "Phi"), ctypes.byref(acc_s),
            self._p(ll_frames, f64, "ll_frames"), self._p(ll_utts, f64, "ll_utts"),
            self._p(objective, f64, "objective"), int(bool(update_sigma)), int(bool(realign)),
            ctypes.byref(h)))
        return EMGraph(self, h, (X, utt_off, n, f, S, phi, Phi, acc, ll_frames, ll_utts, objective))

    # ---------------------------------------------------- learned selection
    def feature_stats(self, X, stream=None):
        mean = torch.empty(self.D, dtype=torch.float32, device=self.device)
        std = torch.empty(self.D, dtype=torch.float32, device=self.device)
        self._check(self.lib.ivx_feature_stats(self.h, self._p(X, torch.float32, "X"), X.shape[0],
                                               self._p(mean, torch.float32, "mean"),
                                               self._p(std, torch.float32, "std"), _stream(stream)))
        return mean, std

    def selector_set(self, params, mean, std, H1=512, H2=512, k=20, min_mass=0.99,
                     max_train_batch=0, stream=None):
        self.sel_dims = SelectorDims(H1, H2, k, min_mass, max_train_batch)
        f = torch.float32
        self._check(self.lib.ivx_selector_set(self.h, ctypes.byref(self.sel_dims),
                                              self._p(params, f, "params"), self._p(mean, f, "mean"),
                                              self._p(std, f, "std"), _stream(stream)))

    def pruned_set(self, k=20, prune=0.025, stream=None):
        self._check(self.lib.ivx_pruned_set(self.h, int(k), float(prune), _stream(stream)))

    def selector_param_count(self) -> int:
        return int(self.lib.ivx_selector_param_count(self.h))

    def selector_get(self, stream=None):
        out = torch.empty(self.selector_param_count(), dtype=torch.float32, device=self.device)
        self._check(self.lib.ivx_selector_get(self.h, self._p(out, torch.float32, "params"),
                                              _stream(stream)))
        return out

    def selector_forward(self, X, h1=None, h2=None, z=None, prop=None, mass=None, fallback=None,
                         stream=None):
        self._check(self.lib.ivx_selector_forward(
            self.h, self._p(X, torch.float32, "X"), X.shape[0], self._p(h1, torch.bfloat16, "h1"),
            self._p(h2, torch.bfloat16, "h2"), self._p(z, torch.float32, "z"),
            self._p(prop, torch.int32, "prop"), self._p(mass, torch.float32, "mass"),
            self._p(fallback, torch.int32, "fallback"), _stream(stream)))

    def selector_grad(self, X, frame_idx, post_idx, post_val, grad=None, loss=None, stream=None):
        self._check(self.lib.ivx_selector_grad(
            self.h, self._p(X, torch.float32, "X"), X.shape[0],
            self._p(frame_idx, torch.int64, "frame_idx"), frame_idx.shape[0],
            self._p(post_idx, torch.int32, "post_idx"), self._p(post_val, torch.float32, "post_val"),
            self._p(grad, torch.float32, "grad"), self._p(loss, torch.float64, "loss"),
            _stream(stream)))

    def selector_train_step(self, X, frame_idx, post_idx, post_val, lr, loss=None, stream=None):
        self._check(self.lib.ivx_selector_train_step(
            self.h, self._p(X, torch.float32, "X"), X.shape[0],
            self._p(frame_idx, torch.int64, "frame_idx"), frame_idx.shape[0],
            self._p(post_idx, torch.int32, "post_idx"), self._p(post_val, torch.float32, "post_val"),
            float(lr), self._p(loss, torch.float64, "loss"), _stream(stream)))

    def selector_counts(self, stream=None):
        a, b = _I64(), _I64()
        self._check(self.lib.ivx_selector_counts(self.h, ctypes.byref(a), ctypes.byref(b),
                                                 _stream(stream)))
        return a.value, b.value

    # ---------------------------------------------------------------- autotuner
    def autotune(self, X, utt_off, stream=None) -> dict:
        t = Tuning()
        self._check(self.lib.ivx_autotune(self.h, self._p(X, torch.float32, "X"),
                                          self._p(utt_off, torch.int64, "utt_off"),
                                          utt_off.shape[0] - 1, X.shape[0], ctypes.byref(t),
                                          _stream(stream)))
        return t.as_dict()

    def tuning_get(self) -> dict:
        t = Tuning()
        self._check(self.lib.ivx_tuning_get(self.h, ctypes.byref(t)))
        return t.as_dict()

    def tuning_set(self, **kw):
        t = Tuning(**{**self.tuning_get(), **kw})
        self._check(self.lib.ivx_tuning_set(self.h, ctypes.byref(t)))

    # ---------------------------------------------------------------- tracing
    def profile_enable(self, capacity=4096):
        self._check(self.lib.ivx_profile_enable(self.h, int(capacity)))

    def profile_read(self):
        """{group: (total ms, calls)} of the event pairs recorded since the last read."""
        n = len(PROFILE_GROUPS)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        self._check(self.lib.ivx_profile_read(self.h, ms, calls, n))
        return {g: (ms[i], calls[i]) for i, g in enumerate(PROFILE_GROUPS)}


class EMGraph:
    """A captured EM iteration; launch() runs one iteration on the current stream."""

    def __init__(self, ctx: Context, handle, keep):
        self.ctx, self.h, self._keep = ctx, handle, keep

    def launch(self, stream=None):
        self.ctx._check(self.ctx.lib.ivx_graph_launch(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ivx_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host(a, dtype, name):
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"{name}: expected a C-contiguous numpy array of {np.dtype(dtype)}")
    return ctypes.c_void_p(a.ctypes.data)


def plan_batches(utt_off: np.ndarray, max_utts: int, max_frames: int) -> np.ndarray:
    """ivx_plan_batches (host only): first utterance of every batch, then U."""
    lib = load()
    U = len(utt_off) - 1
    starts = np.zeros(max(U, 0) + 1, dtype=np.int64)
    nb = ctypes.c_int64()
    st = lib.ivx_plan_batches(_host(utt_off, np.int64, "utt_off"), U, int(max_utts),
                              int(max_frames), ctypes.c_void_p(starts.ctypes.data), len(starts),
                              ctypes.byref(nb))
    if st != 0:
        raise IvxError(st, lib.ivx_last_error().decode(errors="replace"))
    return starts[:nb.value + 1].copy()


class Stream:
    """ivx_stream: batches of host-resident utterances through pinned slots,
    uploaded and processed while the next batch loads."""

    def __init__(self, ctx: Context, max_batch_utts: int, max_batch_frames: int, loaders=4,
                 slots=4):
        self.ctx = ctx
        cfg = StreamConfig(max_batch_utts, max_batch_frames, loaders, slots)
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.ivx_stream_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    @staticmethod
    def _source(fn, D):
        """Wraps fn(u0, u1, out) (out: [frames, D] float32 view to fill) as a
        frame source; an exception in fn stops the pass."""
        if fn is None:
            return FrameSource()

        def cb(user, u0, u1, off, dst):
            try:
                nf = int(off[u1] - off[u0])
                if nf > 0:
                    buf = (ctypes.c_float * (nf * D)).from_address(dst)
                    fn(int(u0), int(u1), np.frombuffer(buf, dtype=np.float32).reshape(nf, D))
                return 0
            except Exception:  # reported by the library as a failed source
                return 1
        return FrameSource(cb)

    def em_pass(self, utt_off, acc: "Accumulators", X=None, source=None, S_acc=None,
                ll_frames=None, ll_utts=None, phi_out=None, prec=IVX_FP32, sel=IVX_SEL_ALL,
                stream=None):
        c = self.ctx
        U = len(utt_off) - 1
        src = self._source(source, c.D)
        s = acc.struct()
        c._check(c.lib.ivx_stream_em_pass(
            self.h, None if X is None else _host(X, np.float32, "X"), src, None,
            _host(utt_off, np.int64, "utt_off"), U, prec, sel,
            c._p(S_acc, torch.float64, "S_acc"), c._p(ll_frames, torch.float64, "ll_frames"),
            c._p(ll_utts, torch.float64, "ll_utts"), ctypes.byref(s),
            c._p(phi_out, torch.float32, "phi_out"), _stream(stream)))

    def extract(self, utt_off, phi, X=None, source=None, prec=IVX_FP32, sel=IVX_SEL_ALL,
                stream=None):
        c = self.ctx
        U = len(utt_off) - 1
        src = self._source(source, c.D)
        c._check(c.lib.ivx_stream_extract(
            self.h, None if X is None else _host(X, np.float32, "X"), src, None,
            _host(utt_off, np.int64, "utt_off"), U, prec, sel, c._p(phi, torch.float32, "phi"),
            _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ivx_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eer(scores: np.ndarray, is_target: np.ndarray) -> float:
    """ivx_eer (host only)."""
    lib = load()
    s = np.ascontiguousarray(scores, dtype=np.float32)
    t = np.ascontiguousarray(is_target, dtype=np.uint8)
    out = ctypes.c_double()
    st = lib.ivx_eer(ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(t.ctypes.data), len(s),
                     ctypes.byref(out))
    if st != 0:
        raise IvxError(st, lib.ivx_last_error().decode(errors="replace"))
    return out.value


class Backend:
    """ivx_backend: whitening, length norm, LDA, two-covariance PLDA and trial
    scoring on device tensors."""

    def __init__(self, max_dim: int, max_n: int, max_classes: int, device: int = 0):
        self.lib = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        self._check(self.lib.ivx_backend_create(max_dim, max_n, max_classes, device,
                                                ctypes.byref(h)))
        self.h = h

    def _check(self, status):
        if status != 0:
            raise IvxError(status, self.lib.ivx_last_error().decode(errors="replace"))

    def _p(self, t, dtype, name):
        return _ptr(t, dtype, name, self.device)

    def whitening(self, X, stream=None):
        n, dim = X.shape
        f64 = torch.float64
        mean = torch.empty(dim, dtype=f64, device=self.device)
        W = torch.empty((dim, dim), dtype=f64, device=self.device)
        self._check(self.lib.ivx_backend_whitening(self.h, self._p(X, torch.float32, "X"), n, dim,
                                                   self._p(mean, f64, "mean"),
                                                   self._p(W, f64, "W"), _stream(stream)))
        return mean, W

    def lnorm(self, X, mean=None, W=None, stream=None):
        n, dim = X.shape
        Y = torch.empty_like(X)
        self._check(self.lib.ivx_backend_lnorm(
            self.h, self._p(X, torch.float32, "X"), n, dim, self._p(mean, torch.float64, "mean"),
            self._p(W, torch.float64, "W"), self._p(Y, torch.float32, "Y"), _stream(stream)))
        return Y

    def lda(self, X, labels, K, out_dim, stream=None):
        n, dim = X.shape
        f64 = torch.float64
        V = torch.empty((dim, out_dim), dtype=f64, device=self.device)
        ev = torch.empty(out_dim, dtype=f64, device=self.device)
        self._check(self.lib.ivx_backend_lda(
            self.h, self._p(X, torch.float32, "X"), n, dim, self._p(labels, torch.int32, "labels"),
            K, out_dim, self._p(V, f64, "V"), self._p(ev, f64, "eigval"), _stream(stream)))
        return V, ev

    def project(self, X, V, stream=None):
        n, dim = X.shape
        out_dim = V.shape[1]
        Y = torch.empty((n, out_dim), dtype=torch.float32, device=self.device)
        self._check(self.lib.ivx_backend_project(
            self.h, self._p(X, torch.float32, "X"), n, dim, self._p(V, torch.float64, "V"),
            out_dim, self._p(Y, torch.float32, "Y"), _stream(stream)))
        return Y

    def plda_fit(self, Y, labels, K, stream=None):
        n, d = Y.shape
        f64 = torch.float64
        mu = torch.empty(d, dtype=f64, device=self.device)
        A = torch.empty((d, d), dtype=f64, device=self.device)
        psi = torch.empty(d, dtype=f64, device=self.device)
        self._check(self.lib.ivx_backend_plda_fit(
            self.h, self._p(Y, torch.float32, "Y"), n, d, self._p(labels, torch.int32, "labels"),
            K, self._p(mu, f64, "mu"), self._p(A, f64, "A"), self._p(psi, f64, "psi"),
            _stream(stream)))
        return mu, A, psi

    def plda_score(self, model, Y1, Y2, trials, stream=None):
        mu, A, psi = model
        d = mu.shape[0]
        T = trials.shape[0]
        scores = torch.empty(T, dtype=torch.float32, device=self.device)
        f64 = torch.float64
        self._check(self.lib.ivx_backend_plda_score(
            self.h, self._p(mu, f64, "mu"), self._p(A, f64, "A"), self._p(psi, f64, "psi"), d,
            self._p(Y1, torch.float32, "Y1"), Y1.shape[0], self._p(Y2, torch.float32, "Y2"),
            Y2.shape[0], self._p(trials, torch.int32, "trials"), T,
            self._p(scores, torch.float32, "scores"), _stream(stream)))
        return scores

    def status(self, stream=None):
        self._check(self.lib.ivx_backend_status(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.ivx_backend_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Accumulators:
    """Device FP64 accumulator buffers for tv_mstep_accumulate (zeroed)."""

    def __init__(self, ctx: Context):
        f, dev = torch.float64, ctx.device
        self.A = torch.zeros((ctx.C, ctx.TP), dtype=f, device=dev)
        self.Cc = torch.zeros((ctx.C, ctx.D, ctx.R), dtype=f, device=dev)
        self.N = torch.zeros(ctx.C, dtype=f, device=dev)
        self.h = torch.zeros(ctx.R, dtype=f, device=dev)
        self.H = torch.zeros(ctx.TP, dtype=f, device=dev)
        self.count = torch.zeros(1, dtype=f, device=dev)

    def zero_(self):
        for t in (self.A, self.Cc, self.N, self.h, self.H, self.count):
            t.zero_()
        return self

    def struct(self) -> Accum:
        return Accum(self.A.data_ptr(), self.Cc.data_ptr(), self.N.data_ptr(), self.h.data_ptr(),
                     self.H.data_ptr(), self.count.data_ptr())
