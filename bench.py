#!/usr/bin/env python3
"""Throughput of one full TV-model EM iteration on one MI355X.

A step is one pass of the whole hot path over the workload: frame posteriors
against the full-covariance UBM over all C components, Baum-Welch n, f and S,
the E-step, the M-step accumulators, the FP64 M-step solve (T and Sigma),
minimum divergence and the UBM-mean realignment.

Workload (default): D=60 features, C=2048 full-covariance components, R=400,
4000 synthetic utterances of 500-1500 frames (~4M frames), seeded generator
(``synth``).  ``value`` is utterances per second of whole EM iterations with
the features resident in HBM; frame posteriors per second and the split of
the step time are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n-utts U] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TV EM utts/s + frame posteriors/s at C=2048,D=60,R=400 vs FP32 plain"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# BF16 MFMA products per FP32 product in the BF16 frame filter (operands split
# into high and low BF16 parts: hi*hi + hi*lo + lo*hi)
BF16_PRODUCTS = 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shape", type=int, default=2, help="workload shape id (synth.SHAPES)")
    ap.add_argument("--n-utts", type=int, default=None, help="first U utterances only")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frame-utts", type=int, default=40,
                    help="oracle baseline: utterances for posteriors + n/f/S (all threads)")
    ap.add_argument("--cpu-estep-utts", type=int, default=400,
                    help="oracle baseline: utterances for E-step + accumulation (all threads)")
    ap.add_argument("--cpu-components", type=int, default=256,
                    help="oracle baseline: components of the per-component fixed work")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 form")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device-to-device once "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the EM iteration replayed from a captured HIP graph")
    ap.add_argument("--form-steps", type=int, default=5,
                    help="timed steps of each secondary form (BF16, graph, standard, streamed, "
                         "pruned, learned); at most --steps")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batching workload (20,000 log-uniform utterances)")
    ap.add_argument("--batching-steps", type=int, default=3,
                    help="timed steps (eager and graph replay) of the batching workload")
    ap.add_argument("--learned-steps", type=int, default=3000,
                    help="training steps of the learned selector (0: skip the learned form)")
    ap.add_argument("--learned-batch", type=int, default=4096)
    ap.add_argument("--learned-sweep", type=str, default="",
                    help="widths:training-utterances:steps lists, e.g. '512,1024,2048:400,1600:3000', "
                         "several separated by ';': train the selector at each width and "
                         "training-set size and report held-out loss, missed mass and fallback "
                         "(off by default)")
    ap.add_argument("--no-standard", action="store_true",
                    help="skip the standard-formulation timing")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streamed-from-host timing")
    ap.add_argument("--stream-batch-utts", type=int, default=500)
    ap.add_argument("--stream-batch-frames", type=int, default=600_000)
    ap.add_argument("--stream-loaders", type=int, default=4)
    ap.add_argument("--no-backend", action="store_true",
                    help="skip the back-end timing on synthetic speakers")
    ap.add_argument("--no-pruned", action="store_true",
                    help="skip the pruned alignment (diagonal-UBM top-20, drop < 0.025)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of timing the candidates")
    ap.add_argument("--tune", type=str, default="",
                    help="launch-shape fields set after the autotuner, e.g. 'estep_global=1,"
                         "mstep_left=0' (see ivx_tuning)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel, workload, frames):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when there is none for this workload and frame count, or when
    the kernel's source file changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    try:
        src = os.path.join(ROOT, vals["source"])
        if source_digest(src) != vals["source_sha256_16"] or int(vals["frames"]) != frames:
            return None
        return int(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError, OSError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rates(wl, n_frame, n_estep, n_comp, pre=None):
    """Times the FP64 oracle, as it stands, on bounded samples of the workload
    with the BLAS threads currently allowed:
      * posteriors over all C + n/f/S on the first ``n_frame`` utterances;
      * E-step + accumulation on ``n_estep`` utterances whose statistics are
        those of the frame sample repeated (the cost does not depend on the
        values);
      * the per-component fixed work (V/U precompute, M-step solve, T update
        of minimum divergence) on the first ``n_comp`` components, scaled to C.
    ``pre`` passes the full V/U precompute for the E-step when it is at hand
    (else it is computed here, untimed beyond the component sample).
    Returns the rates, the extrapolated utts/s of a whole iteration at the
    workload's U, and the full precompute for reuse."""
    import numpy as np
    import oracle
    C = wl.shape.C
    off = wl.utt_off[: n_frame + 1]
    F = int(off[-1])
    X = wl.X[:F]
    T, Sigma, p = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    t0 = time.perf_counter()
    gamma, lse = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    n, f, S = oracle.bw_stats(X, off, gamma)
    t_frame = time.perf_counter() - t0
    cs = slice(0, n_comp)
    t0 = time.perf_counter()
    oracle.tv_precompute(T[cs], Sigma[cs])
    t_pre = (time.perf_counter() - t0) * C / n_comp
    if pre is None:
        pre = oracle.tv_precompute(T, Sigma)
    reps = -(-n_estep // n_frame)
    ne = np.tile(n, (reps, 1))[:n_estep]
    fe = np.tile(f, (reps, 1, 1))[:n_estep]
    t0 = time.perf_counter()
    e = oracle.estep(ne, fe, T, Sigma, p, pre=pre)
    acc = oracle.accumulate(ne, fe, e["phi"], e["Phi"])
    t_utt = time.perf_counter() - t0
    sub = dict(N=acc["N"][cs], A=acc["A"][cs], Cc=acc["Cc"][cs])
    t0 = time.perf_counter()
    T1, _, _ = oracle.mstep(sub, S[cs], T[cs], Sigma[cs])
    oracle.mindiv(acc["hsum"] / acc["count"], acc["Hsum"] / acc["count"], T1)
    t_fixed = t_pre + (time.perf_counter() - t0) * C / n_comp
    U = wl.U
    total = U * (t_frame / n_frame + t_utt / n_estep) + t_fixed
    return dict(value=U / total, frames_per_s=F / t_frame, estep_utts_per_s=n_estep / t_utt,
                fixed_s=t_fixed, frames=F), pre


def cpu_baseline(wl, n_frame, n_estep, n_comp, n_frame_1t, n_estep_1t):
    """The FP64 oracle on the host cores, all BLAS threads and one thread.

    ``value`` is utts/s of a whole EM iteration at the workload's U,
    extrapolated from bounded samples (see _oracle_rates); ``one_thread``
    holds the same figures with a single BLAS thread on smaller samples."""
    from threadpoolctl import threadpool_info, threadpool_limits
    ncpu = os.cpu_count() or 1
    with threadpool_limits(1):
        one, pre = _oracle_rates(wl, n_frame_1t, n_estep_1t, n_comp)
    with threadpool_limits(ncpu):
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        allt, _ = _oracle_rates(wl, n_frame, n_estep, n_comp, pre=pre)
    r = lambda x: round(float(x), 3)  # noqa: E731
    return {
        "value": r(allt["value"]),
        "unit": "utts/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 oracle, {threads} BLAS threads: posteriors over all C and n/f/S on the "
                   f"first {n_frame} utterances ({allt['frames']} frames), E-step + accumulation "
                   f"on {n_estep} utterances (the sample's statistics repeated), precompute + "
                   f"M-step solve + min-div T update on {n_comp} of {wl.shape.C} components "
                   f"scaled to C; whole iteration extrapolated to U={wl.U}"),
        "cpu_model": _cpu_model(),
        "cpu_count": ncpu,
        "frames_per_s": r(allt["frames_per_s"]),
        "estep_utts_per_s": r(allt["estep_utts_per_s"]),
        "fixed_s_per_iteration": r(allt["fixed_s"]),
        "one_thread": {"value": r(one["value"]), "frames_per_s": r(one["frames_per_s"]),
                       "estep_utts_per_s": r(one["estep_utts_per_s"]),
                       "fixed_s_per_iteration": r(one["fixed_s"]),
                       "sample": f"first {n_frame_1t} utterances ({one['frames']} frames), "
                                 f"E-step on {n_estep_1t}, {n_comp} components"},
    }


def learned_form(args, ctx, wl, X, step, timed, reset_model, phi, K, W, dev):
    """Trains the learned selector on the GPU (exact all-component posteriors
    of the first tenth of the utterances as targets), then reports its
    accuracy on the other utterances and the throughput of the EM iteration
    with IVX_SEL_LEARNED, against the plain all-component form."""
    import numpy as np
    import torch

    import synth
    from paper_1906_08556_amd import ivx
    C, D, U, F = wl.shape.C, wl.shape.D, wl.U, wl.F
    H, k, B = 512, 20, args.learned_batch
    Utr = max(1, U // 10)
    Ftr = int(wl.utt_off[Utr])
    reset_model()
    pi = torch.empty((F, 16), dtype=torch.int32, device=dev)
    pv = torch.empty((F, 16), dtype=torch.float32, device=dev)
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv)
    mean, std = ctx.feature_stats(X[:Ftr])
    params = torch.from_numpy(synth.mlp_init(D, H, H, C, seed=args.seed)).to(dev)
    ctx.selector_set(params, mean, std, H1=H, H2=H, k=k, min_mass=0.99, max_train_batch=B)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_steps = args.learned_steps
    for i in range(n_steps):
        fidx = torch.from_numpy(synth.sample_frames(Ftr, B, seed=i)).to(dev)
        ctx.selector_train_step(X, fidx, pi, pv, 1e-3 if i < 0.7 * n_steps else 3e-4, loss=loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ctx.sync_status()
    # held-out accuracy: proposal mass, fallback, posterior mass the proposals miss
    Fe = F - Ftr
    prop = torch.empty((Fe, k), dtype=torch.int32, device=dev)
    mass = torch.empty(Fe, dtype=torch.float32, device=dev)
    ctx.selector_forward(X[Ftr:], prop=prop, mass=mass)
    fb = mass < 0.99
    miss = torch.empty(Fe, dtype=torch.float64, device=dev)
    for r0 in range(0, Fe, 1 << 18):
        r1 = min(Fe, r0 + (1 << 18))
        a = pi[Ftr + r0:Ftr + r1].long()
        hit = ((a.unsqueeze(2) == prop[r0:r1].long().unsqueeze(1)) & (a.unsqueeze(2) >= 0)).any(2)
        miss[r0:r1] = 1.0 - (pv[Ftr + r0:Ftr + r1].double() * hit).sum(1)
    kept = ~fb
    # throughput of the whole EM iteration with the learned selection
    el, ph, prof = timed(0, K, W, sel=ivx.IVX_SEL_LEARNED)
    nfb, pairs = ctx.selector_counts()
    mlp_ms = prof["sel_mlp"][0] / K
    mlp_tflops = 2.0 * (D * H + H * H + H * C) * F / (mlp_ms / 1e3) / 1e12 if mlp_ms > 0 else None
    # one iteration of each form from the same model: i-vectors
    outs = []
    for sel in (ivx.IVX_SEL_ALL, ivx.IVX_SEL_LEARNED):
        reset_model()
        step(0, sel=sel)
        ctx.sync_status()
        outs.append(phi.double().cpu().numpy())
    a, b = outs
    cos = (a * b).sum(1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
    m = miss[kept].cpu().numpy() if bool(kept.any()) else np.zeros(1)
    return {
        "utts_per_s": round(U * K / el, 3), "ms_per_step": round(el * 1e3 / K, 3), "steps": K,
        "frame_posteriors_per_s": round(F * K / (ph["frame"] / 1e3), 1),
        "train": {"steps": n_steps, "batch": B, "seconds": round(t_train, 2),
                  "final_loss": round(loss.item(), 4), "train_utterances": Utr},
        "heldout": {"frames": Fe, "fallback_fraction": round(float(fb.float().mean()), 4),
                    "missed_mass_kept_mean": float(m.mean()),
                    "missed_mass_kept_p99": float(np.quantile(m, 0.99)),
                    "missed_mass_all_mean": float(miss.mean())},
        "timed_pass": {"fallback_frames": nfb, "scored_pairs": pairs},
        "network_kernels": {"ms_per_step": round(mlp_ms, 3), "achieved_bf16_tflops":
                            None if mlp_tflops is None else round(mlp_tflops, 2),
                            "peak": 2500.0,
                            "frac": None if mlp_tflops is None else round(mlp_tflops / 2500.0, 4)},
        "vs_plain_first_iteration": {"ivector_min_cosine": float(cos.min())},
    }


class _Generator:
    """Generates a seeded workload on a daemon host thread (numpy releases the
    interpreter lock inside its array kernels); join() returns it."""

    def __init__(self, shape_id, seed):
        import threading
        self.result, self.error, self.seconds = None, None, 0.0
        self._t = threading.Thread(target=self._run, args=(shape_id, seed), daemon=True)
        self._t.start()

    def _run(self, shape_id, seed):
        import synth
        t0 = time.time()
        try:
            self.result = synth.make(shape_id, seed=seed)
        except BaseException as e:  # noqa: BLE001  (re-raised in join)
            self.error = e
        self.seconds = time.time() - t0

    def join(self):
        self._t.join()
        if self.error is not None:
            raise self.error
        return self.result


def graph_replay(ctx, reset_model, X, off, n, f, S, phi, Phi, acc, ll_frames, ll_utts, obj, K, W,
                 U):
    """Times the whole EM iteration (posteriors, statistics, E-step,
    accumulation, M-step, minimum divergence, realignment) replayed from one
    captured HIP graph: W untimed replays, then K timed."""
    import torch
    reset_model()
    t0 = time.perf_counter()
    g = ctx.graph_create_em(X, off, n, f, S, phi, Phi, acc, ll_frames, ll_utts, obj)
    t_cap = time.perf_counter() - t0
    for _ in range(W):
        g.launch()
    ctx.sync_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        g.launch()
    torch.cuda.synchronize()
    elg = time.perf_counter() - t0
    ctx.sync_status()
    g.close()
    return {"utts_per_s": round(U * K / elg, 3), "ms_per_step": round(elg * 1e3 / K, 3),
            "steps": K, "capture_and_instantiate_ms": round(t_cap * 1e3, 1)}


def batching_block(args, wl, tuning, dev):
    """The batching workload: 20,000 utterances with log-uniform 200-3000
    frame lengths (~20.5M frames) at D 60, C 2048, R 400, FP32, realignment
    every iteration; whole EM iterations issued eagerly and replayed from a
    captured HIP graph, with the launch shapes tuned on the headline workload."""
    import torch
    from paper_1906_08556_amd import ivx
    sh = wl.shape
    C, D, R, U, F = sh.C, sh.D, sh.R, wl.U, wl.F
    K, W = max(1, args.batching_steps), 1
    ctx = ivx.Context(C, D, R, U, F)
    if tuning:
        ctx.tuning_set(**tuning)
    X = torch.from_numpy(wl.X).to(dev)
    off = torch.from_numpy(wl.utt_off).to(dev)
    w_d, mu_d, cov_d = (torch.from_numpy(a).to(dev) for a in (wl.w, wl.mu, wl.cov))
    T0 = torch.from_numpy(wl.T_init).to(dev)
    f64 = torch.float64
    n = torch.empty((U, C), dtype=torch.float32, device=dev)
    f = torch.empty((U, C, D), dtype=torch.float32, device=dev)
    S = torch.zeros((C, D * (D + 1) // 2), dtype=f64, device=dev)
    phi = torch.empty((U, R), dtype=torch.float32, device=dev)
    Phi = torch.empty((U, R * (R + 1) // 2), dtype=torch.float32, device=dev)
    llf, llu, obj = (torch.zeros(1, dtype=f64, device=dev) for _ in range(3))
    acc = ctx.new_accum()

    def reset_model():
        ctx.set_ubm(w_d, mu_d, cov_d)
        ctx.init_tv(T0, 100.0)

    def step():
        S.zero_()
        llf.zero_()
        llu.zero_()
        acc.zero_()
        ctx.bw_stats(X, off, n, f, S_acc=S, ll_acc=llf)
        ctx.tv_estep(n, f, phi, Phi=Phi, ll_acc=llu)
        ctx.tv_mstep_accumulate(n, f, phi, Phi, acc)
        ctx.tv_mstep_solve(acc, S, update_sigma=True, ll_sum=llu, objective=obj)
        ctx.tv_mindiv(acc)
        ctx.ubm_update_means()

    reset_model()
    for _ in range(W):
        step()
    ctx.sync_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.sync_status()
    obj_eager = obj.item()
    graph = graph_replay(ctx, reset_model, X, off, n, f, S, phi, Phi, acc, llf, llu, obj, K, W, U)
    lens = wl.utt_off[1:] - wl.utt_off[:-1]
    out = {"workload": f"shape4:{sh.name}", "utterances": U, "frames": F,
           "lengths": {"min": int(lens.min()), "mean": round(float(lens.mean()), 1),
                       "max": int(lens.max()), "distribution": sh.lengths},
           "eager": {"utts_per_s": round(U * K / el, 3), "ms_per_step": round(el * 1e3 / K, 3),
                     "frame_posteriors_per_s_whole_step": round(F * K / el, 1), "steps": K},
           "graph_replay": graph,
           "graph_vs_eager": round(graph["utts_per_s"] / (U * K / el), 4),
           "objective_after_eager_steps": obj_eager,
           "step": "posteriors+n/f/S+E-step+accumulate+M-step(T,Sigma)+min-div+realign"}
    del acc
    ctx.close()
    return out


def learned_sweep(args, ctx, wl, X, dev):
    """Selector width and training-set size against held-out accuracy on the
    workload's own data: for each (H, training utterances) a 60-H-H-C network
    is trained from the same initialisation recipe on the exact all-component
    posteriors of the first utterances and evaluated on the last tenth of the
    utterances (cross-entropy against the exact posteriors, mass the top-k
    proposals miss, fallback fraction)."""
    import numpy as np
    import torch

    import synth
    runs = []
    for spec in args.learned_sweep.split(";"):
        widths, sizes, steps = spec.split(":")
        runs += [(int(h), int(n), int(steps)) for h in widths.split(",") for n in sizes.split(",")]
    C, D, U, F = wl.shape.C, wl.shape.D, wl.U, wl.F
    k, B = 20, args.learned_batch
    pi = torch.empty((F, 16), dtype=torch.int32, device=dev)
    pv = torch.empty((F, 16), dtype=torch.float32, device=dev)
    ctx.ubm_posteriors(X, post_idx=pi, post_val=pv)
    Ue = U - U // 10
    Fe0 = int(wl.utt_off[Ue])
    Xe = X[Fe0:]
    Fe = F - Fe0
    eidx = torch.arange(Fe0, min(F, Fe0 + (1 << 16)), dtype=torch.int64, device=dev)
    out = []
    for H, Utr, steps in runs:
        if True:
            Utr = min(Utr, Ue)
            Ftr = int(wl.utt_off[Utr])
            mean, std = ctx.feature_stats(X[:Ftr])
            params = torch.from_numpy(synth.mlp_init(D, H, H, C, seed=args.seed)).to(dev)
            ctx.selector_set(params, mean, std, H1=H, H2=H, k=k, min_mass=0.99, max_train_batch=B)
            loss = torch.zeros(1, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                fidx = torch.from_numpy(synth.sample_frames(Ftr, B, seed=i)).to(dev)
                ctx.selector_train_step(X, fidx, pi, pv, 1e-3 if i < 0.7 * steps else 3e-4,
                                        loss=loss)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            train_loss = loss.item()
            # held-out cross-entropy on up to 65,536 frames of the last utterances
            hl = torch.zeros(1, dtype=torch.float64, device=dev)
            tot, nbt = 0.0, 0
            for b0 in range(0, eidx.shape[0], B):
                ctx.selector_grad(X, eidx[b0:b0 + B], pi, pv, loss=hl)
                tot += hl.item()
                nbt += 1
            held_loss = tot / max(1, nbt)
            prop = torch.empty((Fe, k), dtype=torch.int32, device=dev)
            mass = torch.empty(Fe, dtype=torch.float32, device=dev)
            ctx.selector_forward(Xe, prop=prop, mass=mass)
            miss = torch.empty(Fe, dtype=torch.float64, device=dev)
            for r0 in range(0, Fe, 1 << 18):
                r1 = min(Fe, r0 + (1 << 18))
                a = pi[Fe0 + r0:Fe0 + r1].long()
                hit = ((a.unsqueeze(2) == prop[r0:r1].long().unsqueeze(1)) & (a.unsqueeze(2) >= 0)).any(2)
                miss[r0:r1] = 1.0 - (pv[Fe0 + r0:Fe0 + r1].double() * hit).sum(1)
            ctx.sync_status()
            row = {"H": H, "train_utterances": Utr, "train_frames": Ftr, "steps": steps,
                   "batch": B, "train_seconds": round(t_train, 2),
                   "train_loss_last_batch": round(train_loss, 4),
                   "heldout_loss": round(held_loss, 4),
                   "heldout_missed_mass_mean": round(float(miss.mean()), 4),
                   "heldout_fallback_fraction": round(float((mass < 0.99).float().mean()), 4)}
            log(f"[bench] learned sweep: {row}")
            out.append(row)
    return {"workload_frames": F, "heldout_utterances": U - Ue, "k": k,
            "loss": "soft-target cross-entropy against the exact all-component posteriors",
            "runs": out}


def backend_block(ctx, wl0, dev):
    """Sec. 4.1 back-end at the paper's dimensions on synthetic speakers drawn
    from a full-size model (D 60, C 2048, R 400): i-vectors extracted with it in the
    standard formulation, centring + whitening + length norm, LDA 400 -> 200
    and PLDA trained on half of the speakers, all pairs of the other half
    scored, EER."""
    import numpy as np
    import torch

    import synth
    from paper_1906_08556_amd import ivx
    t0 = time.time()
    # the model of the T-std reading (shape 6): frames stay near their
    # components, so UBM alignments follow the generating components
    wl, lab = synth.speakers(6, n_spk=400, per_spk=8, lengths="uniform:200:600", rho=0.5)
    gen_s = time.time() - t0
    R = wl.shape.R
    U = wl.U
    X = torch.from_numpy(wl.X).to(dev)
    off = torch.from_numpy(wl.utt_off).to(dev)
    ctx.set_ubm(torch.from_numpy(wl.w).to(dev), torch.from_numpy(wl.mu).to(dev),
                torch.from_numpy(wl.cov).to(dev))
    ctx.set_tv(torch.from_numpy(wl.T_true).to(dev), torch.from_numpy(wl.cov).to(dev),
               torch.zeros(R, dtype=torch.float64, device=dev))
    ctx.set_bias(torch.from_numpy(wl.mu).to(dev))
    phi = torch.empty((U, R), dtype=torch.float32, device=dev)
    ctx.extract_ivectors(X, off, phi)        # warm-up (TV precompute)
    ctx.sync_status()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.extract_ivectors(X, off, phi)
    torch.cuda.synchronize()
    ext_s = time.perf_counter() - t
    ctx.set_bias(None)
    be = ivx.Backend(512, U, 400)
    train = torch.from_numpy(lab < 200).to(dev)
    lab_tr = torch.from_numpy(lab[lab < 200]).to(dev)
    Xtr, Xte = phi[train].contiguous(), phi[~train].contiguous()
    times = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        times[name] = round((time.perf_counter() - t1) * 1e3, 3)
        return out

    mean, W = timed("whitening_ms", lambda: be.whitening(Xtr))
    Ytr = timed("lnorm_train_ms", lambda: be.lnorm(Xtr, mean, W))
    Yte = be.lnorm(Xte, mean, W)
    V, _ = timed("lda_400_to_200_ms", lambda: be.lda(Ytr, lab_tr, 200, 200))
    Ptr, Pte = be.project(Ytr, V), be.project(Yte, V)
    model = timed("plda_fit_ms", lambda: be.plda_fit(Ptr, lab_tr, 200))
    lte = lab[lab >= 200]
    i, j = np.triu_indices(len(lte), k=1)
    trials = torch.from_numpy(np.stack([i, j], axis=1).astype(np.int32)).to(dev)
    tgt = lte[i] == lte[j]
    be.plda_score(model, Pte, Pte, trials)   # warm-up
    scores = timed("score_ms", lambda: be.plda_score(model, Pte, Pte, trials))
    be.status()
    eer = ivx.eer(scores.cpu().numpy(), tgt)
    be.close()
    return {"speakers": 400, "utterances": U, "frames": int(wl.F), "rho": 0.5,
            "extract_utts_per_s": round(U / ext_s, 1), "eer": round(eer, 5),
            "trials": int(len(tgt)), "target_trials": int(tgt.sum()),
            "score_trials_per_s": round(len(tgt) / (times["score_ms"] / 1e3), 1),
            "times": times, "data_generation_s": round(gen_s, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout "
              "is described in DESIGN.md and not measured here.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1906_08556_amd import ivx

    t0 = time.time()
    wl = synth.make(args.shape, seed=args.seed, n_utts=args.n_utts)
    sh = wl.shape
    log(f"[bench] workload shape {args.shape}: U={wl.U} F={wl.F} D={sh.D} C={sh.C} R={sh.R} "
        f"(generated in {time.time() - t0:.1f}s)")
    # the batching workload (20,000 log-uniform utterances) is generated on a
    # host thread while the GPU runs the forms below (kernel launches are
    # asynchronous, so the thread does not enter the timed regions' GPU time)
    gen4 = None
    if not args.no_batching and args.shape != 4:
        gen4 = _Generator(4, args.seed)
    C, D, R, U, F = sh.C, sh.D, sh.R, wl.U, wl.F
    dev = torch.device("cuda", 0)
    ctx = ivx.Context(C, D, R, U, F)
    X = torch.from_numpy(wl.X).to(dev)
    off = torch.from_numpy(wl.utt_off).to(dev)
    ctx.set_ubm(torch.from_numpy(wl.w).to(dev), torch.from_numpy(wl.mu).to(dev),
                torch.from_numpy(wl.cov).to(dev))
    ctx.init_tv(torch.from_numpy(wl.T_init).to(dev), 100.0)
    n = torch.empty((U, C), dtype=torch.float32, device=dev)
    f = torch.empty((U, C, D), dtype=torch.float32, device=dev)
    S = torch.zeros((C, D * (D + 1) // 2), dtype=torch.float64, device=dev)
    ll_frames = torch.zeros(1, dtype=torch.float64, device=dev)
    phi = torch.empty((U, R), dtype=torch.float32, device=dev)
    Phi = torch.empty((U, R * (R + 1) // 2), dtype=torch.float32, device=dev)
    ll_utt = torch.zeros(1, dtype=torch.float64, device=dev)
    obj = torch.zeros(1, dtype=torch.float64, device=dev)
    acc = ctx.new_accum()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(max(args.steps, 1))]
    w_d = torch.from_numpy(wl.w).to(dev)
    mu_d = torch.from_numpy(wl.mu).to(dev)
    cov_d = torch.from_numpy(wl.cov).to(dev)
    T0_d = torch.from_numpy(wl.T_init).to(dev)

    def reset_model(form="augmented"):
        ctx.set_ubm(w_d, mu_d, cov_d)
        if form == "standard":
            ctx.init_tv_standard(T0_d)
        else:
            ctx.init_tv(T0_d, 100.0)

    def step(prec, e=None, sel=ivx.IVX_SEL_ALL, form="augmented"):
        S.zero_()
        ll_frames.zero_()
        ll_utt.zero_()
        acc.zero_()
        if e is not None:
            e[0].record()
        ctx.bw_stats(X, off, n, f, S_acc=S, ll_acc=ll_frames, prec=prec, sel=sel)
        if e is not None:
            e[1].record()
        ctx.tv_estep(n, f, phi, Phi=Phi, ll_acc=ll_utt, prec=prec)
        ctx.tv_mstep_accumulate(n, f, phi, Phi, acc)
        ctx.tv_mstep_solve(acc, S, update_sigma=True, ll_sum=ll_utt, objective=obj)
        ctx.tv_mindiv(acc)          # the context's formulation decides the form
        if form == "augmented":
            ctx.ubm_update_means()
        if e is not None:
            e[2].record()

    def timed(prec, steps, warmup, sel=ivx.IVX_SEL_ALL, form="augmented"):
        reset_model(form)
        for _ in range(warmup):
            step(prec, sel=sel, form=form)
        ctx.sync_status()
        ctx.profile_enable(8192)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(prec, ev[i], sel=sel, form=form)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        phase = {"frame": sum(ev[i][0].elapsed_time(ev[i][1]) for i in range(steps)),
                 "em": sum(ev[i][1].elapsed_time(ev[i][2]) for i in range(steps))}
        prof = ctx.profile_read()
        ctx.profile_enable(0)
        ctx.sync_status()
        return el, phase, prof

    tuning = None
    if not args.no_autotune:
        reset_model()
        t0 = time.time()
        tuning = ctx.autotune(X, off)
        log(f"[bench] autotuned launch shapes {tuning} in {time.time() - t0:.1f}s")
    if args.tune:
        ctx.tuning_set(**{k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))})
        tuning = ctx.tuning_get()
        log(f"[bench] launch shapes set to {tuning}")
    K = args.steps
    Ks, Ws = max(1, min(K, args.form_steps)), min(args.warmup, 2)
    elapsed, phase, prof = timed(0, K, args.warmup)
    if args.copy_calib_mib > 0:
        nbytes = args.copy_calib_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nbytes} bytes read and written")
        del src, dst
    ms_step = elapsed * 1e3 / K
    value = U * K / elapsed
    frames_per_s = F * K / (phase["frame"] / 1e3)
    em_utts_per_s = U * K / (phase["em"] / 1e3)

    # roofline of the dominant kernel: the expanded-feature frame GEMM, one
    # persistent launch per pass that scores every frame against all C
    # components (2 K C FLOPs per frame, the method's count)
    Kexp = (D + 1) * (D + 2) // 2
    tune_now = ctx.tuning_get()
    flop_per_frame = 2.0 * Kexp * C
    fs_ms, fs_calls = prof["frame_select"]
    fs_avg_s = fs_ms / max(fs_calls, 1) / 1e3
    achieved = flop_per_frame * F / fs_avg_s / 1e12
    roof = {"kernel": "k_frame_tile", "bound": "mfma", "achieved": round(achieved, 2),
            "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("k_frame_tile", f"shape{args.shape}", F),
            "avg_launch_ms": round(fs_avg_s * 1e3, 3), "launches_per_step": fs_calls // K,
            "flop_per_frame_per_launch": flop_per_frame, "frames_per_launch": F,
            "components_per_launch": C}
    log("[bench] FP32 kernel groups (ms per step): " + ", ".join(
        f"{k}={v[0] / K:.2f}" for k, v in prof.items() if v[1]))
    log(f"[bench] objective after last step: {obj.item():.6e}")

    bf16 = None
    if not args.no_bf16:
        el16, ph16, prof16 = timed(1, Ks, Ws)
        fs16_ms, fs16_calls = prof16["frame_select"]
        fs16_avg_s = fs16_ms / max(fs16_calls, 1) / 1e3
        bf16_peak = 2500.0
        # the method's FLOPs (2 K per frame and component) counted once; the
        # MFMA instructions execute more (split operands), reported apart
        ach16 = flop_per_frame * F / fs16_avg_s / 1e12
        log("[bench] BF16 kernel groups (ms per step): " + ", ".join(
            f"{k}={v[0] / Ks:.2f}" for k, v in prof16.items() if v[1]))
        # one iteration of each form from the same initial model: BF16 vs FP32
        outs = {}
        for prec in (0, 1):
            reset_model()
            step(prec)
            ctx.sync_status()
            outs[prec] = (phi.double().cpu().numpy(), obj.item())
        a, b = outs[1][0], outs[0][0]
        cos = (a * b).sum(1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
        bf16 = {"utts_per_s": round(U * Ks / el16, 3), "ms_per_step": round(el16 * 1e3 / Ks, 3),
                "steps": Ks,
                "frame_posteriors_per_s": round(F * Ks / (ph16["frame"] / 1e3), 1),
                "tv_em_utts_per_s": round(U * Ks / (ph16["em"] / 1e3), 3),
                "frame_kernel": {"kernel": "k_frame_tile_bf16", "achieved_bf16_tflops": round(ach16, 2),
                                 "peak": bf16_peak, "frac": round(ach16 / bf16_peak, 4),
                                 "flops_counted": "method (2 K per frame and component, once)",
                                 "mfma_products_per_method_product": BF16_PRODUCTS,
                                 "hardware_mfma_tflops": round(BF16_PRODUCTS * ach16, 2),
                                 "avg_launch_ms": round(fs16_avg_s * 1e3, 3),
                                 "components_per_launch": C},
                "vs_fp32_form_first_iteration": {
                    "ivector_min_cosine": float(cos.min()),
                    "objective_rel_diff": abs(outs[1][1] - outs[0][1]) / abs(outs[0][1])}}
        log(f"[bench] BF16 form: {bf16}")

    graph = None
    if not args.no_graph:
        graph = graph_replay(ctx, reset_model, X, off, n, f, S, phi, Phi, acc, ll_frames, ll_utt,
                             obj, Ks, Ws, U)
        graph["eager_utts_per_s_same_run"] = round(value, 3)
        log(f"[bench] graph replay: {graph}")

    standard = None
    if not args.no_standard:
        # Sec. 2.1 model with centred statistics, Sigma update and the
        # P1-only minimum divergence; no realignment
        els, phs, profs = timed(0, Ks, Ws, form="standard")
        standard = {"utts_per_s": round(U * Ks / els, 3), "ms_per_step": round(els * 1e3 / Ks, 3),
                    "steps": Ks,
                    "tv_em_utts_per_s": round(U * Ks / (phs["em"] / 1e3), 3),
                    "stats_S_ms_per_step": round(profs["stats_S"][0] / Ks, 3),
                    "stats_nf_ms_per_step": round(profs["stats_nf"][0] / Ks, 3),
                    "objective_after_last_step": obj.item(),
                    "step": "posteriors+centred n/f/S+E-step(p=0)+accumulate+M-step(T,Sigma)"
                            "+min-div(P1)"}
        log(f"[bench] standard formulation: {standard}")

    streamed = None
    if not args.no_stream:
        # the same iteration with the frames left in host memory: batches of
        # utterances stream through pinned slots while the previous batch
        # computes; a context sized for one batch, not for the corpus
        bu, bfr = args.stream_batch_utts, args.stream_batch_frames
        ctx2 = ivx.Context(C, D, R, bu, bfr)
        ctx2.tuning_set(**ctx.tuning_get())
        st = ivx.Stream(ctx2, bu, bfr, loaders=args.stream_loaders, slots=4)
        nb = len(ivx.plan_batches(wl.utt_off, bu, bfr)) - 1
        S2 = torch.zeros_like(S)
        llf2, llu2, obj2 = (torch.zeros(1, dtype=torch.float64, device=dev) for _ in range(3))
        acc2 = ctx2.new_accum()

        def reset2():
            ctx2.set_ubm(w_d, mu_d, cov_d)
            ctx2.init_tv(T0_d, 100.0)

        def sstep():
            S2.zero_()
            llf2.zero_()
            llu2.zero_()
            acc2.zero_()
            st.em_pass(wl.utt_off, acc2, X=wl.X, S_acc=S2, ll_frames=llf2, ll_utts=llu2)
            ctx2.tv_mstep_solve(acc2, S2, update_sigma=True, ll_sum=llu2, objective=obj2)
            ctx2.tv_mindiv(acc2)
            ctx2.ubm_update_means()

        reset2()
        sstep()
        ctx2.sync_status()
        reset_model()
        step(0)
        ctx.sync_status()
        obj_res, obj_str = obj.item(), obj2.item()
        T_res, T_str = ctx.get_tv()[0], ctx2.get_tv()[0]
        t_rel = ((T_str - T_res).norm() / T_res.norm()).item()
        reset2()
        for _ in range(Ws):
            sstep()
        ctx2.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(Ks):
            sstep()
        torch.cuda.synchronize()
        els = time.perf_counter() - t0
        ctx2.sync_status()
        streamed = {"utts_per_s": round(U * Ks / els, 3), "ms_per_step": round(els * 1e3 / Ks, 3),
                    "steps": Ks,
                    "batches_per_step": nb, "batch_limits": {"utterances": bu, "frames": bfr},
                    "loaders": args.stream_loaders, "host_bytes_per_step": int(wl.X.nbytes),
                    "vs_resident_first_iteration": {
                        "objective_rel_diff": abs(obj_str - obj_res) / abs(obj_res),
                        "T_rel_diff": t_rel}}
        log(f"[bench] streamed from host: {streamed}")
        st.close()
        del acc2, S2
        ctx2.close()

    backend = None
    if not args.no_backend:
        backend = backend_block(ctx, wl, dev)
        log(f"[bench] back-end on synthetic speakers: {backend}")

    pruned = None
    if not args.no_pruned:
        ctx.pruned_set(20, 0.025)
        elp, php, profp = timed(0, Ks, Ws, sel=ivx.IVX_SEL_PRUNED)
        outs = []
        for sel in (ivx.IVX_SEL_ALL, ivx.IVX_SEL_PRUNED):
            reset_model()
            step(0, sel=sel)
            ctx.sync_status()
            outs.append(phi.double().cpu().numpy())
        a, b = outs
        cos = (a * b).sum(1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
        pruned = {"utts_per_s": round(U * Ks / elp, 3), "ms_per_step": round(elp * 1e3 / Ks, 3),
                  "steps": Ks,
                  "frame_posteriors_per_s": round(F * Ks / (php["frame"] / 1e3), 1),
                  "diag_select_ms_per_step": round(profp["sel_mlp"][0] / Ks, 3),
                  "scoring_ms_per_step": round(profp["sel_score"][0] / Ks, 3),
                  "vs_plain_first_iteration": {"ivector_min_cosine": float(cos.min())}}
        log(f"[bench] pruned alignment: {pruned}")

    learned = None
    if args.learned_steps > 0:
        learned = learned_form(args, ctx, wl, X, step, timed, reset_model, phi, Ks, Ws, dev)
        log(f"[bench] learned selection: {learned}")

    sweep = None
    if args.learned_sweep:
        sweep = learned_sweep(args, ctx, wl, X, dev)

    batching = None
    if gen4 is not None:
        wl4 = gen4.join()
        log(f"[bench] batching workload: U={wl4.U} F={wl4.F} (generated in {gen4.seconds:.1f}s "
            "beside the GPU work)")
        batching = batching_block(args, wl4, tune_now, dev)
        del wl4
        log(f"[bench] batching workload: {batching}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample ...")
        t0 = time.time()
        nf = min(args.cpu_frame_utts, U)
        cpu = cpu_baseline(wl, nf, args.cpu_estep_utts, min(args.cpu_components, C),
                           max(1, nf // 8), max(1, args.cpu_estep_utts // 20))
        log(f"[bench] cpu baseline ({time.time() - t0:.0f}s): {cpu}")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "utts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"shape{args.shape}:{sh.name}", "D": D, "C": C, "R": R,
                   "utterances": U, "frames": F,
                   "step": "posteriors+n/f/S+E-step+accumulate+M-step(T,Sigma)+min-div+realign"},
        "frame_posteriors_per_s": round(frames_per_s, 1),
        "tv_em_utts_per_s": round(em_utts_per_s, 3),
        "phase_ms_per_step": {"frame_stage": round(phase["frame"] / K, 3),
                              "em_stage": round(phase["em"] / K, 3)},
        "roofline": roof,
        "tuning": tuning,
        "bf16_form": bf16,
        "graph_replay": graph,
        "batching_loguniform": batching,
        "standard_formulation": standard,
        "backend_synthetic_speakers": backend,
        "streamed_from_host": streamed,
        "pruned_alignment": pruned,
        "learned_selection": learned,
        "learned_sweep": sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
