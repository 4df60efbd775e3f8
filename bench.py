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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shape", type=int, default=2, help="workload shape id (synth.SHAPES)")
    ap.add_argument("--n-utts", type=int, default=None, help="first U utterances only")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-utts", type=int, default=6)
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 form")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device-to-device once "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--graph", action="store_true",
                    help="also time the EM iteration replayed from a captured HIP graph")
    ap.add_argument("--learned-steps", type=int, default=3000,
                    help="training steps of the learned selector (0: skip the learned form)")
    ap.add_argument("--learned-batch", type=int, default=4096)
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


def cpu_baseline(wl, n_sample):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload.

    Per-utterance work (posteriors over all C, n/f/S, E-step, accumulation)
    is timed on the first ``n_sample`` utterances; the per-iteration fixed
    work (V_c / U_c precompute, M-step solve, minimum divergence) is timed
    once and spread over the workload's U utterances.  Returns utts/s of a
    whole EM iteration at the workload's U.
    """
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_info

    a, b = 0, n_sample
    off = wl.utt_off[: b + 1]
    F = int(off[-1])
    X = wl.X[:F]
    tv = oracle.init_tv(wl.mu, wl.cov, wl.T_init)
    t0 = time.perf_counter()
    gamma, lse = oracle.posteriors(oracle.frame_loglik(X, wl.w, wl.mu, wl.cov))
    n, f, S = oracle.bw_stats(X, off, gamma)
    t_frame = time.perf_counter() - t0
    t0 = time.perf_counter()
    V, Uc = oracle.tv_precompute(*tv[:2])
    t_pre = time.perf_counter() - t0
    del V, Uc
    t0 = time.perf_counter()
    e = oracle.estep(n, f, *tv)
    acc = oracle.accumulate(n, f, e["phi"], e["Phi"])
    t_utt = time.perf_counter() - t0 - t_pre  # estep() repeats the precompute
    t0 = time.perf_counter()
    T1, S1, _ = oracle.mstep(acc, S, tv[0], tv[1])
    h, H = acc["hsum"] / acc["count"], acc["Hsum"] / acc["count"]
    oracle.mindiv(h, H, T1)
    t_fixed_m = time.perf_counter() - t0
    U = wl.U
    per_utt = (t_frame + max(t_utt, 0.0)) / n_sample
    fixed = t_pre + t_fixed_m
    total = per_utt * U + fixed
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {
        "value": U / total,
        "unit": "utts/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"first {n_sample} utterances ({F} frames) for posteriors, n/f/S, E-step and "
                   f"accumulation; one V/U precompute, M-step solve and min-div; scaled to U={U} "
                   f"(frame part {t_frame:.1f}s, E-step part {max(t_utt, 0):.1f}s, fixed "
                   f"{fixed:.1f}s)"),
        "frames_per_s": F / t_frame,
    }


def learned_form(args, ctx, wl, X, step, timed, reset_model, phi, K, dev):
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
    el, ph, prof = timed(0, K, args.warmup, sel=ivx.IVX_SEL_LEARNED)
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
        "utts_per_s": round(U * K / el, 3), "ms_per_step": round(el * 1e3 / K, 3),
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
    K = args.steps
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
    # launch per tile of 32 * frame_ncb components (Cpad / tile launches per
    # pass over the frames)
    Kexp = (D + 1) * (D + 2) // 2
    tune_now = ctx.tuning_get()
    tile = 256 if tune_now["frame_ncb"] == 8 else 128
    flop_per_frame_tile = 2.0 * Kexp * tile
    fs_ms, fs_calls = prof["frame_select"]
    fs_avg_s = fs_ms / max(fs_calls, 1) / 1e3
    achieved = flop_per_frame_tile * F / fs_avg_s / 1e12
    roof = {"kernel": "k_frame_tile", "bound": "mfma", "achieved": round(achieved, 2),
            "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("k_frame_tile", f"shape{args.shape}", F),
            "avg_launch_ms": round(fs_avg_s * 1e3, 3), "launches_per_step": fs_calls // K,
            "flop_per_frame_per_launch": flop_per_frame_tile, "frames_per_launch": F,
            "components_per_launch": tile}
    log("[bench] FP32 kernel groups (ms per step): " + ", ".join(
        f"{k}={v[0] / K:.2f}" for k, v in prof.items() if v[1]))
    log(f"[bench] objective after last step: {obj.item():.6e}")

    bf16 = None
    if not args.no_bf16:
        el16, ph16, prof16 = timed(1, K, args.warmup)
        fs16_ms, fs16_calls = prof16["frame_select"]
        fs16_avg_s = fs16_ms / max(fs16_calls, 1) / 1e3
        bf16_peak = 2500.0
        tile16 = 256 if tune_now["frame_ncb_bf16"] == 8 else 128
        # three BF16 products (hi*hi, hi*lo, lo*hi) per FP32 one
        ach16 = 3.0 * 2.0 * Kexp * tile16 * F / fs16_avg_s / 1e12
        log("[bench] BF16 kernel groups (ms per step): " + ", ".join(
            f"{k}={v[0] / K:.2f}" for k, v in prof16.items() if v[1]))
        # one iteration of each form from the same initial model: BF16 vs FP32
        outs = {}
        for prec in (0, 1):
            reset_model()
            step(prec)
            ctx.sync_status()
            outs[prec] = (phi.double().cpu().numpy(), obj.item())
        a, b = outs[1][0], outs[0][0]
        cos = (a * b).sum(1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
        bf16 = {"utts_per_s": round(U * K / el16, 3), "ms_per_step": round(el16 * 1e3 / K, 3),
                "frame_posteriors_per_s": round(F * K / (ph16["frame"] / 1e3), 1),
                "tv_em_utts_per_s": round(U * K / (ph16["em"] / 1e3), 3),
                "frame_kernel": {"kernel": "k_frame_tile_bf16", "achieved_bf16_tflops": round(ach16, 2),
                                 "peak": bf16_peak, "frac": round(ach16 / bf16_peak, 4),
                                 "avg_launch_ms": round(fs16_avg_s * 1e3, 3),
                                 "components_per_launch": tile16},
                "vs_fp32_form_first_iteration": {
                    "ivector_min_cosine": float(cos.min()),
                    "objective_rel_diff": abs(outs[1][1] - outs[0][1]) / abs(outs[0][1])}}
        log(f"[bench] BF16 form: {bf16}")

    graph = None
    if args.graph:
        reset_model()
        g = ctx.graph_create_em(X, off, n, f, S, phi, Phi, acc, ll_frames, ll_utt, obj)
        for _ in range(args.warmup):
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
        graph = {"utts_per_s": round(U * K / elg, 3), "ms_per_step": round(elg * 1e3 / K, 3)}
        log(f"[bench] graph replay: {graph}")

    standard = None
    if not args.no_standard:
        # Sec. 2.1 model with centred statistics, Sigma update and the
        # P1-only minimum divergence; no realignment
        els, phs, profs = timed(0, K, args.warmup, form="standard")
        standard = {"utts_per_s": round(U * K / els, 3), "ms_per_step": round(els * 1e3 / K, 3),
                    "tv_em_utts_per_s": round(U * K / (phs["em"] / 1e3), 3),
                    "stats_S_ms_per_step": round(profs["stats_S"][0] / K, 3),
                    "stats_nf_ms_per_step": round(profs["stats_nf"][0] / K, 3),
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
        for _ in range(args.warmup):
            sstep()
        ctx2.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            sstep()
        torch.cuda.synchronize()
        els = time.perf_counter() - t0
        ctx2.sync_status()
        streamed = {"utts_per_s": round(U * K / els, 3), "ms_per_step": round(els * 1e3 / K, 3),
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
        elp, php, profp = timed(0, K, args.warmup, sel=ivx.IVX_SEL_PRUNED)
        outs = []
        for sel in (ivx.IVX_SEL_ALL, ivx.IVX_SEL_PRUNED):
            reset_model()
            step(0, sel=sel)
            ctx.sync_status()
            outs.append(phi.double().cpu().numpy())
        a, b = outs
        cos = (a * b).sum(1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
        pruned = {"utts_per_s": round(U * K / elp, 3), "ms_per_step": round(elp * 1e3 / K, 3),
                  "frame_posteriors_per_s": round(F * K / (php["frame"] / 1e3), 1),
                  "diag_select_ms_per_step": round(profp["sel_mlp"][0] / K, 3),
                  "scoring_ms_per_step": round(profp["sel_score"][0] / K, 3),
                  "vs_plain_first_iteration": {"ivector_min_cosine": float(cos.min())}}
        log(f"[bench] pruned alignment: {pruned}")

    learned = None
    if args.learned_steps > 0:
        learned = learned_form(args, ctx, wl, X, step, timed, reset_model, phi, K, dev)
        log(f"[bench] learned selection: {learned}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample ...")
        cpu = cpu_baseline(wl, min(args.cpu_sample_utts, U))
        log(f"[bench] cpu baseline: {cpu['value']:.3f} utts/s, {cpu['frames_per_s']:.0f} frames/s "
            f"({cpu['cores']} threads)")
        cpu.pop("frames_per_s")

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
        "standard_formulation": standard,
        "backend_synthetic_speakers": backend,
        "streamed_from_host": streamed,
        "pruned_alignment": pruned,
        "learned_selection": learned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
