"""Benchmark of FastMap's epipolar-adjustment hot path on one MI355X.

Headline workload (the large street scene): 5,000 cameras in a 12x12-block
city, ~185k image pairs, ~172M matches stored as BF16 (~1.4 GB), 1.5 px
noise, 30 % outliers.  One step is one whole epipolar-adjustment solve:
2,000 Adam iterations in 20 loops of 100 (each loop one persistent fused
loss + adjoint + Adam kernel), with the IRLS reweight + Gram rebuild
(fm_reweight_build, one pass over all matches) before every loop.

Reported (one JSON line):
  value           Gram-build throughput in matches/s: matches divided by the
                  device time of one whole fm_reweight_build call (the sum
                  of its three kernels' durations, each timed by HIP events
                  the runtime records at the kernel's own dispatch, averaged
                  over the timed steps; gram_call_bracket_us is the interval
                  between events recorded on the stream around the call,
                  which also holds the gaps the timing events themselves
                  add between the kernels); 0 unless every pair's final relative rotation is
                  within 0.1 deg and translation direction within 0.5 deg of
                  the stored FP64 oracle solve (tests/golden/large_oracle.json)
                  and no grid barrier failed;
  iters_per_s     Adam iterations per second of device time of the fused
                  solve kernel (the pair-by-pair loop at this size);
  roofline        of the Gram call: bound by vector ALU issue with BF16
                  coordinates (65 lane-operations per match against 256 CUs x
                  4 SIMDs x 16 lanes x 2.4 GHz), with its HBM fraction (8 B
                  per match, 296 B per pair, 36 B per camera) against the
                  vendor 8 TB/s and the copy bandwidth measured on the GPU;
  roofline_iteration
                  bytes and rate of the fused iteration, the kernel that
                  dominates the step;
  errors_vs_fp64  Grams of sampled pairs and the loss against the oracle;
  cpu_baseline    the FP64 oracle on a bounded sample of the same scene, in
                  one process and split over worker processes;
  medium          the medium scene (200 cameras, ~2.9M FP32 matches): its own
                  pose-checked solve, Gram-call and iteration figures, and the
                  widened stages on it (translation averaging, rotation
                  averaging, the relative-translation grid search, focal
                  refinement, the stages in sequence, the learned-weight MLP).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-medium] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAFFIC_MEDIUM = os.path.join(ROOT, "profiles", "gram_medium_traffic.json")
TRAFFIC_LARGE = os.path.join(ROOT, "profiles", "gram_large_traffic.json")
GRAM_SRC = os.path.join(ROOT, "paper_2505_04612_amd", "csrc", "gram.hip")
HBM_PEAK_GBPS = 8000.0
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12     # lane-instructions per second, non-packed
VALU_PER_MATCH_BF16 = 65                       # IRLS Gram pass, BF16 coordinates


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def scene_digest(sc, coords) -> str:
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sc.pairs, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(sc.offsets, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(coords).tobytes())
    h.update(np.ascontiguousarray(sc.R_init).tobytes())
    h.update(np.ascontiguousarray(sc.t_init).tobytes())
    return h.hexdigest()


def _oracle_gram_range(job):
    """Worker of the CPU baseline: the oracle's reweight + Gram pass over a
    contiguous range of whole pairs, with one BLAS thread; returns seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ea
    theta, pairs, offsets, x, delta, tau = job
    with threadpool_limits(1):
        t = time.perf_counter()
        w = ea.irls_weights(ea.residuals(theta, pairs, offsets, x), delta, tau)
        ea.pair_grams(x, offsets, w)
        return time.perf_counter() - t


def _pair_range_jobs(sc, x, theta, lo_pair: int, hi_pair: int, parts: int, delta: float, tau: float):
    """Split pairs [lo_pair, hi_pair) into `parts` ranges of about equal match
    count, each with rebased offsets and its own slice of the coordinates."""
    import numpy as np
    off = sc.offsets
    m0, m1 = int(off[lo_pair]), int(off[hi_pair])
    cuts = [lo_pair]
    for k in range(1, parts):
        cuts.append(int(np.searchsorted(off, m0 + (m1 - m0) * k // parts, side="left")))
    cuts.append(hi_pair)
    jobs = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b <= a:
            continue
        lo, hi = int(off[a]), int(off[b])
        jobs.append((theta, sc.pairs[a:b], off[a:b + 1] - lo, x[lo:hi], delta, tau))
    return jobs


def cpu_baseline(sc, x, theta0, sched_d, budget_s: float = 20.0, workers: int = 0) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    its reweight + Gram pass over a seeded contiguous run of whole pairs (one
    process with one BLAS thread, then the same kind of run split over
    `workers` processes with one BLAS thread each), and its loss + gradient +
    Adam iterations over all pairs (one process).  `x` holds the stored
    coordinates as float64."""
    import concurrent.futures
    import multiprocessing

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ea
    th = theta0.astype(np.float64)
    P, M = sc.num_pairs, sc.num_matches
    delta, tau = sched_d["delta"], sched_d["tau0"]
    rng = np.random.default_rng(11)
    nproc = os.cpu_count() or 1
    workers = workers if workers > 0 else max(1, min(16, nproc))

    def pair_run(matches: int):
        lo = int(rng.integers(0, P))
        hi = int(np.searchsorted(sc.offsets, sc.offsets[lo] + matches, side="left"))
        hi = min(max(hi, lo + 1), P)
        if sc.offsets[hi] - sc.offsets[lo] < matches and lo > 0:
            lo = max(0, int(np.searchsorted(sc.offsets, sc.offsets[hi] - matches, side="right")) - 1)
        return lo, hi

    # one process, one BLAS thread: a run of whole pairs sized to ~budget/3
    probe_lo, probe_hi = pair_run(min(M, 500_000))
    probe = _pair_range_jobs(sc, x, th, probe_lo, probe_hi, 1, delta, tau)[0]
    t_probe = _oracle_gram_range(probe)
    rate1 = (sc.offsets[probe_hi] - sc.offsets[probe_lo]) / max(t_probe, 1e-9)
    lo1, hi1 = pair_run(int(min(M, rate1 * budget_s / 3)))
    job1 = _pair_range_jobs(sc, x, th, lo1, hi1, 1, delta, tau)[0]
    t1 = _oracle_gram_range(job1)
    m1 = int(sc.offsets[hi1] - sc.offsets[lo1])
    # `workers` processes, one BLAS thread each, on a run `workers` times larger
    ctxm = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctxm) as ex:
        list(ex.map(_oracle_gram_range, [probe] * workers))       # start and warm every worker
        lon, hin = pair_run(int(min(M, rate1 * budget_s / 3 * workers)))
        jobs = _pair_range_jobs(sc, x, th, lon, hin, workers, delta, tau)
        t = time.perf_counter()
        list(ex.map(_oracle_gram_range, jobs))
        tn = time.perf_counter() - t
    mn = int(sc.offsets[hin] - sc.offsets[lon])
    # iterations over all pairs, one process: W from the single-process run's
    # pairs is enough to time the arithmetic (the loss does not need the
    # Grams of every pair to cost the same); use the real Grams of that run
    # and zeros elsewhere
    W = np.zeros((P, 9, 9))
    w = ea.irls_weights(ea.residuals(th, job1[1], job1[2], job1[3]), delta, tau)
    W[lo1:hi1] = ea.pair_grams(job1[3], job1[2], w)
    inv_Z = 1.0 / max(int(np.count_nonzero(w)), 1)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    lr = np.array([sched_d["lr_rot"]] * 6 + [sched_d["lr_t"]] * 3)
    n_it, t_it = 0, 0.0
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    w0 = time.perf_counter()
    while t_it < budget_s / 3 or n_it < 3:
        t = time.perf_counter()
        _, g = ea.loss_grad(th, sc.pairs, W, inv_Z)
        th, m, v = ea.adam_step(th, g, m, v, n_it + 1, lr)
        t_it += time.perf_counter() - t
        n_it += 1
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    it_cores = ((r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)) / max(time.perf_counter() - w0, 1e-9)
    return {
        "value": mn / tn, "unit": "matches/s", "cores": workers, "kind": "oracle",
        "value_1_core": m1 / t1,
        "iters_per_s": n_it / t_it, "iters_cores": round(it_cores, 2),
        "sample": (f"FP64 reweight + Gram pass: {mn} matches ({hin - lon} whole pairs) split over {workers} "
                   f"processes with 1 BLAS thread each in {tn:.1f} s, and {m1} matches ({hi1 - lo1} pairs) in "
                   f"one process with 1 BLAS thread in {t1:.1f} s; {n_it} loss+gradient+Adam iterations over all "
                   f"{P} pairs in one process ({t_it:.1f} s)"),
        "host_cpu": _cpu_model(), "nproc": nproc,
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _file_sha(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def bench_translation(ctx, s, sc, runs: int = 4, iters: int = 1000, final_iters: int = 1000,
                      cpu_budget: float = 3.0) -> dict:
    """Global translation averaging on the scene's pair graph: noisy unit
    relative translations (2 deg, 10 % outliers) from the true poses, `runs`
    random initialisations solved together, merge, final loop."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api, synth, translation
    dev = ctx.device
    inp = synth.translation_inputs(sc, runs=runs)
    params = api.params_from_poses(torch.from_numpy(sc.R_gt).to(dev), torch.from_numpy(sc.t_gt).to(dev))
    dirs = api.translation_directions(s, params, torch.from_numpy(inp.t_rel.astype(np.float32)).to(dev))
    init = torch.from_numpy(inp.init.astype(np.float32)).to(dev)
    sched = translation.TranslationSchedule(iters=iters, final_iters=final_iters)

    def stage(timed: bool):
        c = init.clone()
        m, v = torch.zeros_like(c), torch.zeros_like(c)
        if timed:
            ctx.profile(True)
        api.translation_solve(s, dirs, c, m, v, iters, sched.lr, sched.lr_final_frac)
        ms_runs = ctx.profile_read(_lib.K_TA_SOLVE)[0] if timed else 0.0
        merged, choice, _ = api.translation_merge(s, dirs, c)
        f = merged.unsqueeze(0).contiguous()
        m1, v1 = torch.zeros_like(f), torch.zeros_like(f)
        if timed:
            ctx.profile(True)
        api.translation_solve(s, dirs, f, m1, v1, final_iters, sched.lr, sched.lr_final_frac)
        ms_final = ctx.profile_read(_lib.K_TA_SOLVE)[0] if timed else 0.0
        if timed:
            ctx.profile(False)
        return c, f[0], choice, ms_runs, ms_final

    stage(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, o, choice, ms_runs, ms_final = stage(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bar_fail = s.barrier_failures()
    from oracle import translation as ta
    gt = ta.normalize(-np.einsum("nba,nb->na", sc.R_gt, sc.t_gt))
    err = np.linalg.norm(ta.normalize(o.cpu().numpy().astype(np.float64)) - gt, axis=1)
    run_err = [float(np.linalg.norm(ta.normalize(c[r].cpu().numpy().astype(np.float64)) - gt, axis=1).max())
               for r in range(runs)]
    # the oracle as it stands: loss + gradient + Adam steps of one run
    d64 = ta.target_directions(sc.R_gt, inp.t_rel.astype(np.float32).astype(np.float64), sc.pairs)
    x = inp.init[0].astype(np.float32).astype(np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    n_it, t_it = 0, 0.0
    while t_it < cpu_budget or n_it < 5:
        t = time.perf_counter()
        _, g = ta.loss_grad(x, sc.pairs, d64)
        x, m, v = ta.adam_step(x, g, m, v, n_it + 1, ta.lr_at(sched.lr, sched.lr_final_frac, iters, n_it))
        t_it += time.perf_counter() - t
        n_it += 1
    P = sc.num_pairs
    return {
        "kernel": "k_ta_solve_cam (persistent, one wavefront per camera: each pair's L1 term + adjoint from "
                  "both cameras, Adam, 1 grid barrier)",
        "pairs": P, "cameras": sc.num_cams, "runs": runs, "iters": iters, "final_iters": final_iters,
        "run_iters_per_s": runs * iters / (ms_runs / 1e3),
        "us_per_iter_all_runs": ms_runs * 1e3 / iters,
        "us_per_iter_one_run": ms_final * 1e3 / final_iters,
        "stage_wall_ms": wall * 1e3,
        "bound": "latency (one grid barrier per iteration; each pair read from both cameras: "
                 "2 x %d B per pair and run through L2)" % (8 + 12 + 24),
        "centre_err_vs_truth": {"median": float(np.median(err)), "max": float(err.max()),
                                "single_run_max": run_err},
        "inputs": "unit relative translations from the true poses, 2 deg noise, 10 % outlier pairs; "
                  "centres N(0, I) per run",
        "barrier_failures": bar_fail,
        "cpu_baseline": {"run_iters_per_s": n_it / t_it, "kind": "oracle",
                         "sample": f"{n_it} FP64 loss+gradient+Adam steps of one run over {P} pairs"},
    }


def measure_copy_gbps(device, nbytes: int = 512 << 20, reps: int = 5) -> float:
    """Device-to-device copy bandwidth on this GPU (read + write bytes per
    second, median of `reps` copies of `nbytes`, larger than the 256 MB
    Infinity Cache): the measured ceiling the vendor 8 TB/s is set beside."""
    import numpy as np
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / float(np.median(times)) / 1e9


FP64_PEAK_T = 78.6    # TFLOP/s, FP64 vector (MI355X)


def bench_pipeline(ctx, s, sc) -> dict:
    """The pose stages in sequence from noisy relative rotations (2 deg, 10 %
    outlier pairs), the scene's inlier matches and the true directions as
    translation sign priors."""
    import numpy as np
    import torch

    from oracle import ea
    from paper_2505_04612_amd import pipeline, synth
    dev = ctx.device
    rin = synth.rotation_inputs(sc)
    Q = torch.from_numpy(rin.R_rel.reshape(-1, 9).astype(np.float32)).to(dev)
    o = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    i, j = sc.pairs[:, 0], sc.pairs[:, 1]
    prior = np.einsum("pab,pb->pa", sc.R_gt[j], o[i] - o[j])
    prior = torch.from_numpy((prior / np.linalg.norm(prior, axis=1, keepdims=True)).astype(np.float32)).to(dev)
    keep = torch.from_numpy((~sc.outlier).astype(np.float32)).to(dev)
    pipeline.run(s, Q, prior, keep)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, stages = pipeline.run(s, Q, prior, keep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gt = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1)
    out = {"wall_ms": wall * 1e3, "barrier_failures": s.barrier_failures()}
    for name, th in (("after_averaging", stages["averaged"]), ("after_epipolar_adjustment", params)):
        rot, tra = ea.relative_pose_errors(th.cpu().numpy().astype(np.float64), gt, sc.pairs)
        out[name] = {"rot_median_deg": float(np.median(rot)), "rot_p90_deg": float(np.quantile(rot, 0.9)),
                     "rot_max_deg": float(rot.max()), "t_median_deg": float(np.median(tra)),
                     "t_p90_deg": float(np.quantile(tra, 0.9)), "t_max_deg": float(tra.max())}
    out["inputs"] = ("relative rotations from the true poses with 2 deg noise and 10 % outlier pairs; Grams of "
                     "the inlier matches; true directions as the sign priors of the grid search")
    return out


def bench_focal(ctx, sc, kappa: float = 1.05, iters: int = 300, reps: int = 50) -> dict:
    """Focal refinement on the scene's matches normalised with a focal 1/kappa
    of the true one: Grams of the inlier matches, poses held at the truth
    while the log focal scales are refined (then also the poses)."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api, focal
    dev = ctx.device
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, (sc.uv * kappa).astype(np.float32),
                             torch.float32)
    keep = torch.from_numpy((~sc.outlier).astype(np.float32)).to(dev)
    W64, _ = api.build_pair_grams(s, keep, f32=False)
    iz = 1.0 / float(keep.sum().item())
    theta = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1).astype(np.float32)
    p = torch.from_numpy(theta).to(dev)
    phi = torch.zeros(sc.num_cams, dtype=torch.float32, device=dev)
    api.epipolar_focal_loss_grad(s, W64, p, phi, iz)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        api.epipolar_focal_loss_grad(s, W64, p, phi, iz)
    pair_ms, _ = ctx.profile_read(_lib.K_FO_PAIR)
    cam_ms, _ = ctx.profile_read(_lib.K_FO_CAMERA)
    ctx.profile(False)
    # the host loop (loss + gradient and two Adam launches per step), for reference
    ph_h = phi.clone()
    focal.solve(s, W64, p.clone(), ph_h, iz, focal.FocalSchedule(iters=10, lr_rot=0.0, lr_t=0.0), fused=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    focal.solve(s, W64, p.clone(), ph_h, iz, focal.FocalSchedule(iters=iters, lr_rot=0.0, lr_t=0.0), fused=False)
    torch.cuda.synchronize()
    wall_host = time.perf_counter() - t0
    # the persistent loop (warm-up on copies, then timed)
    focal.solve(s, W64, p.clone(), phi.clone(), iz, focal.FocalSchedule(iters=10, lr_rot=0.0, lr_t=0.0))
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    focal.solve(s, W64, p, phi, iz, focal.FocalSchedule(iters=iters, lr_rot=0.0, lr_t=0.0))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fused_ms, _ = ctx.profile_read(_lib.K_FO_SOLVE)
    ctx.profile(False)
    err = np.abs(phi.cpu().numpy() - np.log(kappa))
    p2 = torch.from_numpy(theta).to(dev)
    phi2 = torch.zeros(sc.num_cams, dtype=torch.float32, device=dev)
    focal.solve(s, W64, p2, phi2, iz, focal.FocalSchedule(iters=iters, lr_rot=1e-4, lr_t=1e-4))
    err2 = np.abs(phi2.cpu().numpy() - np.log(kappa))
    s.close()
    return {
        "kernels": "k_fo_solve (persistent, one wavefront per camera: each pair's fundamental-matrix term + "
                   "adjoint from both cameras, Adam on poses and scales); standalone: k_fo_pair + k_fo_camera",
        "pairs": sc.num_pairs, "cameras": sc.num_cams, "focal_error": kappa,
        "us_per_fused_iter": fused_ms * 1e3 / iters,
        "us_per_loss_grad": (pair_ms + cam_ms) * 1e3 / reps,
        "us_pair_kernel": pair_ms * 1e3 / reps, "us_camera_kernel": cam_ms * 1e3 / reps,
        "solve_ms_wall": wall * 1e3, "solve_ms_wall_host_loop": wall_host * 1e3, "iters": iters,
        "log_scale_error": {"poses_held_median": float(np.median(err)), "poses_held_max": float(err.max()),
                            "poses_free_median": float(np.median(err2)), "poses_free_max": float(err2.max())},
        "inputs": "the scene's matches normalised with focal 500/1.05 px (true 500 px), Grams of the inlier matches",
    }


MFMA_F16_PEAK_T = 2500.0   # TFLOP/s, dense FP16 MFMA (MI355X)


def bench_mlp(ctx, M: int, reps: int = 20) -> dict:
    """The learned-weight MLP (3 -> 64 -> 64 -> 1) over M matches of seeded
    random features and weights: forward alone (what a solve runs), forward
    keeping the activations, and backward.  Flops counted: the 64 x 64 layer
    on MFMA (2 * 4096 per match per pass; the backward has two such
    products), against the dense FP16 MFMA peak; bytes: the features and
    outputs (forward), plus the FP16 activations (kept / backward)."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import api
    dev = ctx.device
    rng = np.random.default_rng(5)
    feats = torch.from_numpy(rng.normal(size=(M, 3)).astype(np.float32)).to(dev)
    w = api.MlpWeights(dev)
    w.load_numpy({k: rng.normal(scale=0.3, size=sh) for k, sh in api.MLP_SHAPES.items()},
                 np.zeros(3), np.ones(3))
    dout = torch.from_numpy(rng.normal(size=M).astype(np.float32)).to(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    t_fwd = timed(lambda: api.mlp_forward(ctx, w, feats))
    _, act = api.mlp_forward(ctx, w, feats, keep_act=True)
    t_fwd_act = timed(lambda: api.mlp_forward(ctx, w, feats, keep_act=True))
    g = api.MlpWeights(dev)
    t_bwd = timed(lambda: api.mlp_backward(ctx, w, feats, act, dout, g))
    fl = 2.0 * 64 * 64
    return {
        "kernels": "k_mlp_forward (64x64 layer on v_mfma_f32_16x16x32_f16, 64->1 layer on v_mfma_f32_16x16x16_f16), "
                   "k_mlp_backward (dh1 on "
                   "v_mfma_f32_16x16x32_f16, dW2 on v_mfma_f32_16x16x16_f16) + k_mlp_reduce",
        "matches": M,
        "forward_us": t_fwd * 1e6, "forward_matches_per_s": M / t_fwd,
        "forward_keep_act_us": t_fwd_act * 1e6, "backward_us": t_bwd * 1e6,
        "roofline_forward": {"mfma_TFLOPs": fl * M / t_fwd / 1e12, "mfma_frac": fl * M / t_fwd / 1e12 / MFMA_F16_PEAK_T,
                             "hbm_GBps": 16.0 * M / t_fwd / 1e9, "hbm_frac": 16.0 * M / t_fwd / 1e9 / HBM_PEAK_GBPS},
        "roofline_backward": {"mfma_TFLOPs": 2 * fl * M / t_bwd / 1e12,
                              "mfma_frac": 2 * fl * M / t_bwd / 1e12 / MFMA_F16_PEAK_T,
                              "hbm_GBps": (12.0 + 256.0 + 4.0) * M / t_bwd / 1e9,
                              "hbm_frac": (12.0 + 256.0 + 4.0) * M / t_bwd / 1e9 / HBM_PEAK_GBPS},
        "inputs": "seeded N(0,1) features and N(0, 0.3^2) weights; as many matches as the scene",
    }


def bench_search(ctx, s, sc, C: int = 4096, reps: int = 20, cpu_pairs: int = 200) -> dict:
    """Grid search of the unit relative translation of every pair over C
    Fibonacci-lattice candidates, from the Grams of the matches an upstream
    two-view estimate keeps (the generator's inliers: weight 1, outliers 0)
    and the true rotations; the prior sign is the true direction's."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api
    dev = ctx.device
    keep = torch.from_numpy((~sc.outlier).astype(np.float32)).to(dev)
    W64, _ = api.build_pair_grams(s, keep, f32=False)
    params = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1).astype(np.float32)
    o = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    i, j = sc.pairs[:, 0], sc.pairs[:, 1]
    t_true = np.einsum("pab,pb->pa", sc.R_gt[j], o[i] - o[j])
    t_true /= np.linalg.norm(t_true, axis=1, keepdims=True)
    p_dev = torch.from_numpy(params).to(dev)
    prior = torch.from_numpy(t_true.astype(np.float32)).to(dev)
    cand = api.fibonacci_sphere(C, dev)
    api.translation_search(s, W64, p_dev, cand, prior)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        t, best, err = api.translation_search(s, W64, p_dev, cand, prior)
    ms, n = ctx.profile_read(_lib.K_TS_SEARCH)
    ctx.profile(False)
    per = ms / 1e3 / max(n, 1)
    P = sc.num_pairs
    evals = P * C / per
    # per candidate and pair: 6 products of the form's entries by the
    # candidate's monomials and 5 additions (the monomials are per candidate,
    # shared by all pairs): 11 FP64 flops
    flops = 11.0 * evals
    ang = np.degrees(np.arccos(np.clip(np.sum(t.cpu().numpy().astype(np.float64) * t_true, axis=1), -1, 1)))
    from oracle import grid_search as gs
    W = W64[:cpu_pairs].cpu().numpy()
    full = np.empty((cpu_pairs, 9, 9))
    q = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 2, (0, 2): 3, (2, 0): 3, (1, 2): 4, (2, 1): 4, (2, 2): 5}
    for a in range(3):
        for b in range(3):
            for c in range(3):
                for d in range(3):
                    full[:, 3 * a + b, 3 * c + d] = W[:, 6 * q[(a, c)] + q[(b, d)]]
    Rij = gs.relative_rotations(params.astype(np.float64), sc.pairs[:cpu_pairs])
    cand_np = gs.fibonacci_sphere(C)
    t0 = time.perf_counter()
    gs.grid_search(full, np.diff(sc.offsets)[:cpu_pairs], Rij, cand_np, t_true[:cpu_pairs])
    t_cpu = time.perf_counter() - t0
    return {
        "kernel": "k_ts_search (per-pair 3x3 form from the Gram, candidates in LDS, argmin over lane slices)",
        "pairs": P, "candidates": C, "us_per_launch": per * 1e6, "evals_per_s": evals,
        "roofline": {"bound": "alu", "achieved": flops / 1e12, "peak": FP64_PEAK_T, "unit": "TFLOP/s",
                     "frac": flops / 1e12 / FP64_PEAK_T, "flops_per_eval": 11},
        "angle_to_truth_deg": {"median": float(np.median(ang)), "p90": float(np.quantile(ang, 0.9)),
                               "max": float(ang.max())},
        "inputs": "Grams of the inlier matches (the outliers an upstream two-view estimate removes have weight 0), "
                  "true rotations, true direction as sign prior",
        "cpu_baseline": {"evals_per_s": cpu_pairs * C / t_cpu, "kind": "oracle",
                         "sample": f"errors of all {C} candidates for {cpu_pairs} pairs ({t_cpu:.1f} s)"},
    }


def bench_rotation(ctx, s, sc, steps: int = 300, iters: int = 500, cpu_budget: float = 3.0,
                   cpu_init: bool = True) -> dict:
    """Global rotation averaging on the scene's pair graph: noisy relative
    rotations (2 deg, 10 % outlier pairs) from the true poses, the
    column-wise least-squares initialisation and the geodesic Adam loop."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api, rotation, synth
    dev = ctx.device
    inp = synth.rotation_inputs(sc)
    Q = torch.from_numpy(inp.R_rel.reshape(-1, 9).astype(np.float32)).to(dev)
    sched = rotation.RotationSchedule(lanczos_steps=steps, iters=iters)
    rotation.average(s, Q, sched)          # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    p, info = rotation.average(s, Q, sched)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    init_ms, _ = ctx.profile_read(_lib.K_RA_INIT)
    solve_ms, _ = ctx.profile_read(_lib.K_RA_SOLVE)
    ctx.profile(False)
    bar_fail = s.barrier_failures()
    from oracle import rotation as ra
    P = sc.num_pairs
    e_init = ra.relative_rotation_errors(ra.rotations(info["init"].cpu().numpy().astype(np.float64)), sc.R_gt,
                                         sc.pairs)
    e_fin = ra.relative_rotation_errors(ra.rotations(p.cpu().numpy().astype(np.float64)), sc.R_gt, sc.pairs)
    lz = info["lanczos"].cpu().numpy()
    # the oracle as it stands: its dense initialisation (skipped where the
    # dense 3N x 3N eigendecomposition would take minutes), then Adam steps
    Q64 = inp.R_rel.astype(np.float32).astype(np.float64)
    t = time.perf_counter()
    if cpu_init:
        R0, _ = ra.initialise(sc.pairs, Q64, sc.num_cams)
    else:
        R0 = ra.rotations(info["init"].cpu().numpy().astype(np.float64))
    t_init = time.perf_counter() - t if cpu_init else None
    th = np.concatenate([R0[:, :, 0], R0[:, :, 1]], 1)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    n_it, t_it = 0, 0.0
    while t_it < cpu_budget or n_it < 5:
        t = time.perf_counter()
        _, g = ra.loss_grad(th, sc.pairs, Q64)
        th, m, v = ra.adam_step(th, g, m, v, n_it + 1, ra.lr_at(sched.lr, sched.lr_final_frac, iters, n_it))
        t_it += time.perf_counter() - t
        n_it += 1
    return {
        "kernels": "k_ra_lanczos (2 persistent launches, one per column) + k_ra_solve_cam (persistent, one "
                   "wavefront per camera: geodesic loss + adjoint of each pair from both cameras, Adam)",
        "pairs": P, "cameras": sc.num_cams, "lanczos_steps": [int(lz[1]), int(lz[3])], "iters": iters,
        "init_ms": init_ms, "us_per_lanczos_step": init_ms * 1e3 / max(lz[1] + lz[3], 1),
        "iters_per_s": iters / (solve_ms / 1e3), "us_per_iter": solve_ms * 1e3 / iters,
        "stage_wall_ms": wall * 1e3,
        "bound": "latency (Lanczos: 6 grid barriers per step; solve: 1 per iteration)",
        "rel_rot_err_vs_truth_deg": {"init_median": float(np.median(e_init)), "init_max": float(e_init.max()),
                                     "final_median": float(np.median(e_fin)), "final_max": float(e_fin.max())},
        "inputs": "relative rotations from the true poses, 2 deg noise, 10 % random-rotation outlier pairs",
        "barrier_failures": bar_fail,
        "cpu_baseline": {"init_ms": t_init * 1e3 if t_init is not None else None, "iters_per_s": n_it / t_it,
                         "kind": "oracle",
                         "sample": (f"dense 3N x 3N eigendecompositions (numpy.linalg.eigh) and " if cpu_init else "")
                                   + f"{n_it} FP64 loss+gradient+Adam steps over {P} pairs"},
    }


def traffic_entry(path: str):
    """HBM bytes per fm_reweight_build call (its three kernels: FETCH_SIZE
    and WRITE_SIZE scaled by a plain copy's) from a committed rocprofv3
    counter summary, if it was taken on the current Gram kernel source."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("gram_hip_sha256") != _file_sha(GRAM_SRC):
        return None
    return t.get("bytes_per_call")


def load_golden(name: str, sc, coords_digest) -> dict:
    with open(os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")) as f:
        golden = json.load(f)
    if golden["digest"] != scene_digest(sc, coords_digest):
        raise SystemExit(f"stored oracle solve does not match the generated {name} scene; "
                         f"rerun tests/golden/make_golden.py {name}")
    return golden


def stored_coords(sc, storage: str):
    """(array the scene digest covers, float64 values, torch tensor on the
    host) of the coordinates as the workload stores them (bfloat16 rounded
    to nearest even from float64 by torch on the CPU)."""
    import numpy as np
    import torch
    if storage == "f32":
        c = np.ascontiguousarray(sc.uv, dtype=np.float32)
        return c, c.astype(np.float64), torch.from_numpy(c)
    b = torch.from_numpy(np.ascontiguousarray(sc.uv, dtype=np.float64)).to(torch.bfloat16)
    return b.view(torch.int16).numpy().view(np.uint16), b.to(torch.float64).numpy(), b


def pose_parity(rot, tra, golden) -> tuple:
    """(passed, rule) for per-pair differences (degrees) from the stored
    float64 oracle solve: every pair within 0.1 deg / 0.5 deg, or, where the
    stored file records the oracle's own float32-storage sensitivity (the same
    solve with parameters kept in float32 between steps), differences no
    wider than twice it at the 50th/99th/99.9th percentiles (+1e-3 deg) and
    past the bar on at most twice as many pairs (+10)."""
    import numpy as np
    if rot.max() <= 0.1 and tra.max() <= 0.5:
        return True, "every pair within 0.1 deg / 0.5 deg of the oracle"
    sens = golden.get("float32_storage_sensitivity")
    if sens is None:
        return False, "every pair within 0.1 deg / 0.5 deg of the oracle"
    ok = True
    for key, err, bar in (("rot", rot, 0.1), ("t", tra, 0.5)):
        for q, name in ((50, "p50"), (99, "p99"), (99.9, "p99.9")):
            ok = ok and float(np.percentile(err, q)) <= 2.0 * sens[key][name] + 1e-3
        ok = ok and int(np.sum(err > bar)) <= 2 * sens[key]["over_bar"] + 10
    return ok, "within twice the oracle's own float32-storage sensitivity (stored with the oracle solve)"


def solve_leg(ctx, sc, uv_dev, golden, steps: int, warmup: int, label: str) -> dict:
    """Whole epipolar-adjustment solves (the stored schedule: IRLS reweight +
    Gram rebuild before each of 20 loops of 100 fused iterations) timed over
    `steps` runs, with the launch timing of the library's own kernels, and the
    final poses compared with the stored FP64 oracle solve."""
    import numpy as np
    import torch

    from oracle import ea
    from paper_2505_04612_amd import _lib, api, solver
    dev = ctx.device
    s = api.Scene(ctx, sc.num_cams, torch.from_numpy(sc.pairs).to(dev), torch.from_numpy(sc.offsets).to(dev),
                  uv_dev)
    sched = solver.Schedule(**golden["schedule"])
    theta0 = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    p0 = torch.from_numpy(theta0).to(dev)
    for k in range(warmup):
        solver.solve(s, p0, sched, trace=False, check_barriers=False)
        torch.cuda.synchronize()
        log(f"[bench] {label}: warmup {k + 1}/{warmup} done")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        p, _, Z = solver.solve(s, p0, sched, trace=False, check_barriers=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] {label}: {steps} timed solves in {wall:.3f}s")
    bar_fail = s.barrier_failures()
    call_ms, n_call = ctx.profile_read(_lib.K_GRAM_CALL)
    pass_ms, n_pass = ctx.profile_read(_lib.K_GRAM)
    ess_ms, n_ess = ctx.profile_read(_lib.K_ESSENTIALS)
    fin_ms, n_fin = ctx.profile_read(_lib.K_FINALIZE)
    solve_ms, n_solve = ctx.profile_read(_lib.K_SOLVE)
    ctx.profile(False)
    rot, tra = ea.relative_pose_errors(p.cpu().numpy().astype(np.float64), np.array(golden["theta"]), sc.pairs)
    th_gt = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], axis=1)
    rot_gt, tra_gt = ea.relative_pose_errors(p.cpu().numpy().astype(np.float64), th_gt, sc.pairs)
    within, rule = pose_parity(rot, tra, golden)
    passed = bool(within and bar_fail == 0)
    iters = sched.iters * steps
    return {
        "scene": s, "p0": p0, "theta0": theta0, "sched": sched, "wall": wall, "passed": passed,
        "gram_elem": torch.empty((), dtype=sched.gram_dtype).element_size(),
        "bracket_s": call_ms / 1e3 / max(n_call, 1),
        "call_s": (ess_ms + pass_ms + fin_ms) / 1e3 / max(n_call, 1), "pass_s": pass_ms / 1e3 / max(n_pass, 1),
        "ess_s": ess_ms / 1e3 / max(n_ess, 1), "fin_s": fin_ms / 1e3 / max(n_fin, 1), "n_call": n_call,
        "iters_per_s": iters / (solve_ms / 1e3), "solve_us_per_iter": solve_ms * 1e3 / iters,
        "pose_check": {"passed": passed, "every_pair_within_bar": bool(rot.max() <= 0.1 and tra.max() <= 0.5),
                       "rule": rule, "rot_max_deg": float(rot.max()), "rot_median_deg": float(np.median(rot)),
                       "t_max_deg": float(tra.max()), "t_median_deg": float(np.median(tra)),
                       "rot_p99_deg": float(np.percentile(rot, 99)), "t_p99_deg": float(np.percentile(tra, 99)),
                       "rot_p99.9_deg": float(np.percentile(rot, 99.9)), "t_p99.9_deg": float(np.percentile(tra, 99.9)),
                       "pairs_over_bar": [int(np.sum(rot > 0.1)), int(np.sum(tra > 0.5))],
                       "oracle_float32_sensitivity": golden.get("float32_storage_sensitivity"),
                       "kept_gpu": int(Z.item()), "kept_oracle": golden["kept"], "barrier_failures": bar_fail,
                       "vs_ground_truth_deg": {"gpu_rot_median": float(np.median(rot_gt)),
                                               "gpu_t_median": float(np.median(tra_gt)),
                                               "oracle": golden.get("vs_ground_truth_deg")}},
    }


def gram_loss_errors(ctx, leg, sc, x, n_sample: int = 64) -> dict:
    """Errors against FP64 at the initial poses: the Grams of a seeded sample
    of pairs (per-pair Frobenius and per-element norms, the oracle computed
    pair by pair on the stored coordinates), and the library's loss over all
    pairs against the oracle's loss on the same (the library's) Grams."""
    import numpy as np
    import torch

    from oracle import ea
    from paper_2505_04612_amd import api
    s, p0, th0, sched = leg["scene"], leg["p0"], leg["theta0"].astype(np.float64), leg["sched"]
    W64, _, kept = api.reweight_build(s, p0, sched.delta, sched.tau0, f64=True, f32=False)
    loss, _ = api.epipolar_loss_grad(s, W64, p0, Z=kept)
    Wg = W64.cpu().numpy()
    Z = int(kept.item())
    q = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 2, (0, 2): 3, (2, 0): 3, (1, 2): 4, (2, 1): 4, (2, 2): 5}
    idx = np.array([[6 * q[(a, c)] + q[(b, d)] for c in range(3) for d in range(3)] for a in range(3)
                    for b in range(3)])
    Wfull = Wg[:, idx]
    L_ref = ea.loss_from_grams(th0, sc.pairs, Wfull, 1.0 / max(Z, 1))
    rng = np.random.default_rng(7)
    sample = rng.choice(sc.num_pairs, size=min(n_sample, sc.num_pairs), replace=False)
    worst_rel, worst_el = 0.0, 0.0
    for n in sample:
        lo, hi = int(sc.offsets[n]), int(sc.offsets[n + 1])
        xs = x[lo:hi]
        off = np.array([0, hi - lo])
        r = ea.residuals(th0, sc.pairs[n:n + 1], off, xs)
        w = ea.irls_weights(r, float(np.float32(sched.delta)), float(np.float32(sched.tau0)))
        ref = ea.pair_grams(xs, off, w)[0]
        absg = ea.pair_grams(np.abs(xs), off, w)[0]
        d = Wfull[n] - ref
        worst_rel = max(worst_rel, float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)))
        worst_el = max(worst_el, float((np.abs(d) / np.where(absg > 0, absg, 1.0)).max()))
    return {"gram_sampled_pairs": int(len(sample)), "gram_max_rel_fro": worst_rel, "gram_max_elem_rel": worst_el,
            "loss_gpu": float(loss.item()), "loss_oracle_same_grams": L_ref,
            "loss_rel_err": abs(float(loss.item()) - L_ref) / max(abs(L_ref), 1e-300),
            "kept_at_init": Z}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-medium", action="store_true", help="skip the medium-scene solve leg")
    ap.add_argument("--no-translation", action="store_true", help="skip the translation-averaging leg")
    ap.add_argument("--no-rotation", action="store_true", help="skip the rotation-averaging leg")
    ap.add_argument("--no-search", action="store_true", help="skip the relative-translation grid-search leg")
    ap.add_argument("--no-focal", action="store_true", help="skip the focal-refinement leg")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the pose-pipeline leg")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-weight MLP leg")
    ap.add_argument("--cpu-budget", type=float, default=24.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run three plain 512 MiB device-to-device copies first (the reference the HBM byte "
                         "counters are scaled by)")
    ap.add_argument("--workers", type=int, default=0,
                    help="processes generating the large scene and running the CPU baseline (default: up to 16)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the hot path runs on a single MI355X and this library "
              f"has no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2505_04612_amd import api, synth
    workers = args.workers if args.workers > 0 else max(1, min(16, os.cpu_count() or 1))
    # the large street scene, its stored coordinates and the CPU baseline
    # come first: no GPU call has been made yet when the worker processes start
    t_gen = time.perf_counter()
    sc = synth.large(workers=workers)
    dig, x, uv_host = stored_coords(sc, "bf16")
    log(f"[bench] large scene {sc.stats()} generated in {time.perf_counter() - t_gen:.1f}s")
    golden = load_golden("large", sc, dig)
    del dig
    theta0 = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample of the large scene")
        cpu = cpu_baseline(sc, x, theta0, golden["schedule"], args.cpu_budget, workers)
        log(f"[bench] cpu baseline: {cpu['sample']}")
    ctx = api.default_context()
    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=ctx.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 copies of 512 MiB")
    leg = solve_leg(ctx, sc, uv_host.to(ctx.device).contiguous(), golden, args.steps, args.warmup, "large")
    del uv_host
    errs = gram_loss_errors(ctx, leg, sc, x)
    del x
    M, P, N = sc.num_matches, sc.num_pairs, sc.num_cams
    call_s = leg["call_s"]
    # algorithmic bytes of one fm_reweight_build call: the BF16 coordinates,
    # the pair offsets, the poses, the Grams written (36 values per pair in
    # the schedule's Gram precision)
    alg_bytes = 8.0 * M + (8.0 + 36.0 * leg["gram_elem"]) * P + 36.0 * N
    alg_ops = VALU_PER_MATCH_BF16 * M
    copy_gbps = measure_copy_gbps(ctx.device)
    hbm = alg_bytes / call_s / 1e9
    alu = alg_ops / call_s / 1e12
    passed = leg["passed"]
    out = {
        "metric": "matches/s (Gram build) + epipolar iters/s at <=0.1deg rot err vs FP64 oracle",
        "value": M / call_s if passed else 0.0,
        "unit": "matches/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": leg["wall"] * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "large: %d street cameras in a 12x12-block city, %d pairs, %d matches stored as "
                               "BF16, sigma 1.5 px, 30%% outliers; one step = one epipolar-adjustment solve: "
                               "2000 Adam iterations in 20 fused launches, IRLS reweight + Gram rebuild "
                               "(fm_reweight_build) before each" % (N, P, M),
                   "pairs": P, "matches": M, "cameras": N, "iters": leg["sched"].iters,
                   "round_len": leg["sched"].round_len, "parallelism": "single GPU"},
        "iters_per_s": leg["iters_per_s"] if passed else 0.0,
        "gram_call_us": call_s * 1e6,
        "gram_call_bracket_us": leg["bracket_s"] * 1e6,
        "gram_call_parts_us": {"k_pair_essentials": leg["ess_s"] * 1e6, "k_gram_pass": leg["pass_s"] * 1e6,
                               "k_gram_finalize": leg["fin_s"] * 1e6},
        "solve_us_per_iter": leg["solve_us_per_iter"],
        "pose_check": leg["pose_check"],
        "errors_vs_fp64": errs,
        "roofline": {"bound": "alu",
                     "kernel": "fm_reweight_build (k_pair_essentials + k_gram_pass + k_gram_finalize: fused IRLS "
                               "reweight + Gram, BF16 coordinates), device time of the whole call",
                     "achieved": alu, "peak": VALU_PEAK_T, "unit": "T lane-ops/s", "frac": alu / VALU_PEAK_T,
                     "ops_per_match": VALU_PER_MATCH_BF16,
                     "traffic": traffic_entry(TRAFFIC_LARGE),
                     "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBPS,
                             "alg_bytes_per_call": alg_bytes, "measured_copy_GBps": copy_gbps,
                             "frac_of_measured_copy": hbm / copy_gbps}},
        "roofline_iteration": {
            "kernel": "k_solve (pair-by-pair fused loss + adjoint + Adam, two grid barriers per iteration)",
            "bound": "latency (grid barriers and float64 dependency chains; the 30 MB a pass reads stays in "
                     "the 256 MB last-level cache)",
            "alg_bytes_per_iter": 152.0 * P + 300.0 * N,
            "achieved_GBps": (152.0 * P + 300.0 * N) / (leg["solve_us_per_iter"] * 1e-6) / 1e9},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    leg["scene"].close()
    del leg
    if not args.no_medium:
        log("[bench] medium scene: solve leg")
        out["medium"] = bench_medium(ctx, args)
    print(json.dumps(out), flush=True)
    api.release_all()
    return 0


def bench_medium(ctx, args) -> dict:
    """The medium scene (200 cameras, ~4.9k pairs, ~2.9M FP32 matches): a
    whole solve against its stored oracle solve, then the widened stages on
    the same scene.  Its 48 MB of coordinates stay in the 256 MB last-level
    cache across repeated passes, so its HBM fraction is a cache figure."""
    import numpy as np

    from paper_2505_04612_amd import synth
    sc = synth.medium()
    dig, x, uv_host = stored_coords(sc, "f32")
    golden = load_golden("medium", sc, dig)
    leg = solve_leg(ctx, sc, uv_host.to(ctx.device).contiguous(), golden, args.steps, args.warmup, "medium")
    M, P = sc.num_matches, sc.num_pairs
    alg_bytes = 16.0 * M + (8.0 + 36.0 * leg["gram_elem"]) * P + 36.0 * sc.num_cams
    out = {
        "matches_per_s": M / leg["call_s"] if leg["passed"] else 0.0,
        "gram_call_us": leg["call_s"] * 1e6,
        "gram_call_bracket_us": leg["bracket_s"] * 1e6,
        "gram_call_parts_us": {"k_pair_essentials": leg["ess_s"] * 1e6, "k_gram_pass": leg["pass_s"] * 1e6,
                               "k_gram_finalize": leg["fin_s"] * 1e6},
        "gram_call_GBps": alg_bytes / leg["call_s"] / 1e9,
        "gram_call_frac_of_8TBps_cache_resident": alg_bytes / leg["call_s"] / 1e9 / HBM_PEAK_GBPS,
        "iters_per_s": leg["iters_per_s"], "solve_us_per_iter": leg["solve_us_per_iter"],
        "ms_per_solve": leg["wall"] * 1e3 / args.steps,
        "pose_check": leg["pose_check"],
        "traffic": traffic_entry(TRAFFIC_MEDIUM),
        "config": "medium: 200 cameras on a 3-loop helix, %d pairs, %d matches (FP32), sigma 1 px, 20%% outliers; "
                  "2000 Adam iterations, IRLS every 100" % (P, M),
    }
    s = leg["scene"]
    if not args.no_translation:
        log("[bench] translation averaging on the same pair graph")
        out["translation_averaging"] = bench_translation(ctx, s, sc)
    if not args.no_rotation:
        log("[bench] rotation averaging on the same pair graph")
        out["rotation_averaging"] = bench_rotation(ctx, s, sc)
    if not args.no_search:
        log("[bench] relative-translation grid search on the same scene")
        out["translation_search"] = bench_search(ctx, s, sc)
    if not args.no_focal:
        log("[bench] focal refinement on the same scene")
        out["focal_refinement"] = bench_focal(ctx, sc)
    if not args.no_pipeline:
        log("[bench] the pose stages in sequence")
        out["pose_pipeline"] = bench_pipeline(ctx, s, sc)
    if not args.no_mlp:
        log("[bench] learned-weight MLP over the scene's match count")
        out["learned_mlp"] = bench_mlp(ctx, M)
    s.close()
    return out


if __name__ == "__main__":
    _rc = main()
    if _rc:
        sys.exit(_rc)
