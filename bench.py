"""Benchmark of FastMap's epipolar-adjustment hot path on one MI355X.

Workload (the medium scene): 200 cameras on a 3-loop helix, ~4.9k image
pairs, ~2.9M matches stored as float32, 1 px noise, 20 % outliers.  One step
is one whole epipolar-adjustment solve: 2,000 Adam iterations in 20 loops of
100 (each loop one persistent fused loss+adjoint+Adam kernel), with the IRLS
reweight + Gram rebuild (one pass over all matches) before every loop.

Reported (one JSON line):
  value           Gram-build throughput in matches/s: matches streamed by the
                  fused reweight + Gram pass divided by that kernel's device
                  time (HIP events on its stream, over the timed steps); 0 if
                  the final poses miss the oracle by more than 0.1 deg rotation
                  or 0.5 deg translation direction;
  iters_per_s     Adam iterations per second of device time of the fused
                  solve kernel;
  roofline        of the Gram pass (HBM-bound: 16 B per match read, 72 B per
                  pair (E_n) read and 288 B per pair (FP64 Gram) written per
                  launch); `traffic` is the HBM bytes the byte counters saw
                  for it (profiles/gram_medium_traffic.json), when they were
                  taken on the current kernel source;
  cpu_baseline    the FP64 oracle on a bounded sample of the same workload;
  translation_averaging
                  the stage before epipolar adjustment on the same pair graph
                  (Sec. 3.3, Global Translation): 4 runs from random centres
                  in one persistent launch of 1,000 Adam steps, the merge,
                  and a final 1,000-step loop; device time per iteration,
                  accuracy against the true centres, and the FP64 oracle's
                  iteration rate on a bounded sample;
  translation_search
                  the relative-translation grid search on the same scene
                  (appendix on global translation): 4,096 candidates per
                  pair against each pair's Gram; candidate evaluations per
                  second against the FP64 vector peak, accuracy against the
                  true directions, and the FP64 oracle's rate;
  focal_refinement
                  focal lengths inside epipolar adjustment (Sec. 3.3) on the
                  same scene with coordinates normalised by a focal 5 % off:
                  device time of one loss + gradient evaluation and the
                  recovered focal scales after 300 Adam steps;
  pose_pipeline   the stages in sequence on the same scene (rotation
                  averaging, grid search, translation averaging, then the
                  epipolar solve from their poses): wall time and accuracy
                  against the true poses after the averaging stages and
                  after epipolar adjustment;
  rotation_averaging
                  the first pose stage on the same pair graph (Sec. 3.3,
                  Global Rotation): the column-wise least-squares
                  initialisation (two Lanczos eigenvector solves) and 500
                  Adam steps on the geodesic objective; device times,
                  accuracy against the true rotations, and the FP64 oracle
                  (dense eigendecomposition, iterations) on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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

GOLDEN = os.path.join(ROOT, "tests", "golden", "medium_oracle.json")
TRAFFIC = os.path.join(ROOT, "profiles", "gram_medium_traffic.json")
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


def cpu_baseline(sc, coords, theta0, sched_d, budget_s: float = 20.0) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample: repeated reweight +
    Gram passes over the whole scene, then Adam iterations, ~budget_s total."""
    import numpy as np
    from oracle import ea
    x = coords.astype(np.float64)
    th = theta0.astype(np.float64)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    w0 = time.perf_counter()
    n_build = 0
    t_build = 0.0
    while t_build < budget_s * 0.6 or n_build < 1:
        t = time.perf_counter()
        w = ea.irls_weights(ea.residuals(th, sc.pairs, sc.offsets, x), sched_d["delta"], sched_d["tau0"])
        W = ea.pair_grams(x, sc.offsets, w)
        t_build += time.perf_counter() - t
        n_build += 1
    inv_Z = 1.0 / max(int(np.count_nonzero(w)), 1)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    n_it = 0
    t_it = 0.0
    lr = np.array([sched_d["lr_rot"]] * 6 + [sched_d["lr_t"]] * 3)
    while t_it < budget_s * 0.4 or n_it < 10:
        t = time.perf_counter()
        L, g = ea.loss_grad(th, sc.pairs, W, inv_Z)
        th, m, v = ea.adam_step(th, g, m, v, n_it + 1, lr)
        t_it += time.perf_counter() - t
        n_it += 1
    wall = time.perf_counter() - w0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {
        "value": sc.num_matches * n_build / t_build, "unit": "matches/s",
        "iters_per_s": n_it / t_it,
        "cores": max(1, round(cpu / wall)),
        "kind": "oracle",
        "sample": f"{n_build} FP64 reweight+Gram passes over all {sc.num_matches} matches and {n_it} "
                  f"loss+gradient+Adam iterations over {sc.num_pairs} pairs ({wall:.1f} s)",
        "host_cpu": _cpu_model(), "nproc": os.cpu_count(),
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
        "kernels": "k_mlp_forward (64x64 layer on v_mfma_f32_16x16x16_f16), k_mlp_backward + k_mlp_reduce",
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


def traffic_entry(alg_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current Gram kernel source."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("gram_hip_sha256") != _file_sha(GRAM_SRC):
        return None
    return t.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-translation", action="store_true", help="skip the translation-averaging leg")
    ap.add_argument("--no-rotation", action="store_true", help="skip the rotation-averaging leg")
    ap.add_argument("--no-search", action="store_true", help="skip the relative-translation grid-search leg")
    ap.add_argument("--no-focal", action="store_true", help="skip the focal-refinement leg")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the pose-pipeline leg")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-weight MLP leg")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", choices=["medium", "large"], default="medium",
                    help="medium (default, the metric's workload) or large (5,000 cameras, ~200M BF16 "
                         "matches: Gram-pass and iteration throughput with sampled Gram parity)")
    ap.add_argument("--scale", type=float, default=1.0, help="camera-count scale of the large workload")
    ap.add_argument("--workers", type=int, default=0,
                    help="processes generating the large workload (default: up to 16; 1 = no child processes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the hot path runs on a single MI355X and this library "
              f"has no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    if args.workload == "large":
        return bench_large(args)

    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api, solver, synth

    t_gen = time.perf_counter()
    sc = synth.medium()
    coords = sc.uv.astype(np.float32)
    log(f"[bench] scene {sc.stats()} generated in {time.perf_counter() - t_gen:.1f}s")
    with open(GOLDEN) as f:
        golden = json.load(f)
    if golden["digest"] != scene_digest(sc, coords):
        raise SystemExit("stored oracle result does not match the generated scene; rerun tests/golden/make_golden.py")
    sd = golden["schedule"]
    sched = solver.Schedule(**sd)
    ctx = api.default_context()
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, coords, torch.float32)
    theta0 = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    p0 = torch.from_numpy(theta0).to(ctx.device)

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=ctx.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 copies of 512 MiB")
    for k in range(args.warmup):
        solver.solve(s, p0, sched, trace=False)
        torch.cuda.synchronize()
        log(f"[bench] warmup {k + 1}/{args.warmup} done")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        p, _, Z = solver.solve(s, p0, sched, trace=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] {args.steps} timed steps in {wall:.3f}s")
    bar_fail = s.barrier_failures()
    gram_ms, n_gram = ctx.profile_read(_lib.K_GRAM)
    ess_ms, n_ess = ctx.profile_read(_lib.K_ESSENTIALS)
    fin_ms, n_fin = ctx.profile_read(_lib.K_FINALIZE)
    solve_ms, n_solve = ctx.profile_read(_lib.K_SOLVE)
    ctx.profile(False)

    # pose check against the stored FP64 oracle solve
    from oracle import ea
    rot, tra = ea.relative_pose_errors(p.cpu().numpy().astype(np.float64), np.array(golden["theta"]), sc.pairs)
    passed = bool(rot.max() <= 0.1 and tra.max() <= 0.5 and bar_fail == 0)

    M, P = sc.num_matches, sc.num_pairs
    gram_s = gram_ms / 1e3 / max(n_gram, 1)
    matches_per_s = M / gram_s
    alg_bytes = 16.0 * M + (72.0 + 288.0) * P     # coordinates, E_n in, FP64 Gram out
    achieved = alg_bytes / gram_s / 1e9
    iters = sched.iters * args.steps
    iters_per_s = iters / (solve_ms / 1e3)
    traffic = traffic_entry(alg_bytes)
    copy_gbps = measure_copy_gbps(ctx.device)     # after the timed region
    out = {
        "metric": "matches/s (Gram build) + epipolar iters/s at <=0.1deg rot err vs FP64 oracle",
        "value": matches_per_s if passed else 0.0,
        "unit": "matches/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "medium: 200 cameras on a 3-loop helix, %d pairs, %d matches (FP32), "
                               "sigma 1 px, 20%% outliers; 2000 Adam iterations, IRLS every 100" % (P, M),
                   "pairs": P, "matches": M, "cameras": sc.num_cams, "iters": sched.iters,
                   "round_len": sched.round_len, "parallelism": "single GPU"},
        "iters_per_s": iters_per_s,
        "gram_pass_us": gram_s * 1e6,
        "gram_aux_us": {"essentials": ess_ms * 1e3 / max(n_ess, 1), "finalize": fin_ms * 1e3 / max(n_fin, 1)},
        "solve_kernel_us_per_iter": solve_ms * 1e3 / iters,
        "pose_check": {"passed": passed, "rot_max_deg": float(rot.max()), "rot_median_deg": float(np.median(rot)),
                       "t_max_deg": float(tra.max()), "t_median_deg": float(np.median(tra)),
                       "kept_gpu": int(Z.item()), "kept_oracle": golden["kept"], "barrier_failures": bar_fail},
        "roofline": {"bound": "hbm", "kernel": "k_gram_pass (fused IRLS reweight + Gram, float32 coords)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes,
                     "measured_copy_GBps": copy_gbps, "frac_of_measured_copy": achieved / copy_gbps},
    }
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
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(sc, coords, theta0, sd, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


def bench_large(args) -> int:
    """Large street scene: the fused reweight + Gram pass over ~200M BF16 matches
    (1.6 GB per pass, far beyond the 256 MB last-level cache) and the fused
    iteration over ~250k pairs; Grams of sampled pairs are checked against the
    oracle computed one pair at a time."""
    import numpy as np
    import torch

    from paper_2505_04612_amd import _lib, api, solver, synth
    t_gen = time.perf_counter()
    workers = args.workers if args.workers > 0 else max(1, min(16, (os.cpu_count() or 1)))
    sc = synth.large(scale=args.scale, workers=workers)   # before any GPU call
    log(f"[bench] large scene {sc.stats()} generated in {time.perf_counter() - t_gen:.1f}s")
    ctx = api.default_context()
    dev = ctx.device
    uv = torch.from_numpy(sc.uv).to(dev).to(torch.bfloat16).contiguous()
    s = api.Scene(ctx, sc.num_cams, torch.from_numpy(sc.pairs).to(dev), torch.from_numpy(sc.offsets).to(dev), uv)
    theta0 = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    p0 = torch.from_numpy(theta0).to(dev)
    M, P = sc.num_matches, sc.num_pairs
    sched = solver.Schedule()
    out64 = torch.empty((P, 36), dtype=torch.float64, device=dev)
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    for _ in range(max(args.warmup, 1)):
        api.reweight_build(s, p0, sched.delta, sched.tau0, out=(out64, None, kept))
    torch.cuda.synchronize()
    log("[bench] warm")
    ctx.profile(True)
    t0 = time.perf_counter()
    reps = max(args.steps, 1) * 4
    for _ in range(reps):
        api.reweight_build(s, p0, sched.delta, sched.tau0, out=(out64, None, kept))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gram_ms, n_gram = ctx.profile_read(_lib.K_GRAM)
    ess_ms, _ = ctx.profile_read(_lib.K_ESSENTIALS)
    fin_ms, _ = ctx.profile_read(_lib.K_FINALIZE)
    ctx.profile(False)
    log(f"[bench] {reps} Gram passes in {wall:.3f}s")
    # one optimisation loop of the fused solve
    m = torch.zeros_like(p0)
    v = torch.zeros_like(p0)
    p = p0.clone()
    api.epipolar_solve(s, out64, p, m, v, 10, sched.lr_rot, sched.lr_t, sched.lr_final_frac, 0, 100, Z=kept)
    torch.cuda.synchronize()
    ctx.profile(True)
    K = 100
    api.epipolar_solve(s, out64, p, m, v, K, sched.lr_rot, sched.lr_t, sched.lr_final_frac, 10, 200, Z=kept)
    solve_ms, _ = ctx.profile_read(_lib.K_SOLVE)
    ctx.profile(False)
    log(f"[bench] {K} fused iterations in {solve_ms:.2f} ms")
    # sampled parity of the Gram against the oracle, one pair at a time
    from oracle import ea
    api.reweight_build(s, p0, sched.delta, sched.tau0, out=(out64, None, kept))
    W = out64.cpu().numpy()
    rng = np.random.default_rng(7)
    sample = rng.choice(P, size=min(48, P), replace=False)
    worst_rel, worst_el = 0.0, 0.0
    for n in sample:
        lo, hi = int(sc.offsets[n]), int(sc.offsets[n + 1])
        x = uv[lo:hi].to(torch.float32).cpu().numpy().astype(np.float64)
        off = np.array([0, hi - lo])
        r = ea.residuals(theta0.astype(np.float64), sc.pairs[n:n + 1], off, x)
        w = ea.irls_weights(r, float(np.float32(sched.delta)), float(np.float32(sched.tau0)))
        ref = ea.pair_grams(x, off, w)[0]
        absg = ea.pair_grams(np.abs(x), off, w)[0]
        q = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 2, (0, 2): 3, (2, 0): 3, (1, 2): 4, (2, 1): 4, (2, 2): 5}
        G = np.array([[W[n, 6 * q[(a, c)] + q[(b, d)]] for c in range(3) for d in range(3)]
                      for a in range(3) for b in range(3)])
        d = G - ref
        worst_rel = max(worst_rel, float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)))
        worst_el = max(worst_el, float((np.abs(d) / np.where(absg > 0, absg, 1.0)).max()))
    gram_s = gram_ms / 1e3 / max(n_gram, 1)
    alg_bytes = 8.0 * M + (72.0 + 288.0) * P      # coordinates, E_n in, FP64 Gram out
    achieved = alg_bytes / gram_s / 1e9
    copy_gbps = measure_copy_gbps(ctx.device)     # after the timed region
    out = {
        "metric": "matches/s (Gram build) + epipolar iters/s at <=0.1deg rot err vs FP64 oracle",
        "value": M / gram_s, "unit": "matches/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": wall * 1e3 / reps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "large: %d street cameras, %d pairs, %d matches (BF16), sigma 1.5 px, "
                               "30%% outliers; fused IRLS reweight + Gram pass" % (sc.num_cams, P, M),
                   "pairs": P, "matches": M, "cameras": sc.num_cams, "parallelism": "single GPU"},
        "iters_per_s": K / (solve_ms / 1e3),
        "gram_pass_us": gram_s * 1e6,
        "gram_aux_us": {"essentials": ess_ms * 1e3 / max(n_gram, 1), "finalize": fin_ms * 1e3 / max(n_gram, 1)},
        "sampled_gram_parity": {"pairs": int(len(sample)), "max_rel_fro": worst_rel, "max_elem_rel": worst_el},
        "roofline": {"bound": "hbm", "kernel": "k_gram_pass (fused IRLS reweight + Gram, bf16 coords)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "alg_bytes_per_launch": alg_bytes,
                     "measured_copy_GBps": copy_gbps, "frac_of_measured_copy": achieved / copy_gbps,
                     # with 8 B per match the pass issues more VALU work than HBM time:
                     # VALU instructions per match (gfx950 assembly of the kernel) against
                     # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
                     "valu": {"instr_per_match": VALU_PER_MATCH_BF16,
                              "achieved_T_lane_instr_per_s": VALU_PER_MATCH_BF16 * M / gram_s / 1e12,
                              "peak_T_lane_instr_per_s": VALU_PEAK_T,
                              "frac": VALU_PER_MATCH_BF16 * M / gram_s / 1e12 / VALU_PEAK_T}},
    }
    if not args.no_translation:
        log("[bench] translation averaging on the large pair graph")
        out["translation_averaging"] = bench_translation(ctx, s, sc)
    if not args.no_rotation:
        log("[bench] rotation averaging on the large pair graph")
        out["rotation_averaging"] = bench_rotation(ctx, s, sc, cpu_init=False)
    if not args.no_search:
        log("[bench] relative-translation grid search on the large scene")
        out["translation_search"] = bench_search(ctx, s, sc)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    _rc = main()
    if _rc:
        sys.exit(_rc)
