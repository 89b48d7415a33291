"""Learned robust weights for epipolar adjustment, with IRLS as fallback.

The paper robustifies the L2 epipolar objective by IRLS: weights 1/|r| at
the current poses, recomputed after every optimisation loop (Sec. 3.3).
Here a 3 -> 64 -> 64 -> 1 MLP proposes each match's weight directly from
features (log residual, log pair size, parallax), so after a short warm-up
one Gram build replaces the remaining IRLS rebuilds: the first
`warm_rounds` loops of the plain schedule run as usual, the network weighs
every match at the poses they reach, and the remaining Adam steps run on
that one Gram.  The network is trained on the targets the method's own
converged IRLS solves produce, omega_bar = delta / max(|r|, delta) (0 for
filtered matches), from features at the same warm-up poses, with the
library's MFMA forward/backward kernels and its Adam kernel.

A tail of `tail_rounds` plain IRLS loops (final filter threshold, learning
rate from the middle of the plain schedule's range down to its end) then
takes the learned solution to the IRLS weighting.  Fallback: if the tail
moves the relative rotation of more than a tenth of the pairs by over
0.1 deg, or their translation direction by over 0.5 deg (the
90th percentile of the per-pair changes, so a few pairs with an
ill-conditioned baseline do not decide alone), the full plain IRLS schedule
is run from the initial poses instead, so plain IRLS remains the reference
for pose accuracy.

    python -m paper_2505_04612_amd.learned --train 64 --test 16 --out results.json
"""
from __future__ import annotations

import argparse
import concurrent.futures
import dataclasses
import json
import math
import sys
import time

import numpy as np
import torch

from . import api, solver, synth


@dataclasses.dataclass
class LearnedSchedule:
    warm_rounds: int = 2         # plain IRLS loops before the network weighs the matches
    iters: int = 600             # Adam steps on the learned-weight Gram
    tail_rounds: int = 3         # plain IRLS loops after them (their movement is the fallback check)
    lr_rot: float = 3e-3
    lr_t: float = 1e-2
    lr_final_frac: float = 1e-3
    delta: float = 1e-4
    check_rot_deg: float = 0.1   # fallback thresholds on the per-pair changes
    check_t_deg: float = 0.5
    check_quantile: float = 0.9


def _pose_changes(pa: np.ndarray, pb: np.ndarray, pairs: np.ndarray):
    """Per-pair relative-rotation and translation-direction change (deg)
    between two parameter sets; the sign of t is ignored."""
    def rot(p):
        a1, a2 = p[:, 0:3], p[:, 3:6]
        b1 = a1 / np.linalg.norm(a1, axis=1, keepdims=True)
        u2 = a2 - np.sum(b1 * a2, axis=1, keepdims=True) * b1
        b2 = u2 / np.linalg.norm(u2, axis=1, keepdims=True)
        return np.stack([b1, b2, np.cross(b1, b2)], axis=-1)
    pa, pb = pa.astype(np.float64), pb.astype(np.float64)
    Ra, Rb = rot(pa), rot(pb)
    i, j = pairs[:, 0], pairs[:, 1]
    Qa = Ra[j] @ np.swapaxes(Ra[i], 1, 2)
    Qb = Rb[j] @ np.swapaxes(Rb[i], 1, 2)
    ta = pa[j, 6:9] - np.einsum("pab,pb->pa", Qa, pa[i, 6:9])
    tb = pb[j, 6:9] - np.einsum("pab,pb->pa", Qb, pb[i, 6:9])
    D = Qa @ np.swapaxes(Qb, 1, 2)
    c = (np.trace(D, axis1=1, axis2=2) - 1) / 2
    ax = np.stack([D[:, 2, 1] - D[:, 1, 2], D[:, 0, 2] - D[:, 2, 0], D[:, 1, 0] - D[:, 0, 1]], -1)
    r_err = np.degrees(np.arctan2(0.5 * np.linalg.norm(ax, axis=1), c))
    ua = ta / np.linalg.norm(ta, axis=1, keepdims=True)
    ub = tb / np.linalg.norm(tb, axis=1, keepdims=True)
    t_err = np.degrees(np.arctan2(np.linalg.norm(np.cross(ua, ub), axis=1), np.abs(np.sum(ua * ub, axis=1))))
    return r_err, t_err


def _relative_pose_change(pa: np.ndarray, pb: np.ndarray, pairs: np.ndarray, q: float = 1.0):
    """Quantile q (1 = max) of the per-pair relative-rotation and
    translation-direction changes (deg): the host-side decision of the
    fallback rule."""
    r, t = _pose_changes(pa, pb, pairs)
    return float(np.quantile(r, q)), float(np.quantile(t, q))


def irls_targets(scene: api.Scene, params0: torch.Tensor, sched: solver.Schedule, warm_rounds: int = 2):
    """Features at the warm-up poses (the first warm_rounds loops of the plain
    schedule) and converged-IRLS weight targets in [0, 1]."""
    p, _, _ = solver.solve(scene, params0, sched, trace=False)
    tau_final = solver.tau_at(sched, max(sched.iters // sched.round_len - 1, 0))
    w, _, _ = api.reweight(scene, p, sched.delta, tau_final)
    target = w * sched.delta
    p_warm = params0
    if warm_rounds > 0:
        p_warm, _, _ = solver.solve(scene, params0, sched, trace=False, rounds=warm_rounds)
    feats = api.match_features(scene, p_warm, sched.delta)
    return feats, target, p


@dataclasses.dataclass
class TrainCfg:
    steps: int = 3000
    batch: int = 65536
    lr: float = 2e-3
    lr_final_frac: float = 0.05
    seed: int = 0


def train_mlp(ctx: api.Context, feats: torch.Tensor, target: torch.Tensor, cfg: TrainCfg, progress=None):
    """Minimise sum (mlp(f) - target)^2 over minibatches with the library's
    forward, backward and Adam kernels.  Returns (weights, loss history);
    `progress(step, loss)` is called with each history entry."""
    dev = ctx.device
    mean = feats.mean(dim=0)
    std = feats.std(dim=0).clamp_min(1e-6)
    rng = np.random.default_rng(cfg.seed)
    w = api.MlpWeights(dev, mean=mean.contiguous(), std=std.contiguous())
    for k, s in api.MLP_SHAPES.items():
        if k.startswith("W"):
            w.views[k].copy_(torch.from_numpy(rng.normal(0.0, math.sqrt(2.0 / s[1]), size=s).astype(np.float32)))
    m = torch.zeros_like(w.flat)
    v = torch.zeros_like(w.flat)
    g = api.MlpWeights(dev)
    lr = torch.empty(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg.seed)
    M = feats.shape[0]
    hist = []
    for step in range(1, cfg.steps + 1):
        idx = torch.randint(0, M, (cfg.batch,), device=dev, generator=gen)
        fb = feats[idx].contiguous()
        tb = target[idx]
        out, act = api.mlp_forward(ctx, w, fb, keep_act=True)
        dout = (2.0 / cfg.batch) * (out - tb)
        api.mlp_backward(ctx, w, fb, act, dout.contiguous(), g)
        lr.fill_(cfg.lr * cfg.lr_final_frac ** ((step - 1) / cfg.steps))
        api.adam_step(ctx, w.flat, g.flat, m, v, step, lr, 0.9, 0.999, 1e-8)
        if step % 100 == 0 or step == 1:
            hist.append((step, float(torch.mean((out - tb) ** 2).item())))
            if progress is not None:
                progress(*hist[-1])
    return w, hist


def learned_solve(scene: api.Scene, params0: torch.Tensor, w: api.MlpWeights, ls: LearnedSchedule,
                  fallback: solver.Schedule):
    """Solve with MLP-proposed weights after a short plain warm-up; returns
    (params, info)."""
    ctx = scene.ctx
    warm = ls.warm_rounds * fallback.round_len
    p = params0.detach().clone().contiguous()
    if ls.warm_rounds > 0:
        p, _, _ = solver.solve(scene, params0, fallback, trace=False, rounds=ls.warm_rounds)
    feats = api.match_features(scene, p, ls.delta)
    omega, _ = api.mlp_forward(ctx, w, feats, out_scale=1.0 / ls.delta)
    W64, _ = api.build_pair_grams(scene, omega, f64=True, f32=False)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    api.epipolar_solve(scene, W64, p, m, v, ls.iters, ls.lr_rot, ls.lr_t, ls.lr_final_frac, warm, warm + ls.iters,
                       inv_Z=1.0 / max(scene.num_matches, 1))
    # a tail of plain IRLS loops from the learned solution, at the final
    # filter threshold and with the learning rate falling from the geometric
    # middle of the plain schedule's range to its end; how far the tail moves
    # the learned solution decides the fallback
    p_learned = p.clone()
    tau = solver.tau_at(fallback, max(fallback.iters // fallback.round_len - 1, 0))
    half = math.sqrt(fallback.lr_final_frac)
    T = max(ls.tail_rounds, 1)
    tail = dataclasses.replace(fallback, iters=T * fallback.round_len, tau0=tau, lr_rot=fallback.lr_rot * half,
                               lr_t=fallback.lr_t * half, lr_final_frac=half)
    p_chk = p.clone()
    for r in range(T):
        Wt, Zt = solver._grams(scene, p_chk, tail, solver.tau_at(tail, r))
        m.zero_()
        v.zero_()
        api.epipolar_solve(scene, Wt, p_chk, m, v, tail.round_len, tail.lr_rot, tail.lr_t, tail.lr_final_frac,
                           r * tail.round_len, tail.iters, 0, tail.beta1, tail.beta2, tail.eps, Z=Zt)
    d_rot, d_t = _relative_pose_change(p_learned.cpu().numpy(), p_chk.cpu().numpy(), scene.pairs.cpu().numpy(),
                                       ls.check_quantile)
    info = {"check_rot_deg": d_rot, "check_t_deg": d_t, "fallback": False, "params_learned": p_learned}
    if d_rot > ls.check_rot_deg or d_t > ls.check_t_deg:
        # the learned weights missed the IRLS optimum: plain IRLS from the
        # initial poses decides the result
        info["fallback"] = True
        p_chk, _, _ = solver.solve(scene, params0, fallback, trace=False)
    return p_chk, info


def _gen(seed: int, n_cams: int, n_points: int):
    sc = synth.learned(seed=seed, n_cams=n_cams, n_points=n_points)
    return {"seed": seed, "pairs": sc.pairs, "offsets": sc.offsets, "uv": sc.uv.astype(np.float32),
            "R_gt": sc.R_gt, "t_gt": sc.t_gt, "R_init": sc.R_init, "t_init": sc.t_init, "stats": sc.stats()}


def _pose_err(p: np.ndarray, R_gt, t_gt, pairs):
    """Median and max relative rotation / translation-direction error (deg)
    against ground truth (sign of t ignored)."""
    gt = np.concatenate([R_gt[:, :, 0], R_gt[:, :, 1], t_gt], axis=1)
    rot, tra = _pose_changes(p, gt, pairs)
    return {"rot_med": float(np.median(rot)), "rot_max": float(rot.max()),
            "t_med": float(np.median(tra)), "t_max": float(tra.max())}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--cams", type=int, default=300)
    ap.add_argument("--points", type=int, default=280_000)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--samples", type=int, default=400_000, help="training matches kept per scene")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--learned-iters", type=int, default=600)
    ap.add_argument("--warm-rounds", type=int, default=2)
    ap.add_argument("--tail-rounds", type=int, default=3)
    ap.add_argument("--out", default="learned_results.json")
    args = ap.parse_args(argv)
    t0 = time.time()
    train_seeds = list(range(100, 100 + args.train))
    test_seeds = list(range(200, 200 + args.test))
    scenes = []
    with concurrent.futures.ProcessPoolExecutor(max_workers=args.workers) as ex:
        for sc in ex.map(_gen, train_seeds + test_seeds, [args.cams] * (args.train + args.test),
                         [args.points] * (args.train + args.test)):
            scenes.append(sc)
            print(f"[learned] scene {len(scenes)}/{args.train + args.test} (seed {sc['seed']}) "
                  f"{time.time() - t0:.0f}s", flush=True)
    print(f"[learned] generated {len(scenes)} scenes in {time.time() - t0:.0f}s "
          f"(e.g. {scenes[0]['stats']})", flush=True)
    ctx = api.default_context()
    dev = ctx.device
    sched = solver.Schedule(iters=2000, round_len=100)
    feats_all, tgt_all = [], []
    rng = np.random.default_rng(0)
    for sc in scenes[:args.train]:
        s = api.Scene.from_numpy(ctx, len(sc["R_gt"]), sc["pairs"], sc["offsets"], sc["uv"], torch.float32)
        p0 = torch.from_numpy(np.concatenate([sc["R_init"][:, :, 0], sc["R_init"][:, :, 1], sc["t_init"]],
                                             axis=1).astype(np.float32)).to(dev)
        f, t, _ = irls_targets(s, p0, sched, args.warm_rounds)
        M = f.shape[0]
        keep = torch.from_numpy(rng.choice(M, size=min(args.samples, M), replace=False)).to(dev)
        feats_all.append(f[keep])
        tgt_all.append(t[keep])
        s.close()
    feats = torch.cat(feats_all).contiguous()
    tgt = torch.cat(tgt_all).contiguous()
    print(f"[learned] targets from {args.train} IRLS solves: {feats.shape[0]} samples "
          f"({time.time() - t0:.0f}s)", flush=True)
    w, hist = train_mlp(ctx, feats, tgt, TrainCfg(steps=args.steps),
                        progress=lambda k, l: print(f"[learned] step {k} loss {l:.4g}", flush=True)
                        if k % 500 == 0 else None)
    print(f"[learned] trained: loss {hist[0][1]:.4g} -> {hist[-1][1]:.4g} ({time.time() - t0:.0f}s)", flush=True)
    ls = LearnedSchedule(iters=args.learned_iters, warm_rounds=args.warm_rounds, tail_rounds=args.tail_rounds)
    rows = []
    for sc in scenes[args.train:]:
        # plain method: FP32 coordinates, IRLS every loop; learned form: BF16
        # coordinates (mixed precision), MLP weights, one Gram build
        s = api.Scene.from_numpy(ctx, len(sc["R_gt"]), sc["pairs"], sc["offsets"], sc["uv"], torch.float32)
        s16 = api.Scene.from_numpy(ctx, len(sc["R_gt"]), sc["pairs"], sc["offsets"], sc["uv"], torch.bfloat16)
        p0 = torch.from_numpy(np.concatenate([sc["R_init"][:, :, 0], sc["R_init"][:, :, 1], sc["t_init"]],
                                             axis=1).astype(np.float32)).to(dev)
        solver.solve(s, p0, sched, trace=False)            # warm-up of both paths
        learned_solve(s16, p0, w, ls, sched)
        torch.cuda.synchronize()
        a = time.perf_counter()
        p_irls, _, _ = solver.solve(s, p0, sched, trace=False)
        torch.cuda.synchronize()
        t_irls = time.perf_counter() - a
        a = time.perf_counter()
        p_l, info = learned_solve(s16, p0, w, ls, sched)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - a
        s16.close()
        e_irls = _pose_err(p_irls.cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        e_l = _pose_err(p_l.cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        e_lo = _pose_err(info.pop("params_learned").cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        d = _relative_pose_change(p_l.cpu().numpy(), p_irls.cpu().numpy(), sc["pairs"])
        rows.append({"seed": sc["seed"], "irls_s": t_irls, "learned_s": t_l, "irls_err_deg": e_irls,
                     "learned_err_deg": e_l, "learned_before_check_err_deg": e_lo, "learned_vs_irls_max_deg": d,
                     **info})
        print(f"[learned] seed {sc['seed']}: IRLS {t_irls * 1e3:.1f} ms err {e_irls}, learned "
              f"{t_l * 1e3:.1f} ms err {e_l} fallback {info['fallback']}", flush=True)
        s.close()
    res = {"train_scenes": args.train, "test_scenes": args.test, "samples": int(feats.shape[0]),
           "train_loss": hist, "test": rows, "wall_s": time.time() - t0,
           "weights": {k: v.tolist() for k, v in w.to_numpy().items()},
           "feat_mean": w.mean.cpu().tolist(), "feat_std": w.std.cpu().tolist()}
    with open(args.out, "w") as f:
        json.dump(res, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
