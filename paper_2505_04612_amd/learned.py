"""Learned robust weights for epipolar adjustment, with IRLS as the judge.

The paper robustifies the L2 epipolar objective by IRLS: weights 1/|r| at
the current poses, recomputed after every optimisation loop (Sec. 3.3).
Here a 3 -> 64 -> 64 -> 1 MLP proposes each match's weight directly from
features (log residual, log pair size, parallax), so one Gram build stands
in for an IRLS rebuild: the first `warm_rounds` loops of the plain
schedule run as usual, the network weighs every match at the poses they
reach, and `iters` Adam steps run on that one Gram (at the schedule
position of the loop it replaces).  The network's weights approximate the
converged IRLS weights, so that short segment brings the poses closer to
the solution than a plain IRLS loop at the same position, and the stopping
rule below fires loops earlier.  The network is trained on the
targets the method's own converged IRLS solves produce, omega_bar =
delta / max(|r|, delta) (0 for filtered matches), from features at the same
warm-up poses, with the library's MFMA forward/backward kernels and its
Adam kernel.

Plain IRLS loops then continue from the learned solution at their own
schedule positions (threshold and learning rate), and after each one
fm_pose_change measures, on the device, how far it moved every pair's
relative rotation and translation direction.  Once a loop moves at most
`check_frac` of the pairs by more than 0.1 deg rotation or 0.5 deg
translation direction, the solve is taken as converged and stops; otherwise
the plain loops run to the end of the schedule (the fallback: it costs the
rest of the plain schedule, never a restart).  `plain_converged_solve` is
plain IRLS under the same stopping rule, the fair comparison for what the
network buys.

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
    iters: int = 50              # Adam steps on the learned-weight Gram (at the schedule position of the loop it
                                 # stands in for; measured on held-out scenes, time against plain IRLS under the
                                 # same stopping rule: 50 steps 0.79x (80 cameras) / 0.87x (300 cameras), 100 steps
                                 # 0.89x / 0.93x, 600 steps 1.6x, all but 600 at equal accuracy)
    delta: float = 1e-4
    check_rot_deg: float = 0.1   # a loop that moves a pair by more than these has not converged
    check_t_deg: float = 0.5
    check_frac: float = 0.1      # converged: at most this fraction of the pairs moved beyond them


def _pose_changes(pa: np.ndarray, pb: np.ndarray, pairs: np.ndarray):
    """Per-pair relative-rotation and translation-direction change (deg)
    between two parameter sets; the sign of t is ignored.  Host-side
    evaluation helper (accuracy reports against ground truth); the solve's
    own convergence test runs on the device (fm_pose_change)."""
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


def _plain_loops(scene: api.Scene, p: torch.Tensor, plain: solver.Schedule, first: int, ls: LearnedSchedule,
                 stop_early: bool):
    """Plain IRLS loops first, first+1, ... of the schedule (threshold and
    learning rate at their own positions) from poses p, updated in place.
    With stop_early, after each loop fm_pose_change compares the poses
    before and after it and the loops stop once it moved at most
    ls.check_frac of the pairs beyond the thresholds.  Returns (loops run,
    converged)."""
    R = plain.round_len
    loops = -(-plain.iters // R)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    limit = ls.check_frac * scene.num_pairs
    run = 0
    for k in range(first, loops):
        prev = p.clone() if stop_early else None
        W, Z = solver._grams(scene, p, plain, solver.tau_at(plain, k))
        m.zero_()
        v.zero_()
        K = min(R, plain.iters - k * R)
        api.epipolar_solve(scene, W, p, m, v, K, plain.lr_rot, plain.lr_t, plain.lr_final_frac, k * R, plain.iters,
                           0, plain.beta1, plain.beta2, plain.eps, Z=Z)
        run += 1
        if stop_early:
            counts, _, _ = api.pose_change(scene, prev, p, ls.check_rot_deg, ls.check_t_deg)
            n_rot, n_t = (int(x) for x in counts.tolist())
            if n_rot <= limit and n_t <= limit:
                scene.require_barriers_ok()
                return run, True
    scene.require_barriers_ok()
    return run, False


def plain_converged_solve(scene: api.Scene, params0: torch.Tensor, plain: solver.Schedule,
                          ls: LearnedSchedule = LearnedSchedule()):
    """Plain IRLS (every loop reweighted, from the initial poses) under the
    learned form's stopping rule; returns (params, info)."""
    p = params0.detach().clone().contiguous()
    loops, conv = _plain_loops(scene, p, plain, 0, ls, True)
    return p, {"loops": loops, "converged": conv}


def learned_solve(scene: api.Scene, params0: torch.Tensor, w: api.MlpWeights, ls: LearnedSchedule,
                  plain: solver.Schedule):
    """Solve with MLP-proposed weights after a short plain warm-up, then plain
    IRLS loops to convergence (or to the end of the schedule); returns
    (params, info)."""
    ctx = scene.ctx
    R = plain.round_len
    warm = ls.warm_rounds * R
    p = params0.detach().clone().contiguous()
    if ls.warm_rounds > 0:
        p, _, _ = solver.solve(scene, params0, plain, trace=False, rounds=ls.warm_rounds)
    feats = api.match_features(scene, p, ls.delta)
    omega, _ = api.mlp_forward(ctx, w, feats, out_scale=1.0 / ls.delta)
    W64, _ = api.build_pair_grams(scene, omega, f64=True, f32=False)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    api.epipolar_solve(scene, W64, p, m, v, ls.iters, plain.lr_rot, plain.lr_t, plain.lr_final_frac, warm,
                       plain.iters, inv_Z=1.0 / max(scene.num_matches, 1))
    p_learned = p.clone()
    first = ls.warm_rounds + -(-ls.iters // R)
    loops, conv = _plain_loops(scene, p, plain, first, ls, True)
    return p, {"params_learned": p_learned, "tail_loops": loops, "converged": conv,
               "fallback": not conv, "loops_total": ls.warm_rounds + loops}


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
    ap.add_argument("--learned-iters", type=int, default=LearnedSchedule.iters)
    ap.add_argument("--warm-rounds", type=int, default=2)
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
    ls = LearnedSchedule(iters=args.learned_iters, warm_rounds=args.warm_rounds)
    rows = []
    for sc in scenes[args.train:]:
        # plain method: FP32 coordinates, IRLS every loop; learned form: BF16
        # coordinates (mixed precision), MLP weights, one Gram build
        s = api.Scene.from_numpy(ctx, len(sc["R_gt"]), sc["pairs"], sc["offsets"], sc["uv"], torch.float32)
        s16 = api.Scene.from_numpy(ctx, len(sc["R_gt"]), sc["pairs"], sc["offsets"], sc["uv"], torch.bfloat16)
        p0 = torch.from_numpy(np.concatenate([sc["R_init"][:, :, 0], sc["R_init"][:, :, 1], sc["t_init"]],
                                             axis=1).astype(np.float32)).to(dev)
        solver.solve(s, p0, sched, trace=False)            # warm-up of the paths
        plain_converged_solve(s, p0, sched, ls)
        learned_solve(s16, p0, w, ls, sched)
        torch.cuda.synchronize()
        a = time.perf_counter()
        p_irls, _, _ = solver.solve(s, p0, sched, trace=False)
        torch.cuda.synchronize()
        t_irls = time.perf_counter() - a
        a = time.perf_counter()
        p_pc, info_pc = plain_converged_solve(s, p0, sched, ls)
        torch.cuda.synchronize()
        t_pc = time.perf_counter() - a
        a = time.perf_counter()
        p_l, info = learned_solve(s16, p0, w, ls, sched)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - a
        s16.close()
        e_irls = _pose_err(p_irls.cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        e_pc = _pose_err(p_pc.cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        e_l = _pose_err(p_l.cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        e_lo = _pose_err(info.pop("params_learned").cpu().numpy(), sc["R_gt"], sc["t_gt"], sc["pairs"])
        r_d, t_d = _pose_changes(p_l.cpu().numpy(), p_irls.cpu().numpy(), sc["pairs"])
        rows.append({"seed": sc["seed"], "irls_s": t_irls, "plain_converged_s": t_pc, "learned_s": t_l,
                     "irls_err_deg": e_irls, "plain_converged_err_deg": e_pc, "learned_err_deg": e_l,
                     "learned_before_tail_err_deg": e_lo, "plain_converged": info_pc,
                     "learned_vs_irls_max_deg": (float(r_d.max()), float(t_d.max())), **info})
        print(f"[learned] seed {sc['seed']}: IRLS {t_irls * 1e3:.1f} ms rot med {e_irls['rot_med']:.3f}; plain "
              f"with the stopping rule {t_pc * 1e3:.1f} ms ({info_pc['loops']} loops) rot med "
              f"{e_pc['rot_med']:.3f}; learned {t_l * 1e3:.1f} ms ({info['loops_total']} loops, converged "
              f"{info['converged']}) rot med {e_l['rot_med']:.3f}", flush=True)
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
