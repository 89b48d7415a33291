"""Learned-weight form end to end on small helix scenes (GPU): the network is
trained by the library's own forward/backward/Adam kernels on converged-IRLS
targets; on held-out scenes the learned solve (one Gram from the network's
weights in place of the middle IRLS loops, then plain IRLS loops until a
loop moves at most 10 % of the pairs by more than 0.1 deg / 0.5 deg) is
timed and scored against plain IRLS over the full schedule and against
plain IRLS under the same stopping rule; a garbage network leaves the work
to the plain loops and still ends at plain IRLS accuracy."""
import time

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _scene(seed, ctx, dtype=torch.float32):
    from paper_2505_04612_amd import api, synth
    sc = synth.learned(seed=seed, n_cams=80, n_points=40_000)
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, dtype)
    p0 = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    return sc, s, torch.from_numpy(p0).to(ctx.device)


@pytest.fixture(scope="module")
def trained():
    from paper_2505_04612_amd import api, learned, solver
    ctx = api.default_context()
    sched = solver.Schedule(iters=2000, round_len=100)
    feats, tgts = [], []
    for seed in (100, 101, 102, 103):
        sc, s, p0 = _scene(seed, ctx)
        f, t, _ = learned.irls_targets(s, p0, sched)
        assert torch.all((t >= 0) & (t <= 1))
        feats.append(f)
        tgts.append(t)
        s.close()
    w, hist = learned.train_mlp(ctx, torch.cat(feats).contiguous(), torch.cat(tgts).contiguous(),
                                learned.TrainCfg(steps=800, batch=16384))
    return ctx, sched, w, hist


def test_training_reduces_loss(trained):
    _, _, _, hist = trained
    assert hist[-1][1] < 0.5 * hist[0][1], hist


def _timed(fn, reps=3):
    """Result of the last run and the shortest wall time of `reps` runs."""
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - a)
    return out, best


def test_learned_solve_against_plain_irls_on_held_out_scenes(trained):
    """Held-out scenes 200-203: the learned path (BF16 coordinates) against
    plain IRLS (FP32 coordinates, all 20 loops) and against plain IRLS with
    the same stopping rule.  Asserted: the learned result is as accurate as
    plain IRLS under the same rule (median relative rotation and
    translation-direction error against the truth within 10 % or 0.05 deg),
    and it takes less time than plain IRLS under that rule (measured 0.79x
    over held-out scenes 200-207 with the default 50 learned steps; 600
    steps took 1.6x, as long as the IRLS loops they replaced).  The full
    schedule ends more accurate (median 0.12-0.14 deg against 0.19-0.22 deg
    with either rule) at about twice the time of either ruled path."""
    from paper_2505_04612_amd import learned, solver
    ctx, sched, w, _ = trained
    ls = learned.LearnedSchedule()
    rows = []
    for seed in (200, 201, 202, 203):
        sc, s, p0 = _scene(seed, ctx)
        _, s16, _ = _scene(seed, ctx, torch.bfloat16)
        # warm-up of every path, then the shortest of three timed runs each
        solver.solve(s, p0, sched, trace=False)
        learned.plain_converged_solve(s, p0, sched, ls)
        learned.learned_solve(s16, p0, w, ls, sched)
        (p_irls, _, _), t_irls = _timed(lambda: solver.solve(s, p0, sched, trace=False))
        (p_pc, info_pc), t_pc = _timed(lambda: learned.plain_converged_solve(s, p0, sched, ls))
        (p_l, info), t_l = _timed(lambda: learned.learned_solve(s16, p0, w, ls, sched))
        e = {k: learned._pose_err(p.cpu().numpy(), sc.R_gt, sc.t_gt, sc.pairs)
             for k, p in (("irls", p_irls), ("plain_conv", p_pc), ("learned", p_l))}
        rows.append((seed, t_irls, t_pc, t_l, info_pc["loops"], info["loops_total"], info["converged"], e))
        print(f"seed {seed}: plain IRLS {t_irls * 1e3:.1f} ms rot/t med {e['irls']['rot_med']:.3f}/"
              f"{e['irls']['t_med']:.3f}; plain + stopping rule {t_pc * 1e3:.1f} ms, {info_pc['loops']} loops, "
              f"{e['plain_conv']['rot_med']:.3f}/{e['plain_conv']['t_med']:.3f}; learned {t_l * 1e3:.1f} ms, "
              f"{info['loops_total']} loops (converged {info['converged']}), "
              f"{e['learned']['rot_med']:.3f}/{e['learned']['t_med']:.3f} deg")
        s.close()
        s16.close()
    t_irls = sum(r[1] for r in rows)
    t_pc = sum(r[2] for r in rows)
    t_l = sum(r[3] for r in rows)
    print(f"totals: plain IRLS {t_irls * 1e3:.1f} ms, plain + stopping rule {t_pc * 1e3:.1f} ms, learned "
          f"{t_l * 1e3:.1f} ms: learned / plain IRLS {t_l / t_irls:.2f}, learned / plain + rule {t_l / t_pc:.2f}")
    for seed, _, _, _, _, _, _, e in rows:
        for k in ("rot_med", "t_med"):
            assert e["learned"][k] <= max(1.1 * e["plain_conv"][k], e["plain_conv"][k] + 0.05), (seed, k, e)
            assert e["learned"][k] <= e["irls"][k] + 0.15, (seed, k, e)
    assert t_l <= 1.1 * t_irls, (t_l, t_irls)
    assert t_l < t_pc, ("the learned path is not faster than plain IRLS under the same rule", t_l, t_pc)


def test_garbage_network_leaves_the_work_to_plain_loops(trained):
    """A network whose weights are all ~0 makes a zero Gram, so the learned
    block leaves the poses where they were; the plain loops after it must do
    the work (more loops than with the trained network) and end at plain
    IRLS accuracy under the same stopping rule."""
    from paper_2505_04612_amd import api, learned
    ctx, sched, w_good, _ = trained
    sc, s, p0 = _scene(201, ctx)
    w = api.MlpWeights(ctx.device)
    w.views["b3"].fill_(-30.0)           # sigmoid ~ 0: every weight ~ 0
    ls = learned.LearnedSchedule(warm_rounds=0)
    p_l, info = learned.learned_solve(s, p0, w, ls, sched)
    _, info_good = learned.learned_solve(s, p0, w_good, ls, sched)
    assert info["tail_loops"] >= info_good["tail_loops"], (info, info_good)
    assert info["tail_loops"] >= 2, info
    # plain IRLS under the same stopping rule is the reference
    p_pc, _ = learned.plain_converged_solve(s, p0, sched, ls)
    e_pc = learned._pose_err(p_pc.cpu().numpy(), sc.R_gt, sc.t_gt, sc.pairs)
    e_l = learned._pose_err(p_l.cpu().numpy(), sc.R_gt, sc.t_gt, sc.pairs)
    assert e_l["rot_med"] <= 1.5 * e_pc["rot_med"] + 0.05, (e_l, e_pc)


def test_pose_change_counts_match_host_angles(trained):
    """fm_pose_change against the host evaluation of the same angles on two
    parameter sets a loop apart."""
    from paper_2505_04612_amd import api, learned, solver
    ctx, sched, _, _ = trained
    sc, s, p0 = _scene(202, ctx)
    p1, _, _ = solver.solve(s, p0, solver.Schedule(iters=100, round_len=100), trace=False)
    counts, rot, tr = api.pose_change(s, p0, p1, 0.1, 0.5, per_pair=True)
    r_h, t_h = learned._pose_changes(p0.cpu().numpy(), p1.cpu().numpy(), sc.pairs)
    assert np.allclose(rot.cpu().numpy(), r_h, rtol=1e-5, atol=1e-6)
    assert np.allclose(tr.cpu().numpy(), t_h, rtol=1e-5, atol=1e-6)
    c = counts.cpu().numpy()
    assert abs(int(c[0]) - int(np.sum(r_h > 0.1))) <= 1 and abs(int(c[1]) - int(np.sum(t_h > 0.5))) <= 1
    z, _, _ = api.pose_change(s, p1, p1, 1e-6, 1e-6)
    assert z.cpu().tolist() == [0, 0]
