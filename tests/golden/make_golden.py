"""Write the stored oracle solves that the benchmark's pose check and the
whole-solve GPU tests compare with.

Calls only the input generator and the FP64 oracle (never the HIP path).
Each workload is solved with the default schedule (2,000 Adam steps,
IRLS reweighting every 100) from its seeded initial poses, on the
coordinates exactly as the workload stores them:

    medium    200 cameras, ~4.9k pairs, ~2.9M matches, float32 coordinates
    diffprec  1,000 cameras, ~34k pairs, ~25M matches, bfloat16 coordinates
    large     5,000 street cameras, ~185k pairs, ~172M matches, bfloat16
              coordinates (about half an hour of CPU)

Schedule constants are the float32 values the GPU library receives, so both
sides use identical thresholds and rates.

Each file also records how far the oracle's own solve moves when its
parameters are kept in float32 between Adam steps (all arithmetic still
float64; the storage the GPU library uses): percentiles of the per-pair
relative-rotation and translation-direction differences between that solve
and the float64 one, the number of pairs beyond 0.1 deg / 0.5 deg, and its
final kept-match count.
`--sensitivity` adds only this block to an existing file (whose float64
solve this script wrote).

    python tests/golden/make_golden.py [--sensitivity] [medium|diffprec|large ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ea  # noqa: E402
from paper_2505_04612_amd import synth  # noqa: E402

STORAGE = {"medium": "f32", "diffprec": "bf16", "large": "bf16"}


def f32(x):
    return float(np.float32(x))


def scene_digest(sc, coords) -> str:
    """SHA-256 over the pair list, offsets, stored coordinates and initial
    poses; `coords` is the array of stored values (float32, or the bfloat16
    bit patterns as uint16)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sc.pairs, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(sc.offsets, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(coords).tobytes())
    h.update(np.ascontiguousarray(sc.R_init).tobytes())
    h.update(np.ascontiguousarray(sc.t_init).tobytes())
    return h.hexdigest()


def stored_coords(sc, storage: str):
    """(digest array, float64 values) of the coordinates as the workload
    stores them; bfloat16 is rounded to nearest even from float64 by torch on
    the CPU, as the library's scene upload does."""
    if storage == "f32":
        c = np.ascontiguousarray(sc.uv, dtype=np.float32)
        return c, c.astype(np.float64)
    import torch
    b = torch.from_numpy(np.ascontiguousarray(sc.uv, dtype=np.float64)).to(torch.bfloat16)
    return b.view(torch.int16).numpy().view(np.uint16), b.to(torch.float64).numpy()


def make_scene(name: str):
    if name == "large":
        return synth.large(workers=min(8, os.cpu_count() or 1))
    return synth.make(name)


SCHEDULE = dict(iters=2000, round_len=100, lr_rot=3e-3, lr_t=1e-2, lr_final_frac=1e-3, beta1=0.9,
                beta2=0.999, eps=1e-12, irls=True, delta=1e-4, tau0=0.1, tau_min=0.01)


def oracle_schedule(d=SCHEDULE) -> ea.Schedule:
    kw = {k: (f32(v) if isinstance(v, float) else v) for k, v in d.items()}
    return ea.Schedule(**kw)


def solve_one(name: str) -> dict:
    t0 = time.time()
    sc = make_scene(name)
    digest_arr, x = stored_coords(sc, STORAGE[name])
    print(f"[golden] {name}: {sc.stats()} in {time.time() - t0:.1f}s", flush=True)
    th0 = ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)
    hist = []
    stop = threading.Event()

    def progress():
        while not stop.wait(60.0):
            print(f"[golden] {name}: {len(hist)} of 20 loops started, {time.time() - t0:.0f}s", flush=True)

    th_prog = threading.Thread(target=progress, daemon=True)
    th_prog.start()
    try:
        th, trace, w = ea.solve(th0.astype(np.float64), sc.pairs, sc.offsets, x, oracle_schedule(), history=hist)
    finally:
        stop.set()
    th_gt = ea.params_from_poses(sc.R_gt, sc.t_gt)
    rot, tra = ea.relative_pose_errors(th, th_gt, sc.pairs)
    return {
        "workload": name, "seed": sc.seed, "storage": STORAGE[name], "stats": sc.stats(),
        "digest": scene_digest(sc, digest_arr), "schedule": SCHEDULE,
        "theta": th.tolist(), "kept": int(np.count_nonzero(w)), "final_loss": float(trace[-1]),
        "kept_per_loop": [h["Z"] for h in hist],
        "vs_ground_truth_deg": {"rot_median": float(np.median(rot)), "rot_max": float(rot.max()),
                                "t_median": float(np.median(tra)), "t_max": float(tra.max())},
        "oracle_seconds": time.time() - t0,
    }


def _f32(theta):
    return theta.astype(np.float32).astype(np.float64)


def error_summary(rot: np.ndarray, tra: np.ndarray) -> dict:
    """Percentiles (50, 99, 99.9, 100) of per-pair rotation and translation
    differences in degrees, and the pairs beyond 0.1 deg / 0.5 deg."""
    def q(a):
        return {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99)),
                "p99.9": float(np.percentile(a, 99.9)), "max": float(a.max())}
    return {"rot": {**q(rot), "over_bar": int(np.sum(rot > 0.1))},
            "t": {**q(tra), "over_bar": int(np.sum(tra > 0.5))}}


def sensitivity(name: str, golden: dict) -> dict:
    """The float32-storage solve of the same workload against the stored
    float64 solve."""
    t0 = time.time()
    sc = make_scene(name)
    digest_arr, x = stored_coords(sc, STORAGE[name])
    assert scene_digest(sc, digest_arr) == golden["digest"], "scene does not match the stored solve"
    th0 = ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)
    th, _, w = ea.solve(th0.astype(np.float64), sc.pairs, sc.offsets, x, oracle_schedule(), store=_f32)
    rot, tra = ea.relative_pose_errors(th, np.array(golden["theta"]), sc.pairs)
    out = error_summary(rot, tra)
    out["kept"] = int(np.count_nonzero(w))
    out["seconds"] = time.time() - t0
    return out


def main(argv):
    only_sens = "--sensitivity" in argv
    names = [a for a in argv if not a.startswith("--")] or ["medium"]
    for name in names:
        path = os.path.join(HERE, f"{name}_oracle.json")
        if only_sens:
            with open(path) as f:
                out = json.load(f)
        else:
            out = solve_one(name)
        out["float32_storage_sensitivity"] = sensitivity(name, out)
        with open(path, "w") as f:
            json.dump(out, f)
        print(json.dumps({k: v for k, v in out.items() if k != "theta"}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
