"""Write the stored oracle results the benchmark's pose check compares with.

Calls only the input generator and the FP64 oracle (never the HIP path):
the medium workload (200 cameras, ~4.9k pairs, ~2.9M matches, FP32-stored
coordinates), solved with the default schedule (2,000 Adam steps, IRLS
reweighting every 100).  Schedule constants are the float32 values the GPU
library receives, so both sides use identical thresholds and rates.

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ea  # noqa: E402
from paper_2505_04612_amd import synth  # noqa: E402


def f32(x):
    return float(np.float32(x))


def scene_digest(sc, coords) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sc.pairs, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(sc.offsets, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(coords).tobytes())
    h.update(np.ascontiguousarray(sc.R_init).tobytes())
    h.update(np.ascontiguousarray(sc.t_init).tobytes())
    return h.hexdigest()


SCHEDULE = dict(iters=2000, round_len=100, lr_rot=3e-3, lr_t=1e-2, lr_final_frac=1e-3, beta1=0.9,
                beta2=0.999, eps=1e-12, irls=True, delta=1e-4, tau0=0.1, tau_min=0.01)


def oracle_schedule(d=SCHEDULE) -> ea.Schedule:
    kw = {k: (f32(v) if isinstance(v, float) else v) for k, v in d.items()}
    return ea.Schedule(**kw)


def main():
    t0 = time.time()
    sc = synth.medium()
    coords = sc.uv.astype(np.float32)
    th0 = ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)
    th, trace, w = ea.solve(th0.astype(np.float64), sc.pairs, sc.offsets, coords.astype(np.float64),
                            oracle_schedule())
    th_gt = ea.params_from_poses(sc.R_gt, sc.t_gt)
    rot, tra = ea.relative_pose_errors(th, th_gt, sc.pairs)
    out = {
        "workload": "medium", "seed": sc.seed, "storage": "f32", "stats": sc.stats(),
        "digest": scene_digest(sc, coords), "schedule": SCHEDULE,
        "theta": th.tolist(), "kept": int(np.count_nonzero(w)), "final_loss": float(trace[-1]),
        "vs_ground_truth_deg": {"rot_median": float(np.median(rot)), "rot_max": float(rot.max()),
                                "t_median": float(np.median(tra)), "t_max": float(tra.max())},
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "medium_oracle.json"), "w") as f:
        json.dump(out, f)
    print(json.dumps({k: v for k, v in out.items() if k != "theta"}))


if __name__ == "__main__":
    main()
