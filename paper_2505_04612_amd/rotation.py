"""Global rotation averaging (FastMap, arXiv 2505.04612, Sec. 3.3 "Global
Rotation"; appendix on rotation initialisation), host orchestration of the
library's kernels:

  1. initial rotations from the column-wise least-squares problems
     (fm_rotation_init: Lanczos on the GPU for each column's eigenvector);
  2. K Adam steps on the geodesic objective L_R over the 6D parameters in
     one persistent launch (fm_rotation_solve).

Every step runs in the HIP library; this module only allocates tensors and
sequences the calls.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class RotationSchedule:
    lanczos_steps: int = 300    # per eigenvector (at most 3N)
    iters: int = 500            # Adam steps on L_R
    lr: float = 1e-2            # initial learning rate on (a1, a2)
    lr_final_frac: float = 1e-2 # exponential decay to lr * frac over the loop
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12
    seed: int = 0               # start vectors of the two Lanczos runs


def average(scene: api.Scene, Rrel: torch.Tensor, sched: RotationSchedule = RotationSchedule(),
            trace: bool = False):
    """World-to-camera rotation parameters [N,6] (a1, a2) from the measured
    relative rotations Rrel [P,9] (row-major).  Returns (params, info) with
    the initial parameters, the Lanczos eigenvalues and steps, and, if
    `trace`, the loss trace of the solve.  Raises FastMapError if a
    persistent launch's grid barrier timed out."""
    N = scene.num_cams
    start = torch.from_numpy(np.random.default_rng(sched.seed).normal(size=(2, 3 * N))).to(scene.ctx.device)
    p0, lz = api.rotation_init(scene, Rrel, start, sched.lanczos_steps)
    p = p0.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    tr = torch.empty(sched.iters, dtype=torch.float64, device=p.device) if trace else None
    api.rotation_solve(scene, Rrel, p, m, v, sched.iters, sched.lr, sched.lr_final_frac, beta1=sched.beta1,
                       beta2=sched.beta2, eps=sched.eps, loss_trace=tr)
    scene.require_barriers_ok()
    info = {"init": p0, "lanczos": lz}
    if trace:
        info["trace"] = tr
    return p, info
