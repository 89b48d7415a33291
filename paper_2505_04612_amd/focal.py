"""Focal-length refinement inside epipolar adjustment (FastMap, arXiv
2505.04612, Sec. 3.3: the focal lengths built into the essential matrices).
By default the whole Adam loop is one persistent launch
(fm_epipolar_focal_solve); `fused=False` runs it step by step from the host:
one fm_epipolar_focal_loss_grad (pair and camera kernels), one fm_adam_step
over the poses and one over the log focal scales per step.  The learning
rates decay exponentially from lr0 to lr0 * frac over the loop.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class FocalSchedule:
    iters: int = 300
    lr_rot: float = 3e-3
    lr_t: float = 1e-2
    lr_phi: float = 1e-2
    lr_final_frac: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12


def solve(scene: api.Scene, W36: torch.Tensor, params: torch.Tensor, phi: torch.Tensor, inv_Z: float,
          sched: FocalSchedule = FocalSchedule(), trace: bool = False, fused: bool = True):
    """Refine poses [N,9] and log focal scales [N] in place; returns the loss
    trace (host list) if `trace`.  Raises FastMapError if the persistent
    launch's grid barrier timed out."""
    ctx = scene.ctx
    N = scene.num_cams
    mp, vp = torch.zeros_like(params), torch.zeros_like(params)
    mf, vf = torch.zeros_like(phi), torch.zeros_like(phi)
    if fused:
        tr = torch.empty(sched.iters, dtype=torch.float64, device=params.device) if trace else None
        api.epipolar_focal_solve(scene, W36, params, phi, mp, vp, mf, vf, sched.iters, sched.lr_rot, sched.lr_t,
                                 sched.lr_phi, sched.lr_final_frac, beta1=sched.beta1, beta2=sched.beta2,
                                 eps=sched.eps, inv_Z=inv_Z, loss_trace=tr)
        scene.require_barriers_ok()
        return tr.cpu().tolist() if trace else None
    lr0 = np.tile(np.array([sched.lr_rot] * 6 + [sched.lr_t] * 3, np.float32), N)
    lr_p = torch.empty(9 * N, dtype=torch.float32, device=params.device)
    lr_f = torch.empty(1, dtype=torch.float32, device=params.device)
    out = []
    for k in range(sched.iters):
        f = sched.lr_final_frac ** (k / sched.iters)
        lr_p.copy_(torch.from_numpy(lr0 * np.float32(f)))
        lr_f.fill_(float(sched.lr_phi * f))
        loss, g, gp = api.epipolar_focal_loss_grad(scene, W36, params, phi, inv_Z, want_loss=trace)
        if trace:
            out.append(loss)
        api.adam_step(ctx, params.view(-1), g.view(-1), mp.view(-1), vp.view(-1), k + 1, lr_p, sched.beta1,
                      sched.beta2, sched.eps)
        api.adam_step(ctx, phi, gp, mf, vf, k + 1, lr_f, sched.beta1, sched.beta2, sched.eps)
    return [float(x.item()) for x in out] if trace else None
