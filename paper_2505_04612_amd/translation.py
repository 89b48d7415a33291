"""Global translation averaging (FastMap, arXiv 2505.04612, Sec. 3.3 "Global
Translation"; appendix on multiple initialisations), host orchestration of
the library's kernels:

  1. targets o^{i->j} = -R_j^T t^{i->j} per pair (fm_translation_directions);
  2. R independent runs of K Adam steps on L_t from random centres, all runs
     in one persistent launch (fm_translation_solve);
  3. merge: each run aligned (centroid to the origin, unit mean norm), each
     camera taken from the run with its lowest mean pair term
     (fm_translation_merge);
  4. a final loop of K_final steps from the merged centres.

Every step runs in the HIP library; this module only allocates tensors and
sequences the calls.
"""
from __future__ import annotations

import dataclasses

import torch

from . import api


@dataclasses.dataclass
class TranslationSchedule:
    iters: int = 1000           # Adam steps of each independent run
    final_iters: int = 1000     # Adam steps of the loop from the merged centres
    lr: float = 3e-2            # initial learning rate on the centres
    lr_final_frac: float = 1e-2 # the rate decays exponentially to lr * frac over a loop
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12


def average(scene: api.Scene, dirs: torch.Tensor, init: torch.Tensor,
            sched: TranslationSchedule = TranslationSchedule(), trace: bool = False):
    """Camera centres [N,3] from targets `dirs` [P,3] and initial centres
    `init` [runs,N,3] (one random initialisation per run).  Returns
    (centres, info) with the runs' final centres, the merge choice and, if
    `trace`, the loss traces of the runs and of the final loop.  Raises
    FastMapError if a persistent launch's grid barrier timed out."""
    R = int(init.shape[0])
    runs = init.clone()
    m = torch.zeros_like(runs)
    v = torch.zeros_like(runs)
    tr = torch.empty((R, sched.iters), dtype=torch.float64, device=runs.device) if trace else None
    api.translation_solve(scene, dirs, runs, m, v, sched.iters, sched.lr, sched.lr_final_frac,
                          beta1=sched.beta1, beta2=sched.beta2, eps=sched.eps, loss_trace=tr)
    merged, choice, cam = api.translation_merge(scene, dirs, runs)
    final = merged.unsqueeze(0).contiguous()
    m1 = torch.zeros_like(final)
    v1 = torch.zeros_like(final)
    tr1 = torch.empty((1, sched.final_iters), dtype=torch.float64, device=runs.device) if trace else None
    api.translation_solve(scene, dirs, final, m1, v1, sched.final_iters, sched.lr, sched.lr_final_frac,
                          beta1=sched.beta1, beta2=sched.beta2, eps=sched.eps, loss_trace=tr1)
    scene.require_barriers_ok()
    info = {"runs": runs, "merged": merged, "choice": choice, "cam_loss": cam}
    if trace:
        info["trace_runs"] = tr
        info["trace_final"] = tr1[0]
    return final[0], info
