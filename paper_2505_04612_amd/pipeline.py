"""FastMap's global pose stages in sequence (arXiv 2505.04612, Sec. 3.3 and
the appendix), every step in the library's kernels; the host only sequences
the calls and converts between parameter layouts:

  1. global rotations: column-wise least-squares initialisation, then the
     geodesic objective (rotation.average);
  2. relative translations: grid search over candidate directions on each
     pair's Gram with the relative rotations of step 1
     (fm_translation_search); the sign comes from the caller's prior;
  3. camera centres: translation averaging from several random starts,
     merged (translation.average);
  4. epipolar adjustment from those poses (solver.solve: IRLS loops of the
     fused loss + adjoint + Adam kernel).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import api, rotation, solver, translation


@dataclasses.dataclass
class PipelineConfig:
    rotation: rotation.RotationSchedule = dataclasses.field(default_factory=rotation.RotationSchedule)
    candidates: int = 4096
    translation: translation.TranslationSchedule = dataclasses.field(default_factory=translation.TranslationSchedule)
    runs: int = 4
    seed: int = 5
    ea: solver.Schedule = dataclasses.field(default_factory=lambda: solver.Schedule(iters=2000, round_len=100))


def run(scene: api.Scene, Rrel: torch.Tensor, t_prior: torch.Tensor, weights: torch.Tensor | None = None,
        cfg: PipelineConfig = PipelineConfig()):
    """Poses [N,9] (a1, a2, t) from measured relative rotations Rrel [P,9],
    the scene's matches (Grams with `weights`, e.g. the matches an upstream
    two-view estimate keeps) and prior relative-translation directions
    t_prior [P,3] (only their signs are used).  Returns (params, stages)
    with the intermediate results."""
    dev = scene.ctx.device
    N = scene.num_cams
    p6, rinfo = rotation.average(scene, Rrel, cfg.rotation)
    W64, _ = api.build_pair_grams(scene, weights, f32=False)
    p9 = torch.cat([p6, torch.zeros((N, 3), dtype=torch.float32, device=dev)], 1).contiguous()
    t_rel, _, _ = api.translation_search(scene, W64, p9, api.fibonacci_sphere(cfg.candidates, dev), t_prior)
    dirs = api.translation_directions(scene, p9, t_rel)
    init = torch.from_numpy(np.random.default_rng(cfg.seed).normal(size=(cfg.runs, N, 3)).astype(np.float32)).to(dev)
    centres, tinfo = translation.average(scene, dirs, init, cfg.translation)
    theta0 = api.poses_from_centres(scene.ctx, p6.contiguous(), centres.contiguous())
    params, _, _ = solver.solve(scene, theta0, cfg.ea, trace=False)
    return params, {"rotations": p6, "t_rel": t_rel, "centres": centres, "averaged": theta0}
