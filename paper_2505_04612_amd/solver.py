"""Host orchestration of epipolar adjustment on the GPU (Sec. 3.3).

A solve is a sequence of optimisation loops.  Each loop builds the weighted
per-pair Grams (the first from IRLS weights at the initial poses, or from unit
weights), then runs its Adam steps in one persistent fused kernel
(fm_epipolar_solve).  Between loops the weights are recomputed at the current
poses with a filter threshold that halves from tau0 down to tau_min
(fm_reweight_build, one pass over the matches).  Z (the number of kept
matches) stays on the device, so a whole solve needs no host round trip.
"""
from __future__ import annotations

import dataclasses

import torch

from . import api


@dataclasses.dataclass
class Schedule:
    iters: int = 500              # total Adam steps
    round_len: int = 100          # Adam steps per optimisation loop
    lr_rot: float = 3e-3          # initial lr on the 6D rotation parameters
    lr_t: float = 1e-2            # initial lr on the translations
    lr_final_frac: float = 1e-3   # lr decays exponentially to lr0*frac over the solve
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12
    irls: bool = True             # reweight between loops
    delta: float = 1e-4           # floor of |r| in the IRLS weight 1/max(|r|, delta)
    tau0: float = 0.1             # first filter threshold on |r|
    tau_min: float = 0.01         # threshold floor
    first_round_unit_weights: bool = False
    gram_dtype: torch.dtype = torch.float32  # Gram precision the iterations read (the float32 copy of the
                                             # float64 per-pair sums: half the bytes of each iteration)
    blocks: int = 0               # fused loop grid: 0 automatic, > 0 workgroups of the pair loop, < 0 the camera loop


def tau_at(s: Schedule, k: int) -> float:
    """Threshold of the k-th reweighting: tau0 halved k times, floored."""
    return max(s.tau0 * 0.5 ** k, s.tau_min)


def _grams(scene, params, s: Schedule, tau: float | None):
    f64 = s.gram_dtype == torch.float64
    if tau is None:
        W64, W32 = api.build_pair_grams(scene, None, f64=f64, f32=not f64)
        return (W64 if f64 else W32), None
    W64, W32, kept = api.reweight_build(scene, params, s.delta, tau, f64=f64, f32=not f64)
    return (W64 if f64 else W32), kept


def solve(scene: api.Scene, params0: torch.Tensor, s: Schedule, trace: bool = True, rounds: int | None = None,
          check_barriers: bool = True):
    """Run the schedule from params0 [N,9] float32.  Returns (params, loss
    trace [iters] float64 or None, Z [1] int64 or None for unit weights).
    `rounds` stops after that many optimisation loops (the schedule's learning
    rates and thresholds are those of the full run).  With `check_barriers`
    the call ends by synchronising the device and raises FastMapError if a
    grid barrier of the fused loops timed out (their results would then be
    invalid); without it the caller reads scene.barrier_failures() itself."""
    dev = scene.ctx.device
    params = params0.detach().to(dev, torch.float32).clone().contiguous()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    losses = torch.empty(s.iters, dtype=torch.float64, device=dev) if trace else None
    k_rw = 0
    if s.irls and not s.first_round_unit_weights:
        W, Z = _grams(scene, params, s, tau_at(s, 0))
        k_rw = 1
    else:
        W, Z = _grams(scene, params, s, None)
    inv_Z = 1.0 / max(scene.num_matches, 1)
    done = 0
    stop = s.iters if rounds is None else min(s.iters, rounds * s.round_len)
    while done < stop:
        K = min(s.round_len, s.iters - done)
        m.zero_()
        v.zero_()
        api.epipolar_solve(scene, W, params, m, v, K, s.lr_rot, s.lr_t, s.lr_final_frac, done, s.iters, 0,
                           s.beta1, s.beta2, s.eps, inv_Z=None if Z is not None else inv_Z, Z=Z,
                           loss_trace=losses[done:done + K] if trace else None, blocks=s.blocks)
        done += K
        if s.irls and done < stop:
            W, Z = _grams(scene, params, s, tau_at(s, k_rw))
            k_rw += 1
    if check_barriers:
        scene.require_barriers_ok()
    return params, losses, Z
