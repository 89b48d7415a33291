"""Shared test helpers: cached seeded scenes and tolerance checks."""
from __future__ import annotations

import functools

import numpy as np
import torch

from paper_2505_04612_amd import synth

# q(a, c): position of x~[a] x~[c] in p = (u^2, uv, v^2, u, v, 1)
_Q = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 2, (0, 2): 3, (2, 0): 3, (1, 2): 4, (2, 1): 4, (2, 2): 5}


def expand36(W36: np.ndarray) -> np.ndarray:
    """Expand the documented compact layout W36[n][6 q(a,c) + q(b,d)] into the
    full 9x9 W_{(ab),(cd)} (written here from the ABI documentation)."""
    P = W36.shape[0]
    out = np.empty((P, 9, 9), dtype=W36.dtype)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                for d in range(3):
                    out[:, 3 * a + b, 3 * c + d] = W36[:, 6 * _Q[(a, c)] + _Q[(b, d)]]
    return out


@functools.lru_cache(maxsize=None)
def scene(name: str, **kw) -> synth.Scene:
    return synth.make(name, **kw)


def stored(uv: np.ndarray, dtype: torch.dtype) -> np.ndarray:
    """The float64 value of the coordinates as the workload stores them."""
    return torch.from_numpy(np.ascontiguousarray(uv)).to(dtype).to(torch.float64).numpy()


def gram_errors(W_gpu: np.ndarray, W_ref: np.ndarray, W_abs: np.ndarray):
    """(max per-pair normwise relative error, max elementwise error relative to
    the sum of absolute terms)."""
    d = W_gpu - W_ref
    nrm = np.linalg.norm(W_ref.reshape(len(W_ref), -1), axis=1)
    dn = np.linalg.norm(d.reshape(len(d), -1), axis=1)
    rel = np.where(nrm > 0, dn / np.where(nrm > 0, nrm, 1), dn)
    el = np.abs(d) / np.where(W_abs > 0, W_abs, 1.0)
    return float(rel.max(initial=0.0)), float(el.max(initial=0.0))


def f32(x: float) -> float:
    return float(np.float32(x))
