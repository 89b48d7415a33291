"""Torch-facing wrappers of the C ABI.

PyTorch only supplies device memory and the current HIP stream; every
computation happens in the library's kernels.  Functions take and return
CUDA (HIP) tensors on the context's device.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import FastMapError, check

_DTYPES = {torch.float64: _lib.FM_F64, torch.float32: _lib.FM_F32, torch.bfloat16: _lib.FM_BF16}


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require(t: torch.Tensor, dtype, shape, name: str, device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name}: expected device {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise FastMapError(_lib.FM_EHIP, "no HIP device available")
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = self.lib.fm_create(ctypes.byref(h), device)
        if rc != _lib.FM_OK:
            raise FastMapError(rc, f"fm_create({device}) failed")
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.fm_destroy(self.handle)
            self.handle = None

    def set_check(self, enable: bool) -> None:
        """Turn the library's device-side data checks on or off (fm_set_check)."""
        check(self.handle, self.lib.fm_set_check(self.handle, 1 if enable else 0))

    def check(self) -> int:
        """Synchronise the current stream and read and clear the device check
        flag (fm_check).  Returns 0, or raises FastMapError(FM_EDEVICE_CHECK)
        whose `flags` attribute holds the FM_CHECK_* bits that were set."""
        f = ctypes.c_uint32(0)
        rc = self.lib.fm_check(self.handle, _stream(), ctypes.byref(f))
        if rc != _lib.FM_OK:
            err = FastMapError(rc, self.lib.fm_last_error(self.handle).decode())
            err.flags = int(f.value)
            raise err
        return 0

    def profile(self, enable: bool) -> None:
        """Start (clearing earlier records) or stop launch timing."""
        check(self.handle, self.lib.fm_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self, kernel: int) -> tuple[float, int]:
        """(summed device milliseconds, launches) of one kernel id (_lib.K_*)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(self.handle, self.lib.fm_profile_read(self.handle, kernel, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Context | None = None
_live_scenes: "weakref.WeakSet[Scene]" = weakref.WeakSet()


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(torch.cuda.current_device())
    return _default_ctx


def release_all() -> None:
    """Destroy every live scene and the default context now (explicitly, at
    the end of a program, so that no library call runs inside the
    interpreter's exit); later calls make a new default context."""
    global _default_ctx
    for s in list(_live_scenes):
        s.close()
    if _default_ctx is not None:
        _default_ctx.close()
        _default_ctx = None


@atexit.register
def _shutdown() -> None:
    """Release what release_all() would, if the program did not, while the
    HIP runtime is still up (interpreter teardown order is otherwise
    unspecified)."""
    try:
        release_all()
    except Exception:
        pass


class Scene:
    """Pairs, CSR offsets and match coordinates resident on the device, plus
    the library's derived index data and workspace (fm_scene)."""

    def __init__(self, ctx: Context, num_cams: int, pairs: torch.Tensor, offsets: torch.Tensor,
                 uv: torch.Tensor):
        self.ctx = ctx
        dev = ctx.device
        P = int(pairs.shape[0]) if pairs.ndim == 2 else 0
        M = int(uv.shape[0])
        _require(pairs, torch.int32, (P, 2), "pairs", dev)
        _require(offsets, torch.int64, (P + 1,), "offsets", dev)
        if uv.dtype not in _DTYPES:
            raise TypeError(f"uv dtype {uv.dtype} not supported (float64, float32, bfloat16)")
        _require(uv, uv.dtype, (M, 4), "uv", dev)
        self.num_cams, self.num_pairs, self.num_matches = int(num_cams), P, M
        self.pairs, self.offsets, self.uv = pairs, offsets, uv
        self.dtype = uv.dtype
        h = ctypes.c_void_p()
        rc = ctx.lib.fm_scene_create(ctx.handle, P, M, int(num_cams), _ptr(offsets), _ptr(pairs), _ptr(uv),
                                     _DTYPES[uv.dtype], _stream(), ctypes.byref(h))
        check(ctx.handle, rc)
        self.handle = h
        _live_scenes.add(self)

    @classmethod
    def from_numpy(cls, ctx: Context, num_cams: int, pairs: np.ndarray, offsets: np.ndarray,
                   uv: np.ndarray, dtype: torch.dtype = torch.float32) -> "Scene":
        dev = ctx.device
        uv_t = torch.from_numpy(np.ascontiguousarray(uv, dtype=np.float64)).to(dtype).to(dev)
        return cls(ctx, num_cams,
                   torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).to(dev),
                   torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(dev),
                   uv_t.contiguous())

    @property
    def work_items(self) -> int:
        return int(self.ctx.lib.fm_scene_work_items(self.handle))

    def barrier_failures(self) -> int:
        """Failed grid barriers of the fused solve on this scene since the last
        call (synchronises the device); 0 unless a launch was invalid."""
        n = ctypes.c_int64(0)
        check(self.ctx.handle, self.ctx.lib.fm_solve_barrier_failures(self.ctx.handle, self.handle, ctypes.byref(n)))
        return int(n.value)

    def require_barriers_ok(self) -> None:
        """Raise FastMapError if a grid barrier of a persistent launch on this
        scene timed out since the last query (its results are then invalid);
        synchronises the device."""
        failed = self.barrier_failures()
        if failed:
            raise FastMapError(_lib.FM_EHIP, f"{failed} grid barrier wait(s) of a persistent launch timed out; "
                                             "its results are invalid")

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.ctx.lib.fm_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_from_poses(R: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Pack world-to-camera poses as the library's parameter rows
    (a1, a2, t) = (first column of R, second column of R, t), float32."""
    return torch.cat([R[:, :, 0], R[:, :, 1], t], dim=1).to(torch.float32).contiguous()


# ------------------------------------------------------------------ a1

def build_pair_grams(scene: Scene, weights: torch.Tensor | None = None, f64: bool = True, f32: bool = True):
    """W36 per pair (float64 and/or float32 copies); see include/fastmap_hip.h."""
    dev, P = scene.ctx.device, scene.num_pairs
    if weights is not None:
        _require(weights, torch.float32, (scene.num_matches,), "weights", dev)
    W64 = torch.empty((P, 36), dtype=torch.float64, device=dev) if f64 else None
    W32 = torch.empty((P, 36), dtype=torch.float32, device=dev) if f32 else None
    check(scene.ctx.handle, scene.ctx.lib.fm_build_pair_grams(scene.ctx.handle, scene.handle, _ptr(weights),
                                                              _ptr(W64), _ptr(W32), _stream()))
    return W64, W32


# ------------------------------------------------------------------ a2

def reweight(scene: Scene, params: torch.Tensor, delta: float, tau: float, residuals: bool = False):
    """IRLS weights (and residuals) at `params`; returns (weights, resid|None, kept[1] int64)."""
    dev = scene.ctx.device
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    w = torch.empty(scene.num_matches, dtype=torch.float32, device=dev)
    r = torch.empty(scene.num_matches, dtype=torch.float32, device=dev) if residuals else None
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_reweight(scene.ctx.handle, scene.handle, _ptr(params), float(delta),
                                                      float(tau), _ptr(w), _ptr(r), _ptr(kept), _stream()))
    return w, r, kept


def reweight_build(scene: Scene, params: torch.Tensor, delta: float, tau: float, f64: bool = True,
                   f32: bool = True, out: tuple | None = None):
    """Fused reweight + Gram build; returns (W64|None, W32|None, kept[1] int64)."""
    dev, P = scene.ctx.device, scene.num_pairs
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    if out is not None:
        W64, W32, kept = out
    else:
        W64 = torch.empty((P, 36), dtype=torch.float64, device=dev) if f64 else None
        W32 = torch.empty((P, 36), dtype=torch.float32, device=dev) if f32 else None
        kept = torch.empty(1, dtype=torch.int64, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_reweight_build(scene.ctx.handle, scene.handle, _ptr(params),
                                                            float(delta), float(tau), _ptr(W64), _ptr(W32),
                                                            _ptr(kept), _stream()))
    return W64, W32, kept


# ------------------------------------------------------------------ a3 + a4

def _wdtype(W36: torch.Tensor) -> int:
    if W36.dtype == torch.float64:
        return _lib.FM_F64
    if W36.dtype == torch.float32:
        return _lib.FM_F32
    raise TypeError("W36 must be float64 or float32")


def epipolar_loss_grad(scene: Scene, W36: torch.Tensor, params: torch.Tensor, inv_Z: float | None = None,
                       Z: torch.Tensor | None = None, want_loss: bool = True, want_grad: bool = True):
    """(loss[1] float64 | None, grad [N,9] float32 | None) at `params`."""
    dev = scene.ctx.device
    _require(W36, W36.dtype, (scene.num_pairs, 36), "W36", dev)
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    if Z is not None:
        _require(Z, torch.int64, (1,), "Z", dev)
    elif inv_Z is None:
        raise ValueError("give inv_Z or Z")
    loss = torch.empty(1, dtype=torch.float64, device=dev) if want_loss else None
    grad = torch.empty((scene.num_cams, 9), dtype=torch.float32, device=dev) if want_grad else None
    check(scene.ctx.handle, scene.ctx.lib.fm_epipolar_loss_grad(
        scene.ctx.handle, scene.handle, _ptr(W36), _wdtype(W36), _ptr(params),
        float(inv_Z if inv_Z is not None else 0.0), _ptr(Z), _ptr(loss), _ptr(grad), _stream()))
    return loss, grad


# ------------------------------------------------------------------ a5

def adam_step(ctx: Context, params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              step: int, lr: torch.Tensor, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12) -> None:
    """In-place Adam update of a flat float32 tensor; lr is a device tensor with
    one value or one value per element."""
    n = params.numel()
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        if t.dtype != torch.float32 or t.numel() != n or not t.is_contiguous() or t.device != ctx.device:
            raise ValueError(f"{name}: contiguous float32 with {n} elements on {ctx.device} required")
    if lr.dtype != torch.float32 or lr.numel() not in (1, n) or lr.device != ctx.device:
        raise ValueError("lr: float32 device tensor with 1 or n elements required")
    stride = 0 if lr.numel() == 1 else 1
    check(ctx.handle, ctx.lib.fm_adam_step(ctx.handle, n, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step),
                                           _ptr(lr), stride, beta1, beta2, eps, _stream()))


# ------------------------------------------------------------------ fused loop

def epipolar_solve(scene: Scene, W36: torch.Tensor, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                   K: int, lr_rot: float, lr_t: float, lr_final_frac: float, lr_step0: int, lr_total: int,
                   adam_step0: int = 0, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12,
                   inv_Z: float | None = None, Z: torch.Tensor | None = None,
                   loss_trace: torch.Tensor | None = None, blocks: int = 0) -> None:
    """K fused iterations (loss + adjoint + Adam) in one persistent kernel;
    params, m, v are updated in place; loss_trace [K] float64 optional."""
    dev = scene.ctx.device
    _require(W36, W36.dtype, (scene.num_pairs, 36), "W36", dev)
    for name, t in (("params", params), ("m", m), ("v", v)):
        _require(t, torch.float32, (scene.num_cams, 9), name, dev)
    if loss_trace is not None:
        _require(loss_trace, torch.float64, (K,), "loss_trace", dev)
    if Z is not None:
        _require(Z, torch.int64, (1,), "Z", dev)
    elif inv_Z is None:
        raise ValueError("give inv_Z or Z")
    cfg = _lib.AdamCfg(lr_rot, lr_t, lr_final_frac, beta1, beta2, eps, lr_step0, lr_total, adam_step0, blocks)
    check(scene.ctx.handle, scene.ctx.lib.fm_epipolar_solve(
        scene.ctx.handle, scene.handle, _ptr(W36), _wdtype(W36), _ptr(params), _ptr(m), _ptr(v), int(K),
        ctypes.byref(cfg), float(inv_Z if inv_Z is not None else 0.0), _ptr(Z), _ptr(loss_trace), _stream()))


# ------------------------------------------------------------------ focal refinement

def epipolar_focal_loss_grad(scene: Scene, W36: torch.Tensor, params: torch.Tensor, phi: torch.Tensor,
                             inv_Z: float | None = None, Z: torch.Tensor | None = None, want_loss: bool = True):
    """(loss [1] float64 | None, grad [N,9] float32, gphi [N] float32) of the
    epipolar loss with per-camera log focal scales phi (fundamental matrices)."""
    dev = scene.ctx.device
    _require(W36, W36.dtype, (scene.num_pairs, 36), "W36", dev)
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    _require(phi, torch.float32, (scene.num_cams,), "phi", dev)
    if Z is not None:
        _require(Z, torch.int64, (1,), "Z", dev)
    elif inv_Z is None:
        raise ValueError("give inv_Z or Z")
    loss = torch.empty(1, dtype=torch.float64, device=dev) if want_loss else None
    grad = torch.empty((scene.num_cams, 9), dtype=torch.float32, device=dev)
    gphi = torch.empty(scene.num_cams, dtype=torch.float32, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_epipolar_focal_loss_grad(
        scene.ctx.handle, scene.handle, _ptr(W36), _wdtype(W36), _ptr(params), _ptr(phi),
        float(inv_Z if inv_Z is not None else 0.0), _ptr(Z), _ptr(loss), _ptr(grad), _ptr(gphi), _stream()))
    return loss, grad, gphi


def epipolar_focal_solve(scene: Scene, W36: torch.Tensor, params: torch.Tensor, phi: torch.Tensor,
                         m: torch.Tensor, v: torch.Tensor, m_phi: torch.Tensor, v_phi: torch.Tensor, K: int,
                         lr_rot: float, lr_t: float, lr_phi: float, lr_final_frac: float, lr_step0: int = 0,
                         lr_total: int | None = None, adam_step0: int = 0, beta1: float = 0.9,
                         beta2: float = 0.999, eps: float = 1e-12, inv_Z: float | None = None,
                         Z: torch.Tensor | None = None, loss_trace: torch.Tensor | None = None) -> None:
    """K fused Adam steps on poses [N,9] and log focal scales [N] (one
    persistent kernel); params, phi and their moments are updated in place;
    loss_trace [K] float64 optional."""
    dev = scene.ctx.device
    _require(W36, W36.dtype, (scene.num_pairs, 36), "W36", dev)
    for name, t in (("params", params), ("m", m), ("v", v)):
        _require(t, torch.float32, (scene.num_cams, 9), name, dev)
    for name, t in (("phi", phi), ("m_phi", m_phi), ("v_phi", v_phi)):
        _require(t, torch.float32, (scene.num_cams,), name, dev)
    if loss_trace is not None:
        _require(loss_trace, torch.float64, (K,), "loss_trace", dev)
    if Z is not None:
        _require(Z, torch.int64, (1,), "Z", dev)
    elif inv_Z is None:
        raise ValueError("give inv_Z or Z")
    cfg = _lib.AdamCfg(lr_rot, lr_t, lr_final_frac, beta1, beta2, eps, lr_step0,
                       K if lr_total is None else lr_total, adam_step0, 0)
    check(scene.ctx.handle, scene.ctx.lib.fm_epipolar_focal_solve(
        scene.ctx.handle, scene.handle, _ptr(W36), _wdtype(W36), _ptr(params), _ptr(phi), _ptr(m), _ptr(v),
        _ptr(m_phi), _ptr(v_phi), int(K), ctypes.byref(cfg), float(lr_phi),
        float(inv_Z if inv_Z is not None else 0.0), _ptr(Z), _ptr(loss_trace), _stream()))


# ------------------------------------------------------------------ translation averaging

def _runs_of(scene: Scene, centres: torch.Tensor) -> int:
    if centres.ndim != 3 or centres.shape[1:] != (scene.num_cams, 3):
        raise ValueError(f"centres: expected [runs, {scene.num_cams}, 3], got {tuple(centres.shape)}")
    return int(centres.shape[0])


def translation_directions(scene: Scene, params: torch.Tensor, t_rel: torch.Tensor) -> torch.Tensor:
    """Targets -R_j^T t_rel per pair [P,3] float32 (R_j from params' 6D rotation)."""
    dev = scene.ctx.device
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    _require(t_rel, torch.float32, (scene.num_pairs, 3), "t_rel", dev)
    d = torch.empty((scene.num_pairs, 3), dtype=torch.float32, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_translation_directions(scene.ctx.handle, scene.handle, _ptr(params),
                                                                    _ptr(t_rel), _ptr(d), _stream()))
    return d


def translation_loss_grad(scene: Scene, dirs: torch.Tensor, centres: torch.Tensor, want_loss: bool = True,
                          want_grad: bool = True):
    """(loss [runs] float64 | None, grad [runs,N,3] float32 | None) of L_t."""
    dev = scene.ctx.device
    R = _runs_of(scene, centres)
    _require(dirs, torch.float32, (scene.num_pairs, 3), "dirs", dev)
    _require(centres, torch.float32, (R, scene.num_cams, 3), "centres", dev)
    loss = torch.empty(R, dtype=torch.float64, device=dev) if want_loss else None
    grad = torch.empty((R, scene.num_cams, 3), dtype=torch.float32, device=dev) if want_grad else None
    check(scene.ctx.handle, scene.ctx.lib.fm_translation_loss_grad(scene.ctx.handle, scene.handle, _ptr(dirs), R,
                                                                   _ptr(centres), _ptr(loss), _ptr(grad), _stream()))
    return loss, grad


def translation_solve(scene: Scene, dirs: torch.Tensor, centres: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                      K: int, lr: float, lr_final_frac: float, lr_step0: int = 0, lr_total: int | None = None,
                      adam_step0: int = 0, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12,
                      loss_trace: torch.Tensor | None = None, blocks: int = 0) -> None:
    """K fused Adam iterations on L_t for every run (one persistent kernel);
    centres, m, v [runs,N,3] are updated in place; loss_trace [runs,K] optional."""
    dev = scene.ctx.device
    R = _runs_of(scene, centres)
    _require(dirs, torch.float32, (scene.num_pairs, 3), "dirs", dev)
    for name, t in (("centres", centres), ("m", m), ("v", v)):
        _require(t, torch.float32, (R, scene.num_cams, 3), name, dev)
    if loss_trace is not None:
        _require(loss_trace, torch.float64, (R, K), "loss_trace", dev)
    cfg = _lib.AdamCfg(0.0, lr, lr_final_frac, beta1, beta2, eps, lr_step0, lr_total if lr_total else K,
                       adam_step0, blocks)
    check(scene.ctx.handle, scene.ctx.lib.fm_translation_solve(
        scene.ctx.handle, scene.handle, _ptr(dirs), R, _ptr(centres), _ptr(m), _ptr(v), int(K), ctypes.byref(cfg),
        _ptr(loss_trace), _stream()))


def translation_merge(scene: Scene, dirs: torch.Tensor, centres: torch.Tensor):
    """(merged [N,3] float32, choice [N] int32, cam_loss [runs,N] float64)."""
    dev = scene.ctx.device
    R = _runs_of(scene, centres)
    _require(dirs, torch.float32, (scene.num_pairs, 3), "dirs", dev)
    _require(centres, torch.float32, (R, scene.num_cams, 3), "centres", dev)
    merged = torch.empty((scene.num_cams, 3), dtype=torch.float32, device=dev)
    choice = torch.empty(scene.num_cams, dtype=torch.int32, device=dev)
    cam = torch.empty((R, scene.num_cams), dtype=torch.float64, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_translation_merge(scene.ctx.handle, scene.handle, _ptr(dirs), R,
                                                               _ptr(centres), _ptr(merged), _ptr(choice), _ptr(cam),
                                                               _stream()))
    return merged, choice, cam


def fibonacci_sphere(C: int, device) -> torch.Tensor:
    """C near-uniform unit vectors (golden-angle spiral) [C,3] float64 on
    `device`: the default candidate set of translation_search."""
    k = torch.arange(C, dtype=torch.float64, device=device)
    z = 1.0 - 2.0 * (k + 0.5) / C
    r = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], dim=1).contiguous()


def translation_search(scene: Scene, W36: torch.Tensor, params: torch.Tensor, cand: torch.Tensor,
                       t_prior: torch.Tensor):
    """(t [P,3] float32, best [P] int32, err_min [P] float64): the candidate
    with the lowest mean squared epipolar error per pair, signed like t_prior."""
    dev, P = scene.ctx.device, scene.num_pairs
    _require(W36, torch.float64, (P, 36), "W36", dev)
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    C = int(cand.shape[0])
    _require(cand, torch.float64, (C, 3), "cand", dev)
    _require(t_prior, torch.float32, (P, 3), "t_prior", dev)
    t = torch.empty((P, 3), dtype=torch.float32, device=dev)
    best = torch.empty(P, dtype=torch.int32, device=dev)
    err = torch.empty(P, dtype=torch.float64, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_translation_search(
        scene.ctx.handle, scene.handle, _ptr(W36), _ptr(params), _ptr(cand), C, _ptr(t_prior), _ptr(t), _ptr(best),
        _ptr(err), _stream()))
    return t, best, err


def pose_change(scene: Scene, params_a: torch.Tensor, params_b: torch.Tensor, rot_deg: float, t_deg: float,
                per_pair: bool = False):
    """Per-pair relative-pose change between two parameter sets (fm_pose_change):
    returns (counts [2] int64 device tensor: pairs over rot_deg, pairs over
    t_deg; rot [P] | None; t [P] | None), angles in degrees."""
    dev, P = scene.ctx.device, scene.num_pairs
    _require(params_a, torch.float32, (scene.num_cams, 9), "params_a", dev)
    _require(params_b, torch.float32, (scene.num_cams, 9), "params_b", dev)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    rot = torch.empty(P, dtype=torch.float32, device=dev) if per_pair else None
    tr = torch.empty(P, dtype=torch.float32, device=dev) if per_pair else None
    check(scene.ctx.handle, scene.ctx.lib.fm_pose_change(scene.ctx.handle, scene.handle, _ptr(params_a),
                                                         _ptr(params_b), float(rot_deg), float(t_deg), _ptr(rot),
                                                         _ptr(tr), _ptr(counts), _stream()))
    return counts, rot, tr


def poses_from_centres(ctx: Context, params6: torch.Tensor, centres: torch.Tensor) -> torch.Tensor:
    """(a1, a2, t = -R o) [N,9] float32 from rotation parameters [N,6] and
    camera centres [N,3]."""
    N = int(params6.shape[0])
    _require(params6, torch.float32, (N, 6), "params6", ctx.device)
    _require(centres, torch.float32, (N, 3), "centres", ctx.device)
    out = torch.empty((N, 9), dtype=torch.float32, device=ctx.device)
    check(ctx.handle, ctx.lib.fm_poses_from_centres(ctx.handle, N, _ptr(params6), _ptr(centres), _ptr(out),
                                                    _stream()))
    return out


# ------------------------------------------------------------------ rotation averaging

def rotation_loss_grad(scene: Scene, Rrel: torch.Tensor, params6: torch.Tensor, want_loss: bool = True,
                       want_grad: bool = True):
    """(loss [1] float64 | None, grad [N,6] float32 | None) of L_R."""
    dev = scene.ctx.device
    _require(Rrel, torch.float32, (scene.num_pairs, 9), "Rrel", dev)
    _require(params6, torch.float32, (scene.num_cams, 6), "params6", dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev) if want_loss else None
    grad = torch.empty((scene.num_cams, 6), dtype=torch.float32, device=dev) if want_grad else None
    check(scene.ctx.handle, scene.ctx.lib.fm_rotation_loss_grad(scene.ctx.handle, scene.handle, _ptr(Rrel),
                                                                _ptr(params6), _ptr(loss), _ptr(grad), _stream()))
    return loss, grad


def rotation_solve(scene: Scene, Rrel: torch.Tensor, params6: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                   K: int, lr: float, lr_final_frac: float, lr_step0: int = 0, lr_total: int | None = None,
                   adam_step0: int = 0, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12,
                   loss_trace: torch.Tensor | None = None, blocks: int = 0) -> None:
    """K fused Adam iterations on L_R (one persistent kernel); params6, m, v
    [N,6] are updated in place; loss_trace [K] float64 optional."""
    dev = scene.ctx.device
    _require(Rrel, torch.float32, (scene.num_pairs, 9), "Rrel", dev)
    for name, t in (("params6", params6), ("m", m), ("v", v)):
        _require(t, torch.float32, (scene.num_cams, 6), name, dev)
    if loss_trace is not None:
        _require(loss_trace, torch.float64, (K,), "loss_trace", dev)
    cfg = _lib.AdamCfg(lr, 0.0, lr_final_frac, beta1, beta2, eps, lr_step0, lr_total if lr_total else K,
                       adam_step0, blocks)
    check(scene.ctx.handle, scene.ctx.lib.fm_rotation_solve(
        scene.ctx.handle, scene.handle, _ptr(Rrel), _ptr(params6), _ptr(m), _ptr(v), int(K), ctypes.byref(cfg),
        _ptr(loss_trace), _stream()))


def rotation_init(scene: Scene, Rrel: torch.Tensor, start: torch.Tensor, steps: int = 300, blocks: int = 0):
    """(params [N,6] float32, info [4] float64) from the column-wise
    least-squares initialisation; start [2, 3N] float64 random vectors."""
    dev = scene.ctx.device
    _require(Rrel, torch.float32, (scene.num_pairs, 9), "Rrel", dev)
    _require(start, torch.float64, (2, 3 * scene.num_cams), "start", dev)
    params = torch.empty((scene.num_cams, 6), dtype=torch.float32, device=dev)
    info = torch.zeros(4, dtype=torch.float64, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_rotation_init(scene.ctx.handle, scene.handle, _ptr(Rrel), _ptr(start),
                                                           int(steps), int(blocks), _ptr(params), _ptr(info),
                                                           _stream()))
    return params, info


# ------------------------------------------------------------------ a9: learned weights

MLP_SHAPES = {"W1": (64, 3), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}


class MlpWeights:
    """The MLP's float32 weights as views into one flat device tensor (so one
    fm_adam_step updates them all), plus the feature standardisation."""

    def __init__(self, device, flat: torch.Tensor | None = None, mean=None, std=None):
        n = sum(int(np.prod(s)) for s in MLP_SHAPES.values())
        self.flat = torch.zeros(n, dtype=torch.float32, device=device) if flat is None else flat
        assert self.flat.numel() == n and self.flat.dtype == torch.float32
        self.views = {}
        o = 0
        for k, s in MLP_SHAPES.items():
            c = int(np.prod(s))
            self.views[k] = self.flat[o:o + c].view(*s)
            o += c
        self.mean = torch.zeros(3, dtype=torch.float32, device=device) if mean is None else mean
        self.std = torch.ones(3, dtype=torch.float32, device=device) if std is None else std

    def struct(self):
        v = self.views
        return _lib.Mlp(*(_ptr(v[k]) for k in MLP_SHAPES), _ptr(self.mean), _ptr(self.std))

    def grad_struct(self, g: "MlpWeights"):
        return _lib.MlpGrad(*(_ptr(g.views[k]) for k in MLP_SHAPES))

    def load_numpy(self, params: dict, mean, std) -> None:
        for k in MLP_SHAPES:
            self.views[k].copy_(torch.as_tensor(np.asarray(params[k], dtype=np.float32)))
        self.mean.copy_(torch.as_tensor(np.asarray(mean, dtype=np.float32)))
        self.std.copy_(torch.as_tensor(np.asarray(std, dtype=np.float32)))

    def to_numpy(self) -> dict:
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self.views.items()}


def match_features(scene: Scene, params: torch.Tensor, delta: float) -> torch.Tensor:
    """[M,3] float32 features (log max(|r|, delta), log |Q_n|, parallax)."""
    dev = scene.ctx.device
    _require(params, torch.float32, (scene.num_cams, 9), "params", dev)
    f = torch.empty((scene.num_matches, 3), dtype=torch.float32, device=dev)
    check(scene.ctx.handle, scene.ctx.lib.fm_match_features(scene.ctx.handle, scene.handle, _ptr(params),
                                                            float(delta), _ptr(f), _stream()))
    return f


def mlp_forward(ctx: Context, w: MlpWeights, feats: torch.Tensor, out_scale: float = 1.0,
                keep_act: bool = False):
    """(out [M] float32, act [M,128] float16 | None)."""
    M = int(feats.shape[0])
    _require(feats, torch.float32, (M, 3), "feats", ctx.device)
    out = torch.empty(M, dtype=torch.float32, device=ctx.device)
    act = torch.empty((M, 128), dtype=torch.float16, device=ctx.device) if keep_act else None
    st = w.struct()
    check(ctx.handle, ctx.lib.fm_mlp_forward(ctx.handle, M, _ptr(feats), ctypes.byref(st), float(out_scale),
                                             _ptr(out), _ptr(act), _stream()))
    return out, act


def mlp_backward(ctx: Context, w: MlpWeights, feats: torch.Tensor, act: torch.Tensor, dout: torch.Tensor,
                 grad: MlpWeights | None = None) -> MlpWeights:
    """Gradients of sum(dout * out) into `grad` (allocated if None)."""
    M = int(feats.shape[0])
    _require(feats, torch.float32, (M, 3), "feats", ctx.device)
    _require(act, torch.float16, (M, 128), "act", ctx.device)
    _require(dout, torch.float32, (M,), "dout", ctx.device)
    g = grad if grad is not None else MlpWeights(ctx.device)
    st, gs = w.struct(), w.grad_struct(g)
    check(ctx.handle, ctx.lib.fm_mlp_backward(ctx.handle, M, _ptr(feats), ctypes.byref(st), _ptr(act),
                                              _ptr(dout), ctypes.byref(gs), _stream()))
    return g
