"""Seeded synthetic scenes for epipolar adjustment.

This module only *makes inputs*: camera poses, 3D points, their projections
with pixel noise and outliers, the image-pair list and the per-pair match
lists (CSR, sorted by pair).  It holds none of the method's arithmetic (no
essential matrices, Grams, losses or parameterisation), so the FP64 oracle and
the HIP path can both consume its output without sharing compute code.

Conventions (the paper's problem statement, Sec. 3.3 "Epipolar Adjustment"):
  * world-to-camera poses: X_cam = R_i X + t_i, camera centre o_i = -R_i^T t_i;
  * pinhole camera, focal 500 px, 640x480 image, principal point at the image
    centre (Sec. 3.1 "Camera Assumptions"), so normalised coordinates are
    u = (px - 320) / 500, v = (py - 240) / 500;
  * image pair n = (i_n, j_n) with i_n < j_n; x1 lies in image i_n, x2 in j_n;
  * matches are stored as one [M, 4] array (u1, v1, u2, v2) sorted by pair,
    with int64 offsets [P + 1].

Scene recipes (sizes follow the five workloads the hot path is measured on):
  tiny     20 cameras on a sphere, 2,000 points, FP64, sigma 0.5 px, 10 % outliers
  medium   200 cameras on a 3-turn helix, 165k points, log-normal tracks (mean 6),
           ~4.8k pairs / ~3M matches, FP32, sigma 1 px, 20 % outliers
  diffprec 1,000 nadir cameras on a 20x50 serpentine grid over a relief plane,
           power-law pair sizes on [20, 20k], BF16, sigma 1 px, 25 % outliers
  learned  as medium with 300 cameras (~5M matches)
  large    5,000 street cameras in a city-block grid, facade points,
           ~250k pairs / ~200M matches, BF16, sigma 1.5 px, 30 % outliers
Every scene is reproducible from (recipe, seed); the pose initialisation uses
seed + 10,000.  Epipolar adjustment refines poses that earlier stages
(rotation and translation averaging) already estimated, so the initial poses
are the true ones perturbed: tiny uses 5 deg rotation noise and 0.1 centre
noise (radius-5 rig); the other recipes use 1 deg and a centre noise of a few
percent of the camera spacing.  `init_trans="random"` gives N(0, I) centres.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FOCAL = 500.0
WIDTH = 640.0
HEIGHT = 480.0
CX = WIDTH / 2.0
CY = HEIGHT / 2.0


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    R_gt: np.ndarray        # [N,3,3] float64 world-to-camera rotations
    t_gt: np.ndarray        # [N,3]   float64 world-to-camera translations
    R_init: np.ndarray      # [N,3,3] initial rotations
    t_init: np.ndarray      # [N,3]   initial translations
    pairs: np.ndarray       # [P,2] int32, i < j
    offsets: np.ndarray     # [P+1] int64 CSR offsets into the match arrays
    uv: np.ndarray          # [M,4] float64 normalised (u1, v1, u2, v2)
    outlier: np.ndarray     # [M] bool, True where x2 was replaced by a random pixel
    storage: str            # "f64" | "f32" | "bf16": dtype the workload stores coords in
    sigma_px: float
    outlier_frac: float

    @property
    def num_cams(self) -> int:
        return int(self.R_gt.shape[0])

    @property
    def num_pairs(self) -> int:
        return int(self.pairs.shape[0])

    @property
    def num_matches(self) -> int:
        return int(self.uv.shape[0])

    def pair_sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def stats(self) -> dict:
        sz = self.pair_sizes()
        return {
            "name": self.name, "seed": self.seed, "cams": self.num_cams,
            "pairs": self.num_pairs, "matches": self.num_matches,
            "pair_size_mean": float(sz.mean()) if sz.size else 0.0,
            "pair_size_p50": float(np.percentile(sz, 50)) if sz.size else 0.0,
            "pair_size_p99": float(np.percentile(sz, 99)) if sz.size else 0.0,
            "pair_size_max": int(sz.max()) if sz.size else 0,
            "storage": self.storage,
        }


# ---------------------------------------------------------------- helpers

def _normalize(v, axis=-1):
    return v / np.linalg.norm(v, axis=axis, keepdims=True)


def _look_at(centres: np.ndarray, targets: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera rotations whose optical (z) axis points at `targets`.

    Rows of R are the camera axes (x right, y down, z forward) in world frame.
    """
    z = _normalize(targets - centres)
    up = np.broadcast_to(np.asarray(up, dtype=np.float64), z.shape)
    x = np.cross(z, up)
    bad = np.linalg.norm(x, axis=-1) < 1e-6
    if np.any(bad):
        x[bad] = np.cross(z[bad], np.array([0.0, 1.0, 0.0]))
    x = _normalize(x)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=-2)


def _axis_angle(axis: np.ndarray, angle: np.ndarray) -> np.ndarray:
    """Rodrigues' formula, batched: rotation by `angle` about unit `axis`."""
    axis = _normalize(axis)
    k = np.zeros(axis.shape[:-1] + (3, 3))
    k[..., 0, 1], k[..., 0, 2] = -axis[..., 2], axis[..., 1]
    k[..., 1, 0], k[..., 1, 2] = axis[..., 2], -axis[..., 0]
    k[..., 2, 0], k[..., 2, 1] = -axis[..., 1], axis[..., 0]
    a = np.asarray(angle)[..., None, None]
    eye = np.eye(3)
    return eye + np.sin(a) * k + (1.0 - np.cos(a)) * (k @ k)


def _jitter(R: np.ndarray, rng, max_deg: float) -> np.ndarray:
    """Yaw/pitch jitter U(+-max_deg) applied in the camera frame."""
    n = R.shape[0]
    yaw = np.deg2rad(rng.uniform(-max_deg, max_deg, n))
    pitch = np.deg2rad(rng.uniform(-max_deg, max_deg, n))
    Ry = _axis_angle(np.tile([0.0, 1.0, 0.0], (n, 1)), yaw)
    Rx = _axis_angle(np.tile([1.0, 0.0, 0.0], (n, 1)), pitch)
    return Rx @ Ry @ R


def _project_px(R, t, X):
    """Pixel coordinates and depth of world points X [K,3] in cameras (R,t) [K,...]."""
    Xc = np.einsum("kab,kb->ka", R, X) + t
    z = Xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        px = FOCAL * Xc[:, 0] / z + CX
        py = FOCAL * Xc[:, 1] / z + CY
    return px, py, z


def _in_frame(px, py, z):
    return (z > 1e-6) & (px >= 0) & (px < WIDTH) & (py >= 0) & (py < HEIGHT)


def _to_normalised(px, py):
    return (px - CX) / FOCAL, (py - CY) / FOCAL


def _init_poses(R_gt, t_gt, seed, rot_deg=5.0, trans="perturbed", centre_sigma=0.1):
    """Initial poses: rotation = Exp(rot_deg * k) R_gt with k uniform on S^2.
    Translation: "perturbed" = true camera centres plus N(0, centre_sigma^2 I)
    per axis; "random" = camera centres ~ N(0, I); "gt" = true centres."""
    rng = np.random.default_rng(seed + 10_000)
    n = R_gt.shape[0]
    axis = _normalize(rng.normal(size=(n, 3)))
    R_init = _axis_angle(axis, np.full(n, np.deg2rad(rot_deg))) @ R_gt
    o_gt = -np.einsum("nba,nb->na", R_gt, t_gt)
    if trans == "random":
        o = rng.normal(size=(n, 3))
    elif trans == "perturbed":
        o = o_gt + rng.normal(0.0, centre_sigma, size=(n, 3))
    else:
        o = o_gt
    t_init = -np.einsum("nab,nb->na", R_init, o)
    return R_init, t_init


def _assemble(name, seed, R_gt, t_gt, cam_a, cam_b, uv, outl, min_matches, storage,
              sigma, frac, init_kw):
    init_kw = {k: v for k, v in init_kw.items() if v is not None}
    init_kw.setdefault("centre_sigma", 0.1)
    """Sort matches by pair, drop pairs with fewer than `min_matches`, build CSR."""
    n = R_gt.shape[0]
    key = cam_a.astype(np.int64) * n + cam_b.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key, uv, outl = key[order], uv[order], outl[order]
    uniq, start, counts = np.unique(key, return_index=True, return_counts=True)
    keep = counts >= min_matches
    sel = np.repeat(keep, counts)
    uv, outl = uv[sel], outl[sel]
    uniq, counts = uniq[keep], counts[keep]
    pairs = np.stack([uniq // n, uniq % n], axis=1).astype(np.int32)
    offsets = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    R_init, t_init = _init_poses(R_gt, t_gt, seed, **init_kw)
    return Scene(name, seed, R_gt, t_gt, R_init, t_init, pairs, offsets,
                 np.ascontiguousarray(uv), outl, storage, sigma, frac)


def _observe(rng, R, t, X, sigma):
    px, py, z = _project_px(R, t, X)
    ok = _in_frame(px, py, z)
    px = px + rng.normal(0.0, sigma, px.shape)
    py = py + rng.normal(0.0, sigma, py.shape)
    return px, py, ok


def _make_matches(rng, R_gt, t_gt, cam_a, cam_b, X, sigma, frac, obs_a=None, obs_b=None):
    """Matches for co-visible points X seen by cameras cam_a (first) and cam_b.

    A fraction `frac` of matches become outliers: the second image's pixel is
    replaced by a uniform random pixel.  Returns uv [K,4] float64 and the mask.
    """
    k = X.shape[0]
    if obs_a is None:
        pa, qa, _ = _observe(rng, R_gt[cam_a], t_gt[cam_a], X, sigma)
    else:
        pa, qa = obs_a
    if obs_b is None:
        pb, qb, _ = _observe(rng, R_gt[cam_b], t_gt[cam_b], X, sigma)
    else:
        pb, qb = obs_b
    outl = rng.random(k) < frac
    no = int(outl.sum())
    pb = pb.copy(); qb = qb.copy()
    pb[outl] = rng.uniform(0.0, WIDTH, no)
    qb[outl] = rng.uniform(0.0, HEIGHT, no)
    u1, v1 = _to_normalised(pa, qa)
    u2, v2 = _to_normalised(pb, qb)
    return np.stack([u1, v1, u2, v2], axis=1), outl


# ---------------------------------------------------------------- recipes

def tiny(seed: int = 0, n_cams: int = 20, n_points: int = 2000, sigma: float = 0.5,
         frac: float = 0.10, min_matches: int = 30, init_trans: str = "perturbed",
         init_sigma: float | None = None) -> Scene:
    """20 cameras uniform on a sphere of radius 5 looking at the origin with
    +-10 deg yaw/pitch jitter; 2,000 points in the unit cube, each with a random
    normal (visible from the front half-space only)."""
    rng = np.random.default_rng(seed)
    c = 5.0 * _normalize(rng.normal(size=(n_cams, 3)))
    R = _jitter(_look_at(c, np.zeros_like(c)), rng, 10.0)
    t = -np.einsum("nab,nb->na", R, c)
    X = rng.uniform(-0.5, 0.5, size=(n_points, 3))
    nrm = _normalize(rng.normal(size=(n_points, 3)))
    vis = np.zeros((n_cams, n_points), dtype=bool)
    for i in range(n_cams):
        px, py, z = _project_px(np.broadcast_to(R[i], (n_points, 3, 3)), t[i], X)
        vis[i] = _in_frame(px, py, z) & (np.einsum("kd,kd->k", nrm, c[i] - X) > 0)
    ca, cb, pts = [], [], []
    for i in range(n_cams):
        for j in range(i + 1, n_cams):
            idx = np.nonzero(vis[i] & vis[j])[0]
            if idx.size >= min_matches:
                ca.append(np.full(idx.size, i)); cb.append(np.full(idx.size, j)); pts.append(idx)
    ca = np.concatenate(ca); cb = np.concatenate(cb); pts = np.concatenate(pts)
    uv, outl = _make_matches(rng, R, t, ca, cb, X[pts], sigma, frac)
    return _assemble("tiny", seed, R, t, ca, cb, uv, outl, min_matches, "f64", sigma, frac,
                     {"trans": init_trans, "centre_sigma": init_sigma})


def _helix_scene(name, seed, n_cams, n_points, sigma, frac, storage, min_matches=30, extent=1.0,
                 track_mean=6.0, track_sigma=0.4, init_trans="perturbed", init_sigma=0.02,
                 init_rot_deg=1.0):
    rng = np.random.default_rng(seed)
    phi = 2.0 * math.pi * 3.0 * np.arange(n_cams) / n_cams
    z = np.linspace(-2.0, 2.0, n_cams)
    c = np.stack([5.0 * np.cos(phi), 5.0 * np.sin(phi), z], axis=1)
    R = _jitter(_look_at(c, np.zeros_like(c)), rng, 3.0)
    t = -np.einsum("nab,nb->na", R, c)
    X = rng.uniform(-extent, extent, size=(n_points, 3))
    nrm = _normalize(rng.normal(size=(n_points, 3)))
    # visibility [n_points, n_cams]
    vis = np.zeros((n_points, n_cams), dtype=bool)
    pix = np.zeros((n_points, n_cams, 2))
    for i in range(n_cams):
        px, py, zz = _project_px(np.broadcast_to(R[i], (n_points, 3, 3)), t[i], X)
        vis[:, i] = _in_frame(px, py, zz) & (np.einsum("kd,kd->k", nrm, c[i] - X) > 0)
        pix[:, i, 0] = px + rng.normal(0.0, sigma, n_points)
        pix[:, i, 1] = py + rng.normal(0.0, sigma, n_points)
    mu = math.log(track_mean) - 0.5 * track_sigma ** 2
    L = np.round(rng.lognormal(mu, track_sigma, n_points)).astype(np.int64)
    nvis = vis.sum(axis=1)
    L = np.minimum(np.maximum(L, 2), nvis)
    start_u = rng.random(n_points)
    # tracks: contiguous runs of visible cameras (in trajectory order); all
    # pairwise matches of a track (track completion)
    ca, cb, pa, pb = [], [], [], []
    tri_cache = {}
    for p in range(n_points):
        l = int(L[p])
        if l < 2:
            continue
        cams = np.nonzero(vis[p])[0]
        s = int(start_u[p] * (cams.size - l + 1))
        run = cams[s:s + l]
        if l not in tri_cache:
            tri_cache[l] = np.triu_indices(l, 1)
        a, b = tri_cache[l]
        ca.append(run[a]); cb.append(run[b]); pa.append(np.full(a.size, p))
    ca = np.concatenate(ca); cb = np.concatenate(cb); pts = np.concatenate(pa)
    obs_a = (pix[pts, ca, 0], pix[pts, ca, 1])
    obs_b = (pix[pts, cb, 0], pix[pts, cb, 1])
    uv, outl = _make_matches(rng, R, t, ca, cb, X[pts], sigma, frac, obs_a, obs_b)
    return _assemble(name, seed, R, t, ca, cb, uv, outl, min_matches, storage, sigma, frac,
                     {"trans": init_trans, "centre_sigma": init_sigma, "rot_deg": init_rot_deg})


def medium(seed: int = 1, n_cams: int = 200, n_points: int = 165_000, sigma: float = 1.0,
           frac: float = 0.20, init_trans: str = "perturbed",
           init_sigma: float = 0.02, init_rot_deg: float = 1.0) -> Scene:
    """200 cameras on a 3-loop helix (radius 5, z in [-2, 2]) aimed at the
    origin; points in [-1, 1]^3 with random normals; each point's track is a
    contiguous run (log-normal length, mean 6, log-sd 0.4) of the cameras that
    see it.  165k points give ~4.8k pairs and ~3M matches (the workload's
    "~4k pairs, ~3M matches"; a 50k-point cloud with mean-6 tracks yields only
    ~0.9M matches once pairs below 30 matches are dropped)."""
    return _helix_scene("medium", seed, n_cams, n_points, sigma, frac, "f32",
                        init_trans=init_trans, init_sigma=init_sigma, init_rot_deg=init_rot_deg)


def learned(seed: int = 100, n_cams: int = 300, n_points: int = 280_000, sigma: float = 1.0,
            frac: float = 0.20, init_trans: str = "perturbed",
            init_sigma: float = 0.02, init_rot_deg: float = 1.0) -> Scene:
    """The medium recipe with 300 cameras (~5M matches); seeds 100-163 train,
    200-215 are held out."""
    return _helix_scene("learned", seed, n_cams, n_points, sigma, frac, "f32",
                        init_trans=init_trans, init_sigma=init_sigma, init_rot_deg=init_rot_deg)


def _powerlaw_sizes(rng, n, lo, hi, alpha):
    """Sizes k on [lo, hi] with density proportional to k^-alpha (inverse CDF)."""
    a1 = 1.0 - alpha
    u = rng.random(n)
    k = (lo ** a1 + u * (hi ** a1 - lo ** a1)) ** (1.0 / a1)
    return np.floor(k).astype(np.int64)


def _relief(x, y):
    return 0.08 * np.sin(0.9 * x) * np.cos(0.7 * y) + 0.05 * np.sin(2.3 * x + 1.1 * y)


def diffprec(seed: int = 2, nx: int = 20, ny: int = 50, height: float = 1.0,
             spacing: float = 0.17, sigma: float = 1.0, frac: float = 0.25,
             alpha: float = 1.45, size_lo: int = 20, size_hi: int = 20_000,
             max_pairs: int | None = None, init_trans: str = "perturbed",
             init_sigma: float = 0.01, init_rot_deg: float = 1.0) -> Scene:
    """1,000 nadir cameras on a 20x50 serpentine grid at height 1 over a relief
    ground plane; every pair of cameras whose footprints overlap gets a
    power-law number of matches (density k^-1.45 on [20, 20k]) sampled from
    ground points in the overlap."""
    rng = np.random.default_rng(seed)
    gx, gy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    gx = np.where(gy % 2 == 0, gx, nx - 1 - gx)            # serpentine order
    xs = gx.reshape(-1) * spacing
    ys = gy.reshape(-1) * spacing
    n = xs.size
    c = np.stack([xs, ys, np.full(n, height)], axis=1)
    c[:, :2] += rng.normal(0.0, 0.01, (n, 2))
    c[:, 2] += rng.normal(0.0, 0.02, n)
    # nadir: z axis down; heading alternates with the serpentine rows
    heading = np.where(gy.reshape(-1) % 2 == 0, 0.0, math.pi)
    R = np.zeros((n, 3, 3))
    ch, sh = np.cos(heading), np.sin(heading)
    R[:, 0] = np.stack([ch, sh, np.zeros(n)], axis=1)           # x_cam
    R[:, 2] = np.tile([0.0, 0.0, -1.0], (n, 1))                  # z_cam (down)
    R[:, 1] = np.cross(R[:, 2], R[:, 0])                         # y_cam
    R = _jitter(R, rng, 3.0)
    t = -np.einsum("nab,nb->na", R, c)
    # candidate pairs: footprint centres close enough to overlap
    half_w = height * (WIDTH / 2) / FOCAL
    half_h = height * (HEIGHT / 2) / FOCAL
    ii, jj = np.triu_indices(n, 1)
    dx = np.abs(xs[ii] - xs[jj]); dy = np.abs(ys[ii] - ys[jj])
    reach = 2 * min(half_w, half_h) * 0.85
    cand = (dx < reach) & (dy < reach)
    ii, jj = ii[cand], jj[cand]
    if max_pairs is not None and ii.size > max_pairs:
        sel = np.sort(rng.choice(ii.size, max_pairs, replace=False))
        ii, jj = ii[sel], jj[sel]
    k = _powerlaw_sizes(rng, ii.size, size_lo, size_hi, alpha)
    ca = np.repeat(ii, k); cb = np.repeat(jj, k)
    # sample ground points in the overlap of the two footprints (square window
    # around the midpoint), retry points that fall outside either image
    X = np.zeros((ca.size, 3))
    todo = np.arange(ca.size)
    for _ in range(40):
        if todo.size == 0:
            break
        a, b = ca[todo], cb[todo]
        mx = 0.5 * (c[a, 0] + c[b, 0]); my = 0.5 * (c[a, 1] + c[b, 1])
        wx = np.maximum(reach - np.abs(c[a, 0] - c[b, 0]), 0.05) * 0.5
        wy = np.maximum(reach - np.abs(c[a, 1] - c[b, 1]), 0.05) * 0.5
        x = mx + rng.uniform(-1, 1, todo.size) * wx
        y = my + rng.uniform(-1, 1, todo.size) * wy
        P = np.stack([x, y, _relief(x, y)], axis=1)
        pa, qa, za = _project_px(R[a], t[a], P)
        pb, qb, zb = _project_px(R[b], t[b], P)
        ok = _in_frame(pa, qa, za) & _in_frame(pb, qb, zb)
        X[todo[ok]] = P[ok]
        todo = todo[~ok]
    keep = np.ones(ca.size, dtype=bool)
    keep[todo] = False
    ca, cb, X = ca[keep], cb[keep], X[keep]
    uv, outl = _make_matches(rng, R, t, ca, cb, X, sigma, frac)
    return _assemble("diffprec", seed, R, t, ca, cb, uv, outl, 20, "bf16", sigma, frac,
                     {"trans": init_trans, "centre_sigma": init_sigma, "rot_deg": init_rot_deg})


def _street_matches(args):
    """Facade matches for a block of pairs of the street scene (worker)."""
    (seed, chunk, ii, jj, k, R, t, c, horiz, line, street, heading, sigma, frac) = args
    rng = np.random.default_rng([seed, 1, chunk])
    ca = np.repeat(ii, k); cb = np.repeat(jj, k)
    X = np.zeros((ca.size, 3))
    todo = np.arange(ca.size)
    for _ in range(40):
        if todo.size == 0:
            break
        a, b = ca[todo], cb[todo]
        # a random facade point ahead of the leading camera of the pair, on
        # one of the two building faces lining the street
        hz = horiz[a]
        al_a = np.where(hz, c[a, 0], c[a, 1])
        al_b = np.where(hz, c[b, 0], c[b, 1])
        sg = heading[a]
        front = np.where(sg > 0, np.maximum(al_a, al_b), np.minimum(al_a, al_b))
        along_p = front + sg * rng.uniform(1.0, 40.0, todo.size)
        side = line[a] + np.where(rng.random(todo.size) < 0.5, 0.5, -0.5) * street
        hgt = rng.uniform(0.0, 8.0, todo.size)
        P = np.stack([np.where(hz, along_p, side), np.where(hz, side, along_p), hgt], axis=1)
        pa_, qa_, za = _project_px(R[a], t[a], P)
        pb_, qb_, zb = _project_px(R[b], t[b], P)
        ok = _in_frame(pa_, qa_, za) & _in_frame(pb_, qb_, zb)
        X[todo[ok]] = P[ok]
        todo = todo[~ok]
    keep = np.ones(ca.size, dtype=bool)
    keep[todo] = False
    ca, cb, X = ca[keep], cb[keep], X[keep]
    uv, outl = _make_matches(rng, R, t, ca, cb, X, sigma, frac)
    counts = np.bincount(np.repeat(np.arange(ii.size), k)[keep], minlength=ii.size)
    return uv.astype(np.float32), outl, counts


def large(seed: int = 3, blocks: int = 12, block: float = 10.0, street: float = 2.0,
          n_cams: int = 5000, pairs_per_cam: int = 100, mean_matches: float = 800.0,
          sigma: float = 1.5, frac: float = 0.30, init_trans: str = "perturbed",
          init_sigma: float = 0.03, init_rot_deg: float = 1.0, scale: float = 1.0,
          workers: int = 1, pairs_per_chunk: int = 2000) -> Scene:
    """5,000 street-level cameras in a blocks x blocks city grid, all cameras
    of a street heading the same way along it, with +-15 deg yaw jitter; matches are facade points (the two
    building faces lining the street) seen by two cameras on the same street.
    Each camera is paired with up to ~100 neighbours along its street, pair
    sizes follow a power law with mean ~800 matches (~250k pairs, ~200M
    matches).  Matches are generated per block of pairs with a generator
    seeded by (seed, block), so `workers` processes give the same scene; the
    coordinates are kept as float32 (the workload stores them as bf16).
    `scale` < 1 shrinks the camera count (and so pairs and matches)."""
    rng = np.random.default_rng(seed)
    n_cams = max(8, int(n_cams * scale))
    pitch = block + street
    extent = blocks * pitch
    n_streets = 2 * (blocks + 1)
    # each camera: a street (horizontal or vertical), position along it, heading sign
    st = rng.integers(0, n_streets, n_cams)
    horiz = st < (blocks + 1)
    line = (st % (blocks + 1)) * pitch + street / 2          # street centre coordinate
    along = rng.uniform(0, extent, n_cams)
    lateral = rng.uniform(-0.3, 0.3, n_cams) * street
    order = np.lexsort((along, st))
    st, horiz, line, along, lateral = st[order], horiz[order], line[order], along[order], lateral[order]
    street_sign = np.where(rng.random(n_streets) < 0.5, 1.0, -1.0)   # one heading per street
    sign = street_sign[st]
    cx = np.where(horiz, along, line + lateral)
    cy = np.where(horiz, line + lateral, along)
    cz = np.full(n_cams, 1.6) + rng.normal(0, 0.05, n_cams)
    c = np.stack([cx, cy, cz], axis=1)
    fwd = np.where(horiz[:, None], np.stack([sign, 0 * sign, 0 * sign], 1),
                   np.stack([0 * sign, sign, 0 * sign], 1))
    R = _jitter(_look_at(c, c + fwd), rng, 15.0)
    t = -np.einsum("nab,nb->na", R, c)
    # neighbours along the same street (cameras are sorted by street, position)
    half = pairs_per_cam // 2
    ii, jj = [], []
    bounds = np.searchsorted(st, np.arange(n_streets + 1))
    for s_ in range(n_streets):
        lo, hi = bounds[s_], bounds[s_ + 1]
        m = hi - lo
        if m < 2:
            continue
        for d in range(1, min(half, m - 1) + 1):
            a_ = np.arange(lo, hi - d)
            ii.append(a_); jj.append(a_ + d)
    ii = np.concatenate(ii); jj = np.concatenate(jj)
    o = np.lexsort((jj, ii))
    ii, jj = ii[o], jj[o]
    k = _powerlaw_sizes(rng, ii.size, 20, 20_000, 1.45)
    k = np.maximum(20, np.round(k * (mean_matches / max(k.mean(), 1.0)))).astype(np.int64)
    k = np.minimum(k, 20_000)
    jobs = []
    for ch, lo in enumerate(range(0, ii.size, pairs_per_chunk)):
        sl = slice(lo, lo + pairs_per_chunk)
        jobs.append((seed, ch, ii[sl], jj[sl], k[sl], R, t, c, horiz, line, street, sign, sigma, frac))
    if workers > 1:
        import concurrent.futures
        import multiprocessing
        with concurrent.futures.ProcessPoolExecutor(
                max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
            parts = list(ex.map(_street_matches, jobs))
    else:
        parts = [_street_matches(j) for j in jobs]
    counts = np.concatenate([p[2] for p in parts])
    uv = np.concatenate([p[0] for p in parts])
    outl = np.concatenate([p[1] for p in parts])
    del parts
    keep_pair = counts >= 30
    if not np.all(keep_pair):
        sel = np.repeat(keep_pair, counts)
        uv, outl = uv[sel], outl[sel]
        ii, jj, counts = ii[keep_pair], jj[keep_pair], counts[keep_pair]
    offsets = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    R_init, t_init = _init_poses(R, t, seed, rot_deg=init_rot_deg, trans=init_trans,
                                 centre_sigma=init_sigma)
    return Scene("large", seed, R, t, R_init, t_init, np.stack([ii, jj], 1).astype(np.int32), offsets,
                 uv, outl, "bf16", sigma, frac)


RECIPES = {"tiny": tiny, "medium": medium, "diffprec": diffprec, "learned": learned,
           "large": large}


def make(name: str, **kw) -> Scene:
    return RECIPES[name](**kw)


def noise_free(scene_fn, **kw) -> Scene:
    """The same recipe with zero pixel noise and no outliers."""
    return scene_fn(sigma=0.0, frac=0.0, **kw)


# ------------------------------------------------------------------ translation averaging inputs

@dataclasses.dataclass
class TranslationInputs:
    t_rel: np.ndarray       # [P,3] float64 unit relative translations t^{i->j} (camera j's frame)
    outlier: np.ndarray     # [P] bool, True where t_rel is a random direction
    init: np.ndarray        # [runs,N,3] float64 initial camera centres, N(0, I) per run
    sigma_deg: float
    outlier_frac: float


def translation_inputs(scene: Scene, sigma_deg: float = 2.0, outlier_frac: float = 0.1,
                       runs: int = 4, seed: int | None = None) -> TranslationInputs:
    """Inputs of translation averaging on a scene's pair graph (Sec. 3.3,
    Global Translation): per pair the measured unit direction of camera i's
    centre seen from camera j, t^{i->j} ~ R_j (o_i - o_j) / |o_i - o_j|, with
    Gaussian noise of sigma_deg per axis (radians after conversion) before
    renormalising, and outlier_frac of the pairs replaced by directions
    uniform on the sphere; plus `runs` independent N(0, I) initialisations of
    the N camera centres.  The stage follows rotation averaging, so the
    rotations it uses are the scene's true ones."""
    rng = np.random.default_rng((scene.seed if seed is None else seed) + 20_000)
    R, t = scene.R_gt, scene.t_gt
    o = -np.einsum("nba,nb->na", R, t)
    i, j = scene.pairs[:, 0], scene.pairs[:, 1]
    P = len(scene.pairs)
    tr = _normalize(np.einsum("pab,pb->pa", R[j], o[i] - o[j]))
    tr = _normalize(tr + rng.normal(0.0, np.deg2rad(sigma_deg), size=(P, 3)))
    outl = rng.random(P) < outlier_frac
    tr[outl] = _normalize(rng.normal(size=(int(outl.sum()), 3)))
    init = rng.normal(size=(runs, R.shape[0], 3))
    return TranslationInputs(tr, outl, init, sigma_deg, outlier_frac)


# ------------------------------------------------------------------ rotation averaging inputs

@dataclasses.dataclass
class RotationInputs:
    R_rel: np.ndarray       # [P,3,3] float64 measured relative rotations R^{i->j}
    outlier: np.ndarray     # [P] bool, True where R_rel is a random rotation
    sigma_deg: float
    outlier_frac: float


def rotation_inputs(scene: Scene, sigma_deg: float = 2.0, outlier_frac: float = 0.1,
                    seed: int | None = None) -> RotationInputs:
    """Inputs of rotation averaging on a scene's pair graph (Sec. 3.3, Global
    Rotation): per pair the measured relative rotation R^{i->j} ~ R_j R_i^T,
    rotated by sigma_deg * |N(0, 1)| about a random axis, and outlier_frac of
    the pairs replaced by rotations uniform on SO(3) (random unit quaternions)."""
    rng = np.random.default_rng((scene.seed if seed is None else seed) + 30_000)
    R = scene.R_gt
    i, j = scene.pairs[:, 0], scene.pairs[:, 1]
    P = len(scene.pairs)
    Q = np.einsum("pab,pcb->pac", R[j], R[i])
    axis = _normalize(rng.normal(size=(P, 3)))
    ang = np.deg2rad(sigma_deg) * np.abs(rng.normal(size=P))
    Q = _axis_angle(axis, ang) @ Q
    outl = rng.random(P) < outlier_frac
    q = _normalize(rng.normal(size=(int(outl.sum()), 4)))
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    Q[outl] = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)
    return RotationInputs(Q, outl, sigma_deg, outlier_frac)
