"""Seeded synthetic scenes for the sparse-code uplift, render and decode.

This module draws inputs only: Gaussian parameters, pinhole cameras, Voronoi
region maps, sparse convex region codes, per-Gaussian Top-K tables, codebooks,
query and target vectors.  It contains none of the method's arithmetic
(no projection, compositing, accumulation, Top-K or decoding), so both the
FP64 oracle and the GPU library can consume its arrays without sharing code.

Every generator takes an explicit seed; streams are spawned in a fixed order
from ``numpy.random.SeedSequence`` so the same call always yields the same
arrays on every machine.

Scene shapes mirror the five workloads of the paper's setting (Sec. 5.2 uses
pretrained 3DGS scenes with about a million Gaussians, SAM regions per image
and K-sparse convex codes of Eq. 4):

* ``tiny``      2,000 isotropic Gaussians in the unit cube, 4 views 64x48,
                8 regions per view, M=64, K=4.
* ``scene``     1,000,000 anisotropic Gaussians in a 10x10x4 box, 200 views
                1008x756 on a jittered orbit, 120 regions, M=256, K=8.
* ``render``    the ``scene`` Gaussians with synthetic Top-8 tables over
                M=256, codebook 256x512, 100 views 1440x1080.
* ``backward``  200,000 Gaussians, Top-8 over M=256, codebook 256x512,
                8 views 512x384, unit target feature maps.
* ``large``     3,000,000 Gaussians in a 20x20x6 box, 300 views 1440x1080,
                200 regions, M=512, K=16.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Gaussians", "Camera", "Views", "Scene", "CONFIGS",
    "make_gaussians", "look_at_camera", "orbit_cameras", "circle_cameras",
    "voronoi_region_map", "region_codes", "make_views", "make_scene",
    "random_topk", "random_codebook", "random_unit_vectors", "subset_views",
]


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Gaussians:
    """Structure of arrays, all float32.

    means (N,3) world positions; log_scales (N,3) per-axis log standard
    deviations (activation exp); quats (N,4) rotation quaternions in (w,x,y,z)
    order, not necessarily normalised; opacities (N,) already activated, in (0,1).
    """
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx: np.ndarray) -> "Gaussians":
        return Gaussians(self.means[idx].copy(), self.log_scales[idx].copy(),
                         self.quats[idx].copy(), self.opacities[idx].copy())


@dataclasses.dataclass
class Camera:
    """Pinhole camera, world->camera rotation R (3x3) and translation t.

    Camera axes: +x right, +y down, +z forward.  A world point X maps to
    camera point R X + t and to pixel coordinates (fx x/z + cx, fy y/z + cy);
    pixel (px, py) is sampled at its centre (px + 1/2, py + 1/2).
    """
    R: np.ndarray          # (3,3) float32
    t: np.ndarray          # (3,)  float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def as_row(self) -> np.ndarray:
        """Flat float32 row: R (9), t (3), fx, fy, cx, cy, width, height, near."""
        return np.concatenate([
            np.asarray(self.R, np.float32).reshape(9),
            np.asarray(self.t, np.float32).reshape(3),
            np.array([self.fx, self.fy, self.cx, self.cy,
                      self.width, self.height, self.near], np.float32)])


@dataclasses.dataclass
class Views:
    """Per-view region maps and the sparse convex code of every region.

    region_maps[v] is an (H_v, W_v) int32 map of view-local region ids, -1 for
    pixels that belong to no region.  Region r of view v has global id
    region_base[v] + r; its code occupies row region_base[v] + r of code_idx /
    code_val (k_code slots; unused slots have index -1 and value 0).
    """
    cameras: List[Camera]
    region_maps: List[np.ndarray]
    region_base: np.ndarray     # (V+1,) int64
    code_idx: np.ndarray        # (R_total, k_code) int32
    code_val: np.ndarray        # (R_total, k_code) float32
    m_atoms: int

    @property
    def n_views(self) -> int:
        return len(self.cameras)

    @property
    def k_code(self) -> int:
        return int(self.code_idx.shape[1])


@dataclasses.dataclass
class Scene:
    name: str
    gaussians: Gaussians
    views: Views
    k_top: int
    seed: int


# ----------------------------------------------------------------------------
# primitive generators
# ----------------------------------------------------------------------------
def _streams(seed: int, n: int) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def make_gaussians(seed: int, n: int, box_half: tuple, log_scale_mean: float,
                   log_scale_std: float, isotropic: bool,
                   opacity: str) -> Gaussians:
    """Gaussians uniform in the centred box with half-extents ``box_half``.

    ``opacity`` is ``"uniform"`` for U(0.1, 0.9) or ``"beta"`` for Beta(2,2).
    Isotropic scenes replicate one log-scale to all axes and use the identity
    rotation; anisotropic ones draw per-axis log-scales and quaternions
    uniform on the 3-sphere (normalised Gaussian 4-vectors).
    """
    r_mean, r_scale, r_quat, r_op = _streams(seed, 4)
    half = np.asarray(box_half, np.float64)
    means = (r_mean.random((n, 3)) * 2.0 - 1.0) * half
    if isotropic:
        s = r_scale.normal(log_scale_mean, log_scale_std, size=(n, 1))
        log_scales = np.repeat(s, 3, axis=1)
        quats = np.zeros((n, 4)); quats[:, 0] = 1.0
    else:
        log_scales = r_scale.normal(log_scale_mean, log_scale_std, size=(n, 3))
        q = r_quat.normal(size=(n, 4))
        quats = q / np.linalg.norm(q, axis=1, keepdims=True)
    if opacity == "uniform":
        op = r_op.uniform(0.1, 0.9, size=n)
    elif opacity == "beta":
        op = r_op.beta(2.0, 2.0, size=n)
        op = np.clip(op, 1e-4, 1.0 - 1e-4)
    else:
        raise ValueError(opacity)
    return Gaussians(means.astype(np.float32), log_scales.astype(np.float32),
                     quats.astype(np.float32), op.astype(np.float32))


def look_at_camera(eye, target, width: int, height: int, fov_x_deg: float,
                   up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at ``eye`` looking at ``target`` with world up ``up``.

    Horizontal field of view ``fov_x_deg``; square pixels (fy = fx); principal
    point at the image centre (W/2, H/2).
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), float(np.float32(fx)),
                  float(np.float32(fx)), width / 2.0, height / 2.0, width, height)


def circle_cameras(n: int, radius: float, width: int, height: int,
                   fov_x_deg: float) -> List[Camera]:
    """``n`` cameras evenly spaced on a circle of ``radius`` in the z=0 plane."""
    cams = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        cams.append(look_at_camera((radius * math.cos(a), radius * math.sin(a), 0.0),
                                   (0.0, 0.0, 0.0), width, height, fov_x_deg))
    return cams


def orbit_cameras(seed: int, n: int, radius: float, radius_jitter: float,
                  height_mean: float, height_jitter: float, target_std: float,
                  width: int, height: int, fov_x_deg: float,
                  jitter: bool = True) -> List[Camera]:
    """Jittered orbit: azimuth 2 pi k/n plus U(-1/2,1/2) of one step, radius and
    height jittered uniformly, look-at point N(0, target_std^2) per axis."""
    rng = _streams(seed, 1)[0]
    cams = []
    for k in range(n):
        step = 2.0 * math.pi / n
        az = step * k + (rng.uniform(-0.5, 0.5) * step if jitter else 0.0)
        rad = radius + (rng.uniform(-radius_jitter, radius_jitter) if jitter else 0.0)
        hgt = height_mean + (rng.uniform(-height_jitter, height_jitter) if jitter else 0.0)
        tgt = rng.normal(0.0, target_std, size=3) if jitter else np.zeros(3)
        cams.append(look_at_camera((rad * math.cos(az), rad * math.sin(az), hgt), tgt,
                                   width, height, fov_x_deg))
    return cams


def voronoi_region_map(rng: np.random.Generator, width: int, height: int,
                       n_sites: int) -> np.ndarray:
    """(H, W) int32 map: each pixel centre goes to its nearest site (Euclidean
    distance; sites are uniform in [0,W) x [0,H), so exact ties have
    probability zero).  Nearest-site search uses a k-d tree."""
    from scipy.spatial import cKDTree
    sites = np.stack([rng.uniform(0, width, n_sites), rng.uniform(0, height, n_sites)], 1)
    xs = np.arange(width, dtype=np.float64) + 0.5
    ys = np.arange(height, dtype=np.float64) + 0.5
    X, Y = np.meshgrid(xs, ys)
    _, idx = cKDTree(sites).query(np.stack([X.ravel(), Y.ravel()], 1), workers=-1)
    return idx.reshape(height, width).astype(np.int32)


def region_codes(rng: np.random.Generator, n_regions: int, m_atoms: int,
                 k_code: int) -> tuple:
    """K-sparse convex codes (Eq. 4): ``k_code`` distinct atoms uniform over
    [0, M), values U(0,1) normalised to sum 1."""
    keys = rng.random((n_regions, m_atoms))
    idx = np.argpartition(keys, k_code - 1, axis=1)[:, :k_code].astype(np.int32)
    val = rng.random((n_regions, k_code))
    val = val / val.sum(axis=1, keepdims=True)
    return idx, val.astype(np.float32)


def make_views(seed: int, cameras: List[Camera], n_sites: int, m_atoms: int,
               k_code: int, hole_sites: int = 0) -> Views:
    """Voronoi region maps and codes for every camera.

    ``hole_sites`` of the ``n_sites`` cells (the last ones) are mapped to -1
    ("no region"), which exercises uncovered pixels.
    """
    rng_map, rng_code = _streams(seed, 2)
    maps, bases, idxs, vals = [], [0], [], []
    for cam in cameras:
        m = voronoi_region_map(rng_map, cam.width, cam.height, n_sites)
        if hole_sites:
            m = np.where(m >= n_sites - hole_sites, -1, m).astype(np.int32)
        n_reg = n_sites - hole_sites
        maps.append(m)
        ci, cv = region_codes(rng_code, n_reg, m_atoms, k_code)
        idxs.append(ci); vals.append(cv)
        bases.append(bases[-1] + n_reg)
    return Views(cameras, maps, np.asarray(bases, np.int64),
                 np.concatenate(idxs, 0), np.concatenate(vals, 0), m_atoms)


def subset_views(views: Views, which) -> Views:
    """The views listed in ``which`` (their regions renumbered densely)."""
    which = list(which)
    cams = [views.cameras[v] for v in which]
    maps = [views.region_maps[v] for v in which]
    bases, idxs, vals = [0], [], []
    for v in which:
        lo, hi = views.region_base[v], views.region_base[v + 1]
        idxs.append(views.code_idx[lo:hi]); vals.append(views.code_val[lo:hi])
        bases.append(bases[-1] + (hi - lo))
    return Views(cams, maps, np.asarray(bases, np.int64), np.concatenate(idxs, 0),
                 np.concatenate(vals, 0), views.m_atoms)


def random_topk(seed: int, n: int, m_atoms: int, k: int) -> tuple:
    """Synthetic per-Gaussian Top-K table: k distinct atoms, U(0,1) values
    normalised to sum 1.  Returns (idx int32 (n,k), val float32 (n,k))."""
    rng = _streams(seed, 1)[0]
    out_i = np.empty((n, k), np.int32)
    out_v = np.empty((n, k), np.float32)
    chunk = 1 << 18
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        keys = rng.random((e - s, m_atoms))
        out_i[s:e] = np.argpartition(keys, k - 1, axis=1)[:, :k]
        v = rng.random((e - s, k))
        out_v[s:e] = (v / v.sum(axis=1, keepdims=True)).astype(np.float32)
    return out_i, out_v


def random_codebook(seed: int, m_atoms: int, dim: int) -> np.ndarray:
    """(M, D) float32 codebook, rows N(0,1) then L2-normalised."""
    rng = _streams(seed, 1)[0]
    c = rng.normal(size=(m_atoms, dim))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    return c.astype(np.float32)


def random_unit_vectors(seed: int, n: int, dim: int) -> np.ndarray:
    """(n, dim) float32 unit vectors, isotropic."""
    rng = _streams(seed, 1)[0]
    q = rng.normal(size=(n, dim))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def random_coeff_rows(seed: int, n: int, m_atoms: int, nnz: int = 24, empty_frac: float = 0.1) -> np.ndarray:
    """(n, M) float32 rows shaped like rendered coefficient maps (Eq. 7):
    ``nnz`` distinct atoms per row with U(0,1) weights scaled to a row sum
    1 - T with T ~ U(0,1) (the blend of a few Gaussians' Top-K codes), and a
    fraction ``empty_frac`` of all-zero background rows."""
    rng = _streams(seed, 1)[0]
    nnz = min(nnz, m_atoms)
    out = np.zeros((n, m_atoms), np.float32)
    idx = np.argpartition(rng.random((n, m_atoms)), nnz - 1, axis=1)[:, :nnz]
    v = rng.random((n, nnz))
    v *= (rng.random(n) / v.sum(axis=1))[:, None]
    np.put_along_axis(out, idx, v.astype(np.float32), axis=1)
    out[rng.random(n) < empty_frac] = 0.0
    return out


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
CONFIGS = {
    "tiny": dict(n=2000, box=(0.5, 0.5, 0.5), ls=(-4.0, 0.3), iso=True, op="uniform",
                 views=4, res=(64, 48), sites=8, m=64, k=4),
    "scene": dict(n=1_000_000, box=(5.0, 5.0, 2.0), ls=(-4.5, 0.5), iso=False, op="beta",
                  views=200, res=(1008, 756), sites=120, m=256, k=8,
                  orbit=(12.0, 1.0, 4.0, 1.0, 0.5)),
    "render": dict(n=1_000_000, box=(5.0, 5.0, 2.0), ls=(-4.5, 0.5), iso=False, op="beta",
                   views=100, res=(1440, 1080), m=256, k=8, dim=512,
                   orbit=(12.0, 1.0, 4.0, 1.0, 0.5)),
    "backward": dict(n=200_000, box=(5.0, 5.0, 2.0), ls=(-4.5, 0.5), iso=False, op="beta",
                     views=8, res=(512, 384), m=256, k=8, dim=512,
                     orbit=(12.0, 0.0, 4.0, 0.0, 0.0)),
    "large": dict(n=3_000_000, box=(10.0, 10.0, 3.0), ls=(-4.5, 0.5), iso=False, op="beta",
                  views=300, res=(1440, 1080), sites=200, m=512, k=16,
                  orbit=(24.0, 2.0, 6.0, 2.0, 0.5)),
}
_SEED_BASE = {"tiny": 1000, "scene": 1001, "render": 1002, "backward": 1003, "large": 1004}


def make_scene(name: str, n_views: Optional[int] = None, n_gaussians: Optional[int] = None,
               res: Optional[tuple] = None, hole_sites: int = 0) -> Scene:
    """Build one of the uplift workloads (``tiny``, ``scene``, ``large``).

    ``n_views`` keeps the first views of the workload's camera rig (views are
    additive, so a prefix is an exact sub-problem); ``n_gaussians`` keeps a
    prefix of the Gaussians; ``res`` overrides the image size (focal length
    rescaled to keep the 60 degree horizontal field of view).
    """
    c = CONFIGS[name]
    seed = _SEED_BASE[name]
    s_g, s_cam, s_view = [int(x) for x in np.random.SeedSequence(seed).generate_state(3)]
    n = c["n"] if n_gaussians is None else int(n_gaussians)
    g = make_gaussians(s_g, c["n"], c["box"], c["ls"][0], c["ls"][1], c["iso"], c["op"])
    if n != c["n"]:
        g = g.subset(np.arange(n))
    w, h = c["res"] if res is None else res
    nv = c["views"]
    if name == "tiny":
        cams = circle_cameras(nv, 3.0, w, h, 60.0)
    else:
        r, rj, hm, hj, ts = c["orbit"]
        cams = orbit_cameras(s_cam, nv, r, rj, hm, hj, ts, w, h, 60.0)
    if n_views is not None:
        cams = cams[:n_views]
    views = make_views(s_view, cams, c["sites"], c["m"], c["k"], hole_sites=hole_sites)
    return Scene(name, g, views, c["k"], seed)
