"""3D Gaussian covariance and per-view EWA projection, FP64 (oracle).

Follows the 3DGS preliminaries of Sec. 3: each Gaussian has a centre mu, a
per-axis scale s (given as log-scale, activation exp), a rotation quaternion q
(w,x,y,z, normalised here) and an activated opacity o.  The 3D covariance is
Sigma = R(q) diag(exp(2 s)) R(q)^T.  The 2D footprint G^2D of Eq. 2's
alpha_i = o_i G_i^2D(v,p) is the EWA splat of the tile rasterizer the paper
inherits: Sigma2D = J W Sigma W^T J^T + 0.3 I with the Jacobian J evaluated at
the camera point whose x/z, y/z are clamped to 1.3 tan(half fov).

Readings where the paper is silent (3DGS conventions): near plane 0.2, the
+0.3 px^2 low-pass dilation, the 1.3 Jacobian clamp, pixel (px,py) sampled at
(px+1/2, py+1/2), depth order by the Gaussian centre's view depth rounded to
float32 with ties to the lower Gaussian id.

Parity pinned by: the scalar brute force (``brute``) and the closed forms in
the oracle tests (isotropic on-axis Gaussian, single Gaussian at a pixel centre).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NEAR = 0.2
DILATION = 0.3
JAC_CLAMP = 1.3
ALPHA_MIN = 1.0 / 255.0


def quat_to_rotmat(q: np.ndarray) -> np.ndarray:
    """(N,4) quaternions (w,x,y,z) -> (N,3,3) rotation matrices (normalised first)."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariance3d(log_scales: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """Sigma = R S S^T R^T with S = diag(exp(log_scales)); (N,3,3) FP64."""
    R = quat_to_rotmat(quats)
    s2 = np.exp(2.0 * np.asarray(log_scales, np.float64))
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


@dataclasses.dataclass
class Projection:
    """Per-Gaussian projection into one view (all FP64 unless stated).

    visible   bool, in front of the near plane and able to reach alpha >= 1/255
    z         view depth of the centre
    depth_key float32 rounding of z (the front-to-back sort key)
    mean2d    (N,2) pixel coordinates of the centre
    cov2d     (N,3) dilated 2D covariance (xx, xy, yy)
    conic     (N,3) its inverse (a, b, c): d^T conic d = a dx^2 + 2 b dx dy + c dy^2
    opacity   (N,)
    box       (N,4) inclusive pixel-index box (x0, x1, y0, y1) that contains
              every pixel whose alpha can reach 1/255 (an enumeration aid only,
              widened by one pixel); x0 > x1 means empty
    """
    visible: np.ndarray
    z: np.ndarray
    depth_key: np.ndarray
    mean2d: np.ndarray
    cov2d: np.ndarray
    conic: np.ndarray
    opacity: np.ndarray
    box: np.ndarray


def camera_point(means: np.ndarray, cam) -> np.ndarray:
    """p = R mu + t, each coordinate summed left to right in FP64."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    m = np.asarray(means, np.float64)
    x = R[0, 0] * m[:, 0] + R[0, 1] * m[:, 1] + R[0, 2] * m[:, 2] + t[0]
    y = R[1, 0] * m[:, 0] + R[1, 1] * m[:, 1] + R[1, 2] * m[:, 2] + t[1]
    z = R[2, 0] * m[:, 0] + R[2, 1] * m[:, 1] + R[2, 2] * m[:, 2] + t[2]
    return np.stack([x, y, z], 1)


def project(g, cam, cov3d: np.ndarray | None = None) -> Projection:
    """EWA projection of every Gaussian of ``g`` into camera ``cam``."""
    fx, fy = float(cam.fx), float(cam.fy)
    cx, cy = float(cam.cx), float(cam.cy)
    W, H = int(cam.width), int(cam.height)
    near = float(getattr(cam, "near", NEAR))
    if cov3d is None:
        cov3d = covariance3d(g.log_scales, g.quats)
    p = camera_point(g.means, cam)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    front = z > near
    zs = np.where(front, z, 1.0)
    tan_x = W / (2.0 * fx)
    tan_y = H / (2.0 * fy)
    lim_x, lim_y = JAC_CLAMP * tan_x, JAC_CLAMP * tan_y
    tx = np.clip(x / zs, -lim_x, lim_x) * zs
    ty = np.clip(y / zs, -lim_y, lim_y) * zs
    n = x.shape[0]
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / zs
    J[:, 0, 2] = -fx * tx / (zs * zs)
    J[:, 1, 1] = fy / zs
    J[:, 1, 2] = -fy * ty / (zs * zs)
    Rc = np.asarray(cam.R, np.float64)
    T = J @ Rc                                           # (n,2,3)
    S2 = np.einsum("nij,njk,nlk->nil", T, cov3d, T)      # T Sigma T^T
    sxx = S2[:, 0, 0] + DILATION
    sxy = S2[:, 0, 1]
    syy = S2[:, 1, 1] + DILATION
    det = sxx * syy - sxy * sxy
    conic = np.stack([syy / det, -sxy / det, sxx / det], 1)
    mean2d = np.stack([fx * x / zs + cx, fy * y / zs + cy], 1)
    o = np.asarray(g.opacities, np.float64)
    lo = np.log(np.maximum(255.0 * o, 1e-300))
    reach = lo >= 0.0
    r2 = 2.0 * np.maximum(lo, 0.0)
    hx = np.sqrt(r2 * sxx)
    hy = np.sqrt(r2 * syy)
    visible = front & reach & (det > 0)
    with np.errstate(invalid="ignore"):
        x0 = np.ceil(mean2d[:, 0] - hx - 0.5) - 1
        x1 = np.floor(mean2d[:, 0] + hx - 0.5) + 1
        y0 = np.ceil(mean2d[:, 1] - hy - 0.5) - 1
        y1 = np.floor(mean2d[:, 1] + hy - 0.5) + 1
    x0 = np.clip(np.nan_to_num(x0, nan=W), 0, W); x1 = np.clip(np.nan_to_num(x1, nan=-1), -1, W - 1)
    y0 = np.clip(np.nan_to_num(y0, nan=H), 0, H); y1 = np.clip(np.nan_to_num(y1, nan=-1), -1, H - 1)
    box = np.stack([x0, x1, y0, y1], 1).astype(np.int64)
    visible &= (box[:, 0] <= box[:, 1]) & (box[:, 2] <= box[:, 3])
    return Projection(visible, z, z.astype(np.float32), mean2d,
                      np.stack([sxx, sxy, syy], 1), conic, o, box)


def alpha_at(proj: Projection, i: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Unclamped o * exp(-1/2 d^T conic d) at pixel centres; 0 where the
    exponent is positive (the 3DGS guard, a no-op for positive-definite conics)."""
    dx = px + 0.5 - proj.mean2d[i, 0]
    dy = py + 0.5 - proj.mean2d[i, 1]
    a, b, c = proj.conic[i, 0], proj.conic[i, 1], proj.conic[i, 2]
    power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
    out = proj.opacity[i] * np.exp(np.minimum(power, 0.0))
    return np.where(power > 0.0, 0.0, out)


def tan_half_fov(cam) -> tuple:
    return cam.width / (2.0 * cam.fx), cam.height / (2.0 * cam.fy)


def isotropic_on_axis_alpha(o: float, s: float, z: float, f: float, d: float) -> float:
    """Closed form used as a pin: an isotropic Gaussian of scale s centred on the
    optical axis at depth z has J = diag(f/z, f/z) there, so its 2D variance is
    (s f/z)^2 + 0.3 and alpha at distance d is min(0.99, o exp(-d^2/(2 var)))."""
    var = (s * f / z) ** 2 + DILATION
    return min(0.99, o * math.exp(-d * d / (2.0 * var)))
