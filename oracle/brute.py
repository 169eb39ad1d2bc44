"""Independent scalar brute force (pure Python floats), tiny scenes only.

A second transcription of Eq. 2, Eq. 5 and Eq. 7 that evaluates every
Gaussian at every pixel centre (no boxes, no culling beyond the near plane),
re-derives the 3DGS covariance and EWA projection with the ``math`` module,
and accumulates with dictionaries.  It shares nothing with the vectorised
oracle modules, so agreement between the two pins the vectorised code.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple


def _rot(q):
    w, x, y, z = (float(v) for v in q)
    n = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    return [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def splat(mu, log_scale, quat, opacity, cam):
    """Return (depth32, mx, my, (a, b, c), o) or None when behind the near plane."""
    R = [[float(cam.R[i][j]) for j in range(3)] for i in range(3)]
    t = [float(cam.t[i]) for i in range(3)]
    m = [float(v) for v in mu]
    p = [R[i][0] * m[0] + R[i][1] * m[1] + R[i][2] * m[2] + t[i] for i in range(3)]
    x, y, z = p
    if not z > float(cam.near):
        return None
    fx, fy = float(cam.fx), float(cam.fy)
    limx = 1.3 * (cam.width / (2.0 * fx))
    limy = 1.3 * (cam.height / (2.0 * fy))
    tx = min(limx, max(-limx, x / z)) * z
    ty = min(limy, max(-limy, y / z)) * z
    J = [[fx / z, 0.0, -fx * tx / (z * z)], [0.0, fy / z, -fy * ty / (z * z)]]
    Rq = _rot(quat)
    S = [[math.exp(float(log_scale[i])) if i == j else 0.0 for j in range(3)] for i in range(3)]
    M = _matmul(Rq, S)
    Sigma = _matmul(M, _transpose(M))
    T = _matmul(J, R)
    S2 = _matmul(_matmul(T, Sigma), _transpose(T))
    sxx = S2[0][0] + 0.3; sxy = S2[0][1]; syy = S2[1][1] + 0.3
    det = sxx * syy - sxy * sxy
    conic = (syy / det, -sxy / det, sxx / det)
    mx = fx * x / z + float(cam.cx)
    my = fy * y / z + float(cam.cy)
    import numpy as _np  # only for the float32 rounding of the depth key
    return float(_np.float32(z)), mx, my, conic, float(opacity)


def pixel_weights(gaussians, cam) -> Dict[Tuple[int, int], List[Tuple[int, float]]]:
    """{(px,py): [(gaussian id, e), ...] in composite order} for every pixel."""
    sp = []
    for i in range(gaussians.n):
        s = splat(gaussians.means[i], gaussians.log_scales[i], gaussians.quats[i],
                  gaussians.opacities[i], cam)
        if s is not None:
            sp.append((s[0], i, s))
    sp.sort(key=lambda r: (r[0], r[1]))
    out = {}
    for py in range(cam.height):
        for px in range(cam.width):
            T = 1.0
            lst = []
            for _, i, (_, mx, my, (a, b, c), o) in sp:
                dx = px + 0.5 - mx
                dy = py + 0.5 - my
                power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
                if power > 0.0:
                    continue
                alpha = min(0.99, o * math.exp(power))
                if alpha < 1.0 / 255.0:
                    continue
                test = T * (1.0 - alpha)
                if test < 1e-4:
                    break
                lst.append((i, alpha * T))
                T = test
            out[(px, py)] = (lst, T)
    return out


def uplift(gaussians, views) -> Dict[Tuple[int, int], float]:
    """Algorithm 1 literally: {(gaussian, atom): w} over all views and pixels."""
    w: Dict[Tuple[int, int], float] = {}
    for v in range(views.n_views):
        cam = views.cameras[v]
        pw = pixel_weights(gaussians, cam)
        rmap = views.region_maps[v]
        for (px, py), (lst, _) in pw.items():
            r = int(rmap[py, px])
            if r < 0:
                continue
            g = int(views.region_base[v]) + r
            for i, e in lst:
                for s in range(views.code_idx.shape[1]):
                    j = int(views.code_idx[g, s])
                    if j < 0:
                        continue
                    w[(i, j)] = w.get((i, j), 0.0) + float(views.code_val[g, s]) * e
    return w


def topk(row: List[float], k: int):
    """Eq. 6 by selection: repeatedly take the largest positive value, lowest index on ties."""
    taken = set()
    idx, val = [], []
    for _ in range(k):
        best = -1
        for j, x in enumerate(row):
            if j in taken or not x > 0:
                continue
            if best < 0 or x > row[best]:
                best = j
        if best < 0:
            break
        taken.add(best); idx.append(best); val.append(row[best])
    s = sum(val)
    val = [x / s for x in val] if s > 0 else val
    while len(idx) < k:
        idx.append(-1); val.append(0.0)
    return idx, val


def render(gaussians, topk_idx, topk_val, cam, m_atoms: int):
    """{(px,py): coefficient list of length M} for every pixel (Eq. 7)."""
    pw = pixel_weights(gaussians, cam)
    out = {}
    for key, (lst, _) in pw.items():
        row = [0.0] * m_atoms
        for i, e in lst:
            for s in range(len(topk_idx[i])):
                j = int(topk_idx[i][s])
                if j >= 0:
                    row[j] += float(topk_val[i][s]) * e
        out[key] = row
    return out
