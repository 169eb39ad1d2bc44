"""Sparse coefficient uplift (Eq. 5, Algorithm 1) and Top-K filter (Eq. 6), FP64.

Algorithm 1: every w_i starts at zero; for every view v, pixel p and Gaussian
i in N_{v,p}, each non-zero (atom j, coefficient c_j) of the pixel's sparse
code W_v(p) adds c_j * e_i(v,p) to w_i[j].  Codes are per region (Sec. 4.1):
all pixels of a region share one K-sparse convex code; pixels with region id
-1 carry no code (they still composite).  The normaliser Z_i of Eq. 5 is
omitted: Eq. 6's L1 normalisation subsumes it.

Eq. 6: w_hat_i = Top_K(w_i) / ||Top_K(w_i)||_1.  Readings: entries are ranked
by (value descending, atom index ascending), so exact ties go to the lower
index; only strictly positive entries are kept; fewer than K of them are
padded with (index -1, value 0); a row that is all zero is all padding.

U_v (region_touches) is pinned by the brute force's per-pixel lists and by
the closed forms of a one-region map (U_v = Gaussians that contribute) and
a map with one region per pixel (U_v = contributions).

Parity pinned by: the brute force (per-entry), the invariants row-sum = Z_i,
linearity in the codes, additivity over views, one-hot codes giving per-region
weight sums, a uniform code uplifting to itself, and Top-K against a full sort.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .composite import ambiguity, composite_view
from .project import covariance3d, project


@dataclasses.dataclass
class UpliftResult:
    acc: np.ndarray            # (N, M) FP64 accumulated coefficients (rows may be a subset)
    amb: np.ndarray            # (N, M) FP64 ambiguity mass per entry
    n_contrib: int             # contributions over all views
    count_slack: int           # how far a float32 contribution count may move
    rows: Optional[np.ndarray] # the Gaussian ids of acc's rows (None = all)


def accumulate_view(acc: np.ndarray, amb: np.ndarray, vw, region_map: np.ndarray,
                    base: int, code_idx: np.ndarray, code_val: np.ndarray,
                    row_of: Optional[np.ndarray], m_atoms: int, amb_list=None) -> None:
    """acc[i, j] += c_j * e for every contribution of one view (Alg. 1 inner loops)."""
    rmap = region_map.reshape(-1)
    reg = rmap[vw.pixel]
    has = reg >= 0
    gi = vw.gauss[has]; e = vw.e[has]; g = base + reg[has].astype(np.int64)
    if row_of is not None:
        r = row_of[gi]; keep = r >= 0
        gi, e, g = r[keep], e[keep], g[keep]
    kc = code_idx.shape[1]
    for s in range(kc):
        j = code_idx[g, s].astype(np.int64)
        c = code_val[g, s].astype(np.float64)
        ok = j >= 0
        acc += np.bincount(gi[ok] * m_atoms + j[ok], weights=c[ok] * e[ok],
                           minlength=acc.size).reshape(acc.shape)
    if amb_list:
        for pix, gids, delta, _ in amb_list:
            r0 = rmap[pix]
            if r0 < 0:
                continue
            gg = base + int(r0)
            for s in range(kc):
                j = int(code_idx[gg, s])
                if j < 0:
                    continue
                c = float(code_val[gg, s])
                for gid, d in zip(gids, delta):
                    if d == 0.0:
                        continue
                    row = gid if row_of is None else row_of[gid]
                    if row >= 0:
                        amb[row, j] += c * d


def uplift_accumulate(gaussians, views, rows: Optional[np.ndarray] = None,
                      view_ids=None, track_marginal: bool = True) -> UpliftResult:
    """w_i for every Gaussian (or only ``rows``), summed over ``view_ids``.

    With ``rows`` given, only pixels inside those Gaussians' boxes are
    composited (all Gaussians still take part in the compositing there), which
    yields those rows exactly at a fraction of the cost.
    """
    n = gaussians.n
    m = views.m_atoms
    row_of = None
    nrows = n
    if rows is not None:
        rows = np.asarray(rows, np.int64)
        row_of = -np.ones(n, np.int64); row_of[rows] = np.arange(rows.shape[0])
        nrows = rows.shape[0]
    acc = np.zeros((nrows, m)); amb = np.zeros((nrows, m))
    cov = covariance3d(gaussians.log_scales, gaussians.quats)
    ncon = 0; slack = 0
    vids = range(views.n_views) if view_ids is None else view_ids
    for v in vids:
        cam = views.cameras[v]
        proj = project(gaussians, cam, cov)
        mask = None
        if rows is not None:
            mask = np.zeros(cam.width * cam.height, bool)
            for i in rows:
                if not proj.visible[i]:
                    continue
                x0, x1, y0, y1 = proj.box[i]
                yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
                mask[(yy * cam.width + xx).ravel()] = True
        vw = composite_view(proj, cam.width, cam.height, pixel_mask=mask,
                            track_marginal=track_marginal)
        amb_list = ambiguity(vw.marginal) if track_marginal else None
        if rows is None:
            ncon += vw.n_contrib
            slack += sum(s for *_, s in amb_list) if amb_list else 0
        accumulate_view(acc, amb, vw, views.region_maps[v], int(views.region_base[v]),
                        views.code_idx, views.code_val, row_of, m, amb_list)
    return UpliftResult(acc, amb, ncon, slack, rows)


def region_touches(gaussians, views, view_ids=None) -> np.ndarray:
    """U_v per view: the distinct (Gaussian i, region r) pairs with a
    contribution e_i(v,p) > 0 at some pixel p of region r >= 0, i.e. the
    pairs whose region code Algorithm 1's inner loop adds at least once in
    view v (the unit of Eq. 5's O(|S_i| K) cost once pixels of a region share
    its code).  Returns int64 (number of views,)."""
    cov = covariance3d(gaussians.log_scales, gaussians.quats)
    vids = list(range(views.n_views)) if view_ids is None else list(view_ids)
    out = np.zeros(len(vids), np.int64)
    for k, v in enumerate(vids):
        cam = views.cameras[v]
        vw = composite_view(project(gaussians, cam, cov), cam.width, cam.height, track_marginal=False)
        reg = views.region_maps[v].reshape(-1)[vw.pixel].astype(np.int64)
        has = (reg >= 0) & (vw.e > 0)
        nreg = int(views.region_base[v + 1] - views.region_base[v])
        out[k] = np.unique(vw.gauss[has].astype(np.int64) * max(nreg, 1) + reg[has]).shape[0]
    return out


def topk_rows(acc: np.ndarray, k: int):
    """Eq. 6 per row: (idx int32 (N,K), val FP64 (N,K)), see module docstring."""
    acc = np.asarray(acc, np.float64)
    n, m = acc.shape
    col = np.broadcast_to(np.arange(m), (n, m))
    order = np.lexsort((col, -acc), axis=1)[:, :k]
    top = np.take_along_axis(acc, order, axis=1)
    pos = top > 0
    idx = np.where(pos, order, -1).astype(np.int32)
    val = np.where(pos, top, 0.0)
    s = val.sum(axis=1, keepdims=True)
    val = np.where(s > 0, val / np.where(s > 0, s, 1.0), 0.0)
    if k > m:
        pad = k - m
        idx = np.concatenate([idx, -np.ones((n, pad), np.int32)], 1)
        val = np.concatenate([val, np.zeros((n, pad))], 1)
    return idx, val


def dense_uplift(gaussians, views, codebook: np.ndarray):
    """Dense feature uplift, Eq. 3: f_i = (1/Z_i) sum_{(v,p) in S_i} e_i(v,p) F_v(p)
    with F_v(p) = W_v(p) C the decoded feature of the pixel's region (Eq. 4)
    and Z_i = sum e_i(v,p).  Reading: pixels without a region carry no feature
    and enter neither sum (as in the sparse uplift).  Returns (f (N,D), Z (N,))
    in FP64; rows with Z_i = 0 are zero."""
    C = np.asarray(codebook, np.float64)
    n, d = gaussians.n, C.shape[1]
    R = views.code_idx.shape[0]
    F = np.zeros((R, d))
    for s in range(views.code_idx.shape[1]):
        j = views.code_idx[:, s]
        ok = j >= 0
        F[ok] += views.code_val[ok, s].astype(np.float64)[:, None] * C[j[ok]]
    f = np.zeros((n, d)); Z = np.zeros(n)
    cov = covariance3d(gaussians.log_scales, gaussians.quats)
    for v in range(views.n_views):
        cam = views.cameras[v]
        vw = composite_view(project(gaussians, cam, cov), cam.width, cam.height, track_marginal=False)
        reg = views.region_maps[v].reshape(-1)[vw.pixel]
        has = reg >= 0
        gi, e, g = vw.gauss[has], vw.e[has], int(views.region_base[v]) + reg[has].astype(np.int64)
        np.add.at(f, gi, e[:, None] * F[g])
        Z += np.bincount(gi, weights=e, minlength=n)
    f = np.divide(f, Z[:, None], out=np.zeros_like(f), where=Z[:, None] > 0)
    return f, Z


def row_entropy(acc: np.ndarray) -> np.ndarray:
    """Entropy of each Gaussian's coefficient distribution (App. C.2):
    H(w_i) = -sum_l p_l log p_l over the row normalised to sum one (natural
    log, 0 log 0 = 0); an all-zero row has H = 0.  Reading: the accumulated
    row before Top-K, L1-normalised, as the distribution."""
    a = np.asarray(acc, np.float64)
    s = a.sum(axis=1, keepdims=True)
    p = np.divide(a, s, out=np.zeros_like(a), where=s > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(p > 0, p * np.log(p), 0.0)
    return -t.sum(axis=1)


def uplift(gaussians, views, k: int):
    """Full uplift: accumulate over all views, then Top-K (Alg. 1)."""
    res = uplift_accumulate(gaussians, views)
    idx, val = topk_rows(res.acc, k)
    return idx, val, res
