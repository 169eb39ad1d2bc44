"""Front-to-back alpha compositing weights e = alpha * T, FP64 (oracle).

Eq. 2: e_i(v,p) = alpha_i(v,p) * prod_{j<i} (1 - alpha_j(v,p)) over the
Gaussians N_{v,p} overlapping pixel p, ordered front to back, with
alpha_i = o_i G_i^2D(v,p).  The 3DGS numerics the paper inherits decide which
Gaussians belong to N_{v,p} and when the list ends, taken in this order for
each candidate of the depth-sorted list:

1. alpha = min(0.99, o exp(-1/2 d^T conic d));
2. skip the Gaussian if alpha < 1/255 (it is not in N_{v,p});
3. testT = T (1 - alpha); if testT < 1e-4 the pixel is finished and this
   Gaussian is excluded;
4. otherwise e = alpha T and T = testT.

Reading: the support S_i of Eq. 3/5 is every (v,p) where step 4 runs, with no
3-sigma truncation; boxes are only a conservative enumeration aid.

The FP64 oracle also reports *marginal events*: candidates whose alpha lies
within ``eps_alpha`` (relative) of 1/255 and transmittance tests within
``eps_T`` (relative) of 1e-4.  A float32 implementation may legitimately take
the other branch there; ``ambiguity`` recomposites such pixels with the
decision flipped and returns the exact weight change, which parity tests add
to their tolerance.

Parity pinned by: the scalar brute force, the closed forms (single Gaussian,
two Gaussians on one pixel) and the invariant sum_i e_i(p) = 1 - T_final(p).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .project import ALPHA_MIN, Projection, alpha_at

ALPHA_MAX = 0.99
T_MIN = 1e-4


@dataclasses.dataclass
class ViewWeights:
    """Weights of one view.

    gauss, pixel, e   the contributions (Gaussian id, flat pixel y*W+x, weight)
    t_final           (H*W,) transmittance left at every pixel
    marginal          {flat pixel: candidate list} for pixels with marginal events;
                      each list holds (gauss ids, unclamped-alpha values, event
                      kinds) in composite order, see ``ambiguity``
    """
    gauss: np.ndarray
    pixel: np.ndarray
    e: np.ndarray
    t_final: np.ndarray
    marginal: dict

    @property
    def n_contrib(self) -> int:
        return int(self.gauss.shape[0])


def _band_candidates(proj: Projection, ids: np.ndarray, y0: int, y1: int, width: int,
                     pixel_mask: Optional[np.ndarray]):
    bx0, bx1, by0, by1 = (proj.box[ids, k] for k in range(4))
    sel = (by0 <= y1 - 1) & (by1 >= y0)
    ids = ids[sel]
    gx0 = bx0[sel]; bw = bx1[sel] - gx0 + 1
    gy0 = np.maximum(by0[sel], y0); gy1 = np.minimum(by1[sel], y1 - 1)
    bh = gy1 - gy0 + 1
    cnt = bw * bh
    tot = int(cnt.sum())
    if tot == 0:
        e = np.zeros(0, np.int64)
        return e, e, e
    rep = np.repeat(np.arange(ids.shape[0]), cnt)
    off = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    w = bw[rep]
    px = gx0[rep] + off % w
    py = gy0[rep] + off // w
    gi = ids[rep]
    if pixel_mask is not None:
        keep = pixel_mask[py * width + px]
        gi, px, py = gi[keep], px[keep], py[keep]
    return gi, px, py


def composite_view(proj: Projection, width: int, height: int, band: int = 32,
                   pixel_mask: Optional[np.ndarray] = None, eps_alpha: float = 1e-5,
                   eps_T: float = 1e-4, track_marginal: bool = True) -> ViewWeights:
    """Composite every pixel (or those in ``pixel_mask``) of one view."""
    ids = np.flatnonzero(proj.visible)
    if pixel_mask is not None:
        # keep only Gaussians whose box holds a pixel in scope (summed-area table)
        sat = np.zeros((height + 1, width + 1), np.int64)
        sat[1:, 1:] = pixel_mask.reshape(height, width).cumsum(0).cumsum(1)
        x0, x1, y0, y1 = (proj.box[ids, k] for k in range(4))
        tot = sat[y1 + 1, x1 + 1] - sat[y0, x1 + 1] - sat[y1 + 1, x0] + sat[y0, x0]
        ids = ids[tot > 0]
    t_final = np.ones(width * height)
    out_g, out_p, out_e = [], [], []
    marginal = {}
    lo_thr = ALPHA_MIN * (1.0 - eps_alpha) if track_marginal else ALPHA_MIN
    for y0 in range(0, height, band):
        y1 = min(height, y0 + band)
        gi, px, py = _band_candidates(proj, ids, y0, y1, width, pixel_mask)
        if gi.shape[0] == 0:
            continue
        a_raw = alpha_at(proj, gi, px.astype(np.float64), py.astype(np.float64))
        alpha = np.minimum(ALPHA_MAX, a_raw)
        keep = alpha >= lo_thr
        gi, px, py, alpha = gi[keep], px[keep], py[keep], alpha[keep]
        pix = py * width + px
        order = np.lexsort((gi, proj.depth_key[gi], pix))
        gi, pix, alpha = gi[order], pix[order], alpha[order]
        n = gi.shape[0]
        if n == 0:
            continue
        # rank of each candidate inside its pixel's list
        start = np.ones(n, bool); start[1:] = pix[1:] != pix[:-1]
        first = np.flatnonzero(start)
        gid = np.cumsum(start) - 1
        rank = np.arange(n) - first[gid]
        upix = pix[first]
        T = np.ones(first.shape[0])
        alive = np.ones(first.shape[0], bool)
        e = np.zeros(n)
        mflag = np.zeros(first.shape[0], bool)
        if track_marginal:
            near_a = np.abs(alpha - ALPHA_MIN) <= eps_alpha * ALPHA_MIN
            np.logical_or.at(mflag, gid[near_a], True)
        by_rank = np.argsort(rank, kind="stable")
        counts = np.bincount(rank)
        pos = 0
        for r in range(counts.shape[0]):
            idx = by_rank[pos:pos + counts[r]]; pos += counts[r]
            g = gid[idx]
            act = alive[g] & (alpha[idx] >= ALPHA_MIN)
            idx, g = idx[act], g[act]
            a = alpha[idx]
            testT = T[g] * (1.0 - a)
            stop = testT < T_MIN
            if track_marginal:
                near_t = np.abs(testT - T_MIN) <= eps_T * T_MIN
                mflag[g[near_t]] = True
            go = ~stop
            e[idx[go]] = a[go] * T[g[go]]
            T[g[go]] = testT[go]
            alive[g[stop]] = False
        t_final[upix] = T
        c = e > 0
        out_g.append(gi[c]); out_p.append(pix[c]); out_e.append(e[c])
        if track_marginal and mflag.any():
            for k in np.flatnonzero(mflag):
                s = first[k]
                t = first[k + 1] if k + 1 < first.shape[0] else n
                marginal[int(upix[k])] = (gi[s:t].copy(), alpha[s:t].copy())
    if out_g:
        G = np.concatenate(out_g); P = np.concatenate(out_p); E = np.concatenate(out_e)
    else:
        G = np.zeros(0, np.int64); P = np.zeros(0, np.int64); E = np.zeros(0)
    return ViewWeights(G, P, E, t_final, marginal)


def composite_list(alpha: np.ndarray, flip_alpha: int = -1, flip_stop: int = -1) -> np.ndarray:
    """Scalar compositing of one pixel's depth-sorted candidate list.

    ``flip_alpha`` / ``flip_stop`` invert the skip test or the stop test at
    that list position (used to measure what a marginal event can change).
    Returns the weight of every candidate (0 where it does not contribute).
    """
    T = 1.0
    out = np.zeros(alpha.shape[0])
    for k in range(alpha.shape[0]):
        a = float(alpha[k])
        include = a >= ALPHA_MIN
        if k == flip_alpha:
            include = not include
        if not include:
            continue
        testT = T * (1.0 - a)
        stop = testT < T_MIN
        if k == flip_stop:
            stop = not stop
        if stop:
            break
        out[k] = a * T
        T = testT
    return out


def ambiguity(marginal: dict, eps_alpha: float = 1e-5, eps_T: float = 1e-4):
    """Per marginal pixel, the summed |weight change| of each Gaussian over all
    single flips of marginal decisions, and the change in contribution count.

    Returns a list of (flat pixel, gauss ids, |delta e| per candidate, count slack).
    """
    out = []
    for pix, (gi, alpha) in marginal.items():
        base = composite_list(alpha)
        # replay to find the stop-test values
        T = 1.0
        tests = []
        for k in range(alpha.shape[0]):
            a = float(alpha[k])
            if a < ALPHA_MIN:
                continue
            testT = T * (1.0 - a)
            tests.append((k, testT))
            if testT < T_MIN:
                break
            T = testT
        delta = np.zeros(alpha.shape[0])
        slack = 0
        nb = int((base > 0).sum())
        flips = [("a", k) for k in range(alpha.shape[0])
                 if abs(alpha[k] - ALPHA_MIN) <= eps_alpha * ALPHA_MIN]
        flips += [("t", k) for k, tv in tests if abs(tv - T_MIN) <= eps_T * T_MIN]
        for kind, k in flips:
            alt = composite_list(alpha, flip_alpha=k if kind == "a" else -1,
                                 flip_stop=k if kind == "t" else -1)
            delta += np.abs(alt - base)
            slack += abs(int((alt > 0).sum()) - nb)
        out.append((pix, gi, delta, slack))
    return out
