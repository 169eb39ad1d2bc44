"""Sparse coefficient render (Eq. 7) and codebook decode (Eq. 8), FP64 (oracle).

Eq. 7: W_hat_v(p) = sum_{i in N_{v,p}} w_hat_i e_i(v,p), with e from the same
front-to-back compositing as the uplift; each Gaussian carries K (atom index,
value) pairs, index -1 meaning an empty slot.  Eq. 8: F_v(p) = W_hat_v(p) C
with the codebook C of shape (M, D).

Parity pinned by: sum_m W_hat(p)[m] = 1 - T_final(p) when every w_hat sums to
one; a shared coefficient vector c rendering to (1 - T_final) c; one-hot rows
decoding to codebook rows; and the brute-force weights.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .composite import composite_view
from .project import covariance3d, project


@dataclasses.dataclass
class RenderResult:
    coeff: np.ndarray       # (P, M) FP64 rendered coefficients (P = pixels in scope)
    pixels: np.ndarray      # (P,) flat pixel ids of the rows of coeff
    t_final: np.ndarray     # (P,)
    weights: object         # ViewWeights of the view (for the backward)


def render_coeff(gaussians, topk_idx: np.ndarray, topk_val: np.ndarray, cam, m_atoms: int,
                 pixel_mask: Optional[np.ndarray] = None, track_marginal: bool = False
                 ) -> RenderResult:
    """Rendered coefficient map of one view over ``pixel_mask`` (all pixels if None)."""
    cov = covariance3d(gaussians.log_scales, gaussians.quats)
    proj = project(gaussians, cam, cov)
    vw = composite_view(proj, cam.width, cam.height, pixel_mask=pixel_mask,
                        track_marginal=track_marginal)
    P = cam.width * cam.height
    pixels = np.arange(P) if pixel_mask is None else np.flatnonzero(pixel_mask)
    row = -np.ones(P, np.int64); row[pixels] = np.arange(pixels.shape[0])
    coeff = np.zeros((pixels.shape[0], m_atoms))
    kk = topk_idx.shape[1]
    r = row[vw.pixel]
    for s in range(kk):
        j = topk_idx[vw.gauss, s].astype(np.int64)
        v = topk_val[vw.gauss, s].astype(np.float64)
        ok = j >= 0
        coeff += np.bincount(r[ok] * m_atoms + j[ok], weights=v[ok] * vw.e[ok],
                             minlength=coeff.size).reshape(coeff.shape)
    return RenderResult(coeff, pixels, vw.t_final[pixels], vw)


def decode(coeff: np.ndarray, codebook: np.ndarray) -> np.ndarray:
    """Eq. 8: F = W_hat C, FP64 matrix product."""
    return np.asarray(coeff, np.float64) @ np.asarray(codebook, np.float64)


def relevancy(features: np.ndarray, query: np.ndarray, canon: np.ndarray,
              temperature: float = 10.0) -> np.ndarray:
    """Relevancy score of App. B: min over canonical vectors of
    exp(a F.q) / (exp(a F.q) + exp(a F.c_k)), a = 10."""
    fq = features @ np.asarray(query, np.float64)
    fc = features @ np.asarray(canon, np.float64).T
    return np.min(1.0 / (1.0 + np.exp(temperature * (fc - fq[:, None]))), axis=1)


def relevancy_map(coeff: np.ndarray, codebook: np.ndarray, queries: np.ndarray, canon: np.ndarray,
                  temperature: float = 10.0) -> np.ndarray:
    """Relevancy of every pixel to every query (App. B) on the decoded
    features of Eq. 8: R[p, q] = relevancy(F, queries[q], canon)[p] with
    F = W_hat C in FP64.  Returns [P, Q] float64."""
    F = decode(coeff, codebook)
    return np.stack([relevancy(F, qv, canon, temperature) for qv in np.asarray(queries, np.float64)], axis=1)
