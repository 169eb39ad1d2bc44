"""Gradients of a cosine feature loss through render (Eq. 7) and decode (Eq. 8), FP64.

Loss: L = mean over covered pixels of (1 - cos(F(p), t(p))), F = W_hat C.
A pixel is covered when at least one Gaussian contributes to it (F is 0 and
the cosine undefined elsewhere; those pixels are left out of the loss).

With G(p) = dL/dF(p) = -(1/P_c) (t/(|F||t|) - (F.t) F/(|F|^3 |t|)):
  dL/dC         = sum_p W_hat(p)^T G(p)
  dL/dW_hat(p)  = G(p) C^T
  dL/dw_hat_i[k] = sum_{(v,p)} e_i(v,p) dL/dW_hat_v(p)[idx_ik]
Atom indices and the geometry receive no gradient.

Parity pinned by: FP64 central finite differences (h = 1e-4) of ``loss`` and
the adjoint identity <G, dW C> = <G C^T, dW>.
"""
from __future__ import annotations

import numpy as np


def cosine_loss(F: np.ndarray, targets: np.ndarray, covered: np.ndarray, n_covered: int) -> float:
    F = np.asarray(F, np.float64)[covered]
    t = np.asarray(targets, np.float64)[covered]
    cos = (F * t).sum(1) / (np.linalg.norm(F, axis=1) * np.linalg.norm(t, axis=1))
    return float((1.0 - cos).sum() / n_covered)


def cosine_loss_grad(F: np.ndarray, targets: np.ndarray, covered: np.ndarray,
                     n_covered: int) -> np.ndarray:
    F = np.asarray(F, np.float64)
    t = np.asarray(targets, np.float64)
    G = np.zeros_like(F)
    f, tt = F[covered], t[covered]
    nf = np.linalg.norm(f, axis=1, keepdims=True)
    nt = np.linalg.norm(tt, axis=1, keepdims=True)
    ft = (f * tt).sum(1, keepdims=True)
    G[covered] = -(tt / (nf * nt) - ft * f / (nf ** 3 * nt)) / n_covered
    return G


def codebook_grad(coeff: np.ndarray, G: np.ndarray) -> np.ndarray:
    """dL/dC = W_hat^T G (summed over pixels)."""
    return np.asarray(coeff, np.float64).T @ np.asarray(G, np.float64)


def coeff_grad(weights, pixel_row: np.ndarray, topk_idx: np.ndarray, dW: np.ndarray,
               out: np.ndarray) -> None:
    """out[i, k] += sum over contributions of e * dW[row(p), idx_ik] (one view)."""
    r = pixel_row[weights.pixel]
    ok_pix = r >= 0
    gi = weights.gauss[ok_pix]; e = weights.e[ok_pix]; r = r[ok_pix]
    for k in range(topk_idx.shape[1]):
        j = topk_idx[gi, k].astype(np.int64)
        ok = j >= 0
        np.add.at(out[:, k], gi[ok], e[ok] * dW[r[ok], j[ok]])
