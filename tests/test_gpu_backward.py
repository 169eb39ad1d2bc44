"""GPU backward of render + decode against the FP64 oracle's gradient.

Tolerance (written here), per entry of dL/dw_hat (N, K) and dL/dC (M, D):
    |g_gpu - g_ref| <= 1e-4 |g_ref| + 1e-5 a_ref
where a_ref is the same sum taken over absolute values of its terms (float32
summation error grows with the magnitude of the terms, not with a result that
cancels).  The oracle itself is pinned against FP64 central finite differences
in tests/test_oracle_pins.py.
"""
import numpy as np
import pytest
import torch

import paper_2605_13600_amd as P
import scenegen as sg
from oracle import backward as OB
from oracle import render as OR
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu

REL = 1e-4


def _check_grad(got, ref, absref, name):
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    tol = REL * np.abs(ref) + 1e-5 * absref
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    print(f"[{name}] max err/tol {float((err / np.maximum(tol, 1e-300)).max()):.3g}, max rel err "
          f"{float((err / scale).max()):.3g} (|ref|max {np.abs(ref).max():.3g})")
    assert (err <= tol).all(), (name, float((err / np.maximum(tol, 1e-300)).max()))


def _loss_torch(F, tf, targets, sum_loss=False):
    """mean (or sum) over covered pixels of 1 - cos(F, t); covered = some contribution."""
    tot, ncov = 0.0, 0
    for f, t, T in zip(F, targets, tf):
        cov = (T < 1.0).reshape(-1)
        f2, t2 = f.reshape(-1, f.shape[-1])[cov], t.reshape(-1, t.shape[-1])[cov]
        cos = (f2 * t2).sum(1) / (f2.norm(dim=1) * t2.norm(dim=1))
        tot = tot + (1.0 - cos).sum()
        ncov += int(cov.sum())
    return tot if sum_loss else tot / ncov


def test_backward_matches_oracle_full():
    require_gpu()
    n, m, d, k = 4000, 256, 512, 8
    g = sg.make_gaussians(31, n, (5.0, 5.0, 2.0), -3.4, 0.5, False, "beta")
    cams = sg.orbit_cameras(32, 2, 12.0, 0.0, 4.0, 0.0, 0.0, 128, 96, 60.0, jitter=False)
    ti, tv = sg.random_topk(33, n, m, k)
    C = sg.random_codebook(34, m, d)
    targets = [sg.random_unit_vectors(40 + v, c.width * c.height, d) for v, c in enumerate(cams)]
    dg = P.gaussians_to_device(g)
    dti = torch.from_numpy(ti).cuda()
    dtv = torch.from_numpy(tv).cuda().requires_grad_(True)
    dC = torch.from_numpy(C).cuda().requires_grad_(True)
    Fs, tfs = [], []
    for cam in cams:
        F, tf = P.render_decode(dg, dti, dtv, dC, cam)
        Fs.append(F); tfs.append(tf)
    tt = [torch.from_numpy(t).cuda().reshape(c.height, c.width, d) for t, c in zip(targets, cams)]
    loss = _loss_torch(Fs, tfs, tt)
    loss.backward()
    # oracle gradient (FP64)
    rrs = [OR.render_coeff(g, ti, tv, cam, m) for cam in cams]
    Fr = [OR.decode(rr.coeff, C) for rr in rrs]
    covs = [rr.t_final < 1.0 for rr in rrs]
    ncov = sum(int(c.sum()) for c in covs)
    Lref = sum(OB.cosine_loss(F, t, c, ncov) for F, t, c in zip(Fr, targets, covs))
    assert float(loss) == pytest.approx(Lref, rel=1e-5)
    gC = np.zeros((m, d)); gw = np.zeros((n, k))
    aC = np.zeros((m, d)); aw = np.zeros((n, k))
    Cabs = np.abs(C.astype(np.float64))
    for rr, F, t, c in zip(rrs, Fr, targets, covs):
        G = OB.cosine_loss_grad(F, t, c, ncov)
        rows = np.arange(rr.coeff.shape[0])
        gC += OB.codebook_grad(rr.coeff, G)
        aC += OB.codebook_grad(np.abs(rr.coeff), np.abs(G))
        OB.coeff_grad(rr.weights, rows, ti, G @ C.astype(np.float64).T, gw)
        OB.coeff_grad(rr.weights, rows, ti, np.abs(G) @ Cabs.T, aw)
    _check_grad(dC.grad.cpu().numpy(), gC, aC, "dL/dC")
    _check_grad(dtv.grad.cpu().numpy(), gw, aw, "dL/dw_hat")


def test_backward_workload_size_sampled_gaussians():
    """200,000 Gaussians, Top-8 over M=256, codebook 256x512, 8 views 512x384 (the
    backward workload); sum-of-(1 - cos) loss so the pixel count does not enter;
    dL/dw_hat checked on 500 Gaussians against the oracle restricted to their
    footprints (exact for those rows)."""
    require_gpu()
    n, m, d, k = 200_000, 256, 512, 8
    g = sg.make_gaussians(1003, n, (5.0, 5.0, 2.0), -4.5, 0.5, False, "beta")
    cams = sg.orbit_cameras(1004, 8, 12.0, 0.0, 4.0, 0.0, 0.0, 512, 384, 60.0, jitter=False)
    ti, tv = sg.random_topk(1005, n, m, k)
    C = sg.random_codebook(1006, m, d)
    dg = P.gaussians_to_device(g)
    dti = torch.from_numpy(ti).cuda()
    dtv = torch.from_numpy(tv).cuda().requires_grad_(True)
    dC = torch.from_numpy(C).cuda().requires_grad_(True)
    targets = [sg.random_unit_vectors(2000 + v, 512 * 384, d) for v in range(8)]
    Fs, tfs = [], []
    for cam in cams:
        F, tf = P.render_decode(dg, dti, dtv, dC, cam)
        Fs.append(F); tfs.append(tf)
    tt = [torch.from_numpy(t).cuda().reshape(384, 512, d) for t in targets]
    loss = _loss_torch(Fs, tfs, tt, sum_loss=True)
    loss.backward()
    gw_gpu = dtv.grad.cpu().numpy()
    # pick 500 Gaussians with a non-zero gradient, oracle on their footprints
    rng = np.random.default_rng(7)
    cand = np.flatnonzero(np.abs(gw_gpu).sum(1) > 0)
    rows = rng.choice(cand, 500, replace=False)
    from oracle import project as OP
    gw = np.zeros((500, k))
    aw = np.zeros((500, k))
    row_of = -np.ones(n, np.int64); row_of[rows] = np.arange(500)
    for cam, t in zip(cams, targets):
        proj = OP.project(g, cam)
        mask = np.zeros(cam.width * cam.height, bool)
        for i in rows:
            if proj.visible[i]:
                x0, x1, y0, y1 = proj.box[i]
                yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
                mask[(yy * cam.width + xx).ravel()] = True
        rr = OR.render_coeff(g, ti, tv, cam, m, pixel_mask=mask)
        F = OR.decode(rr.coeff, C)
        cov = rr.t_final < 1.0
        G = OB.cosine_loss_grad(F, t[rr.pixels], cov, 1)
        dW = G @ C.astype(np.float64).T
        prow = -np.ones(cam.width * cam.height, np.int64); prow[rr.pixels] = np.arange(rr.pixels.shape[0])
        w = rr.weights
        sel = row_of[w.gauss] >= 0
        sub = type(w)(row_of[w.gauss[sel]], w.pixel[sel], w.e[sel], w.t_final, {})
        OB.coeff_grad(sub, prow, ti[rows], dW, gw)
        OB.coeff_grad(sub, prow, ti[rows], np.abs(G) @ np.abs(C.astype(np.float64)).T, aw)
    _check_grad(gw_gpu[rows], gw, aw, "dL/dw_hat (500 sampled Gaussians, 8 views 512x384)")
