"""GPU backward of render + decode against the FP64 oracle's gradient.

Tolerance (written here), per entry of dL/dw_hat (N, K) and dL/dC (M, D):
    |g_gpu - g_ref| <= C_SUM u A,   u = 2^-24 (float32 unit roundoff)
where A is the same sum taken over the absolute values of its terms.  Every
term of these sums is formed from float32 inputs (the rendered coefficients,
the transmittance products behind e, the decoded features and the loss
gradient), so each carries a relative error of a few u and the sum an error
of order u A however it is added up; the entries of a gradient cancel to far
below A, so a bar relative to |g| alone cannot be met by float32 arithmetic.
The relative figure err / max(|g|, 1e-3 |g|_inf) is printed for each check.
A missing, doubled or mis-indexed term moves an entry by about A / (number of
terms), orders of magnitude above C_SUM u A at these sizes.  The oracle is
pinned against FP64 central finite differences in tests/test_oracle_pins.py.
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

C_SUM = 8.0         # bar, in units of u A
REL_FLOOR = 1e-3    # printed relative figure: err / max(|g|, 1e-3 |g|_inf)


def _check_grad(got, ref, absref, name):
    """Entry-wise: err <= C_SUM u A; prints the largest err / (u A) and the
    largest err / max(|g|, 1e-3 |g|_inf)."""
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    u = 2.0 ** -24
    c_obs = float((err / np.maximum(absref * u, 1e-300)).max())
    scale = np.maximum(np.abs(ref), REL_FLOOR * np.abs(ref).max())
    rel = float((err / scale).max())
    print(f"[{name}] max err / (u A) {c_obs:.3g} (bar {C_SUM:g}), max err / max(|g|, 1e-3 |g|inf) {rel:.3g}, "
          f"|ref|max {np.abs(ref).max():.3g}", flush=True)
    assert (err <= C_SUM * u * absref).all(), (name, c_obs)


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


def test_backward_workload_size():
    """200,000 Gaussians, Top-8 over M=256, codebook 256x512, 8 views 512x384 (the
    backward workload); sum-of-(1 - cos) loss so the pixel count does not enter.
    dL/dC is checked in full (the oracle renders and decodes every view) and
    dL/dw_hat on 500 sampled Gaussians with a non-zero gradient."""
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
    Fs, tfs, tt = [], [], []
    for v, cam in enumerate(cams):
        F, tf = P.render_decode(dg, dti, dtv, dC, cam)
        Fs.append(F); tfs.append(tf)
        tt.append(torch.from_numpy(sg.random_unit_vectors(2000 + v, 512 * 384, d)).cuda().reshape(384, 512, d))
    loss = _loss_torch(Fs, tfs, tt, sum_loss=True)
    loss.backward()
    del Fs, tt
    gw_gpu = dtv.grad.cpu().numpy()
    gC_gpu = dC.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    cand = np.flatnonzero(np.abs(gw_gpu).sum(1) > 0)
    rows = rng.choice(cand, 500, replace=False)
    row_of = -np.ones(n, np.int64); row_of[rows] = np.arange(500)
    C64 = C.astype(np.float64)
    gC = np.zeros((m, d)); aC = np.zeros((m, d))
    gw = np.zeros((500, k)); aw = np.zeros((500, k))
    for v, cam in enumerate(cams):
        rr = OR.render_coeff(g, ti, tv, cam, m)
        F = OR.decode(rr.coeff, C)
        cov = rr.t_final < 1.0
        G = OB.cosine_loss_grad(F, sg.random_unit_vectors(2000 + v, 512 * 384, d), cov, 1)
        del F
        gC += OB.codebook_grad(rr.coeff, G)
        aC += OB.codebook_grad(np.abs(rr.coeff), np.abs(G))
        w = rr.weights
        sel = row_of[w.gauss] >= 0
        sub = type(w)(row_of[w.gauss[sel]], w.pixel[sel], w.e[sel], w.t_final, {})
        prow = np.arange(cam.width * cam.height)
        OB.coeff_grad(sub, prow, ti[rows], G @ C64.T, gw)
        OB.coeff_grad(sub, prow, ti[rows], np.abs(G) @ np.abs(C64).T, aw)
        print(f"view {v} oracle done", flush=True)
    _check_grad(gC_gpu, gC, aC, "dL/dC (8 views 512x384)")
    _check_grad(gw_gpu[rows], gw, aw, "dL/dw_hat (500 sampled Gaussians, 8 views 512x384)")


def test_backward_is_deterministic_and_leaves_grads_on_overflow():
    """The same backward twice gives bit-identical gradients (fixed summation
    order); a call whose pair capacity is too small reports SCOUP_E_WORKSPACE
    and adds nothing to the gradient buffers."""
    require_gpu()
    import ctypes as C_
    from paper_2605_13600_amd import _lib as L
    n, m, d, k = 4000, 256, 512, 8
    g = sg.make_gaussians(31, n, (5.0, 5.0, 2.0), -3.4, 0.5, False, "beta")
    cam = sg.orbit_cameras(32, 1, 12.0, 0.0, 4.0, 0.0, 0.0, 128, 96, 60.0, jitter=False)[0]
    ti, tv = sg.random_topk(33, n, m, k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    dC = torch.from_numpy(sg.random_codebook(34, m, d)).cuda()
    W = P.render_coeff(dg, dti, dtv, cam, m, dtype="f32")[0]
    gen = torch.Generator(device="cuda").manual_seed(5)
    Gf = torch.randn((96 * 128, d), device="cuda", generator=gen)
    outs = []
    for _ in range(2):
        gw, gc = torch.zeros_like(dtv), torch.zeros_like(dC)
        P.render_backward(dg, dti, dtv, cam, W, dC, Gf, gw, gc)
        outs.append((gw.clone(), gc.clone()))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert float(outs[0][1].abs().max()) > 0 and float(outs[0][0].abs().max()) > 0
    lib = L.load()
    c = P.camera_struct(cam)
    gs = dg.struct()
    cap = 64
    nb = lib.scoup_render_backward_workspace_bytes(n, C_.byref(c), m, d, cap)
    buf = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gw, gc = torch.full_like(dtv, 3.0), torch.full_like(dC, 3.0)
    st = lib.scoup_render_backward(C_.byref(gs), dti.data_ptr(), dtv.data_ptr(), k, m, C_.byref(c), W.data_ptr(),
                                   dC.data_ptr(), d, Gf.data_ptr(), gw.data_ptr(), gc.data_ptr(), buf.data_ptr(),
                                   buf.numel(), None)
    torch.cuda.synchronize()
    assert st == L.E_WORKSPACE and lib.scoup_required_pair_capacity() > cap
    assert bool((gw == 3.0).all()) and bool((gc == 3.0).all())
