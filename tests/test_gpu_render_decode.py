"""GPU parity of the sparse coefficient render (Eq. 7) and the codebook decode (Eq. 8).

Tolerances:
* FP32 coefficient map, per pixel: ||dW||_1 <= 1e-5 ||W_ref||_1 + amb(p) + 1e-9,
  amb(p) the oracle's ambiguity mass of the pixel (|weight change| of its
  marginal decisions; every w_hat sums to one, so it bounds the L1 change);
* BF16 / FP8 maps: elementwise within the format's rounding (2^-8 / 2^-3 relative,
  plus the smallest subnormal for FP8) of the FP32 result;
* decode on seeded float32 inputs: FP32 within 1e-5 relative of the FP64 product
  (row norm), BF16 and FP8 cosine error 1 - cos <= 2e-2 per pixel;
* render + decode end to end: cosine error against the FP64 oracle <= 2e-2 (BF16),
  1e-5 (FP32); statistics printed for FP8.
"""
import numpy as np
import pytest
import torch

import paper_2605_13600_amd as P
import scenegen as sg
from oracle import composite as OC
from oracle import render as OR
from tests import _scenes as S
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu


def _amb_per_pixel(rr, width, height):
    amb = np.zeros(width * height)
    for pix, gi, delta, _ in OC.ambiguity(rr.weights.marginal):
        amb[pix] += delta.sum()
    return amb


def _render_scene(n=20_000, res=(200, 150), m=64, k=4, seed=3):
    g = sg.make_gaussians(seed, n, (5.0, 5.0, 2.0), -3.6, 0.5, False, "beta")
    cams = sg.orbit_cameras(seed + 1, 2, 12.0, 1.0, 4.0, 1.0, 0.5, res[0], res[1], 60.0)
    ti, tv = sg.random_topk(seed + 2, n, m, k)
    return g, cams, ti, tv


@pytest.mark.parametrize("res,m,k", [((200, 150), 64, 4), ((203, 77), 256, 8), ((64, 48), 512, 16)])
def test_render_fp32_matches_oracle(res, m, k):
    require_gpu()
    g, cams, ti, tv = _render_scene(res=res, m=m, k=k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    for cam in cams:
        W, tf, nc, _ = P.render_coeff(dg, dti, dtv, cam, m, dtype="f32")
        torch.cuda.synchronize()
        rr = OR.render_coeff(g, ti, tv, cam, m, track_marginal=True)
        amb = _amb_per_pixel(rr, cam.width, cam.height)
        got = W.cpu().numpy().reshape(-1, m).astype(np.float64)
        err = np.abs(got - rr.coeff).sum(1)
        ref = np.abs(rr.coeff).sum(1)
        assert (err <= 1e-5 * ref + amb + 1e-9).all(), float((err - 1e-5 * ref - amb).max())
        # final transmittance; a marginal decision (see the oracle) may change it
        ok = np.ones(rr.t_final.shape[0], bool)
        ok[list(rr.weights.marginal.keys())] = False
        assert np.allclose(tf.cpu().numpy().reshape(-1)[ok], rr.t_final[ok], rtol=2e-5, atol=1e-7)
        slack = sum(s for *_, s in OC.ambiguity(rr.weights.marginal))
        assert abs(nc - rr.weights.n_contrib) <= slack
        print(f"[render {res} M={m}] contrib={nc} max L1 rel err={float((err / np.maximum(ref, 1e-30)).max()):.3g}")


def test_render_low_precision_outputs():
    require_gpu()
    g, cams, ti, tv = _render_scene(res=(160, 120), m=256, k=8)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    f32, _, _, _ = P.render_coeff(dg, dti, dtv, cams[0], 256, dtype="f32")
    b16, _, _, _ = P.render_coeff(dg, dti, dtv, cams[0], 256, dtype="bf16")
    f8, _, _, sc = P.render_coeff(dg, dti, dtv, cams[0], 256, dtype="fp8")
    a = f32.cpu().numpy().astype(np.float64)
    b = b16.float().cpu().numpy().astype(np.float64)
    assert (np.abs(b - a) <= 2.0 ** -8 * np.abs(a) + 1e-30).all()
    c = f8.view(torch.float8_e4m3fn).float().cpu().numpy().astype(np.float64) / sc
    assert (np.abs(c - a) <= 2.0 ** -3 * np.abs(a) + 2.0 ** -9 / sc).all()
    # the map's FP8 bytes are the OCP E4M3 rounding (nearest even) of the float32
    # rows times the power-of-two scale, bit for bit: torch's CPU conversion
    ref8 = (f32.cpu() * sc).to(torch.float8_e4m3fn).view(torch.uint8)
    assert sc == 256.0 and torch.equal(f8.cpu().view(torch.uint8), ref8)


def _cos_err(F, R, mask=None):
    F = np.asarray(F, np.float64); R = np.asarray(R, np.float64)
    nf, nr = np.linalg.norm(F, axis=1), np.linalg.norm(R, axis=1)
    ok = (nr > 0) if mask is None else mask
    return 1.0 - (F[ok] * R[ok]).sum(1) / (nf[ok] * nr[ok])


@pytest.mark.parametrize("m,d", [(64, 512), (100, 512), (256, 512), (512, 512), (256, 128), (256, 1024)])
def test_decode_against_fp64(m, d):
    require_gpu()
    rng = np.random.default_rng(m + d)
    Pn = 1000 + 77
    A = rng.random((Pn, m)).astype(np.float32)
    A *= (rng.random((Pn, m)) < 0.1)                     # sparse-ish rows like rendered maps
    A[:5] = 0
    C = sg.random_codebook(m, m, d)
    ref = A.astype(np.float64) @ C.astype(np.float64)
    Ct = torch.from_numpy(C).cuda()
    At = torch.from_numpy(A).cuda()
    F32 = P.decode(At, Ct, "f32", out_dtype="f32").cpu().numpy()
    rn = np.linalg.norm(ref, axis=1, keepdims=True)
    assert (np.abs(F32 - ref) <= 1e-5 * rn + 1e-12).all()
    F16 = P.decode(At.to(torch.bfloat16), Ct, "bf16", out_dtype="bf16").float().cpu().numpy()
    e16 = _cos_err(F16, ref)
    q8 = torch.from_numpy(A * 256.0).cuda().to(torch.float8_e4m3fn).view(torch.uint8)
    F8 = P.decode(q8, Ct, "fp8", coeff_scale=256.0, out_dtype="f32").cpu().numpy()
    e8 = _cos_err(F8, ref)
    print(f"[decode M={m} D={d}] cos err bf16 max {e16.max():.2e} fp8 max {e8.max():.2e} mean {e8.mean():.2e}")
    assert e16.max() <= 2e-2 and e8.max() <= 2e-2
    assert np.abs(F16[:5]).max() == 0 and np.abs(F8[:5]).max() == 0


def test_render_decode_end_to_end_scene_rows():
    """The 1M-Gaussian scene's Gaussians with synthetic Top-8 over M=256, codebook
    256x512, one 1440x1080 view; 3000 sampled pixels against the FP64 oracle."""
    require_gpu()
    sc = sg.make_scene("scene", n_views=1)
    g = sc.gaussians
    cam = sg.orbit_cameras(77, 100, 12.0, 1.0, 4.0, 1.0, 0.5, 1440, 1080, 60.0)[0]
    ti, tv = sg.random_topk(11, g.n, 256, 8)
    C = sg.random_codebook(12, 256, 512)
    dg = P.gaussians_to_device(g)
    dti, dtv, Ct = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda(), torch.from_numpy(C).cuda()
    pix = np.random.default_rng(0).choice(1440 * 1080, 3000, replace=False)
    mask = np.zeros(1440 * 1080, bool); mask[pix] = True
    rr = OR.render_coeff(g, ti, tv, cam, 256, pixel_mask=mask)
    Fref = OR.decode(rr.coeff, C)
    cov = rr.t_final < 1.0
    stats = {}
    for dt in ("f32", "bf16", "fp8"):
        W, tf, nc, scl = P.render_coeff(dg, dti, dtv, cam, 256, dtype=dt)
        F = P.decode(W, Ct, dt, coeff_scale=scl, out_dtype="f32" if dt == "f32" else "bf16")
        Fs = F.reshape(-1, 512)[torch.from_numpy(rr.pixels).cuda()].float().cpu().numpy()
        e = _cos_err(Fs, Fref, cov)
        stats[dt] = (float(e.max()), float(np.percentile(e, 99)), float(e.mean()))
    print(f"[render+decode 1440x1080] contrib={nc} covered={int(cov.sum())} cos err (max,p99,mean) {stats}")
    assert stats["f32"][0] <= 1e-5
    assert stats["bf16"][0] <= 2e-2
    assert stats["fp8"][0] <= 2e-2


@pytest.mark.parametrize("res,m,k,d", [((203, 77), 256, 8, 512), ((70, 45), 100, 5, 200), ((64, 48), 512, 16, 1024),
                                       ((33, 17), 64, 4, 128)])
def test_fused_render_equals_render_then_decode(res, m, k, d):
    """scoup_render (Eq. 7 then Eq. 8 in one kernel, rows kept on chip) against
    scoup_decode of the scoup_render_coeff map of the same precision.  With the
    float32 map requested (the backward's path) the rows are summed exactly as
    for the map: features, map and final transmittance bit for bit, in F32,
    BF16 and FP8.  Without it, BF16 / FP8 rows are accumulated on MFMA from
    bfloat16 products: cosine error against the same reference <= 1e-4 (BF16:
    a bfloat16 rounding of each term) or 1e-2 (FP8), inside the 2e-2 bar, and
    a second call gives the same bits."""
    require_gpu()
    g, cams, ti, tv = _render_scene(n=8_000, res=res, m=m, k=k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    Ct = torch.from_numpy(sg.random_codebook(5, m, d)).cuda()
    cam = cams[0]
    W32, tf_ref, nc_ref, _ = P.render_coeff(dg, dti, dtv, cam, m, dtype="f32")
    for dt in ("f32", "bf16", "fp8"):
        for out in ("f32", "bf16"):
            F, Wf, tf, nc = P.render(dg, dti, dtv, Ct, cam, in_dtype=dt, out_dtype=out, want_coeff=True)
            F2, _, _, _ = P.render(dg, dti, dtv, Ct, cam, in_dtype=dt, out_dtype=out)
            Wm, _, _, scl = P.render_coeff(dg, dti, dtv, cam, m, dtype=dt)
            Fref = P.decode(Wm, Ct, dt, coeff_scale=scl, out_dtype=out)
            torch.cuda.synchronize()
            iv = (lambda t: t.view(torch.int16)) if out == "bf16" else (lambda t: t.view(torch.int32))
            assert torch.equal(iv(F), iv(Fref)), (dt, out, float((F.float() - Fref.float()).abs().max()))
            F3, _, _, _ = P.render(dg, dti, dtv, Ct, cam, in_dtype=dt, out_dtype=out)
            torch.cuda.synchronize()
            assert torch.equal(iv(F2), iv(F3)), (dt, out)
            if dt == "f32":
                assert torch.equal(iv(F), iv(F2)), (dt, out)
            else:
                a_ = F2.reshape(-1, d).double().cpu().numpy()
                b_ = Fref.reshape(-1, d).double().cpu().numpy()
                nz = np.linalg.norm(b_, axis=1) > 0
                assert (np.abs(a_[~nz]) == 0).all()
                e = _cos_err(a_[nz], b_[nz])
                # BF16: one bfloat16 rounding per term; FP8: the rows' E4M3 rounding may land
                # on the neighbouring code (3 mantissa bits) for entries that moved by it
                assert e.max() <= (1e-4 if dt == "bf16" else 1e-2), (dt, out, float(e.max()))
            assert torch.equal(Wf.view(torch.int32), W32.view(torch.int32))
            assert torch.equal(tf, tf_ref) and nc == nc_ref
    print(f"[fused render {res} M={m} K={k} D={d}] contrib={nc_ref}: features equal render + decode")


def test_fused_render_full_view_against_oracle():
    """The 1M-Gaussian scene's Gaussians, synthetic Top-8 over M=256, codebook
    256x512, one 1440x1080 view rendered and decoded in one pass; 3000 sampled
    pixels against the FP64 oracle: cosine error <= 1e-5 (FP32), <= 2e-2
    (BF16, FP8)."""
    require_gpu()
    sc = sg.make_scene("scene", n_views=1)
    g = sc.gaussians
    cam = sg.orbit_cameras(78, 100, 12.0, 1.0, 4.0, 1.0, 0.5, 1440, 1080, 60.0)[0]
    ti, tv = sg.random_topk(13, g.n, 256, 8)
    C = sg.random_codebook(14, 256, 512)
    dg = P.gaussians_to_device(g)
    dti, dtv, Ct = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda(), torch.from_numpy(C).cuda()
    pix = np.random.default_rng(1).choice(1440 * 1080, 3000, replace=False)
    mask = np.zeros(1440 * 1080, bool); mask[pix] = True
    rr = OR.render_coeff(g, ti, tv, cam, 256, pixel_mask=mask)
    Fref = OR.decode(rr.coeff, C)
    cov = rr.t_final < 1.0
    stats = {}
    for dt in ("f32", "bf16", "fp8"):
        F, _, tf, nc = P.render(dg, dti, dtv, Ct, cam, in_dtype=dt, out_dtype="f32" if dt == "f32" else "bf16")
        Fs = F.reshape(-1, 512)[torch.from_numpy(rr.pixels).cuda()].float().cpu().numpy()
        e = _cos_err(Fs, Fref, cov)
        stats[dt] = (float(e.max()), float(np.percentile(e, 99)), float(e.mean()))
        assert np.abs(Fs[~cov]).max() == 0 if (~cov).any() else True
    print(f"[fused render 1440x1080] contrib={nc} covered={int(cov.sum())} cos err (max,p99,mean) {stats}")
    assert stats["f32"][0] <= 1e-5
    assert stats["bf16"][0] <= 2e-2
    assert stats["fp8"][0] <= 2e-2


@pytest.mark.parametrize("res,m,k,d", [((203, 77), 256, 8, 512), ((70, 45), 100, 5, 200)])
def test_render_views_equal_single_view_renders(res, m, k, d):
    """scoup_render_views (views in flight, each lane with its own binning
    buffers) against scoup_render on each camera: six views (more than the
    four lanes, so lanes are reused), every decode and output precision, bit
    for bit, with four, three and one views in flight; contributions summed
    over the views."""
    require_gpu()
    n = 8_000
    g = sg.make_gaussians(11, n, (5.0, 5.0, 2.0), -3.6, 0.5, False, "beta")
    cams = sg.orbit_cameras(12, 6, 12.0, 1.0, 4.0, 1.0, 0.5, res[0], res[1], 60.0)
    ti, tv = sg.random_topk(13, n, m, k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    Ct = torch.from_numpy(sg.random_codebook(14, m, d)).cuda()
    old = P.views_in_flight()
    try:
        for dt in ("f32", "bf16", "fp8"):
            for out in ("f32", "bf16"):
                iv = (lambda t: t.view(torch.int16)) if out == "bf16" else (lambda t: t.view(torch.int32))
                refs, nc_sum = [], 0
                for cam in cams:
                    F, _, _, nc = P.render(dg, dti, dtv, Ct, cam, in_dtype=dt, out_dtype=out, want_t_final=False)
                    refs.append(F)
                    nc_sum += nc
                for lanes in (4, 3, 1):
                    P.set_views_in_flight(lanes)
                    Fv, ncv = P.render_views(dg, dti, dtv, Ct, cams, in_dtype=dt, out_dtype=out)
                    torch.cuda.synchronize()
                    assert Fv.shape == (len(cams), res[1], res[0], d)
                    for v, F in enumerate(refs):
                        assert torch.equal(iv(Fv[v]), iv(F)), (dt, out, lanes, v)
                    assert ncv == nc_sum, (dt, out, lanes)
    finally:
        P.set_views_in_flight(old)
    print(f"[render views {res} M={m} K={k} D={d}] 6 views equal single-view renders")


def test_render_views_edge_cases():
    """No views: an empty result.  Cameras of different image sizes: an
    argument error.  A pair capacity below what a view needs: the workspace
    error, and the binding's retry gives the single-view results."""
    require_gpu()
    n, m, k, d = 6_000, 64, 4, 128
    g = sg.make_gaussians(21, n, (5.0, 5.0, 2.0), -3.6, 0.5, False, "beta")
    cams = sg.orbit_cameras(22, 3, 12.0, 1.0, 4.0, 1.0, 0.5, 96, 64, 60.0)
    other = sg.orbit_cameras(23, 1, 12.0, 1.0, 4.0, 1.0, 0.5, 80, 64, 60.0)
    ti, tv = sg.random_topk(24, n, m, k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    Ct = torch.from_numpy(sg.random_codebook(25, m, d)).cuda()
    F0, nc0 = P.render_views(dg, dti, dtv, Ct, [])
    assert F0.shape[0] == 0 and nc0 == 0
    with pytest.raises(P.ScoupError):
        P.render_views(dg, dti, dtv, Ct, list(cams) + list(other))
    from paper_2605_13600_amd import api as A
    A._capacity_cache.pop(("render", n, 96, 64), None)
    Fv, ncv = P.render_views(dg, dti, dtv, Ct, cams, workspace=A.Workspace(dg.means.device), pair_capacity=64)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        F, _, _, _ = P.render(dg, dti, dtv, Ct, cam, want_t_final=False)
        assert torch.equal(Fv[v].view(torch.int16), F.view(torch.int16)), v
