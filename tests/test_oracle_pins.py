"""Pins of the FP64 oracle against the paper's definitions and the mathematics.
# (golden opacities are decimal; inputs are float32, so comparisons allow the
# float32 rounding of the inputs, about 1e-7 relative)

None of these tests touches the GPU library.  Each pin is chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a wrong threshold) fails at least one of them; the
``test_planted_*`` tests plant such mistakes and check that a pin catches them.
"""
import json
import math
import os

import numpy as np
import pytest

import scenegen as sg
from oracle import backward as OB
from oracle import brute as BR
from oracle import composite as OC
from oracle import project as OP
from oracle import render as OR
from oracle import uplift as OU
from tests import _scenes as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _weights(g, cam):
    proj = OP.project(g, cam)
    return OC.composite_view(proj, cam.width, cam.height)


def _pixel_lists(vw, width):
    d = {}
    for gi, p, e in zip(vw.gauss, vw.pixel, vw.e):
        d.setdefault((int(p) % width, int(p) // width), []).append((int(gi), float(e)))
    return d


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("case", GOLD["single_gaussian_at_pixel_centre"]["cases"])
def test_single_gaussian_at_pixel_centre(case):
    cam = S.axis_camera()
    g = S.gaussians([[0, 0, 4.0]], -6.0, [case["o"]])
    vw = _weights(g, cam)
    lists = _pixel_lists(vw, cam.width)
    assert lists[(4, 4)] == [(0, pytest.approx(case["e"], rel=1e-7))]


@pytest.mark.parametrize("case", GOLD["two_gaussians_one_pixel"]["cases"])
def test_two_gaussians_one_pixel(case):
    cam = S.axis_camera()
    # ids deliberately in back-to-front storage order: depth decides, not id
    g = S.gaussians([[0, 0, 6.0], [0, 0, 3.0]], -6.0, [case["o_back"], case["o_front"]])
    vw = _weights(g, cam)
    lst = _pixel_lists(vw, cam.width)[(4, 4)]
    assert [i for i, _ in lst] == [1, 0]
    assert lst[0][1] == pytest.approx(case["e_front"], rel=2e-7)
    assert lst[1][1] == pytest.approx(case["e_back"], rel=2e-7)
    assert vw.t_final[4 * cam.width + 4] == pytest.approx(case["t_final"], rel=1e-6)


def test_saturation_stop():
    case = GOLD["saturation_stop"]["cases"][0]
    cam = S.axis_camera()
    g = S.gaussians([[0, 0, 3.0], [0, 0, 4.0], [0, 0, 5.0]], -6.0, case["o"])
    lst = dict(_pixel_lists(_weights(g, cam), cam.width)[(4, 4)])
    got = [lst.get(i, 0.0) for i in range(3)]
    assert got == pytest.approx(case["e"], rel=1e-6, abs=1e-12)


def test_isotropic_on_axis_closed_form():
    f, z, s, o = 40.0, 5.0, 0.2, 0.7
    cam = S.axis_camera(21, 21, f)
    g = S.gaussians([[0, 0, z]], math.log(s), [o])
    lists = _pixel_lists(_weights(g, cam), cam.width)
    # the closed form takes the float32-rounded inputs the oracle sees
    o, z, f = float(np.float32(o)), float(np.float32(z)), float(np.float32(f))
    s = math.exp(float(np.float32(math.log(s))))
    checked = 0
    for (px, py), lst in lists.items():
        d = math.hypot(px + 0.5 - 10.5, py + 0.5 - 10.5)
        want = OP.isotropic_on_axis_alpha(o, s, z, f, d)
        assert lst[0][1] == pytest.approx(want, rel=1e-13), (px, py)
        checked += 1
    # every pixel where the closed form reaches 1/255 is present, and no other
    want_n = sum(1 for px in range(21) for py in range(21)
                 if OP.isotropic_on_axis_alpha(o, s, z, f, math.hypot(px - 10, py - 10)) >= 1 / 255)
    assert checked == want_n > 20


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed,iso,holes", [(1, True, 0), (2, False, 0), (3, False, 1)])
def test_brute_force_matches_oracle(seed, iso, holes):
    g, views = S.small_scene(seed, n=50, iso=iso, holes=holes)
    res = OU.uplift_accumulate(g, views)
    ref = np.zeros_like(res.acc)
    for (i, j), w in BR.uplift(g, views).items():
        ref[i, j] = w
    assert np.abs(ref - res.acc).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.count_nonzero(ref) == np.count_nonzero(res.acc)
    # per-pixel lists and final transmittance
    cam = views.cameras[0]
    pw = BR.pixel_weights(g, cam)
    vw = _weights(g, cam)
    lists = _pixel_lists(vw, cam.width)
    for (px, py), (lst, T) in pw.items():
        got = lists.get((px, py), [])
        assert [i for i, _ in got] == [i for i, _ in lst]
        assert np.allclose([e for _, e in got], [e for _, e in lst], rtol=1e-13, atol=0)
        assert vw.t_final[py * cam.width + px] == pytest.approx(T, rel=1e-13)


def test_brute_force_tiny_workload_subset():
    sc = sg.make_scene("tiny", n_gaussians=300, res=(32, 24))
    res = OU.uplift_accumulate(sc.gaussians, sc.views)
    ref = np.zeros_like(res.acc)
    for (i, j), w in BR.uplift(sc.gaussians, sc.views).items():
        ref[i, j] = w
    assert np.abs(ref - res.acc).max() <= 1e-13
    assert res.n_contrib > 1000


@pytest.mark.parametrize("seed", [3, 4])
def test_region_touches_brute_force_and_closed_forms(seed):
    g, views = S.small_scene(seed, n=60, holes=1)
    got = OU.region_touches(g, views)
    for v, cam in enumerate(views.cameras):
        rmap = views.region_maps[v]
        pairs = set()
        for (px, py), (lst, _) in BR.pixel_weights(g, cam).items():
            r = int(rmap[py, px])
            if r >= 0:
                pairs.update((i, r) for i, e in lst if e > 0)
        assert got[v] == len(pairs)
    cam = views.cameras[0]
    vw = _weights(g, cam)
    one = sg.Views([cam], [np.zeros((cam.height, cam.width), np.int32)], np.array([0, 1], np.int64),
                   views.code_idx[:1], views.code_val[:1], views.m_atoms)
    assert OU.region_touches(g, one)[0] == np.unique(vw.gauss[vw.e > 0]).shape[0]
    per = np.arange(cam.width * cam.height, dtype=np.int32).reshape(cam.height, cam.width)
    codes_i = np.zeros((per.size, views.code_idx.shape[1]), np.int32)
    codes_v = np.zeros((per.size, views.code_idx.shape[1]), np.float32)
    each = sg.Views([cam], [per], np.array([0, per.size], np.int64), codes_i, codes_v, views.m_atoms)
    assert OU.region_touches(g, each)[0] == int((vw.e > 0).sum())


# ---------------------------------------------------------------- invariants
def test_weights_sum_to_one_minus_transmittance():
    sc = sg.make_scene("tiny")
    for cam in sc.views.cameras:
        vw = _weights(sc.gaussians, cam)
        s = np.bincount(vw.pixel, weights=vw.e, minlength=cam.width * cam.height)
        assert np.allclose(s, 1.0 - vw.t_final, atol=1e-13)
        assert vw.t_final.min() >= 1e-4
        assert s.max() <= 1.0 - 1e-4 + 1e-15


def test_row_sum_equals_total_weight():
    sc = sg.make_scene("tiny")
    res = OU.uplift_accumulate(sc.gaussians, sc.views)
    z = np.zeros(sc.gaussians.n)
    zc = np.zeros(sc.gaussians.n)
    csum = sc.views.code_val.astype(np.float64).sum(1)   # 1 up to float32 rounding
    for v, cam in enumerate(sc.views.cameras):
        vw = _weights(sc.gaussians, cam)
        reg = sc.views.region_maps[v].reshape(-1)[vw.pixel] + sc.views.region_base[v]
        z += np.bincount(vw.gauss, weights=vw.e, minlength=sc.gaussians.n)
        zc += np.bincount(vw.gauss, weights=vw.e * csum[reg], minlength=sc.gaussians.n)
    assert np.allclose(res.acc.sum(1), zc, rtol=1e-12, atol=1e-15)
    assert np.allclose(res.acc.sum(1), z, rtol=1e-6)
    assert (z > 0).sum() > 1000


def test_linear_in_codes_and_additive_over_views():
    sc = sg.make_scene("tiny")
    v = sc.views
    rng = np.random.default_rng(5)
    val2 = rng.random(v.code_val.shape).astype(np.float32)
    v2 = sg.Views(v.cameras, v.region_maps, v.region_base, v.code_idx, val2, v.m_atoms)
    a, b = 0.75, -1.25
    v3 = sg.Views(v.cameras, v.region_maps, v.region_base, v.code_idx,
                  (a * v.code_val.astype(np.float64) + b * val2.astype(np.float64)), v.m_atoms)
    r1 = OU.uplift_accumulate(sc.gaussians, v).acc
    r2 = OU.uplift_accumulate(sc.gaussians, v2).acc
    r3 = OU.uplift_accumulate(sc.gaussians, v3).acc
    assert np.allclose(r3, a * r1 + b * r2, atol=1e-12)
    ra = OU.uplift_accumulate(sc.gaussians, v, view_ids=[0, 1]).acc
    rb = OU.uplift_accumulate(sc.gaussians, v, view_ids=[2, 3]).acc
    assert np.allclose(ra + rb, r1, atol=1e-13)
    sub = sg.subset_views(v, [2, 3])
    assert np.allclose(OU.uplift_accumulate(sc.gaussians, sub).acc, rb, atol=0)


def test_one_hot_codes_give_region_weight_sums():
    g, views = S.small_scene(11, n=60, m=4, k=1, sites=4)
    # code of region r of every view = atom r, value 1
    idx = np.zeros_like(views.code_idx); val = np.ones_like(views.code_val)
    for v in range(views.n_views):
        lo, hi = views.region_base[v], views.region_base[v + 1]
        idx[lo:hi, 0] = np.arange(hi - lo)
    vv = sg.Views(views.cameras, views.region_maps, views.region_base, idx, val, 4)
    acc = OU.uplift_accumulate(g, vv).acc
    want = np.zeros_like(acc)
    for v in range(vv.n_views):
        for (px, py), (lst, _) in BR.pixel_weights(g, vv.cameras[v]).items():
            r = vv.region_maps[v][py, px]
            for i, e in lst:
                want[i, r] += e
    assert np.allclose(acc, want, atol=1e-13)


def test_uniform_code_uplifts_to_itself():
    sc = sg.make_scene("tiny")
    v = sc.views
    c_idx = np.array([5, 17, 40, 63], np.int32)
    c_val = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    vv = sg.Views(v.cameras, v.region_maps, v.region_base,
                  np.tile(c_idx, (v.code_idx.shape[0], 1)),
                  np.tile(c_val, (v.code_val.shape[0], 1)), v.m_atoms)
    idx, val, res = OU.uplift(sc.gaussians, vv, 4)
    touched = res.acc.sum(1) > 0
    assert touched.sum() > 1000
    assert (idx[touched] == np.array([63, 40, 17, 5])).all()
    assert np.allclose(val[touched], np.array([0.4, 0.3, 0.2, 0.1], np.float64)
                       * (1.0 / c_val.astype(np.float64).sum()), rtol=1e-6)
    assert (idx[~touched] == -1).all() and (val[~touched] == 0).all()


def test_dense_feature_uplift_equivalence():
    """Eq. 3 with F = W C equals (acc_i / Z_i) C: the untruncated sparse uplift is lossless."""
    g, views = S.small_scene(21, n=50, m=8, k=3)
    C = sg.random_codebook(3, 8, 6).astype(np.float64)
    acc = OU.uplift_accumulate(g, views).acc
    dense = np.zeros((g.n, 6)); Z = np.zeros(g.n)
    for v in range(views.n_views):
        cam = views.cameras[v]
        for (px, py), (lst, _) in BR.pixel_weights(g, cam).items():
            r = views.region_maps[v][py, px]
            gg = views.region_base[v] + r
            Wp = np.zeros(8)
            Wp[views.code_idx[gg]] = views.code_val[gg]
            F = Wp @ C
            for i, e in lst:
                dense[i] += e * F; Z[i] += e
    t = Z > 0
    assert np.allclose(acc[t] / Z[t, None] @ C, dense[t] / Z[t, None], atol=1e-12)


# ---------------------------------------------------------------- Top-K
@pytest.mark.parametrize("case", GOLD["topk_ties"]["cases"])
def test_topk_golden(case):
    idx, val = OU.topk_rows(np.array([case["row"]]), case["k"])
    assert idx[0].tolist() == case["idx"]
    assert val[0] == pytest.approx(np.array(case["val"]) / max(1e-300, sum(case["val"]) or 1.0)
                                   if sum(case["val"]) else case["val"])


def test_topk_matches_full_sort_and_selection():
    rng = np.random.default_rng(0)
    A = rng.integers(0, 6, size=(300, 24)).astype(np.float64)   # many exact ties and zeros
    A[rng.random(A.shape) < 0.3] = 0
    for k in (1, 4, 8, 30):
        idx, val = OU.topk_rows(A, k)
        for r in range(A.shape[0]):
            srt = sorted(range(24), key=lambda j: (-A[r, j], j))
            pos = [j for j in srt if A[r, j] > 0][:k]
            bi, bv = BR.topk(list(A[r]), k)
            assert idx[r, :len(pos)].tolist() == pos == [j for j in bi if j >= 0]
            assert (idx[r, len(pos):] == -1).all()
            assert np.allclose(val[r], bv, atol=1e-15)


# ---------------------------------------------------------------- render
def test_render_invariants_and_brute():
    g, views = S.small_scene(31, n=50, m=8, k=3)
    cam = views.cameras[1]
    ti, tv = sg.random_topk(4, g.n, 8, 3)
    rr = OR.render_coeff(g, ti, tv, cam, 8)
    assert np.allclose(rr.coeff.sum(1), 1.0 - rr.t_final, atol=1e-12)
    ref = BR.render(g, ti, tv, cam, 8)
    for (px, py), row in ref.items():
        assert np.allclose(rr.coeff[py * cam.width + px], row, atol=1e-14)
    # every Gaussian carrying the same vector c renders (1 - T) c, decodes parallel to c C
    c = np.array([0.5, 0.3, 0.2])
    ti2 = np.tile(np.array([1, 4, 6], np.int32), (g.n, 1)); tv2 = np.tile(c.astype(np.float32), (g.n, 1))
    rr2 = OR.render_coeff(g, ti2, tv2, cam, 8)
    cv = np.zeros(8); cv[[1, 4, 6]] = tv2[0]
    assert np.allclose(rr2.coeff, (1.0 - rr2.t_final)[:, None] * cv[None], atol=1e-13)
    C = sg.random_codebook(9, 8, 16)
    F = OR.decode(rr2.coeff, C)
    cov = rr2.t_final < 1.0
    ref_dir = cv @ C.astype(np.float64)
    cos = F[cov] @ ref_dir / (np.linalg.norm(F[cov], axis=1) * np.linalg.norm(ref_dir))
    assert np.allclose(cos, 1.0, atol=1e-12)
    # one-hot coefficient rows decode to codebook rows
    assert np.allclose(OR.decode(np.eye(8), C), C.astype(np.float64), atol=0)


# ---------------------------------------------------------------- backward
def _loss_of(g, ti, tv, C, cams, targets):
    tot, covs, Fs = 0.0, [], []
    for cam, t in zip(cams, targets):
        rr = OR.render_coeff(g, ti, tv, cam, C.shape[0])
        F = OR.decode(rr.coeff, C)
        cov = rr.t_final < 1.0
        covs.append(cov); Fs.append((rr, F))
    ncov = sum(int(c.sum()) for c in covs)
    for (rr, F), cov, t in zip(Fs, covs, targets):
        tot += OB.cosine_loss(F, t, cov, ncov)
    return tot, Fs, covs, ncov


def test_backward_matches_finite_differences():
    g, views = S.small_scene(41, n=30, res=(12, 10), m=6, k=3)
    cams = views.cameras
    ti, tv = sg.random_topk(5, g.n, 6, 3)
    tv = tv.astype(np.float64)
    C = sg.random_codebook(6, 6, 5).astype(np.float64)
    targets = [sg.random_unit_vectors(7 + v, c.width * c.height, 5).astype(np.float64)
               for v, c in enumerate(cams)]
    L, Fs, covs, ncov = _loss_of(g, ti, tv, C, cams, targets)
    dC = np.zeros_like(C); dw = np.zeros_like(tv)
    for (rr, F), cov, t in zip(Fs, covs, targets):
        G = OB.cosine_loss_grad(F, t, cov, ncov)
        dC += OB.codebook_grad(rr.coeff, G)
        dW = G @ C.T
        row = np.arange(rr.coeff.shape[0])
        OB.coeff_grad(rr.weights, row, ti, dW, dw)
        # adjoint identity <G, dX C> = <G C^T, dX>
        dX = np.random.default_rng(1).normal(size=rr.coeff.shape)
        assert np.vdot(G, dX @ C) == pytest.approx(np.vdot(G @ C.T, dX), rel=1e-12)
    h = 1e-4
    rng = np.random.default_rng(3)
    for _ in range(12):
        i, k = int(rng.integers(g.n)), int(rng.integers(3))
        tp = tv.copy(); tp[i, k] += h
        tm = tv.copy(); tm[i, k] -= h
        fd = (_loss_of(g, ti, tp, C, cams, targets)[0] - _loss_of(g, ti, tm, C, cams, targets)[0]) / (2 * h)
        assert fd == pytest.approx(dw[i, k], rel=1e-6, abs=1e-10)
    for _ in range(8):
        m, d = int(rng.integers(6)), int(rng.integers(5))
        Cp = C.copy(); Cp[m, d] += h
        Cm = C.copy(); Cm[m, d] -= h
        fd = (_loss_of(g, ti, tv, Cp, cams, targets)[0] - _loss_of(g, ti, tv, Cm, cams, targets)[0]) / (2 * h)
        assert fd == pytest.approx(dC[m, d], rel=1e-6, abs=1e-10)
    assert np.abs(dw).max() > 1e-4


# ---------------------------------------------------------------- marginal events
def test_flip_helpers_change_only_marginal_decisions():
    a = np.array([0.5, 1.0 / 255.0 * (1 - 1e-7), 0.3])
    base = OC.composite_list(a)
    assert base[1] == 0.0 and base[2] == pytest.approx(0.3 * 0.5)
    alt = OC.composite_list(a, flip_alpha=1)
    assert alt[1] > 0 and alt[2] < base[2]
    amb = OC.ambiguity({7: (np.array([3, 4, 5]), a)})
    (_, _, delta, slack), = amb
    assert delta[1] == pytest.approx(alt[1]) and slack == 1


# ---------------------------------------------------------------- planted mistakes
def test_planted_conic_sign_is_caught(monkeypatch):
    g, views = S.small_scene(2, n=50)
    cam = views.cameras[0]
    orig = OP.alpha_at

    def bad(proj, i, px, py):
        p2 = OP.Projection(proj.visible, proj.z, proj.depth_key, proj.mean2d, proj.cov2d,
                           proj.conic * np.array([1.0, -1.0, 1.0]), proj.opacity, proj.box)
        return orig(p2, i, px, py)
    monkeypatch.setattr(OC, "alpha_at", bad)
    vw = _weights(g, cam)
    pw = BR.pixel_weights(g, cam)
    lists = _pixel_lists(vw, cam.width)
    def same(a, b):
        return len(a) == len(b) and np.allclose([e for _, e in a], [e for _, e in b])
    mism = sum(1 for key, (lst, _) in pw.items() if not same(lists.get(key, []), lst))
    assert mism > 0


def test_planted_missing_dilation_is_caught(monkeypatch):
    monkeypatch.setattr(OP, "DILATION", 0.0)
    f, z, s, o = 40.0, 5.0, 0.2, 0.7
    cam = S.axis_camera(21, 21, f)
    g = S.gaussians([[0, 0, z]], math.log(s), [o])
    lists = _pixel_lists(_weights(g, cam), cam.width)
    monkeypatch.setattr(OP, "DILATION", 0.3)
    lst = lists[(12, 10)]
    want = OP.isotropic_on_axis_alpha(o, s, z, f, 2.0)
    assert abs(lst[0][1] - want) > 1e-3


def test_planted_depth_order_is_caught(monkeypatch):
    cam = S.axis_camera()
    g = S.gaussians([[0, 0, 6.0], [0, 0, 3.0]], -6.0, [0.8, 0.5])
    proj = OP.project(g, cam)
    proj.depth_key = -proj.depth_key          # back to front
    vw = OC.composite_view(proj, cam.width, cam.height)
    lst = _pixel_lists(vw, cam.width)[(4, 4)]
    case = GOLD["two_gaussians_one_pixel"]["cases"][0]
    assert lst[1][1] != pytest.approx(case["e_back"], abs=1e-6)


def test_row_entropy_pins():
    from scipy.stats import entropy as sp_entropy
    rng = np.random.default_rng(3)
    A = rng.random((50, 40)) * (rng.random((50, 40)) < 0.4)
    A[0] = 0
    A[1] = 0; A[1, 7] = 2.5
    A[2] = 1.0
    H = OU.row_entropy(A)
    assert H[0] == 0.0 and H[1] == 0.0
    assert H[2] == pytest.approx(math.log(40), rel=1e-14)
    for r in range(3, 50):
        assert H[r] == pytest.approx(sp_entropy(A[r]), rel=1e-12, abs=1e-14)
    assert np.allclose(OU.row_entropy(7.0 * A), H, rtol=1e-13)   # scale invariant


def test_dense_uplift_oracle_equals_sparse_times_codebook():
    """Eq. 3 with F = W C is the untruncated sparse uplift (Eq. 5) decoded by C:
    f_i = (acc_i / Z_i) C, with Z_i the row sum of acc when codes sum to one."""
    g, views = S.small_scene(23, n=60, m=8, k=3)
    # exact convex codes so that row sums equal Z
    val = views.code_val.astype(np.float64)
    val /= val.sum(1, keepdims=True)
    vv = sg.Views(views.cameras, views.region_maps, views.region_base, views.code_idx, val, 8)
    C = sg.random_codebook(4, 8, 5).astype(np.float64)
    f, Z = OU.dense_uplift(g, vv, C)
    acc = OU.uplift_accumulate(g, vv).acc
    t = Z > 0
    assert t.sum() > 20
    assert np.allclose(acc.sum(1), Z, rtol=1e-12)
    assert np.allclose(f[t], (acc[t] / Z[t, None]) @ C, atol=1e-12)
    assert (f[~t] == 0).all()


# ---------------------------------------------------------------- relevancy (App. B)
def _orthonormal(rng, n, d):
    q, _ = np.linalg.qr(rng.standard_normal((d, n)))
    return q.T                                           # n orthonormal rows


def test_relevancy_closed_forms():
    """Special cases of the App. B score that reduce to the logistic function
    (scipy's expit): a feature along the query with one canonical vector
    orthogonal to both gives expit(a |F|); a zero feature gives one half."""
    from scipy.special import expit
    rng = np.random.default_rng(11)
    q, c1, c2, c3 = _orthonormal(rng, 4, 16)
    for s in (1.0, -1.0, 0.1, 0.37):
        F = (s * q)[None]
        r = OR.relevancy(F, q, c1[None])
        assert r[0] == pytest.approx(expit(10.0 * s), rel=1e-14)           # a = 10
        assert OR.relevancy(F, q, c1[None], temperature=3.0)[0] == pytest.approx(expit(3.0 * s), rel=1e-14)
    assert OR.relevancy(np.zeros((1, 16)), q, np.stack([c1, c2]))[0] == 0.5
    # the minimum over canonical vectors: a canonical equal to the query caps the score at 1/2
    F = (0.8 * q + 0.3 * c2)[None]
    r = OR.relevancy(F, q, np.stack([c1, q, c3]))
    assert r[0] == pytest.approx(0.5, abs=0)
    # the least favourable canonical vector decides: F.c2 = 0.3 > F.c1 = 0
    assert OR.relevancy(F, q, np.stack([c1, c2]))[0] == pytest.approx(expit(10.0 * (0.8 - 0.3)), rel=1e-14)


def test_relevancy_invariants():
    """With one canonical vector, swapping it with the query maps R to 1 - R;
    the score is independent of the order of the canonical vectors and never
    exceeds the score against any single one of them."""
    rng = np.random.default_rng(12)
    F = rng.standard_normal((200, 24)) * 0.3
    q = rng.standard_normal(24); q /= np.linalg.norm(q)
    cs = rng.standard_normal((4, 24)); cs /= np.linalg.norm(cs, axis=1, keepdims=True)
    r1 = OR.relevancy(F, q, cs[:1]); r1s = OR.relevancy(F, cs[0], q[None])
    assert np.allclose(r1 + r1s, 1.0, atol=1e-15)
    r = OR.relevancy(F, q, cs)
    assert np.allclose(r, OR.relevancy(F, q, cs[::-1]), rtol=1e-14, atol=0)
    for k in range(4):
        assert (r <= OR.relevancy(F, q, cs[k:k + 1]) * (1 + 1e-13)).all()
    assert ((r > 0) & (r < 1)).all()
    # monotone in the query-minus-canonical similarity
    one = OR.relevancy(F, q, cs[:1])
    d = F @ q - F @ cs[0]
    assert (np.diff(one[np.argsort(d)]) >= 0).all()


def test_relevancy_map_is_decode_then_score():
    """The per-query map decodes once (Eq. 8) and scores each query; a
    coefficient row that is one-hot on atom j scores the codebook row C_j."""
    rng = np.random.default_rng(13)
    C = sg.random_codebook(5, 12, 20).astype(np.float64)
    qs = sg.random_unit_vectors(6, 3, 20); cs = sg.random_unit_vectors(7, 4, 20)
    W = np.eye(12)
    R = OR.relevancy_map(W, C, qs, cs)
    assert R.shape == (12, 3)
    for j in range(12):
        for t in range(3):
            assert R[j, t] == pytest.approx(OR.relevancy(C[j:j + 1], qs[t], cs)[0], rel=1e-14)
    W2 = rng.random((30, 12))
    assert np.allclose(OR.relevancy_map(W2, C, qs, cs)[:, 1], OR.relevancy(W2 @ C, qs[1], cs), rtol=1e-13)
