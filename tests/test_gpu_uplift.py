"""GPU parity of the uplift (Eq. 5 / Algorithm 1) and Top-K (Eq. 6) against the oracle.

All calls go through the C ABI (ctypes binding).  Tolerances are defined in
tests/_parity.py.
"""
import numpy as np
import pytest
import torch

import paper_2605_13600_amd as P
import scenegen as sg
from oracle import uplift as OU
from tests import _parity as PT
from tests import _scenes as S
from tests._gpu import require_gpu, to_device

pytestmark = pytest.mark.gpu


def _run(g, v, k):
    dg, dv = to_device(g, v)
    idx, val, acc, nc = P.uplift(dg, dv, k)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), val.cpu().numpy(), acc.cpu().numpy(), nc


def _compare(g, v, k, label):
    idx, val, acc, nc = _run(g, v, k)
    ref = OU.uplift_accumulate(g, v)
    sa = PT.check_acc(acc, ref.acc, ref.amb)
    assert abs(nc - ref.n_contrib) <= ref.count_slack, (nc, ref.n_contrib, ref.count_slack)
    st = PT.check_topk(idx, val, ref.acc, ref.amb, k)
    print(f"[{label}] contrib gpu={nc} ref={ref.n_contrib} acc={sa} topk={st}", flush=True)
    return sa, st, ref


def test_tiny_workload_full():
    """2,000 isotropic Gaussians, 4 views 64x48, 8 regions, M=64, K=4."""
    require_gpu()
    sc = sg.make_scene("tiny")
    sa, st, ref = _compare(sc.gaussians, sc.views, sc.k_top, "tiny")
    assert ref.n_contrib > 50_000 and st["exact"] >= 0.99 * st["rows"]


@pytest.mark.parametrize("res", [(70, 45), (33, 17), (16, 16), (1, 1)])
def test_ragged_tiles_and_holes(res):
    """Partial tiles on the right/bottom edge, pixels with no region (-1)."""
    require_gpu()
    sc = sg.make_scene("tiny", res=res, hole_sites=2)
    _compare(sc.gaussians, sc.views, sc.k_top, f"ragged{res}")


def test_anisotropic_multi_tile():
    """Anisotropic scene-like Gaussians, 30k, 3 views 320x240 (300 tiles), M=256, K=8."""
    require_gpu()
    g = sg.make_gaussians(77, 30_000, (5.0, 5.0, 2.0), -3.5, 0.5, False, "beta")
    cams = sg.orbit_cameras(78, 3, 12.0, 1.0, 4.0, 1.0, 0.5, 320, 240, 60.0)
    v = sg.make_views(79, cams, 40, 256, 8)
    _compare(g, v, 8, "aniso")


def test_large_image_radix_binning():
    """1920x1664 views (49,920 8x8 blocks, above the counting pass's 49,152):
    pairs are emitted Gaussian-major and radix-sorted by block, and the
    emission also leaves each Gaussian's first pair index in its splat for the
    compositing."""
    require_gpu()
    g = sg.make_gaussians(91, 4000, (5.0, 5.0, 2.0), -4.0, 0.3, False, "beta")
    cams = sg.orbit_cameras(92, 2, 12.0, 1.0, 4.0, 1.0, 0.5, 1920, 1664, 60.0)
    v = sg.make_views(93, cams, 40, 64, 4)
    sa, st, ref = _compare(g, v, 4, "radix")
    assert ref.n_contrib > 500_000


def test_dense_tile_sorted_in_global_memory():
    """A tile holding more splats than the LDS sort capacity takes the global sort."""
    require_gpu()
    rng = np.random.default_rng(5)
    n = 6000
    means = np.stack([rng.uniform(-0.02, 0.02, n), rng.uniform(-0.02, 0.02, n), rng.uniform(-0.3, 0.3, n)], 1)
    g = S.gaussians(means, np.log(0.004), rng.uniform(0.05, 0.3, n))
    cam = S.axis_camera(48, 48, 60.0)
    cam = sg.Camera(cam.R, np.array([0, 0, 3.0], np.float32), cam.fx, cam.fy, cam.cx, cam.cy, 48, 48)
    rm = (np.arange(48 * 48).reshape(48, 48) // 300).astype(np.int32) % 3
    idx, val = sg.region_codes(np.random.default_rng(1), 3, 16, 4)
    v = S.views_for([cam], [rm], idx, val, 16)
    _compare(g, v, 4, "dense-tile")


def test_resume_accumulate_equals_full():
    """Views are additive: accumulating two view sets into one buffer equals one call."""
    require_gpu()
    sc = sg.make_scene("tiny")
    dg = P.gaussians_to_device(sc.gaussians)
    full, _ = P.uplift_accumulate(dg, P.views_to_device(sc.views))
    a, _ = P.uplift_accumulate(dg, P.views_to_device(sg.subset_views(sc.views, [0, 1])))
    a, _ = P.uplift_accumulate(dg, P.views_to_device(sg.subset_views(sc.views, [2, 3])), acc=a,
                               accumulate=True)
    torch.cuda.synchronize()
    f, r = full.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64)
    assert np.allclose(f, r, rtol=1e-5, atol=1e-12)


def test_workspace_retry_path_and_view_batches():
    """A pair capacity far too small is reported and the wrapper's retry succeeds;
    summing records one view at a time equals one pass over all views."""
    require_gpu()
    sc = sg.make_scene("tiny")
    dg, dv = to_device(sc.gaussians, sc.views)
    ws = P.api.Workspace()
    from paper_2605_13600_amd import _lib as L
    import ctypes as C
    lib = L.load()
    gs, vs = dg.struct(), dv.struct()
    nb = lib.scoup_uplift_workspace_bytes(dg.n, C.byref(vs), 16, 1)
    buf = ws.get(nb)
    acc0 = torch.zeros((dg.n, 64), dtype=torch.float32, device="cuda")
    st = lib.scoup_uplift_accumulate(C.byref(gs), C.byref(vs), acc0.data_ptr(), 0, 16, 1, buf.data_ptr(),
                                     buf.numel(), None, None)
    assert st == L.E_WORKSPACE and lib.scoup_required_pair_capacity() > 16
    P.api._capacity_cache.clear()
    ref = OU.uplift_accumulate(sc.gaussians, sc.views)
    for vb in (1, 3, 0):
        acc, nc = P.uplift_accumulate(dg, dv, workspace=ws, pair_capacity=1, view_batch=vb)
        PT.check_acc(acc.cpu().numpy(), ref.acc, ref.amb)
        assert abs(nc - ref.n_contrib) <= ref.count_slack


@pytest.mark.parametrize("vb", [1, 0])
def test_resumed_call_over_capacity_leaves_acc_unchanged(vb):
    """Eq. 5 sums over views, so a second call with accumulate=1 resumes over
    further views.  When that call's pair capacity is too small it reports
    SCOUP_E_WORKSPACE before writing anything: acc is bit for bit what it was.
    Repeated with exactly the capacity it asked for, it succeeds (the count
    checked up front is the count its views use) and equals one call over all
    views."""
    require_gpu()
    import ctypes as C
    from paper_2605_13600_amd import _lib as L
    sc = sg.make_scene("tiny")
    lib = L.load()
    dg = P.gaussians_to_device(sc.gaussians)
    full, _ = P.uplift_accumulate(dg, P.views_to_device(sc.views))
    a, _ = P.uplift_accumulate(dg, P.views_to_device(sg.subset_views(sc.views, [0, 1])))
    before = a.clone()
    dv2 = P.views_to_device(sg.subset_views(sc.views, [2, 3]))
    gs, vs = dg.struct(), dv2.struct()
    ws = P.api.Workspace()
    cap = 16
    buf = ws.get(lib.scoup_uplift_workspace_bytes(dg.n, C.byref(vs), cap, vb))
    st = lib.scoup_uplift_accumulate(C.byref(gs), C.byref(vs), a.data_ptr(), 1, cap, vb, buf.data_ptr(),
                                     buf.numel(), None, None)
    torch.cuda.synchronize()
    need = int(lib.scoup_required_pair_capacity())
    assert st == L.E_WORKSPACE and need > cap, (st, need)
    assert torch.equal(a, before)
    buf = ws.get(lib.scoup_uplift_workspace_bytes(dg.n, C.byref(vs), need, vb))
    st = lib.scoup_uplift_accumulate(C.byref(gs), C.byref(vs), a.data_ptr(), 1, need, vb, buf.data_ptr(),
                                     buf.numel(), None, None)
    torch.cuda.synchronize()
    assert st == L.OK, lib.scoup_last_error()
    f, r = full.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64)
    assert np.allclose(f, r, rtol=1e-5, atol=1e-12)
    ref = OU.uplift_accumulate(sc.gaussians, sc.views)
    PT.check_acc(r, ref.acc, ref.amb)


@pytest.mark.parametrize("limit", [1, 64])
def test_deferred_entry_overflow_adds_directly(limit):
    """A per-view deferred-entry buffer capped far below what fragmented maps
    need: the compositing adds the further regions' weights to the
    accumulator itself; every kernel completes and the result still matches
    the oracle (three levels, one of them cut into 1000 regions)."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    levels = [sg.make_views(800 + s, sc.views.cameras, s, 64, 4, hole_sites=1) for s in (8, 300, 1000)]
    dg = P.gaussians_to_device(sc.gaussians)
    try:
        P.set_deferred_entry_limit(limit)
        idxs, vals, accs, nc = P.uplift_levels(dg, [P.views_to_device(v) for v in levels], 4)
        torch.cuda.synchronize()
    finally:
        P.set_deferred_entry_limit(0)
    for lvl, v in enumerate(levels):
        ref = OU.uplift_accumulate(sc.gaussians, v)
        sa = PT.check_acc(accs[lvl].cpu().numpy(), ref.acc, ref.amb)
        PT.check_topk(idxs[lvl].cpu().numpy(), vals[lvl].cpu().numpy(), ref.acc, ref.amb, 4)
        assert abs(nc - ref.n_contrib) <= ref.count_slack
        print(f"[entry limit {limit}, level {lvl}] acc={sa}")


@pytest.mark.parametrize("m,kc", [(64, 5), (512, 16), (96, 3), (64, 12)])
def test_code_widths_of_the_row_build(m, kc):
    """Codes of K_code slots over codebooks of M atoms, full oracle: widths
    that are not a multiple of four (the row build's scalar code loads) and
    12 or 16 (four code quads loaded a chunk ahead, 12 re-reading one)."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    v = sg.make_views(600 + kc, sc.views.cameras, 40, m, kc, hole_sites=1)
    _compare(sc.gaussians, v, kc, f"m{m}-kc{kc}")


def test_large_workload_two_views_sampled_rows():
    """The 3M-Gaussian workload (20x20x6 box, 1440x1080, 200 regions per view,
    16-sparse codes over M=512, Top-16) on two of its views: 300 sampled rows
    against the row-sampled oracle, every sampled row's Top-K checked."""
    require_gpu()
    sc = sg.make_scene("large", n_views=2)
    assert sc.views.m_atoms == 512 and sc.views.k_code == 16 and sc.k_top == 16
    idx, val, acc, nc = _run(sc.gaussians, sc.views, sc.k_top)
    rows = np.random.default_rng(0).choice(sc.gaussians.n, 300, replace=False)
    ref = OU.uplift_accumulate(sc.gaussians, sc.views, rows=rows)
    sa = PT.check_acc(acc[rows], ref.acc, ref.amb)
    st = PT.check_topk(idx[rows], val[rows], ref.acc, ref.amb, sc.k_top)
    print(f"[large-2views] contrib={nc} acc={sa} topk={st}", flush=True)
    assert (ref.acc.sum(1) > 0).sum() > 100


@pytest.mark.parametrize("sites,limit", [(8, 0), (300, 0), (300, 16)])
def test_region_touch_count(sites, limit):
    """U_v summed over views, counted on the device while statistics are on,
    against the oracle's distinct (Gaussian, region) pairs with a contribution;
    with a capped entry buffer the direct adds bound the rest."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    v = sg.make_views(950 + sites, sc.views.cameras, sites, 64, 4, hole_sites=1)
    dg, dv = to_device(sc.gaussians, v)
    try:
        P.set_deferred_entry_limit(limit)
        P.stage_timing(True)
        P.uplift(dg, dv, 4)
        torch.cuda.synchronize()
        st = P.uplift_touch_stats()
    finally:
        P.stage_timing(False)
        P.set_deferred_entry_limit(0)
    ref = OU.uplift_accumulate(sc.gaussians, v)
    u_ref = int(OU.region_touches(sc.gaussians, v).sum())
    print(f"[touches sites={sites} limit={limit}] gpu={st} oracle={u_ref} slack={ref.count_slack}")
    assert st["views"] == v.n_views and st["lost"] == 0
    if limit == 0:
        assert st["direct"] == 0
        assert abs(st["touches"] - u_ref) <= ref.count_slack
    else:
        assert st["direct"] > 0
        assert st["touches"] - ref.count_slack <= u_ref <= st["touches"] + st["direct"] + ref.count_slack


def test_empty_and_invisible():
    require_gpu()
    sc = sg.make_scene("tiny")
    # no Gaussians
    g0 = sc.gaussians.subset(np.arange(0))
    dg, dv = to_device(g0, sc.views)
    acc, nc = P.uplift_accumulate(dg, dv)
    assert acc.shape == (0, 64) and nc == 0
    # every Gaussian behind the cameras' near planes -> all-zero rows -> padding
    g = sc.gaussians.subset(np.arange(100))
    g.means[:] = 0.0
    cams = [sg.Camera(c.R, c.t, c.fx, c.fy, c.cx, c.cy, c.width, c.height, near=10.0) for c in sc.views.cameras]
    v = sg.Views(cams, sc.views.region_maps, sc.views.region_base, sc.views.code_idx, sc.views.code_val, 64)
    idx, val, acc, nc = _run(g, v, 4)
    assert nc == 0 and (acc == 0).all() and (idx == -1).all() and (val == 0).all()


def test_bad_region_id_is_reported():
    require_gpu()
    sc = sg.make_scene("tiny")
    maps = [m.copy() for m in sc.views.region_maps]
    maps[1][10, 10] = 99
    v = sg.Views(sc.views.cameras, maps, sc.views.region_base, sc.views.code_idx, sc.views.code_val, 64)
    dg, dv = to_device(sc.gaussians, v)
    with pytest.raises(P.ScoupError) as ei:
        P.uplift_accumulate(dg, dv)
    assert ei.value.status == -5


def test_bad_code_atom_index_is_reported():
    """A code slot whose atom index is >= m_atoms (every region's first slot):
    the row build leaves it out and the call reports the data error."""
    require_gpu()
    sc = sg.make_scene("tiny")
    ci = sc.views.code_idx.copy()
    ci[:, 0] = 64
    v = sg.Views(sc.views.cameras, sc.views.region_maps, sc.views.region_base, ci, sc.views.code_val, 64)
    dg, dv = to_device(sc.gaussians, v)
    with pytest.raises(P.ScoupError) as ei:
        P.uplift_accumulate(dg, dv)
    assert ei.value.status == -5 and "code atom" in str(ei.value)


@pytest.mark.parametrize("m,k", [(64, 4), (100, 7), (256, 8), (512, 16), (1000, 64)])
def test_topk_kernel_against_oracle_exact(m, k):
    """Top-K alone on a seeded float32 matrix with exact ties and zero rows: indices
    bit-exact (same float32 input on both sides), values within 1e-6."""
    require_gpu()
    rng = np.random.default_rng(m)
    A = rng.integers(0, 40, size=(2000, m)).astype(np.float32) * np.float32(0.125)
    A[rng.random(A.shape) < 0.5] = 0
    A[:7] = 0
    A[7:20, : m // 2] = 1.0
    idx, val = P.topk(torch.from_numpy(A).cuda(), k)
    ri, rv = OU.topk_rows(A.astype(np.float64), k)
    assert (idx.cpu().numpy() == ri).all()
    assert np.allclose(val.cpu().numpy(), rv, rtol=1e-6, atol=1e-7)


def test_full_size_scene_sampled_rows():
    """The 1M-Gaussian, 1008x756 scene on two of its views (views are additive, so
    a view subset is an exact sub-problem); 300 sampled rows against the
    row-sampled oracle, every row's Top-K checked."""
    require_gpu()
    sc = sg.make_scene("scene", n_views=2)
    idx, val, acc, nc = _run(sc.gaussians, sc.views, sc.k_top)
    rows = np.random.default_rng(0).choice(sc.gaussians.n, 300, replace=False)
    ref = OU.uplift_accumulate(sc.gaussians, sc.views, rows=rows)
    sa = PT.check_acc(acc[rows], ref.acc, ref.amb)
    st = PT.check_topk(idx[rows], val[rows], ref.acc, ref.amb, sc.k_top)
    print(f"[scene-2views] contrib={nc} acc={sa} topk={st}", flush=True)
    assert (ref.acc.sum(1) > 0).sum() > 200


def test_three_semantic_levels_in_one_pass():
    """Three region maps over the same cameras (4, 8 and 16 Voronoi cells, own
    codes) uplifted in one compositing pass; each level matches the oracle run
    on that level alone."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    levels = [sg.make_views(500 + s, sc.views.cameras, s, 64, 4, hole_sites=1 if s == 8 else 0)
              for s in (4, 8, 16)]
    dg = P.gaussians_to_device(sc.gaussians)
    idxs, vals, accs, nc, ents = P.uplift_levels(dg, [P.views_to_device(v) for v in levels], 4, entropy=True)
    torch.cuda.synchronize()
    for lvl, v in enumerate(levels):
        ref = OU.uplift_accumulate(sc.gaussians, v)
        sa = PT.check_acc(accs[lvl].cpu().numpy(), ref.acc, ref.amb)
        # entropy of the fused pass, against the oracle on the oracle's rows (1e-4 abs:
        # float32 rows and logs; rows with ambiguity mass are left out)
        He = OU.row_entropy(ref.acc)
        okr = ref.amb.sum(1) == 0
        assert np.allclose(ents[lvl].cpu().numpy()[okr], He[okr], atol=1e-4, rtol=1e-4)
        st = PT.check_topk(idxs[lvl].cpu().numpy(), vals[lvl].cpu().numpy(), ref.acc, ref.amb, 4)
        assert abs(nc - ref.n_contrib) <= ref.count_slack
        print(f"[level {lvl}] acc={sa} topk={st}")


def test_entropy_kernel_against_oracle():
    """Row entropy (App. C.2) on a seeded float32 matrix with zero rows and
    one-hot rows, against the oracle on the same float32 values."""
    require_gpu()
    rng = np.random.default_rng(9)
    A = (rng.random((3000, 256)) * (rng.random((3000, 256)) < 0.05)).astype(np.float32)
    A[:5] = 0
    A[5:9] = 0; A[5:9, 3] = 1.5
    H = P.entropy(torch.from_numpy(A).cuda()).cpu().numpy()
    R = OU.row_entropy(A.astype(np.float64))
    assert (H[:9] == 0).all()
    assert np.allclose(H, R, rtol=1e-5, atol=2e-6)


@pytest.mark.parametrize("d", [64, 512])
def test_dense_feature_uplift_against_oracle(d):
    """Eq. 3 on the same engine: features within 1e-5 relative (row norm) plus
    the ambiguity mass carried through the decoded features; Z within 1e-5."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45), hole_sites=1)
    C = sg.random_codebook(31, 64, d)
    dg, dv = to_device(sc.gaussians, sc.views)
    feat, z, nc = P.uplift_dense(dg, dv, torch.from_numpy(C).cuda())
    torch.cuda.synchronize()
    f_ref, z_ref = OU.dense_uplift(sc.gaussians, sc.views, C)
    amb = OU.uplift_accumulate(sc.gaussians, sc.views).amb
    zr = z.cpu().numpy().astype(np.float64)
    ok = amb.sum(1) == 0
    assert np.allclose(zr[ok], z_ref[ok], rtol=1e-5, atol=1e-9)
    fg = feat.cpu().numpy().astype(np.float64)
    nrm = np.linalg.norm(f_ref, axis=1)
    err = np.linalg.norm(fg - f_ref, axis=1)
    assert (err[ok] <= 1e-5 * nrm[ok] + 1e-7).all(), float((err[ok] / np.maximum(nrm[ok], 1e-30)).max())


def _regions_per_block(v):
    """Largest number of distinct regions in one 8x8 block over the views."""
    best = 0
    for m in v.region_maps:
        H, W = m.shape
        for y in range(0, H, 8):
            for x in range(0, W, 8):
                r = m[y:y + 8, x:x + 8]
                best = max(best, len(np.unique(r[r >= 0])))
    return best


@pytest.mark.parametrize("sites", [150, 1200])
def test_fragmented_regions_per_block(sites):
    """Voronoi maps fine enough that 8x8 blocks hold many regions: the block's
    two record regions, the further-region columns (deferred entries) and,
    at 1200 cells, regions beyond the 16 membership columns (per-region loop)."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    v = sg.make_views(910 + sites, sc.views.cameras, sites, 64, 4, hole_sites=3)
    rb = _regions_per_block(v)
    assert rb >= (17 if sites == 1200 else 4), rb
    _compare(sc.gaussians, v, 4, f"fragmented{sites}")


def test_fragmented_levels_in_one_pass():
    """Four levels (coarse to very fine) in one compositing pass: 8 record
    columns, the remaining 8 columns shared by the fine levels' further
    regions, the rest through the per-region loop; every level matches the
    oracle run on that level alone."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    levels = [sg.make_views(700 + s, sc.views.cameras, s, 64, 4, hole_sites=1) for s in (6, 60, 300, 1000)]
    dg = P.gaussians_to_device(sc.gaussians)
    idxs, vals, accs, nc = P.uplift_levels(dg, [P.views_to_device(v) for v in levels], 4)
    torch.cuda.synchronize()
    for lvl, v in enumerate(levels):
        ref = OU.uplift_accumulate(sc.gaussians, v)
        sa = PT.check_acc(accs[lvl].cpu().numpy(), ref.acc, ref.amb)
        PT.check_topk(idxs[lvl].cpu().numpy(), vals[lvl].cpu().numpy(), ref.acc, ref.amb, 4)
        assert abs(nc - ref.n_contrib) <= ref.count_slack
        print(f"[fragmented level {lvl}] acc={sa}")


def test_dense_feature_uplift_fragmented():
    """Eq. 3 with many regions per block: further regions add w F_r and w
    through the deferred entries and the per-region loop."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    v = sg.make_views(933, sc.views.cameras, 1200, 64, 4, hole_sites=3)
    C = sg.random_codebook(32, 64, 64)
    dg, dv = to_device(sc.gaussians, v)
    feat, z, nc = P.uplift_dense(dg, dv, torch.from_numpy(C).cuda())
    torch.cuda.synchronize()
    f_ref, z_ref = OU.dense_uplift(sc.gaussians, v, C)
    amb = OU.uplift_accumulate(sc.gaussians, v).amb
    ok = amb.sum(1) == 0
    zr = z.cpu().numpy().astype(np.float64)
    assert np.allclose(zr[ok], z_ref[ok], rtol=1e-5, atol=1e-9)
    fg = feat.cpu().numpy().astype(np.float64)
    nrm = np.linalg.norm(f_ref, axis=1)
    err = np.linalg.norm(fg - f_ref, axis=1)
    assert (err[ok] <= 1e-5 * nrm[ok] + 1e-7).all(), float((err[ok] / np.maximum(nrm[ok], 1e-30)).max())


@pytest.mark.parametrize("n", [2, 64, 65, 128, 129, 256, 257, 512, 513, 1024, 1025, 2048, 2049, 4096, 4097])
def test_block_list_lengths_at_sort_class_edges(n):
    """One 8x8 block whose list holds exactly n pairs (every Gaussian covers
    the whole block), for n at the edges of the depth sort's size classes
    (one wave, two and four waves, one workgroup, global memory).  Opacities
    near 1/255 keep every pixel compositing through ~1800 Gaussians, so the
    weight of each one depends on the exact depth order before it; a tenth
    of the Gaussians repeat another's position (equal depths, id order)."""
    require_gpu()
    rng = np.random.default_rng(4000 + n)
    means = np.stack([rng.uniform(-0.05, 0.05, n), rng.uniform(-0.05, 0.05, n), rng.uniform(1.0, 3.0, n)], 1)
    dup = rng.random(n) < 0.1
    dup[0] = False
    means[dup] = means[rng.integers(0, n, int(dup.sum()))]
    g = S.gaussians(means, np.log(30.0), rng.uniform(0.0045, 0.0055, n))
    cam = S.axis_camera(8, 8, 10.0)
    rm = np.zeros((8, 8), np.int32)
    rm[:, 4:] = 1
    idx, val = sg.region_codes(np.random.default_rng(2), 2, 16, 4)
    v = S.views_for([cam], [rm], idx, val, 16)
    sa, st, ref = _compare(g, v, 4, f"list{n}")
    assert ref.n_contrib >= 64 * min(n, 1800)


@pytest.mark.parametrize("vif", [1, 2, 3])
def test_views_in_flight_settings_agree(vif):
    """Fewer views in flight than the default 4 (and a view batch that does
    not divide by it): the same accumulator up to float rounding of the
    deferred entries' order, and the oracle's parity."""
    require_gpu()
    sc = sg.make_scene("tiny", res=(70, 45))
    v = sg.make_views(77, sc.views.cameras, 300, 64, 4, hole_sites=1)
    dg, dv = to_device(sc.gaussians, v)
    try:
        P.set_views_in_flight(vif)
        assert P.views_in_flight() == vif
        _, _, acc_k, nc_k = P.uplift(dg, dv, 4)
        P.set_views_in_flight(4)
        _, _, acc_4, nc_4 = P.uplift(dg, dv, 4)
        torch.cuda.synchronize()
    finally:
        P.set_views_in_flight(4)
    assert nc_k == nc_4
    a, b = acc_k.cpu().numpy(), acc_4.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-5, atol=1e-7)
    ref = OU.uplift_accumulate(sc.gaussians, v)
    PT.check_acc(a, ref.acc, ref.amb)
