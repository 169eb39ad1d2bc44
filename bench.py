#!/usr/bin/env python3
"""Throughput of SCOUP's sparse-code uplift on one MI355X.

One step = the whole uplift of Algorithm 1 over one synthetic scene already
resident in HBM: for every view, projection, tile binning, per-tile depth
sort, front-to-back compositing fused with the weighted sparse accumulation
(Eq. 2, Eq. 5), then the Top-K filter of every Gaussian (Eq. 6).

Default workload ("scene"): 1,000,000 anisotropic Gaussians in a 10x10x4 box,
200 views of 1008x756 on a jittered orbit, 120 Voronoi regions per view,
8-sparse codes over M=256 atoms, Top-K=8.  The metric is Gaussian-pixel
contributions aggregated per second (terms e_i(v,p) > 0 that enter Eq. 5).

Prints one JSON line.  ``--gpus`` above 1 is refused: this build measures a
single GPU (the multi-GPU plan is in the design notes).
"""
from __future__ import annotations

import argparse
import ctypes as C
from ctypes import byref as C_byref, c_double as C_double, c_int64 as C_int64
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
STAGES = ["project", "pair_scan", "emit", "tile_sort", "composite", "topk",
          "render", "decode", "render_backward", "backward_gemm", "row_build", "relevancy", "relevancy_fold",
          "extra_apply"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FLOPS_PER_CONTRIBUTION = 14     # alpha (offsets 2, quadratic form 6, opacity product, clamp) +
                                # compositing (1 - alpha, T (1 - alpha), alpha T, cutoff test); plus one exp
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector peak (256 CU x 2.4 GHz, packed FP32)


def uplift_view_bytes(n, width, height, regions, k_code, touches):
    """Algorithmic HBM bytes of one view of the uplift (Eq. 5 costs
    O(|S_i| K) per Gaussian): read the Gaussians (44 B each), the view's
    region map (4 B per pixel) and code table (8 B per code slot), and per
    distinct (Gaussian, region) pair with weight one code's worth of
    accumulator traffic (8 B per code slot)."""
    return 44 * n + 4 * width * height + 8 * regions * k_code + 8 * k_code * touches


def uplift_step_bytes(n, m, k, view_bytes):
    """Whole uplift: the views plus zeroing the N x M accumulator, reading it
    once for Top-K and writing N x K (index, value) pairs."""
    return view_bytes + 4 * n * m + 4 * n * m + 8 * n * k


def composite_source_hash():
    """Hash of the compositing kernel's source (its section of uplift.hip and
    the device header), to tell whether committed counters still apply."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2605_13600_amd", "csrc")
    up = open(os.path.join(csrc, "uplift.hip")).read()
    a, b = up.index("constexpr int kEStride"), up.index("// Eq. 6 on one row held by a wave")
    h = hashlib.sha256(up[a:b].encode())
    h.update(open(os.path.join(csrc, "scoup_device.h"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per compositing launch from the committed counter summary
    (two rocprofv3 passes scaled by a copy of known size), or None when the
    kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "composite_scene_1M_200views_hbm_counters.md")
    try:
        txt = open(path).read()
    except OSError:
        return None
    vals = dict(ln.split(": ", 1) for ln in txt.splitlines()
                if ln.startswith(("source_sha256: ", "traffic_bytes_per_launch: ")))
    if vals.get("source_sha256") != composite_source_hash():
        return None
    return int(vals["traffic_bytes_per_launch"])


def _oracle_band(job):
    """One worker of the CPU baseline: the FP64 oracle (projection +
    compositing + accumulation) on rows [y0, y0 + rows) of one view of the
    scene workload, all Gaussians.  Returns (contributions, seconds)."""
    view, rows = job
    import numpy as np
    import scenegen as sg
    from oracle import composite as OC
    from oracle import project as OP
    from oracle import uplift as OU
    sc = sg.make_scene("scene", n_views=view + 1)
    cam = sc.views.cameras[view]
    y0 = max(0, cam.height // 2 - rows // 2)
    mask = np.zeros(cam.width * cam.height, bool)
    mask[y0 * cam.width:(y0 + rows) * cam.width] = True
    acc = np.zeros((sc.gaussians.n, sc.views.m_atoms))
    t0 = time.perf_counter()
    proj = OP.project(sc.gaussians, cam)
    vw = OC.composite_view(proj, cam.width, cam.height, pixel_mask=mask, track_marginal=False)
    OU.accumulate_view(acc, None, vw, sc.views.region_maps[view], int(sc.views.region_base[view]),
                       sc.views.code_idx, sc.views.code_val, None, sc.views.m_atoms)
    return vw.n_contrib, time.perf_counter() - t0


def cpu_baseline(workload, rows=96):
    """The FP64 oracle timed on the host: one process per core (spawned, so
    nothing of the GPU process is inherited), each on a band of ``rows`` image
    rows through the centre of a different view of the 1M-Gaussian scene
    (views are additive); rate = all contributions / the slowest worker's
    time.  Then the same band of view 0 alone in this process (one core)."""
    import multiprocessing as mp
    if workload != "scene":
        return None
    # one worker per core of this process's share, at most 16 (the host share
    # of one GPU; each worker holds its own copy of the scene, about 1.5 GB)
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_band, [(v, rows) for v in range(cores)])
    n_all = sum(c for c, _ in res)
    t_all = max(t for _, t in res)
    c1, t1 = _oracle_band((0, rows))
    return dict(value=n_all / t_all, unit="contributions/s", cores=cores, kind="oracle",
                cpu_model=model, value_1core=c1 / t1,
                sample=f"{cores} processes, each the FP64 NumPy oracle (projection of all 1,000,000 Gaussians, "
                       f"compositing and accumulation) on a {rows}-row band through the centre of one of views "
                       f"0..{cores - 1} (1008x756): {n_all} contributions, slowest worker {t_all:.1f} s; "
                       f"one core alone: {c1} contributions of view 0 in {t1:.1f} s")


def bench_render_decode(n_views, gaussians, lib, P, sg, torch, np):
    """Render (Eq. 7) + decode (Eq. 8) of the 1M-Gaussian scene with synthetic
    Top-8 over M=256, codebook 256x512, on the first ``n_views`` of 100 orbit
    views at 1440x1080; FP32, BF16 and FP8 decode inputs.  Also the query
    path: render + fused decode/relevancy (App. B) for 16 query vectors."""
    m, d, k = 256, 512, 8
    cams = sg.orbit_cameras(2002, 100, 12.0, 1.0, 4.0, 1.0, 0.5, 1440, 1080, 60.0)[:n_views]
    ti, tv = sg.random_topk(2003, gaussians.n, m, k)
    cb = sg.random_codebook(2004, m, d)
    dg = P.gaussians_to_device(gaussians)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    dC = torch.from_numpy(cb).cuda()
    n_q = 16
    dQ = torch.from_numpy(sg.random_unit_vectors(2005, n_q, d)).cuda()
    dCanon = torch.from_numpy(sg.random_unit_vectors(2006, 4, d)).cuda()
    px = 1440 * 1080
    res = {"workload": f"render+decode: {gaussians.n} Gaussians, Top-{k} over M={m}, codebook {m}x{d}, "
                       f"{n_views} views 1440x1080", "views": n_views}
    peak = {"f32": (157.3, "TFLOP/s"), "bf16": (2500.0, "TFLOP/s"), "fp8": (5000.0, "TFLOP/s")}
    in_b = {"f32": 4, "bf16": 2, "fp8": 1}
    for dt in ("f32", "bf16", "fp8"):
        out_dt = "f32" if dt == "f32" else "bf16"
        W, _, nc, scl = P.render_coeff(dg, dti, dtv, cams[0], m, dtype=dt)
        F = P.decode(W, dC, dt, coeff_scale=scl, out_dtype=out_dt)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for cam in cams:
            W, _, nc, scl = P.render_coeff(dg, dti, dtv, cam, m, dtype=dt, want_t_final=False)
            F = P.decode(W, dC, dt, coeff_scale=scl, out_dtype=out_dt)
        torch.cuda.synchronize()
        t_rd = time.perf_counter() - t0
        # decode alone, with HIP events on the launch stream
        lib.scoup_stage_timing(1)
        for _ in range(n_views):
            F = P.decode(W, dC, dt, coeff_scale=scl, out_dtype=out_dt)
        tot, cnt = C_double(), C_int64()
        lib.scoup_stage_stats(7, C_byref(tot), C_byref(cnt))
        lib.scoup_stage_timing(0)
        dec_us = tot.value * 1e3 / max(1, cnt.value)
        flops = 2.0 * px * m * d
        bytes_ = px * (m * in_b[dt] + d * (4 if out_dt == "f32" else 2))
        tf = flops / (dec_us * 1e-6) / 1e12
        gbs = bytes_ / (dec_us * 1e-6) / 1e9
        pk, _ = peak[dt]
        res[dt] = {
            "render_decode_mpix_s": round(px * n_views / t_rd / 1e6, 2),
            "decode_mpix_s": round(px / (dec_us * 1e-6) / 1e6, 2),
            "decode_avg_us": round(dec_us, 2),
            "decode_tflops": round(tf, 2), "decode_mfma_frac": round(tf / pk, 4),
            "decode_hbm_gbs": round(gbs, 1), "decode_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "decode_arith_intensity": round(flops / bytes_, 1),
            "decode_mfma_ceiling": round(min(1.0, (flops / bytes_) / (pk * 1e12 / (HBM_PEAK_GBS * 1e9))), 4),
            "contributions_per_view": nc,
        }
        # the one-pass render (Eq. 7 + Eq. 8 fused, coefficient rows kept on chip)
        Ff, _, _, _ = P.render(dg, dti, dtv, dC, cams[0], in_dtype=dt, out_dtype=out_dt, want_t_final=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for cam in cams:
            Ff, _, _, _ = P.render(dg, dti, dtv, dC, cam, in_dtype=dt, out_dtype=out_dt, want_t_final=False)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        del Ff
        # the same views through scoup_render_views, 8 cameras a call, views in flight
        vb = 8
        Fv, _ = P.render_views(dg, dti, dtv, dC, cams[:min(vb, n_views)], in_dtype=dt, out_dtype=out_dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(0, n_views, vb):
            Fv, _ = P.render_views(dg, dti, dtv, dC, cams[i:i + vb], in_dtype=dt, out_dtype=out_dt)
        torch.cuda.synchronize()
        t_fv = time.perf_counter() - t0
        del Fv
        lib.scoup_stage_timing(1)
        for cam in cams[:min(5, n_views)]:
            P.render(dg, dti, dtv, dC, cam, in_dtype=dt, out_dtype=out_dt, want_t_final=False)
        lib.scoup_stage_stats(6, C_byref(tot), C_byref(cnt))
        fk_us = tot.value * 1e3 / max(1, cnt.value)
        lib.scoup_stage_timing(1)
        for cam in cams[:min(5, n_views)]:
            P.render_coeff(dg, dti, dtv, cam, m, dtype=dt, want_t_final=False)
        lib.scoup_stage_stats(6, C_byref(tot), C_byref(cnt))
        map_us = tot.value * 1e3 / max(1, cnt.value)
        lib.scoup_stage_timing(0)
        res[dt]["map_kernel_avg_us"] = round(map_us, 1)
        res[dt]["map_kernel_hbm_frac"] = round((gaussians.n * (48 + 8 * k) + px * m * in_b[dt]) /
                                               (map_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        # algorithmic bytes of the fused kernel: splats + code slots read per Gaussian
        # (48 + 8 K), the feature rows written
        f_bytes = gaussians.n * (48 + 8 * k) + px * d * (4 if out_dt == "f32" else 2)
        res[dt].update({
            "fused_render_mpix_s": round(px * n_views / t_f / 1e6, 2),
            "fused_render_views_mpix_s": round(px * n_views / t_fv / 1e6, 2),
            "fused_kernel_avg_us": round(fk_us, 1),
            "fused_kernel_hbm_frac": round(f_bytes / (fk_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "fused_kernel_tflops": round(2.0 * px * m * d / (fk_us * 1e-6) / 1e12, 1),
        })
        # query path: render + fused decode/relevancy (App. B), 16 queries, 4 canonical vectors
        R = P.relevancy(W, dC, dQ, dCanon, dt, coeff_scale=scl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for cam in cams:
            W, _, nc, scl = P.render_coeff(dg, dti, dtv, cam, m, dtype=dt, want_t_final=False)
            R = P.relevancy(W, dC, dQ, dCanon, dt, coeff_scale=scl)
        torch.cuda.synchronize()
        t_rr = time.perf_counter() - t0
        lib.scoup_stage_timing(1)
        for _ in range(n_views):
            R = P.relevancy(W, dC, dQ, dCanon, dt, coeff_scale=scl)
        lib.scoup_stage_stats(11, C_byref(tot), C_byref(cnt))
        rel_us = tot.value * 1e3 / max(1, cnt.value)
        lib.scoup_stage_stats(12, C_byref(tot), C_byref(cnt))
        prep_us = tot.value * 1e3 / max(1, cnt.value)
        lib.scoup_stage_timing(0)
        rel_bytes = px * (m * in_b[dt] + n_q * 4)
        res[dt].update({
            "render_relevancy_mpix_s": round(px * n_views / t_rr / 1e6, 2),
            "relevancy_avg_us": round(rel_us, 2), "relevancy_fold_avg_us": round(prep_us, 2),
            "relevancy_hbm_gbs": round(rel_bytes / (rel_us * 1e-6) / 1e9, 1),
            "relevancy_hbm_frac": round(rel_bytes / (rel_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
        })
        log(f"render+decode {dt}: {res[dt]}")
    return res


def bench_decode_sweep(lib, P, sg, torch, np, px=1440 * 1080, d=512, reps=5):
    """Decode alone over codebook sizes M in {64, 128, 256, 512} (D = 512,
    one 1440x1080 view of coefficients, sparse rows like rendered maps), FP32 /
    BF16 / FP8 inputs; HIP-event time on the launch stream."""
    out = {}
    rng = np.random.default_rng(7)
    for m in (64, 128, 256, 512):
        A = rng.random((px, m), dtype=np.float32) * (rng.random((px, m), dtype=np.float32) < 0.1)
        At = torch.from_numpy(A).cuda()
        cb = torch.from_numpy(sg.random_codebook(100 + m, m, d)).cuda()
        ins = {"f32": At, "bf16": At.to(torch.bfloat16),
               "fp8": (At * 256.0).to(torch.float8_e4m3fn).view(torch.uint8)}
        row = {}
        for dt in ("f32", "bf16", "fp8"):
            out_dt = "f32" if dt == "f32" else "bf16"
            scl = 256.0 if dt == "fp8" else 1.0
            P.decode(ins[dt], cb, dt, coeff_scale=scl, out_dtype=out_dt)
            lib.scoup_stage_timing(1)
            for _ in range(reps):
                P.decode(ins[dt], cb, dt, coeff_scale=scl, out_dtype=out_dt)
            tot, cnt = C_double(), C_int64()
            lib.scoup_stage_stats(7, C_byref(tot), C_byref(cnt))
            lib.scoup_stage_timing(0)
            us = tot.value * 1e3 / max(1, cnt.value)
            in_b = {"f32": 4, "bf16": 2, "fp8": 1}[dt]
            by = px * (m * in_b + d * (4 if out_dt == "f32" else 2))
            row[dt] = {"mpix_s": round(px / (us * 1e-6) / 1e6, 1), "avg_us": round(us, 1),
                       "tflops": round(2.0 * px * m * d / (us * 1e-6) / 1e12, 1),
                       "hbm_frac": round(by / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
        out[f"M={m}"] = row
        log(f"decode sweep M={m}: {row}")
    return out


def bench_levels_and_dense(sc, P, sg, torch, np, dense_views=20):
    """Three semantic levels in one pass vs three single-level uplifts (all
    views), and the dense feature uplift (Eq. 3, D = 512) vs the sparse uplift
    on the first ``dense_views`` views."""
    out = {}
    v = sc.views
    lv2 = sg.make_views(3001, v.cameras, 60, v.m_atoms, v.k_code)
    lv3 = sg.make_views(3002, v.cameras, 240, v.m_atoms, v.k_code)
    dg = P.gaussians_to_device(sc.gaussians)
    dvs = [P.views_to_device(x) for x in (v, lv2, lv3)]
    ws = P.api.Workspace()
    k = sc.k_top

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    t3, r3 = timed(lambda: P.uplift_levels(dg, dvs, k, workspace=ws))
    t1 = 0.0
    for dv in dvs:
        t, _ = timed(lambda dv=dv: P.uplift(dg, dv, k, workspace=ws))
        t1 += t
    out["levels"] = {"workload": "3 levels (120 / 60 / 240 regions per view), all views",
                     "one_pass_ms": round(t3 * 1e3, 2), "three_uplifts_ms": round(t1 * 1e3, 2),
                     "speedup": round(t1 / t3, 2), "contributions": r3[3]}
    log(f"levels: {out['levels']}")
    sub = sg.subset_views(v, range(min(dense_views, v.n_views)))
    dsub = P.views_to_device(sub)
    cb = torch.from_numpy(sg.random_codebook(3003, v.m_atoms, 512)).cuda()
    ts, _ = timed(lambda: P.uplift(dg, dsub, k, workspace=ws))
    td, _ = timed(lambda: P.uplift_dense(dg, dsub, cb, workspace=ws))
    out["dense_vs_sparse"] = {"workload": f"first {sub.n_views} views, D=512 vs M={v.m_atoms}, K_code={v.k_code}",
                              "sparse_ms": round(ts * 1e3, 2), "dense_ms": round(td * 1e3, 2),
                              "dense_over_sparse": round(td / ts, 2)}
    log(f"dense vs sparse: {out['dense_vs_sparse']}")
    return out


def bench_backward(lib, P, sg, torch, np, n_views=8):
    """Backward of render + decode (float32) on the backward workload: 200,000
    Gaussians, Top-8 over M=256, codebook 256x512, 8 orbit views of 512x384;
    a seeded N(0,1) feature gradient stands in for dL/dF.  HIP-event time of
    the render-backward kernel and of the two GEMMs (dW = G C^T, dC = W^T G)."""
    n, m, d, k = 200_000, 256, 512, 8
    g = sg.make_gaussians(1003, n, (5.0, 5.0, 2.0), -4.5, 0.5, False, "beta")
    cams = sg.orbit_cameras(1004, n_views, 12.0, 0.0, 4.0, 0.0, 0.0, 512, 384, 60.0, jitter=False)
    ti, tv = sg.random_topk(1005, n, m, k)
    dg = P.gaussians_to_device(g)
    dti, dtv = torch.from_numpy(ti).cuda(), torch.from_numpy(tv).cuda()
    dC = torch.from_numpy(sg.random_codebook(1006, m, d)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(1007)
    G = torch.randn((384 * 512, d), device="cuda", generator=gen)
    maps = [P.render_coeff(dg, dti, dtv, cam, m, dtype="f32", want_t_final=False)[0] for cam in cams]
    gw, gc = torch.zeros_like(dtv), torch.zeros_like(dC)
    P.render_backward(dg, dti, dtv, cams[0], maps[0], dC, G, gw, gc)      # warm-up
    torch.cuda.synchronize()
    lib.scoup_stage_timing(1)
    t0 = time.perf_counter()
    for cam, W in zip(cams, maps):
        P.render_backward(dg, dti, dtv, cam, W, dC, G, gw, gc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot, cnt = C_double(), C_int64()
    lib.scoup_stage_stats(8, C_byref(tot), C_byref(cnt))
    bwd_us = tot.value * 1e3 / max(1, cnt.value)
    lib.scoup_stage_stats(9, C_byref(tot), C_byref(cnt))
    gemm_ms = tot.value / max(1, n_views)
    lib.scoup_stage_timing(0)
    px = 384 * 512
    gemm_tf = 2 * 2.0 * px * m * d / (gemm_ms * 1e-3) / 1e12
    out = {"workload": f"backward: {n} Gaussians, Top-{k} over M={m}, codebook {m}x{d}, {n_views} views 512x384",
           "ms_per_view": round(wall * 1e3 / n_views, 3), "mpix_s": round(px * n_views / wall / 1e6, 2),
           "render_backward_avg_us": round(bwd_us, 2), "gemms_ms_per_view": round(gemm_ms, 3),
           "gemm_tflops_f32": round(gemm_tf, 2), "gemm_mfma_frac": round(gemm_tf / 157.3, 4)}
    log(f"backward: {out}")
    return out


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size, for scaling rocprof's FETCH_SIZE /
    WRITE_SIZE counters (the dispatch appears in the same profile)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    return nbytes


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scene", choices=["scene", "tiny", "large"])
    ap.add_argument("--views", type=int, default=None, help="use only the first views (debug)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--render-views", type=int, default=100,
                    help="views of the 1440x1080 render workload to time (0 = skip)")
    ap.add_argument("--decode-sweep", type=int, default=1, help="time decode for M in 64..512 (0 = skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="three-level pass and dense-vs-sparse uplift sections (0 = skip)")
    ap.add_argument("--backward", type=int, default=1, help="time the render + decode backward (0 = skip)")
    ap.add_argument("--views-in-flight", type=int, default=4,
                    help="views projected, binned and composited at once in the timed steps (1..4); the "
                         "per-stage timing step always runs one view at a time")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy (for scaling HBM counters in a profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(views shard across GPUs by design, but no multi-GPU path is built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import scenegen as sg
    import paper_2605_13600_amd as P
    from paper_2605_13600_amd import _lib as L

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lib = L.load()

    t = time.time()
    sc = sg.make_scene(args.workload, n_views=args.views)
    log(f"scene {args.workload}: {sc.gaussians.n} Gaussians, {sc.views.n_views} views "
        f"{sc.views.cameras[0].width}x{sc.views.cameras[0].height}, M={sc.views.m_atoms}, "
        f"K={sc.k_top} generated in {time.time() - t:.1f}s")
    dg = P.gaussians_to_device(sc.gaussians)
    dv = P.views_to_device(sc.views)
    n, m, k = sc.gaussians.n, sc.views.m_atoms, sc.k_top
    acc = torch.empty((n, m), dtype=torch.float32, device="cuda")
    ws = P.api.Workspace()
    stream = torch.cuda.current_stream()

    def step():
        idx, val, a, nc = P.uplift(dg, dv, k, workspace=ws, acc=acc)
        return nc

    P.set_views_in_flight(args.views_in_flight)
    for i in range(args.warmup):
        nc = step()
        log(f"warmup {i} done, contributions {nc}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        nc = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms:.2f} ms/step, {nc} contributions/step")

    # per-stage kernel time with HIP events on the launch stream (one extra step,
    # one view at a time, so that every kernel's events time it alone)
    P.set_views_in_flight(1)
    lib.scoup_stage_timing(1)          # also turns on the uplift's U_v count for this step
    step()
    P.set_views_in_flight(args.views_in_flight)
    touch_stats = P.uplift_touch_stats()
    stages = {}
    for sid, name in enumerate(STAGES):
        tot, cnt = C.c_double(), C.c_int64()
        lib.scoup_stage_stats(sid, C.byref(tot), C.byref(cnt))
        if cnt.value:
            stages[name] = dict(total_ms=round(tot.value, 4), launches=int(cnt.value),
                                avg_us=round(tot.value * 1e3 / cnt.value, 3))
    lib.scoup_stage_timing(0)
    log(f"stages: {json.dumps(stages)}")

    touch = touch_stats
    if touch["views"] != sc.views.n_views or touch["lost"]:
        log(f"touch statistics incomplete: {touch}")

    # roofline of the dominant kernel: the compositing + accumulation kernel
    # (one launch per view), HBM-bound by the algorithmic byte model
    v = sc.views
    u_v = touch["touches"] / max(1, touch["views"])
    regions = int(v.region_base[-1]) / v.n_views
    w0 = v.cameras[0]
    view_bytes = [uplift_view_bytes(n, c.width, c.height, int(v.region_base[i + 1] - v.region_base[i]),
                                    v.k_code, u_v) for i, c in enumerate(v.cameras)]
    per_view = sum(view_bytes) / v.n_views
    comp = stages["composite"]
    comp_s = comp["avg_us"] * 1e-6
    achieved = per_view / comp_s / 1e9
    step_bytes = uplift_step_bytes(n, m, k, sum(view_bytes))
    step_gbs = step_bytes / (ms * 1e-3) / 1e9
    alu = nc / v.n_views * FLOPS_PER_CONTRIBUTION / comp_s / 1e12
    roofline = dict(
        kernel="k_composite_blk", bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
        frac=round(achieved / HBM_PEAK_GBS, 5),
        traffic=measured_traffic() if v.n_views == 200 and args.workload == "scene" else None,
        per_launch=f"one view: 44 N + 4 H W + 8 R_v K_code + 8 K_code U_v = {per_view / 1e6:.1f} MB "
                   f"(U_v = {u_v:.0f} distinct (Gaussian, region) pairs with weight, counted on the device)",
        avg_launch_us=comp["avg_us"],
        step={"bytes": int(step_bytes), "achieved_gbs": round(step_gbs, 1),
              "frac": round(step_gbs / HBM_PEAK_GBS, 5),
              "model": "sum over views of the per-view bytes + 4 N M (zero) + 4 N M (Top-K read) + 8 N K"},
        alu={"achieved_tflops": round(alu, 3), "peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
             "frac": round(alu / FP32_VECTOR_PEAK_TFLOPS, 5),
             "per_contribution": f"{FLOPS_PER_CONTRIBUTION} flops + 1 exp"},
        dominant_stage=max(stages, key=lambda s_: stages[s_]["total_ms"]))

    if args.copy_calibration:
        copy_calibration(torch)
    sweep = bench_decode_sweep(lib, P, sg, torch, np) if args.decode_sweep else None
    extras = bench_levels_and_dense(sc, P, sg, torch, np) if args.extras else None
    backward = bench_backward(lib, P, sg, torch, np) if args.backward else None

    render = None
    if args.render_views > 0:
        render = bench_render_decode(args.render_views, sc.gaussians, lib, P, sg, torch, np)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the CPU sample ...")
        cpu = cpu_baseline(args.workload)
        log(f"cpu baseline: {cpu}")

    w = sc.views.cameras[0]
    out = {
        "metric": "Gaussian-pixel contributions aggregated/s (uplift)",
        "value": nc * args.steps / dt,
        "unit": "contributions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload} uplift: {n} Gaussians, {sc.views.n_views} views "
                        f"{w.width}x{w.height}, M={m}, K_code={sc.views.k_code}, Top-K={k}",
            "contributions_per_step": nc,
            "parallelism": "single GPU",
            "views_in_flight": args.views_in_flight,
        },
        "stages": stages,
        "stages_note": "per-stage kernel times from one extra step with one view in flight",
        "roofline": roofline,
        "cpu_baseline": cpu,
        "render_decode": render,
        "decode_sweep": sweep,
        "extras": extras,
        "backward": backward,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
