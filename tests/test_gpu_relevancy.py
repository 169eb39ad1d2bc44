"""Parity of the fused decode + relevancy kernel (App. B on Eq. 8) with the
oracle: the oracle decodes the stored coefficient map in FP64 and scores
each query; the kernel never forms the features.

Tolerance.  With w the (dequantised) coefficient row of a pixel and S the
codebook folded into a query or canonical vector, the kernel's dot product
s = sum_m w_m S_m carries the rounding of S (2^-24 relative for float32
maps, 2^-16 for the two-term bfloat16 split used with BF16 / FP8 maps) and
float32 accumulation over M terms (M 2^-24), both relative to
B = sum_m |w_m| max |S_m|.  R = sigma(a (s_q - max_c s_c)) moves by at most
a / 4 per unit change of each of the two dot products, so
|dR| <= (a / 2) (u + M 2^-24) B, plus a few float32 ulps from the epilogue.
"""
import numpy as np
import pytest
import torch

import paper_2605_13600_amd as P
import scenegen as sg
from oracle import render as OR
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu

TEMP = 10.0


def _store(rows: np.ndarray, dtype: str, scale: float):
    """Host-side storage of a coefficient map: (device tensor, FP64 values it holds)."""
    t = torch.from_numpy(rows * np.float32(scale))
    if dtype == "f32":
        dev, deq = t, t.double()
    elif dtype == "bf16":
        q = t.to(torch.bfloat16)
        dev, deq = q, q.double()
    else:
        q = t.to(torch.float8_e4m3fn)
        dev, deq = q.view(torch.uint8), q.double()
    return dev.cuda(), (deq / scale).numpy()


def _bound(w: np.ndarray, C, qs, cs, dtype: str) -> np.ndarray:
    S = np.asarray(C, np.float64) @ np.concatenate([qs, cs]).astype(np.float64).T
    u = 2.0 ** -24 if dtype == "f32" else 2.0 ** -16
    m = w.shape[1]
    B = np.abs(w) @ np.abs(S).max(axis=1)
    return 0.5 * TEMP * (u + m * 2.0 ** -24) * B + 4e-6


def _run(rows, C, qs, cs, dtype, scale):
    dev, deq = _store(rows, dtype, scale)
    out = P.relevancy(dev, torch.from_numpy(C).cuda(), torch.from_numpy(qs).cuda(), torch.from_numpy(cs).cuda(),
                      in_dtype=dtype, coeff_scale=scale, temperature=TEMP)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), deq


CASES = [  # (pixels, M, D, Q, n_canon, dtype, scale)
    (805, 64, 96, 16, 4, "f32", 1.0),
    (805, 64, 96, 16, 4, "bf16", 1.0),
    (805, 64, 96, 16, 4, "fp8", 256.0),
    (1000, 37, 40, 5, 3, "f32", 1.0),        # rows of 148 bytes: unaligned bytewise loads
    (1000, 37, 40, 5, 3, "bf16", 4.0),
    (1000, 37, 40, 5, 3, "fp8", 256.0),
    (333, 256, 512, 25, 4, "bf16", 1.0),     # two query groups, ragged second group
    (333, 256, 512, 50, 1, "fp8", 256.0),
    (257, 130, 64, 1, 2, "f32", 1.0),
    (64, 512, 512, 24, 4, "f32", 1.0),
    (1, 8, 16, 3, 4, "bf16", 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "P%d_M%d_D%d_Q%d_c%d_%s" % c[:6])
def test_relevancy_matches_oracle(case):
    require_gpu()
    n, m, d, q, nc, dtype, scale = case
    rows = sg.random_coeff_rows(100 + m, n, m)
    C = sg.random_codebook(200 + m, m, d)
    qs = sg.random_unit_vectors(300 + q, q, d)
    cs = sg.random_unit_vectors(400 + nc, nc, d)
    got, deq = _run(rows, C, qs, cs, dtype, scale)
    ref = OR.relevancy_map(deq, C, qs, cs, TEMP)
    err = np.abs(got - ref)
    tol = _bound(deq, C, qs, cs, dtype)[:, None]
    bad = np.argwhere(err > tol)
    assert bad.size == 0, f"{len(bad)} scores off, first {bad[:3]}, max err {err.max():.3e}"
    # the background rows (w = 0) score exactly 1/2
    empty = np.flatnonzero(np.abs(deq).sum(1) == 0)
    assert (got[empty] == 0.5).all()


def test_relevancy_empty_map():
    require_gpu()
    C = torch.from_numpy(sg.random_codebook(1, 16, 32)).cuda()
    qs = torch.from_numpy(sg.random_unit_vectors(2, 4, 32)).cuda()
    cs = torch.from_numpy(sg.random_unit_vectors(3, 4, 32)).cuda()
    out = P.relevancy(torch.empty((0, 16), device="cuda"), C, qs, cs, in_dtype="f32")
    assert out.shape == (0, 4)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_relevancy_full_view_sampled(dtype):
    """1440 x 1080 pixels, M = 256, D = 512, 16 queries, 4 canonical vectors:
    the launch the benchmark times, checked on 4000 sampled pixels."""
    require_gpu()
    W, H, m, d, q = 1440, 1080, 256, 512, 16
    n = W * H
    pool = sg.random_coeff_rows(7, 1 << 15, m)
    rng = np.random.default_rng(8)
    pick = rng.integers(0, pool.shape[0], n)
    scale = 256.0 if dtype == "fp8" else 1.0
    pool_dev, pool_deq = _store(pool, dtype, scale)
    coeff = pool_dev[torch.from_numpy(pick).cuda()]
    C = sg.random_codebook(9, m, d)
    qs = sg.random_unit_vectors(10, q, d)
    cs = sg.random_unit_vectors(11, 4, d)
    out = P.relevancy(coeff, torch.from_numpy(C).cuda(), torch.from_numpy(qs).cuda(), torch.from_numpy(cs).cuda(),
                      in_dtype=dtype, coeff_scale=scale, temperature=TEMP)
    torch.cuda.synchronize()
    sample = np.concatenate([rng.integers(0, n, 3990), np.arange(n - 10, n)])
    got = out[torch.from_numpy(sample).cuda()].cpu().numpy().astype(np.float64)
    w = pool_deq[pick[sample]]
    ref = OR.relevancy_map(w, C, qs, cs, TEMP)
    tol = _bound(w, C, qs, cs, dtype)[:, None]
    assert (np.abs(got - ref) <= tol).all(), np.abs(got - ref).max()
    assert torch.isfinite(out).all()
