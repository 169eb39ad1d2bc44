"""The C ABI library loads, exports every symbol include/scoup.h declares, and
validates arguments on the host (no device work is started by these calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2605_13600_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "scoup.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(scoup_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    syms = declared_symbols()
    assert len(syms) >= 7
    for s in syms:
        assert hasattr(lib, s), s
        assert s in L.SIGNATURES, f"{s} has no ctypes signature"


def test_version_and_error_strings():
    lib = L.load()
    assert b"gfx950" in lib.scoup_version()
    assert isinstance(lib.scoup_last_error(), bytes)


def test_topk_argument_validation():
    lib = L.load()
    assert lib.scoup_topk(None, 10, 64, 0, None, None, None) == L.E_ARG
    assert lib.scoup_topk(None, 10, 64, 65, None, None, None) == L.E_ARG
    assert lib.scoup_topk(None, 10, 8, 9, None, None, None) == L.E_ARG
    assert lib.scoup_topk(None, 10, 5000, 4, None, None, None) == L.E_ARG
    assert lib.scoup_topk(None, 10, 64, 4, None, None, None) == L.E_ARG
    assert b"NULL" in lib.scoup_last_error()


def _views(width=64, height=48, n_views=1, offsets=None):
    cams = (L.Camera * n_views)()
    for c in cams:
        c.R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
        c.fx = c.fy = 50.0; c.cx = width / 2; c.cy = height / 2
        c.width, c.height, c.near_z = width, height, 0.2
    off = np.array(offsets if offsets is not None else [i * width * height for i in range(n_views + 1)], np.int64)
    base = np.arange(n_views + 1, dtype=np.int64) * 4
    v = L.Views(n_views, cams, 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                base.ctypes.data_as(C.POINTER(C.c_int64)), 1, 1, 4, 64)
    return v, (cams, off, base)


def test_uplift_argument_validation():
    lib = L.load()
    v, keep = _views()
    g = L.Gaussians(10, 1, 1, 1, 1)
    ws = lib.scoup_uplift_workspace_bytes(10, C.byref(v), 0, 0)
    assert ws > 0
    assert lib.scoup_uplift_workspace_bytes(10, C.byref(v), 1 << 20, 1) >= (1 << 20) * 40
    cap = 1 << 16
    ws = lib.scoup_uplift_workspace_bytes(10, C.byref(v), cap, 1)
    # NULL acc / workspace, misaligned workspace, bad K, bad capacity, mismatched map size
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(v), None, 0, cap, 1, 256, ws, None, None) == L.E_ARG
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(v), 256, 0, cap, 1, None, ws, None, None) == L.E_ARG
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(v), 256, 0, cap, 1, 257, ws, None, None) == L.E_ARG
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(v), 256, 0, 0, 1, 256, ws, None, None) == L.E_ARG
    assert lib.scoup_uplift(C.byref(g), C.byref(v), 0, 256, 256, 256, cap, 1, 256, ws, None, None) == L.E_ARG
    assert lib.scoup_uplift(C.byref(g), C.byref(v), 65, 256, 256, 256, cap, 1, 256, ws, None, None) == L.E_ARG
    bad, keep2 = _views(offsets=[0, 100])
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(bad), 256, 0, cap, 1, 256, ws, None, None) == L.E_ARG
    assert b"map_offsets" in lib.scoup_last_error()
    # workspace smaller than the capacity and view batch need
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(v), 256, 0, cap, 1, 256, 1024, None, None) \
        == L.E_WORKSPACE
    assert lib.scoup_required_pair_capacity() > 0
    neg = L.Gaussians(-1, 1, 1, 1, 1)
    assert lib.scoup_uplift_accumulate(C.byref(neg), C.byref(v), 256, 0, cap, 1, 256, ws, None, None) == L.E_ARG
    big, keep3 = _views(width=40000)
    assert lib.scoup_uplift_accumulate(C.byref(g), C.byref(big), 256, 0, cap, 1, 256, ws, None, None) == L.E_ARG


def test_relevancy_argument_validation():
    lib = L.load()
    fake = C.c_void_p(0x1000)          # never dereferenced: every call below fails validation first
    ws = C.c_void_p(0x10000)
    args = dict(coeff=fake, dt=L.F32, scale=1.0, P=100, m=64, cb=fake, d=32, q=fake, nq=16, c=fake, nc=4,
                temp=10.0, out=fake, ws=ws, wsb=1 << 30)

    def call(**kw):
        a = {**args, **kw}
        return lib.scoup_relevancy(a["coeff"], a["dt"], a["scale"], a["P"], a["m"], a["cb"], a["d"], a["q"],
                                   a["nq"], a["c"], a["nc"], a["temp"], a["out"], a["ws"], a["wsb"], None)

    assert call(nc=0) == L.E_ARG and call(nc=5) == L.E_ARG
    assert call(nq=0) == L.E_ARG and call(nq=1025) == L.E_ARG
    assert call(temp=0.0) == L.E_ARG and call(temp=float("inf")) == L.E_ARG
    assert call(m=0) == L.E_ARG and call(d=0) == L.E_ARG and call(dt=7) == L.E_ARG
    assert call(scale=-1.0) == L.E_ARG and call(P=-1) == L.E_ARG
    assert call(q=None) == L.E_ARG and call(out=None) == L.E_ARG and call(c=None) == L.E_ARG
    assert call(ws=C.c_void_p(0x10001)) == L.E_ARG
    assert call(wsb=16) == L.E_WORKSPACE
    assert b"workspace" in lib.scoup_last_error()
    # workspace: one S fragment set per group of 24 queries, two bfloat16 terms for BF16 / FP8 maps
    b24 = lib.scoup_relevancy_workspace_bytes(256, 24, L.BF16)
    assert lib.scoup_relevancy_workspace_bytes(256, 25, L.BF16) == 2 * b24
    assert lib.scoup_relevancy_workspace_bytes(256, 16, L.F32) == 256 * 32 * 4
    assert b24 == 256 * 32 * 2 * 2
    assert lib.scoup_relevancy_workspace_bytes(0, 16, L.F32) == 0
