"""The no-allocation decode entry point (scoup_decode_noalloc) against
scoup_decode, through the C ABI: the same kernels on the same inputs, so the
features must be bit-identical.  Two calls in a row, the second smaller (the
scratch keeps the first call's codebook; the second must not see it), in
every input precision; a codebook larger than the scratch is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen as sg
from paper_2605_13600_amd import _lib as L
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu

_DT = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8_E4M3}


def _coeff(seed, p, m, dt):
    A = torch.from_numpy(sg.random_coeff_rows(seed, p, m)).cuda()
    if dt == "f32":
        return A, 1.0
    if dt == "bf16":
        return A.to(torch.bfloat16), 1.0
    return (A * 256.0).to(torch.float8_e4m3fn).view(torch.uint8), 256.0


def _both(lib, A, scale, dt, cb, out_dt="bf16"):
    p, m = A.shape
    d = cb.shape[1]
    odt = torch.float32 if out_dt == "f32" else torch.bfloat16
    ref = torch.full((p, d), 7.0, dtype=odt, device="cuda")
    got = torch.full((p, d), -7.0, dtype=odt, device="cuda")
    nb = lib.scoup_decode_workspace_bytes(m, d, _DT[dt])
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    st = lib.scoup_decode(A.data_ptr(), _DT[dt], scale, p, m, cb.data_ptr(), d, ref.data_ptr(), _DT[out_dt],
                          ws.data_ptr(), nb, s)
    assert st == L.OK, lib.scoup_last_error()
    st = lib.scoup_decode_noalloc(A.data_ptr(), _DT[dt], scale, p, m, cb.data_ptr(), d, got.data_ptr(),
                                  _DT[out_dt], s)
    assert st == L.OK, lib.scoup_last_error()
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("dt", ["fp8", "bf16", "f32"])
def test_noalloc_decode_equals_workspace_decode_twice(dt):
    require_gpu()
    lib = L.load()
    assert lib.scoup_decode_noalloc_max_bytes() == 8 << 20
    first = (3000, 256, 512, 11)
    second = (777, 128, 200, 12)      # smaller: fewer pixels, atoms and features
    for p, m, d, seed in (first, second):
        A, scale = _coeff(seed, p, m, dt)
        cb = torch.from_numpy(sg.random_codebook(seed + 100, m, d) * (3.0 if seed == 12 else 1.0)).cuda()
        out_dt = "f32" if dt == "f32" else "bf16"
        ref, got = _both(lib, A, scale, dt, cb, out_dt)
        assert torch.equal(ref.view(torch.int16) if ref.dtype == torch.bfloat16 else ref.view(torch.int32),
                           got.view(torch.int16) if got.dtype == torch.bfloat16 else got.view(torch.int32)), \
            (dt, p, m, d, float((ref.float() - got.float()).abs().max()))
        print(f"[noalloc {dt}] {p}x{m} @ {m}x{d}: bit-identical", flush=True)


def test_noalloc_decode_refuses_codebooks_beyond_the_scratch():
    require_gpu()
    lib = L.load()
    m, d = 4096, 1024                  # float32 codebook of 16 MiB
    assert lib.scoup_decode_workspace_bytes(m, d, L.F32) > lib.scoup_decode_noalloc_max_bytes()
    cb = torch.zeros((m, d), dtype=torch.float32, device="cuda")
    out = torch.empty((1, d), dtype=torch.float32, device="cuda")
    A = torch.zeros((1, m), dtype=torch.float32, device="cuda")
    st = lib.scoup_decode_noalloc(A.data_ptr(), L.F32, 1.0, 1, m, cb.data_ptr(), d, out.data_ptr(), L.F32, None)
    assert st == L.E_ARG and b"scratch" in lib.scoup_last_error()
