"""Torch-facing wrappers of the libscoup C ABI.

torch supplies device memory and the stream; every arithmetic step runs in
libscoup's HIP kernels.  Inputs are torch tensors already on the GPU (or
host arrays that these helpers copy there once).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


class ScoupError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libscoup status {status}: {msg}")
        self.status = status


def _check(status: int) -> None:
    if status != L.OK:
        raise ScoupError(status, L.load().scoup_last_error().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclasses.dataclass
class DeviceGaussians:
    """Gaussians on the GPU: means (N,3), log_scales (N,3), quats (N,4) w-first,
    opacities (N,), all float32 contiguous."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def struct(self) -> L.Gaussians:
        return L.Gaussians(self.n, _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats),
                           _ptr(self.opacities))


def camera_struct(cam) -> L.Camera:
    """scoup_camera from any object with R, t, fx, fy, cx, cy, width, height, near."""
    c = L.Camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).reshape(3)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_z = float(getattr(cam, "near", 0.2))
    return c


@dataclasses.dataclass
class DeviceViews:
    """Per-view inputs of the uplift with the region maps and codes on the GPU."""
    cams: Sequence
    region_maps: torch.Tensor      # int32, all views concatenated
    map_offsets: np.ndarray        # int64 (V+1,)
    region_base: np.ndarray        # int64 (V+1,)
    code_idx: torch.Tensor         # int32 (R_total, k_code)
    code_val: torch.Tensor         # float32 (R_total, k_code)
    m_atoms: int

    def __post_init__(self):
        self._cams = (L.Camera * max(1, len(self.cams)))(*[camera_struct(c) for c in self.cams])
        self._moff = np.ascontiguousarray(self.map_offsets, np.int64)
        self._rbase = np.ascontiguousarray(self.region_base, np.int64)

    @property
    def n_views(self) -> int:
        return len(self.cams)

    @property
    def k_code(self) -> int:
        return int(self.code_idx.shape[1])

    def struct(self) -> L.Views:
        return L.Views(self.n_views, self._cams, _ptr(self.region_maps),
                       self._moff.ctypes.data_as(C.POINTER(C.c_int64)),
                       self._rbase.ctypes.data_as(C.POINTER(C.c_int64)),
                       _ptr(self.code_idx), _ptr(self.code_val), self.k_code, int(self.m_atoms))


def gaussians_to_device(g, device="cuda") -> DeviceGaussians:
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
    return DeviceGaussians(f(g.means), f(g.log_scales), f(g.quats), f(g.opacities))


def views_to_device(v, device="cuda") -> DeviceViews:
    """Copy an object with cameras, region_maps, region_base, code_idx, code_val,
    m_atoms (host arrays) to the GPU."""
    maps = [np.ascontiguousarray(m, np.int32).reshape(-1) for m in v.region_maps]
    off = np.zeros(len(maps) + 1, np.int64)
    off[1:] = np.cumsum([m.size for m in maps])
    rm = torch.from_numpy(np.concatenate(maps) if maps else np.zeros(1, np.int32)).to(device)
    ci = torch.as_tensor(np.ascontiguousarray(v.code_idx, np.int32)).to(device)
    cv = torch.as_tensor(np.ascontiguousarray(v.code_val, np.float32)).to(device)
    return DeviceViews(list(v.cameras), rm, off, np.asarray(v.region_base, np.int64), ci, cv,
                       int(v.m_atoms))


_capacity_cache = {}


class Workspace:
    """Grow-only device workspace for the uplift calls."""

    def __init__(self, device="cuda"):
        self.buf = None
        self.device = device

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _workspace(device) -> Workspace:
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


WORKSPACE_LIMIT = 48 << 30   # the uplift workspace is capped here by batching views


def _uplift_call(g: DeviceGaussians, views: DeviceViews, acc: torch.Tensor, accumulate: bool, k: int,
                 idx: Optional[torch.Tensor], val: Optional[torch.Tensor], stream, workspace,
                 pair_capacity: int, view_batch: int):
    lib = L.load()
    dev = g.means.device
    ws = workspace or _workspace(dev)
    gs, vs = g.struct(), views.struct()
    key = ("uplift", g.n, views.n_views, int(views._moff[-1]))
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0), 6 * g.n, 1 << 16)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        vb = int(view_batch) if view_batch else max(1, views.n_views)
        while vb > 1 and lib.scoup_uplift_workspace_bytes(g.n, C.byref(vs), cap, vb) > WORKSPACE_LIMIT:
            vb = (vb + 1) // 2
        nbytes = lib.scoup_uplift_workspace_bytes(g.n, C.byref(vs), cap, vb)
        buf = ws.get(nbytes)
        cnt.zero_()
        if k > 0:
            st = lib.scoup_uplift(C.byref(gs), C.byref(vs), k, _ptr(acc), _ptr(idx), _ptr(val), cap, vb,
                                  _ptr(buf), buf.numel(), _ptr(cnt), _stream(stream))
        else:
            st = lib.scoup_uplift_accumulate(C.byref(gs), C.byref(vs), _ptr(acc), int(accumulate), cap, vb,
                                             _ptr(buf), buf.numel(), _ptr(cnt), _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.1) + 4096
            _capacity_cache[key] = cap
            continue
        _check(st)
        return int(cnt.item())
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def uplift_accumulate(g: DeviceGaussians, views: DeviceViews, acc: Optional[torch.Tensor] = None,
                      accumulate: bool = False, stream=None, workspace: Optional[Workspace] = None,
                      pair_capacity: int = 0, view_batch: int = 0):
    """acc (N, M) float32 += Eq. 5 over every view (zeroed first unless ``accumulate``).
    Returns (acc, n_contrib)."""
    if acc is None:
        acc = torch.empty((g.n, views.m_atoms), dtype=torch.float32, device=g.means.device)
    nc = _uplift_call(g, views, acc, accumulate, 0, None, None, stream, workspace, pair_capacity, view_batch)
    return acc, nc


def uplift_levels(g: DeviceGaussians, levels: Sequence[DeviceViews], k: int, stream=None, workspace=None,
                  pair_capacity: int = 0, view_batch: int = 0, entropy: bool = False):
    """Several semantic levels (same cameras, own region maps and codes) from one
    compositing pass per view.  Returns ([idx], [val], [acc], n_contrib) -- and
    [entropy] last if ``entropy`` -- one entry per level."""
    lib = L.load()
    dev = g.means.device
    nl = len(levels)
    m = levels[0].m_atoms
    accs = [torch.empty((g.n, m), dtype=torch.float32, device=dev) for _ in range(nl)]
    idxs = [torch.empty((g.n, max(k, 1)), dtype=torch.int32, device=dev) for _ in range(nl)]
    vals = [torch.empty((g.n, max(k, 1)), dtype=torch.float32, device=dev) for _ in range(nl)]
    arr = (L.Views * nl)(*[lv.struct() for lv in levels])
    P = C.c_void_p * nl
    pa, pi, pv = P(*[t.data_ptr() for t in accs]), P(*[t.data_ptr() for t in idxs]), P(*[t.data_ptr() for t in vals])
    ents = [torch.empty(g.n, dtype=torch.float32, device=dev) for _ in range(nl)] if entropy else None
    pe = P(*[t.data_ptr() for t in ents]) if entropy else None
    ws = workspace or _workspace(dev)
    gs = g.struct()
    key = ("uplift", g.n, levels[0].n_views, int(levels[0]._moff[-1]))
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0), 6 * g.n, 1 << 16)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        vb = int(view_batch) if view_batch else max(1, levels[0].n_views)
        while vb > 1 and lib.scoup_uplift_levels_workspace_bytes(g.n, nl, arr, cap, vb) > WORKSPACE_LIMIT:
            vb = (vb + 1) // 2
        buf = ws.get(lib.scoup_uplift_levels_workspace_bytes(g.n, nl, arr, cap, vb))
        cnt.zero_()
        st = lib.scoup_uplift_levels(C.byref(gs), nl, arr, k, pa, pi, pv, pe, cap, vb, _ptr(buf), buf.numel(),
                                     _ptr(cnt), _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.1) + 4096
            _capacity_cache[key] = cap
            continue
        _check(st)
        if entropy:
            return idxs, vals, accs, int(cnt.item()), ents
        return idxs, vals, accs, int(cnt.item())
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def uplift_dense(g: DeviceGaussians, views: DeviceViews, codebook: torch.Tensor, stream=None, workspace=None,
                 pair_capacity: int = 0, view_batch: int = 0):
    """Dense feature uplift (Eq. 3) with F_v(p) = W_v(p) C: returns
    (features (N, D) float32, Z (N,) float32, n_contrib)."""
    lib = L.load()
    dev = g.means.device
    d = int(codebook.shape[1])
    feat = torch.empty((g.n, d), dtype=torch.float32, device=dev)
    z = torch.empty(g.n, dtype=torch.float32, device=dev)
    ws = workspace or _workspace(dev)
    gs, vs = g.struct(), views.struct()
    key = ("uplift", g.n, views.n_views, int(views._moff[-1]))
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0), 6 * g.n, 1 << 16)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        vb = int(view_batch) if view_batch else max(1, views.n_views)
        while vb > 1 and lib.scoup_uplift_dense_workspace_bytes(g.n, C.byref(vs), d, cap, vb) > WORKSPACE_LIMIT:
            vb = (vb + 1) // 2
        buf = ws.get(lib.scoup_uplift_dense_workspace_bytes(g.n, C.byref(vs), d, cap, vb))
        cnt.zero_()
        st = lib.scoup_uplift_dense(C.byref(gs), C.byref(vs), _ptr(codebook), d, _ptr(feat), _ptr(z), cap, vb,
                                    _ptr(buf), buf.numel(), _ptr(cnt), _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.1) + 4096
            _capacity_cache[key] = cap
            continue
        _check(st)
        return feat, z, int(cnt.item())
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def entropy(acc: torch.Tensor, stream=None) -> torch.Tensor:
    """Row entropy of the coefficient distribution (App. C.2) of acc (N, M)."""
    lib = L.load()
    n, m = acc.shape
    out = torch.empty(n, dtype=torch.float32, device=acc.device)
    _check(lib.scoup_entropy(_ptr(acc), n, m, _ptr(out), _stream(stream)))
    return out


def topk(acc: torch.Tensor, k: int, stream=None):
    """Eq. 6 per row of acc (N, M): (idx int32 (N,k), val float32 (N,k))."""
    lib = L.load()
    n, m = acc.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=acc.device)
    val = torch.empty((n, k), dtype=torch.float32, device=acc.device)
    _check(lib.scoup_topk(_ptr(acc), n, m, k, _ptr(idx), _ptr(val), _stream(stream)))
    return idx, val


def set_views_in_flight(k: int) -> None:
    """Views the uplift projects, bins and composites at the same time (1..4)."""
    L.load().scoup_set_views_in_flight(int(k))


def views_in_flight() -> int:
    return int(L.load().scoup_views_in_flight())


def stage_timing(enable: bool) -> None:
    """Per-stage kernel timing (HIP events) and uplift statistics on or off
    (turning either way resets the counters)."""
    L.load().scoup_stage_timing(1 if enable else 0)


def uplift_touch_stats() -> dict:
    """Uplift statistics collected while stage timing is on: distinct
    (Gaussian, region) pairs with weight summed over views (U_v), pairs the
    counting set lost, direct further-region adds, views counted."""
    vals = [C.c_uint64() for _ in range(4)]
    L.load().scoup_uplift_touch_stats(*[C.byref(x) for x in vals])
    return dict(zip(("touches", "lost", "direct", "views"), (int(x.value) for x in vals)))


def set_deferred_entry_limit(n: int) -> None:
    """Cap the uplift's per-view buffer of deferred further-region entries at
    ``n`` entries (0 = the workspace's capacity); past it the compositing adds
    those weights to the accumulator directly."""
    L.load().scoup_set_deferred_entry_limit(int(n))


def uplift(g: DeviceGaussians, views: DeviceViews, k: int, stream=None, workspace=None,
           pair_capacity: int = 0, view_batch: int = 0, acc: Optional[torch.Tensor] = None):
    """Algorithm 1: accumulate over all views, then Top-K (fused into the last
    accumulation pass).  Returns (idx (N,k) int32, val (N,k) float32,
    acc (N,M) float32, n_contrib)."""
    dev = g.means.device
    if acc is None:
        acc = torch.empty((g.n, views.m_atoms), dtype=torch.float32, device=dev)
    idx = torch.empty((g.n, k), dtype=torch.int32, device=dev)
    val = torch.empty((g.n, k), dtype=torch.float32, device=dev)
    nc = _uplift_call(g, views, acc, False, k, idx, val, stream, workspace, pair_capacity, view_batch)
    return idx, val, acc, nc


_DT = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8_E4M3}
_TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.uint8}
FP8_COEFF_SCALE = 256.0   # rendered coefficients are <= 1; x256 keeps them inside E4M3's range


def render_coeff(g: DeviceGaussians, topk_idx: torch.Tensor, topk_val: torch.Tensor, cam, m_atoms: int,
                 dtype: str = "f32", scale: Optional[float] = None, want_t_final: bool = True,
                 stream=None, workspace: Optional[Workspace] = None, pair_capacity: int = 0):
    """Eq. 7 for one camera: coefficient map (H, W, M) in ``dtype`` (``f32``,
    ``bf16`` or ``fp8`` = E4M3 bytes scaled by ``scale``), the final
    transmittance (H, W) and the contribution count."""
    lib = L.load()
    dev = g.means.device
    c = camera_struct(cam)
    H, W = int(cam.height), int(cam.width)
    if scale is None:
        scale = FP8_COEFF_SCALE if dtype == "fp8" else 1.0
    out = torch.empty((H, W, m_atoms), dtype=_TORCH_DT[dtype], device=dev)
    tf = torch.empty((H, W), dtype=torch.float32, device=dev) if want_t_final else None
    ws = workspace or _workspace(dev)
    gs = g.struct()
    k = int(topk_idx.shape[1])
    key = ("render", g.n, W, H)
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0))
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        nbytes = lib.scoup_render_workspace_bytes(g.n, C.byref(c), cap)
        buf = ws.get(nbytes)
        cnt.zero_()
        st = lib.scoup_render_coeff(C.byref(gs), _ptr(topk_idx), _ptr(topk_val), k, m_atoms, C.byref(c),
                                    _ptr(out), _DT[dtype], float(scale), _ptr(tf), _ptr(buf), buf.numel(),
                                    _ptr(cnt), _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.25) + 1024
            _capacity_cache[key] = cap
            continue
        _check(st)
        return out, tf, int(cnt.item()), float(scale)
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def render(g: DeviceGaussians, topk_idx: torch.Tensor, topk_val: torch.Tensor, codebook: torch.Tensor, cam,
           in_dtype: str = "bf16", out_dtype: str = "bf16", want_coeff: bool = False, want_t_final: bool = True,
           stream=None, workspace: Optional[Workspace] = None, pair_capacity: int = 0):
    """Sec. 4.3 render in one pass (Eq. 7 then Eq. 8): per-pixel features
    (H, W, D) in ``out_dtype`` decoded on MFMA in ``in_dtype`` from the float32
    coefficient rows, which stay on chip.  Returns (features, coeff (H, W, M)
    float32 or None, t_final (H, W) or None, n_contrib)."""
    lib = L.load()
    dev = g.means.device
    c = camera_struct(cam)
    H, W = int(cam.height), int(cam.width)
    m, d = codebook.shape
    k = int(topk_idx.shape[1])
    feat = torch.empty((H, W, d), dtype=_TORCH_DT[out_dtype], device=dev)
    coeff = torch.empty((H, W, m), dtype=torch.float32, device=dev) if want_coeff else None
    tf = torch.empty((H, W), dtype=torch.float32, device=dev) if want_t_final else None
    ws = workspace or _workspace(dev)
    gs = g.struct()
    key = ("render", g.n, W, H)
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0))
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        nbytes = lib.scoup_render_decode_workspace_bytes(g.n, C.byref(c), m, d, _DT[in_dtype], cap)
        buf = ws.get(nbytes)
        cnt.zero_()
        st = lib.scoup_render(C.byref(gs), _ptr(topk_idx), _ptr(topk_val), k, C.byref(c), _ptr(codebook), m, d,
                              _DT[in_dtype], _ptr(coeff), _ptr(tf), _ptr(feat), _DT[out_dtype], _ptr(buf),
                              buf.numel(), _ptr(cnt), _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.25) + 1024
            _capacity_cache[key] = cap
            continue
        _check(st)
        return feat, coeff, tf, int(cnt.item())
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def render_views(g: DeviceGaussians, topk_idx: torch.Tensor, topk_val: torch.Tensor, codebook: torch.Tensor, cams,
                 in_dtype: str = "bf16", out_dtype: str = "bf16", stream=None, workspace: Optional[Workspace] = None,
                 pair_capacity: int = 0):
    """``render`` for several cameras of one image size, views in flight
    (Sec. 4.3, Eq. 7 then Eq. 8 per view).  Returns (features (V, H, W, D),
    n_contrib over all views); view v equals ``render`` on cams[v]."""
    lib = L.load()
    dev = g.means.device
    cams = list(cams)
    nv = len(cams)
    m, d = codebook.shape
    k = int(topk_idx.shape[1])
    H, W = (int(cams[0].height), int(cams[0].width)) if nv else (0, 0)
    feat = torch.empty((nv, H, W, d), dtype=_TORCH_DT[out_dtype], device=dev)
    if nv == 0:
        return feat, 0
    carr = (L.Camera * nv)(*[camera_struct(c) for c in cams])
    ws = workspace or _workspace(dev)
    gs = g.struct()
    key = ("render", g.n, W, H)
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0))
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(4):
        nbytes = lib.scoup_render_views_workspace_bytes(g.n, C.byref(carr[0]), nv, m, d, _DT[in_dtype], cap)
        buf = ws.get(nbytes)
        cnt.zero_()
        st = lib.scoup_render_views(C.byref(gs), _ptr(topk_idx), _ptr(topk_val), k, carr, nv, _ptr(codebook), m, d,
                                    _DT[in_dtype], _ptr(feat), _DT[out_dtype], _ptr(buf), buf.numel(), _ptr(cnt),
                                    _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.25) + 1024
            _capacity_cache[key] = cap
            continue
        _check(st)
        return feat, int(cnt.item())
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


def decode(coeff: torch.Tensor, codebook: torch.Tensor, in_dtype: str = "bf16", coeff_scale: float = 1.0,
           out_dtype: str = "bf16", stream=None, workspace: Optional[Workspace] = None) -> torch.Tensor:
    """Eq. 8: features = coeff @ codebook on MFMA.  ``coeff`` is (..., M) in
    ``in_dtype`` storage (float32, bfloat16 or E4M3 bytes scaled by
    ``coeff_scale``); ``codebook`` is the float32 (M, D) codebook, converted
    to ``in_dtype`` by the library.  Returns (..., D) in ``out_dtype``."""
    lib = L.load()
    m, d = codebook.shape
    P = coeff.numel() // m
    out = torch.empty((*coeff.shape[:-1], d), dtype=_TORCH_DT[out_dtype], device=coeff.device)
    ws = workspace or Workspace(coeff.device)
    buf = ws.get(lib.scoup_decode_workspace_bytes(m, d, _DT[in_dtype]))
    _check(lib.scoup_decode(_ptr(coeff), _DT[in_dtype], float(coeff_scale), P, m, _ptr(codebook), d,
                            _ptr(out), _DT[out_dtype], _ptr(buf), buf.numel(), _stream(stream)))
    return out


def relevancy(coeff: torch.Tensor, codebook: torch.Tensor, queries: torch.Tensor, canon: torch.Tensor,
              in_dtype: str = "bf16", coeff_scale: float = 1.0, temperature: float = 10.0, stream=None,
              workspace: Optional[Workspace] = None) -> torch.Tensor:
    """App. B relevancy of every pixel to every query on the decoded features
    coeff @ codebook, without forming them.  ``coeff`` is (..., M) in
    ``in_dtype`` storage; ``queries`` (Q, D) and ``canon`` (n_canon <= 4, D)
    are float32.  Returns (..., Q) float32 scores."""
    lib = L.load()
    m, d = codebook.shape
    P = coeff.numel() // m
    q = int(queries.shape[0])
    out = torch.empty((*coeff.shape[:-1], q), dtype=torch.float32, device=coeff.device)
    ws = workspace or Workspace(coeff.device)
    buf = ws.get(lib.scoup_relevancy_workspace_bytes(m, q, _DT[in_dtype]))
    _check(lib.scoup_relevancy(_ptr(coeff), _DT[in_dtype], float(coeff_scale), P, m, _ptr(codebook), d,
                               _ptr(queries), q, _ptr(canon), int(canon.shape[0]), float(temperature),
                               _ptr(out), _ptr(buf), buf.numel(), _stream(stream)))
    return out


def render_backward(g: DeviceGaussians, topk_idx: torch.Tensor, topk_val: torch.Tensor, cam,
                    coeff_map: torch.Tensor, codebook: torch.Tensor, grad_features: torch.Tensor,
                    grad_topk_val: Optional[torch.Tensor] = None, grad_codebook: Optional[torch.Tensor] = None,
                    stream=None, workspace: Optional[Workspace] = None, pair_capacity: int = 0):
    """Backward of render + decode for one camera (float32).  Accumulates into
    (and returns) grad_topk_val (N, K) and grad_codebook (M, D)."""
    lib = L.load()
    dev = g.means.device
    m, d = codebook.shape
    k = int(topk_idx.shape[1])
    if grad_topk_val is None:
        grad_topk_val = torch.zeros_like(topk_val)
    if grad_codebook is None:
        grad_codebook = torch.zeros_like(codebook)
    c = camera_struct(cam)
    ws = workspace or _workspace(dev)
    gs = g.struct()
    key = ("render", g.n, int(cam.width), int(cam.height))
    cap = max(int(pair_capacity), _capacity_cache.get(key, 0))
    for _ in range(4):
        nbytes = lib.scoup_render_backward_workspace_bytes(g.n, C.byref(c), m, d, cap)
        buf = ws.get(nbytes)
        st = lib.scoup_render_backward(C.byref(gs), _ptr(topk_idx), _ptr(topk_val), k, m, C.byref(c),
                                       _ptr(coeff_map), _ptr(codebook), d, _ptr(grad_features),
                                       _ptr(grad_topk_val), _ptr(grad_codebook), _ptr(buf), buf.numel(),
                                       _stream(stream))
        if st == L.E_WORKSPACE:
            cap = int(lib.scoup_required_pair_capacity() * 1.25) + 1024
            _capacity_cache[key] = cap
            continue
        _check(st)
        return grad_topk_val, grad_codebook
    raise ScoupError(L.E_WORKSPACE, "workspace retry limit reached")


class RenderDecode(torch.autograd.Function):
    """features (H, W, D) float32 = decode(render(topk, cam), codebook), with
    gradients for ``topk_val`` and ``codebook`` from libscoup's backward.
    Also returns the final transmittance (H, W) (not differentiable)."""

    @staticmethod
    def forward(ctx, topk_val, codebook, g, topk_idx, cam):
        F, W, tf, _ = render(g, topk_idx, topk_val, codebook, cam, in_dtype="f32", out_dtype="f32",
                             want_coeff=True)
        ctx.save_for_backward(topk_val, codebook, topk_idx, W)
        ctx.g, ctx.cam = g, cam
        ctx.mark_non_differentiable(tf)
        return F, tf

    @staticmethod
    def backward(ctx, dF, dtf):
        topk_val, codebook, topk_idx, W = ctx.saved_tensors
        gv, gc = render_backward(ctx.g, topk_idx, topk_val, ctx.cam, W, codebook, dF.contiguous())
        return gv, gc, None, None, None


def render_decode(g: DeviceGaussians, topk_idx: torch.Tensor, topk_val: torch.Tensor, codebook: torch.Tensor,
                  cam):
    """Differentiable render + decode (float32): returns (features, t_final)."""
    return RenderDecode.apply(topk_val, codebook, g, topk_idx, cam)
