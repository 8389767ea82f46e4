"""Torch-facing wrapper of libqgs: device buffers, streams and autograd.

PyTorch provides memory and the current HIP stream; every step of the
rendering runs in the HIP kernels behind the C ABI (see include/qgs.h).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

SCENE_KEYS = ("center", "quat", "scale", "curv", "opacity", "rgb")
SCENE_SHAPES = {"center": 3, "quat": 4, "scale": 2, "curv": 2, "opacity": 0, "rgb": 3}


def make_camera(cam) -> L.QgsCamera:
    """QgsCamera from an object with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    c = L.QgsCamera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def make_opts(tight_bound: bool = True, **kw) -> L.QgsRenderOpts:
    """qgs_default_opts() with fields replaced by keyword.  `flags` is added to
    the default flags; tight_bound=False clears QGS_TIGHT_BOUND (the k-sigma
    local box without the chord bound)."""
    o = L.qgs_default_opts()
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        elif k == "flags":
            o.flags |= int(v)
        else:
            setattr(o, k, float(v))
    if not tight_bound:
        o.flags &= ~L.QGS_TIGHT_BOUND
    return o


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def scene_to_device(scene, device="cuda") -> dict:
    """Dict of contiguous FP32 device tensors from a scenes.Scene (with "sh"
    [n, K, 3] when the scene has spherical-harmonics colour)."""
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k), np.float32)).to(device) for k in SCENE_KEYS}
    if getattr(scene, "sh", None) is not None:
        t["sh"] = torch.from_numpy(np.ascontiguousarray(scene.sh, np.float32)).to(device)
    return t


def sh_degree_of(t: dict) -> int:
    """Degree of the SH colour of a device scene dict (-1: plain rgb)."""
    sh = t.get("sh")
    if sh is None:
        return -1
    deg = int(round(sh.shape[1] ** 0.5)) - 1
    if (deg + 1) ** 2 != sh.shape[1] or not 0 <= deg <= 3 or sh.shape[-1] != 3:
        raise ValueError("sh must be [n, (degree + 1)^2, 3] with degree 0..3")
    return deg


def _scene_struct(t: dict) -> L.QgsScene:
    s = L.QgsScene()
    for k in SCENE_KEYS + (("sh",) if t.get("sh") is not None else ()):
        x = t[k]
        if x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
            raise ValueError(f"scene tensor {k} must be contiguous float32 on the GPU")
        setattr(s, k, x.data_ptr())
    s.sh_degree = max(sh_degree_of(t), 0)
    s.n = int(t["center"].shape[0])
    return s


@dataclass
class FrameState:
    """Device buffers of one rendered view, kept for the backward pass."""
    n: int
    cam: L.QgsCamera
    records: torch.Tensor
    depth_key: torch.Tensor
    rect: torch.Tensor
    tiles: torch.Tensor
    pair_offset: torch.Tensor
    conic: torch.Tensor
    pair_tile: torch.Tensor
    pair_prim: torch.Tensor
    emit_to_sorted: torch.Tensor
    ranges: torch.Tensor
    tile_order: torch.Tensor
    counters: torch.Tensor
    capacity: int
    num_pairs: int | None
    color: torch.Tensor
    depth: torch.Tensor
    normal: torch.Tensor
    T_final: torch.Tensor
    last: torch.Tensor
    # geometry maps (None unless the renderer computes them)
    curvature: torch.Tensor | None = None
    median_depth: torch.Tensor | None = None
    distortion: torch.Tensor | None = None
    median_pos: torch.Tensor | None = None
    frame: torch.Tensor | None = None  # per-primitive frames for the per-tile sort depth
    flags: int = 0  # the renderer's option flags the state was preprocessed with
    # replay bitmap of the forward for the backward
    steps: torch.Tensor | None = None
    step_count: torch.Tensor | None = None

    def prim_buf(self) -> L.QgsPrimBuf:
        p = L.QgsPrimBuf()
        p.records, p.depth_key, p.rect = _ptr(self.records), _ptr(self.depth_key), _ptr(self.rect)
        p.tiles, p.pair_offset, p.n = _ptr(self.tiles), _ptr(self.pair_offset), self.n
        p.conic = _ptr(self.conic)
        p.frame = _ptr(self.frame) if self.frame is not None else None
        return p

    def lists(self) -> L.QgsTileLists:
        l = L.QgsTileLists()
        l.pair_tile, l.pair_prim = _ptr(self.pair_tile), _ptr(self.pair_prim)
        l.emit_to_sorted = _ptr(self.emit_to_sorted) if self.emit_to_sorted is not None else None
        l.ranges, l.counters, l.capacity = _ptr(self.ranges), _ptr(self.counters), self.capacity
        l.tile_order = _ptr(self.tile_order)
        return l

    def images(self) -> L.QgsImages:
        im = L.QgsImages()
        im.color, im.depth, im.normal = _ptr(self.color), _ptr(self.depth), _ptr(self.normal)
        im.T_final, im.last = _ptr(self.T_final), _ptr(self.last)
        if self.curvature is not None:
            im.curvature, im.median_depth = _ptr(self.curvature), _ptr(self.median_depth)
            im.distortion, im.median_pos = _ptr(self.distortion), _ptr(self.median_pos)
        if self.steps is not None:
            im.steps, im.step_count = _ptr(self.steps), _ptr(self.step_count)
        return im


class Renderer:
    """Renders views of a scene through libqgs.

    capacity: pair-list capacity to start from; grown on demand (exact mode) or
    fixed (exact=False, no host synchronisation; overflow is then reported in
    counters[1]).  geometry: also render the curvature, median-depth and
    depth-distortion maps.
    """

    def __init__(self, device="cuda", opts: L.QgsRenderOpts | None = None, capacity: int = 1 << 20,
                 growth: float = 1.25, geometry: bool = False):
        self.device = torch.device(device)
        self.geometry = bool(geometry)
        self.opts = opts if opts is not None else make_opts()
        self.capacity = int(capacity)
        self.growth = growth
        self._sort_ws = None
        self._bwd_ws = None

    def _workspace(self, attr, nbytes):
        buf = getattr(self, attr)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            setattr(self, attr, buf)
        return buf

    def _alloc_lists(self, st: FrameState, cap: int):
        st.capacity = int(cap)
        st.pair_tile = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        st.pair_prim = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        # the emission map is built only for the deterministic backward
        st.emit_to_sorted = (torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
                             if self.opts.flags & L.QGS_DETERMINISTIC_BWD else None)
        ntiles = st.ranges.numel() // 2
        st.steps = torch.empty(L.replay_words(cap, ntiles), dtype=torch.int64, device=self.device)
        st.step_count = torch.empty(4 * ntiles, dtype=torch.int32, device=self.device)

    def preprocess(self, scene_t: dict, cam) -> FrameState:
        n = int(scene_t["center"].shape[0])
        c = cam if isinstance(cam, L.QgsCamera) else make_camera(cam)
        dev = self.device
        H, W = c.height, c.width
        ntiles = ((W + 15) // 16) * ((H + 15) // 16)
        st = FrameState(
            n=n, cam=c,
            records=torch.empty(max(n, 1) * 32, dtype=torch.float32, device=dev),
            depth_key=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            rect=torch.empty(max(n, 1) * 4, dtype=torch.int32, device=dev),
            tiles=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            pair_offset=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            conic=torch.empty(max(n, 1) * 8, dtype=torch.float64, device=dev),
            pair_tile=None, pair_prim=None, emit_to_sorted=None,
            ranges=torch.empty(2 * ntiles, dtype=torch.int32, device=dev),
            tile_order=torch.empty(ntiles, dtype=torch.int32, device=dev),
            counters=torch.zeros(8, dtype=torch.int32, device=dev),
            capacity=0, num_pairs=None,
            color=torch.empty((3, H, W), dtype=torch.float32, device=dev),
            depth=torch.empty((H, W), dtype=torch.float32, device=dev),
            normal=torch.empty((3, H, W), dtype=torch.float32, device=dev),
            T_final=torch.empty((H, W), dtype=torch.float32, device=dev),
            last=torch.empty((H, W), dtype=torch.int32, device=dev),
            flags=int(self.opts.flags),
        )
        if self.opts.flags & L.QGS_TILE_DEPTH:
            st.frame = torch.empty(max(n, 1) * 16, dtype=torch.float64, device=dev)
        if self.geometry:
            st.curvature = torch.empty((H, W), dtype=torch.float32, device=dev)
            st.median_depth = torch.empty((H, W), dtype=torch.float32, device=dev)
            st.distortion = torch.empty((H, W), dtype=torch.float32, device=dev)
            st.median_pos = torch.empty((H, W), dtype=torch.int32, device=dev)
        L.qgs_preprocess(_scene_struct(scene_t), c, self.opts, st.prim_buf(), _stream())
        return st

    def bin_sort(self, st: FrameState, exact: bool = True):
        self._alloc_lists(st, self.capacity)
        while True:
            sort_bytes, _ = L.qgs_workspace_query(st.n, st.cam, st.capacity, self.opts.flags)
            ws = self._workspace("_sort_ws", sort_bytes)
            status, cnt = L.qgs_bin_sort(st.prim_buf(), st.cam, self.opts, st.lists(), ws.data_ptr(), ws.numel(),
                                         want_count=exact, stream=_stream(), raise_on_capacity=False)
            st.num_pairs = cnt
            if status == L.QGS_ERR_CAPACITY:
                self.capacity = max(int(cnt * self.growth) + 1024, self.capacity)
                self._alloc_lists(st, self.capacity)
                continue
            return st

    def render_fwd(self, st: FrameState):
        L.qgs_render_fwd(st.prim_buf(), st.lists(), st.cam, self.opts, st.images(), _stream())
        return st

    def forward(self, scene_t: dict, cam, exact: bool = True) -> FrameState:
        st = self.preprocess(scene_t, cam)
        self.bin_sort(st, exact=exact)
        return self.render_fwd(st)

    def backward(self, scene_t: dict, st: FrameState, dcolor=None, ddepth=None, dnormal=None,
                 out: dict | None = None, accumulate: bool = False, dcurvature=None, dmedian_depth=None,
                 ddistortion=None, stats: dict | None = None) -> dict:
        """Parameter gradients (dict like the scene's, "sh" included when the
        scene has SH colour).  stats: optional {"screen_grad": [n], "visible":
        [n]} FP32 tensors that the densification statistics are added to."""
        keys = SCENE_KEYS + (("sh",) if scene_t.get("sh") is not None else ())
        if out is None:
            out = {k: torch.empty_like(scene_t[k]) for k in keys}
        g = L.QgsSceneGrads()
        for k in keys:
            setattr(g, k, out[k].data_ptr())
        if stats is not None:
            for k in ("screen_grad", "visible"):
                x = stats[k]
                if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != st.n:
                    raise ValueError(f"stats[{k}] must be a contiguous float32 tensor of n entries")
                setattr(g, k, x.data_ptr())
        dl = L.QgsImageGrads()
        keep = []
        geo = (("dcurvature", dcurvature), ("dmedian_depth", dmedian_depth), ("ddistortion", ddistortion))
        if st.curvature is None and any(t is not None for _, t in geo):
            raise ValueError("geometry gradients need a forward rendered with geometry=True")
        for name, t in (("dcolor", dcolor), ("ddepth", ddepth), ("dnormal", dnormal)) + geo:
            if t is not None:
                t = t.contiguous().float()
                keep.append(t)
                setattr(dl, name, t.data_ptr())
        opts = L.QgsRenderOpts.from_buffer_copy(self.opts)
        if (opts.flags & L.QGS_DETERMINISTIC_BWD) and st.emit_to_sorted is None:
            raise ValueError("the deterministic backward needs lists binned with the deterministic flag")
        if accumulate:
            opts.flags |= L.QGS_ACCUMULATE_GRADS
        _, bwd_bytes = L.qgs_workspace_query(st.n, st.cam, st.capacity, opts.flags)
        ws = self._workspace("_bwd_ws", bwd_bytes)
        L.qgs_render_bwd(_scene_struct(scene_t), st.prim_buf(), st.lists(), st.cam, opts, st.images(), dl, g,
                         ws.data_ptr(), ws.numel(), _stream())
        return out


class QGSRasterize(torch.autograd.Function):
    """colour, depth, normal = QGSRasterize.apply(center, quat, scale, curv,
    opacity, rgb, sh, renderer, camera); sh is None for plain rgb colour; with
    a geometry renderer also curvature, median depth and depth distortion."""

    @staticmethod
    def forward(ctx, center, quat, scale, curv, opacity, rgb, sh, renderer: Renderer, cam):
        scene_t = dict(center=center.contiguous(), quat=quat.contiguous(), scale=scale.contiguous(),
                       curv=curv.contiguous(), opacity=opacity.contiguous(), rgb=rgb.contiguous())
        if sh is not None:
            scene_t["sh"] = sh.contiguous()
        st = renderer.forward(scene_t, cam)
        ctx.renderer = renderer
        ctx.state = st
        ctx.has_sh = sh is not None
        ctx.save_for_backward(*[scene_t[k] for k in SCENE_KEYS + (("sh",) if sh is not None else ())])
        if renderer.geometry:
            return st.color, st.depth, st.normal, st.curvature, st.median_depth, st.distortion
        return st.color, st.depth, st.normal

    @staticmethod
    def backward(ctx, dcolor, ddepth, dnormal, *dgeo):
        keys = SCENE_KEYS + (("sh",) if ctx.has_sh else ())
        scene_t = dict(zip(keys, ctx.saved_tensors))
        dk, dm, dd = (tuple(dgeo) + (None, None, None))[:3]
        g = ctx.renderer.backward(scene_t, ctx.state, dcolor, ddepth, dnormal, dcurvature=dk, dmedian_depth=dm,
                                  ddistortion=dd)
        return (g["center"], g["quat"], g["scale"], g["curv"], g["opacity"], g["rgb"], g.get("sh"), None, None)


def render(scene_t: dict, cam, renderer: Renderer | None = None, geometry: bool = False):
    """Differentiable render of one view: (colour [3,H,W], depth [H,W], normal [3,H,W]), and with
    geometry=True also (curvature [H,W], median depth [H,W], depth distortion [H,W]).  scene_t may
    hold "sh" [n, K, 3] for view-dependent colour."""
    r = renderer if renderer is not None else Renderer(device=scene_t["center"].device, geometry=geometry)
    return QGSRasterize.apply(scene_t["center"], scene_t["quat"], scene_t["scale"], scene_t["curv"],
                              scene_t["opacity"], scene_t["rgb"], scene_t.get("sh"), r, cam)


def signed_scale(x: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """The paper's signed-scale activation s = tanh(t) exp(x) (Sec. 3.2): a
    scale whose sign, and so the paraboloid's type, changes differentiably."""
    return torch.tanh(t) * torch.exp(x)


def signed_scale_to_params(s1, s2, s3):
    """The paper's signed scales (s1, s2, s3) -> (sigma, lambda) of this API:
    sigma_i = |s_i|, lambda_i = sign(s_i) s3 / s_i^2 (Sec. 3.2, curvature paragraph)."""
    sigma = torch.stack([s1.abs(), s2.abs()], -1)
    lam = torch.stack([torch.sign(s1) * s3 / (s1 * s1), torch.sign(s2) * s3 / (s2 * s2)], -1)
    return sigma, lam
