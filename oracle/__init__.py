"""FP64 CPU oracle for the quadric Gaussian splatting rasterizer.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never imports, links or runs anything here.

The arithmetic lives in ``qgs_oracle.c`` (plain C, FP64, OpenMP), which this
module builds with gcc and calls through ctypes.  See the header of that file
for the equations it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qgs_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

# Readings of the unstated constants (the renderer inherits them from the 3DGS
# framework the paper builds on); every one is an input.
DEFAULT_OPTS = dict(near=0.2, k_sigma=3.0, alpha_min=1.0 / 255.0, alpha_max=0.99,
                    T_eps=1e-4, A_eps=1e-6, bg=(0.0, 0.0, 0.0), resort=0, tile_depth=False)

# Margin scales for the discrete decisions: a pixel whose relative distance to a
# decision boundary is below its scale is reported with margin < 1.  Dcond is
# the conditioning of an accepted root's derivative (D relative to B^2 + 4|AC|),
# which matters for gradients only.
DEFAULT_DELTA = dict(A=1e-3, D=1e-6, near=1e-5, E=1e-5, alpha_min=1e-4, T=1e-4,
                     normal=1e-4, clamp=1e-4, median=1e-5, sort=3e-6, Dcond=1e-3)
_DELTA_ORDER = ["A", "D", "near", "E", "alpha_min", "T", "normal", "clamp", "median", "sort", "Dcond"]
KINDS = _DELTA_ORDER
# longest recorded decision path per result of alternatives()
PATH_MAX = 24


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if (not os.path.exists(_SO)) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
        L.oracle_keys.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, f32, f32, P, P, P, P, P, P, P, P, i32, f32]
        L.oracle_keys.restype = None
        L.oracle_bin_sort.argtypes = [i64, P, P, P, P, P, P, i32, i32, i32, i32, i64, P, P, P, P, P, f32]
        L.oracle_bin_sort.restype = i64
        L.oracle_tile_depth_bits.argtypes = [P, i32, i32, P, i32, i32, f64]
        L.oracle_tile_depth_bits.restype = ctypes.c_uint32
        L.oracle_render.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, i32, i32, P, P,
                                    i32, i32, i32, i32, i32,
                                    P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P,
                                    P, i32, P,
                                    i32, i64, P, P, P, P, P, i32, P]
        L.oracle_render.restype = i64
        L.oracle_render_alts.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, i32, i32, P, P,
                                         i32, i32, i32, i32, i32, P, i32, i32,
                                         i64, P, i32, P, P, P, P, P]
        L.oracle_render_alts.restype = i64
        L.oracle_gfun.argtypes = [f64]
        L.oracle_gfun.restype = f64
        L.oracle_gprime.argtypes = [f64]
        L.oracle_gprime.restype = f64
        L.oracle_arc_length.argtypes = [f64, f64]
        L.oracle_arc_length.restype = f64
        L.oracle_local_box.argtypes = [f64, f64, f64, f64, f64, i32, P]
        L.oracle_local_box.restype = None
        L.oracle_tb_frustum.argtypes = [f64, f64, f64, f64, f64, P]
        L.oracle_tb_frustum.restype = None
        L.oracle_blend_k.argtypes = [f32, f32, f32]
        L.oracle_blend_k.restype = f64
        L.oracle_ray_hit.argtypes = [P, P, P, P, P, P, P, P]
        L.oracle_ray_hit.restype = None
        _lib_handle = L
    return _lib_handle


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def cam_array(cam, dtype=np.float32):
    return np.concatenate([np.asarray(cam.R, np.float64).reshape(9), np.asarray(cam.t, np.float64).reshape(3),
                           [cam.fx, cam.fy, cam.cx, cam.cy]]).astype(np.float32).astype(dtype)


def opts_array(opts=None):
    o = dict(DEFAULT_OPTS)
    if opts:
        o.update(opts)
    # thresholds are FP32 values on the GPU; the oracle uses the same values
    vals = [o["near"], o["k_sigma"], o["alpha_min"], o["alpha_max"], o["T_eps"], o["A_eps"], *o["bg"],
            float(o["resort"])]
    return np.asarray(vals, np.float32).astype(np.float64)


def delta_array(delta=None):
    d = dict(DEFAULT_DELTA)
    if delta:
        d.update(delta)
    return np.asarray([d[k] for k in _DELTA_ORDER], np.float64)


def gfun(u: float) -> float:
    return _lib().oracle_gfun(float(u))


def gprime(u: float) -> float:
    return _lib().oracle_gprime(float(u))


def arc_length(a: float, rho: float) -> float:
    return _lib().oracle_arc_length(float(a), float(rho))


def local_box(s1, s2, l1, l2, k=3.0, tight=False):
    """Inflated local box (hx, hy, zlo, zhi) holding a primitive's support."""
    out = np.zeros(4, np.float64)
    _lib().oracle_local_box(float(s1), float(s2), float(l1), float(l2), float(k), int(bool(tight)), _ptr(out))
    return out


def blend_k(opacity, alpha_min=1.0 / 255.0, k=3.0):
    """Cut-off of the tight bounds for a primitive of this opacity (it blends
    only where o G >= alpha_min)."""
    return _lib().oracle_blend_k(float(opacity), float(alpha_min), float(k))


def tb_frustum(s1, s2, l1, l2, k=3.0):
    """The paper's tangent-plane frustum (rho1, rho2, x1, x2, h); measurement only."""
    out = np.zeros(5, np.float64)
    _lib().oracle_tb_frustum(float(s1), float(s2), float(l1), float(l2), float(k), _ptr(out))
    return out


def keys(scene, cam, opts=None, tight=False, paper_tb=False):
    """Key stage: cull flag, FP32 depth key bits, pixel and tile rectangles
    (tight: the chord-bound local box; paper_tb: the rectangle of the paper's
    tangent-plane frustum instead, with no conic test -- measurement only)."""
    o = opts_array(opts)
    n = scene.n
    culled = np.zeros(n, np.uint8)
    depth_bits = np.zeros(n, np.uint32)
    rect_px = np.zeros((n, 4), np.int32)
    rect_tile = np.zeros((n, 4), np.int32)
    tiles = np.zeros(n, np.uint32)
    conic = np.zeros((n, 6), np.float64)
    conic_ok = np.zeros(n, np.uint8)
    frame = np.zeros((n, 16), np.float64)
    arrs = [_f32(a) for a in scene.arrays()]
    camv = cam_array(cam)
    _lib().oracle_keys(n, *[_ptr(a) for a in arrs], _ptr(camv), cam.width, cam.height,
                       ctypes.c_float(o[0]), ctypes.c_float(o[1]),
                       _ptr(culled), _ptr(depth_bits), _ptr(rect_px), _ptr(rect_tile), _ptr(tiles),
                       _ptr(conic), _ptr(conic_ok), _ptr(frame), 2 if paper_tb else int(bool(tight)),
                       ctypes.c_float(o[2]))
    return dict(culled=culled, depth_bits=depth_bits, rect_px=rect_px, rect_tile=rect_tile, tiles=tiles,
                conic=conic, conic_ok=conic_ok, frame=frame, cam=camv, width=cam.width, height=cam.height,
                near=float(o[0]))


def tile_depth_bits(k, p, tx, ty):
    """Per-tile sort depth key of primitive p for tile (tx, ty) (key-stage spec)."""
    return int(_lib().oracle_tile_depth_bits(_ptr(np.ascontiguousarray(k["frame"][p])), int(tx), int(ty),
                                             _ptr(_f64(k["cam"].astype(np.float64))), k["width"], k["height"],
                                             float(k["near"])))


def bin_sort(k, cam, with_seq=False, tile_depth=False):
    """Sorted tile|depth key list and per-tile ranges from the key stage
    (with_seq: also the emission index of every sorted pair)."""
    n = k["culled"].shape[0]
    tx, ty = cam.tiles_x, cam.tiles_y
    ranges = np.zeros((tx * ty, 2), np.uint32)
    L = _lib()
    args = (_ptr(k["culled"]), _ptr(k["depth_bits"]), _ptr(k["rect_tile"]), _ptr(k["conic"]), _ptr(k["conic_ok"]),
            _ptr(k["cam"]), k["width"], k["height"], tx, ty)
    fr = _ptr(k["frame"]) if tile_depth else None
    total = L.oracle_bin_sort(n, *args, 0, None, None, None, _ptr(ranges), fr, ctypes.c_float(k["near"]))
    keys_out = np.zeros(max(total, 1), np.uint64)
    prims = np.zeros(max(total, 1), np.uint32)
    seq = np.zeros(max(total, 1), np.uint32)
    total2 = L.oracle_bin_sort(n, *args, total, _ptr(keys_out), _ptr(prims), _ptr(seq), _ptr(ranges), fr,
                               ctypes.c_float(k["near"]))
    assert total2 == total
    if with_seq:
        return keys_out[:total], prims[:total], ranges, seq[:total]
    return keys_out[:total], prims[:total], ranges


def _render_inputs(scene, cam, opts, window, params64, key_stage, delta, cam_vec64):
    o = opts_array(opts)
    dv = delta_array(delta)
    if key_stage is None:
        key_stage = keys(scene, cam, opts)
    x0, y0, w, h = window if window is not None else (0, 0, cam.width, cam.height)
    prm = params64 if params64 is not None else scene.arrays()
    arrs = [_f64(a) for a in prm[:6]]
    # SH colour: params64 may carry the coefficients as a seventh array
    sh = prm[6] if len(prm) > 6 else scene.sh
    sh64 = _f64(sh) if sh is not None else None
    sh_deg = -1 if sh is None else int(round(np.sqrt(np.asarray(sh).shape[1]))) - 1
    camv = cam_array(cam, np.float64) if cam_vec64 is None else _f64(cam_vec64)
    o_d = dict(DEFAULT_OPTS)
    o_d.update(opts or {})
    keycam = _f64(key_stage["cam"].astype(np.float64))
    fr = _ptr(key_stage["frame"]) if o_d["tile_depth"] else None
    head = [scene.n, *[_ptr(a) for a in arrs], _ptr(key_stage["culled"]), _ptr(key_stage["depth_bits"]),
            fr, _ptr(keycam), _ptr(camv), cam.width, cam.height, _ptr(o), _ptr(dv), x0, y0, w, h]
    # keep the arrays the pointers refer to alive for the call
    keep = (arrs, sh64, camv, keycam, o, dv, key_stage)
    return head, (x0, y0, w, h), sh, sh64, sh_deg, keep


def render(scene, cam, opts=None, window=None, dL=None, nthreads=None, params64=None,
           key_stage=None, delta=None, cam_vec64=None, branch_median=False, forced=None, grad_skip=False):
    """FP64 render of a pixel window (x0, y0, w, h) (default: the full view).

    params64: optional tuple of FP64 parameter arrays overriding the scene's
    (used for finite differences; order and culling still come from the key
    stage of the FP32 scene).  cam_vec64: optional FP64 camera vector
    {R[9], t[3], fx, fy, cx, cy} overriding the FP32 one.  dL: optional (dcolor[3,H,W], ddepth[H,W],
    dnormal[3,H,W]) or (..., dcurvature[H,W], dmedian[H,W], ddistortion[H,W]) over the full view;
    runs the backward.  branch_median: the median depth's decisions count in
    the margin (and branch).  forced: optional (pixels, paths, lengths) -- row-major window pixel
    indices, their decision paths [k, PATH_MAX] and path lengths, as
    alternatives() returns them -- whose near-tied decisions take those outcomes.
    grad_skip: pixels whose gradient margin is below 1 (an ill-conditioned or
    ambiguous derivative) contribute no gradient.
    Returns a dict of window-sized FP64 maps (colour, depth, normal, curvature, median depth,
    depth distortion, final transmittance, blend count, decision margin, gradient margin,
    near-tie kinds as bits of KINDS, the primitive at which the pixel stopped or -1) and, with
    dL, parameter gradients.
    """
    head, (x0, y0, w, h), sh, sh64, sh_deg, keep = _render_inputs(scene, cam, opts, window, params64, key_stage,
                                                                  delta, cam_vec64)
    n = scene.n
    color = np.zeros((3, h, w)); depth = np.zeros((h, w)); normal = np.zeros((3, h, w))
    T = np.zeros((h, w)); nb = np.zeros((h, w), np.int32); margin = np.zeros((h, w))
    gmargin = np.zeros((h, w)); kinds = np.zeros((h, w), np.uint16); stop_id = np.zeros((h, w), np.int64)
    curvature = np.zeros((h, w)); median = np.zeros((h, w)); dist = np.zeros((h, w))
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    grads = None
    gp = [None] * 12
    if dL is not None:
        dc = _f64(dL[0][:, y0:y0 + h, x0:x0 + w])
        dd = _f64(dL[1][y0:y0 + h, x0:x0 + w])
        dn = _f64(dL[2][:, y0:y0 + h, x0:x0 + w])
        extra = [_f64(m[y0:y0 + h, x0:x0 + w]) if m is not None else None for m in
                 (list(dL[3:6]) + [None] * 3)[:3]]
        grads = dict(center=np.zeros((n, 3)), quat=np.zeros((n, 4)), scale=np.zeros((n, 2)),
                     curv=np.zeros((n, 2)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
        if sh is not None:
            grads["sh"] = np.zeros(np.asarray(sh).shape)
        gp = ([_ptr(dc), _ptr(dd), _ptr(dn)] + [_ptr(m) if m is not None else None for m in extra] +
              [_ptr(grads[k]) for k in ("center", "quat", "scale", "curv", "opacity", "rgb")])
    if forced is not None and len(forced[0]) > 0:
        fpix = np.ascontiguousarray(forced[0], np.int32)
        fpath = np.ascontiguousarray(forced[1], np.uint8).reshape(len(fpix), PATH_MAX)
        flen = np.ascontiguousarray(forced[2], np.int32)
        fargs = [len(fpix), _ptr(fpix), _ptr(fpath), _ptr(flen)]
    else:
        fargs = [0, None, None, None]
    ev = _lib().oracle_render(*head, int(nthreads),
                              _ptr(color), _ptr(depth), _ptr(normal), _ptr(T), _ptr(nb), _ptr(margin),
                              _ptr(curvature), _ptr(median), _ptr(dist), *gp,
                              _ptr(sh64) if sh64 is not None else None, sh_deg,
                              _ptr(grads["sh"]) if (grads is not None and sh is not None) else None,
                              int(bool(branch_median)), *fargs, _ptr(gmargin), _ptr(kinds), int(bool(grad_skip)),
                              _ptr(stop_id))
    del keep
    if ev < 0:
        raise ValueError("bad window")
    out = dict(color=color, depth=depth, normal=normal, curvature=curvature, median_depth=median,
               distortion=dist, T_final=T, n_blend=nb, margin=margin, gmargin=gmargin, kinds=kinds,
               stop_id=stop_id, evals=int(ev))
    if grads is not None:
        out["grads"] = grads
    return out


# channel order of the results of alternatives()
ALT_CHANNELS = ("color0", "color1", "color2", "depth", "normal0", "normal1", "normal2", "curvature",
                "median_depth", "distortion", "T_final")


def alternatives(scene, cam, pixels, opts=None, window=None, nthreads=None, key_stage=None, delta=None,
                 branch_median=False, max_leaves=256):
    """Every result the window pixels `pixels` (row-major indices in the window)
    may take when their near-tied decisions go either way (reading R19: FP32 and
    FP64 may decide differently there, and either outcome is correct).
    Returns dict: n[k] results per pixel, overflow[k] (the enumeration was cut
    short), vals[k, max_leaves, 11] (ALT_CHANNELS), paths[k, max_leaves,
    PATH_MAX] and plen[k, max_leaves] (the decision path of each result, for
    render(forced=...)).  Result 0 is the one render() gives."""
    head, _, sh, sh64, sh_deg, keep = _render_inputs(scene, cam, opts, window, None, key_stage, delta, None)
    pix = np.ascontiguousarray(pixels, np.int32).reshape(-1)
    k = len(pix)
    nl = np.zeros(k, np.int32)
    ovf = np.zeros(k, np.uint8)
    vals = np.zeros((k, max_leaves, len(ALT_CHANNELS)))
    paths = np.zeros((k, max_leaves, PATH_MAX), np.uint8)
    plen = np.zeros((k, max_leaves), np.int32)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    if k > 0:
        ev = _lib().oracle_render_alts(*head, int(nthreads), _ptr(sh64) if sh64 is not None else None, sh_deg,
                                       int(bool(branch_median)), k, _ptr(pix), int(max_leaves), _ptr(nl), _ptr(ovf),
                                       _ptr(vals), _ptr(paths), _ptr(plen))
        if ev < 0:
            raise ValueError("bad window or pixel index")
    del keep
    return dict(n=nl, overflow=ovf, vals=vals, paths=paths, plen=plen)


def sh_basis(deg, d):
    """Real SH basis values Y[16] and their gradients dY[16][3] at direction d."""
    Y = np.zeros(16)
    dY = np.zeros((16, 3))
    _lib().oracle_sh_basis(int(deg), _ptr(_f64(d)), _ptr(Y), _ptr(dY))
    return Y, dY


def ray_hit(center, quat, scale, curv, cam_vec64, dcam, opts=None):
    """One ray against one primitive.  Returns a dict of the hit quantities."""
    out = np.zeros(15)
    o = opts_array(opts)
    _lib().oracle_ray_hit(_ptr(_f64(center)), _ptr(_f64(quat)), _ptr(_f64(scale)), _ptr(_f64(curv)),
                          _ptr(_f64(cam_vec64)), _ptr(_f64(dcam)), _ptr(o), _ptr(out))
    return dict(ok=bool(out[0]), linear=bool(out[1]), t=out[2], x=out[3], y=out[4], z=out[5], E=out[6], G=out[7],
                A=out[8], B=out[9], C=out[10], normal=out[11:14].copy(), K=out[14])
