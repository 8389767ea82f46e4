"""ctypes binding of libqgs (include/qgs.h): argument marshalling only.

Every function here has the name of the C entry point it calls and raises
QgsError on a non-zero status.  Loading fails loudly when the library has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqgs.so")

c_void_p, c_int32, c_uint32, c_int64, c_uint64, c_float = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                                            ctypes.c_int64, ctypes.c_uint64, ctypes.c_float)

QGS_OK = 0
QGS_ERR_INVALID_ARG = -1
QGS_ERR_WORKSPACE = -2
QGS_ERR_CAPACITY = -3
QGS_ERR_BUDGET = -4
QGS_ERR_HIP = -5
QGS_ERR_NOT_FOUND = -6
QGS_ERR_STATE = -7

QGS_RECORD_BYTES = 128
QGS_DETERMINISTIC_BWD = 1
QGS_ACCUMULATE_GRADS = 2
QGS_COUNT_EVALS = 4
QGS_TILE_DEPTH = 8
QGS_RESORT = 16
QGS_TIGHT_BOUND = 32
QGS_BWD_STATIC_BYTES = 64 << 20


class QgsScene(ctypes.Structure):
    _fields_ = [("center", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("curv", c_void_p),
                ("opacity", c_void_p), ("rgb", c_void_p), ("n", c_int64), ("sh", c_void_p), ("sh_degree", c_int32),
                ("pad", c_int32)]


class QgsCamera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32)]


class QgsRenderOpts(ctypes.Structure):
    _fields_ = [("near_plane", c_float), ("k_sigma", c_float), ("alpha_min", c_float), ("alpha_max", c_float),
                ("T_eps", c_float), ("A_eps", c_float), ("bg", c_float * 3), ("tile", c_int32), ("flags", c_uint32),
                ("kernel_events", c_void_p * 2)]


class QgsPrimBuf(ctypes.Structure):
    _fields_ = [("records", c_void_p), ("depth_key", c_void_p), ("rect", c_void_p), ("tiles", c_void_p),
                ("pair_offset", c_void_p), ("conic", c_void_p), ("n", c_int64), ("frame", c_void_p)]


class QgsTileLists(ctypes.Structure):
    _fields_ = [("pair_tile", c_void_p), ("pair_prim", c_void_p), ("emit_to_sorted", c_void_p),
                ("ranges", c_void_p), ("tile_order", c_void_p), ("counters", c_void_p), ("capacity", c_uint64)]


class QgsImages(ctypes.Structure):
    _fields_ = [("color", c_void_p), ("depth", c_void_p), ("normal", c_void_p), ("T_final", c_void_p),
                ("last", c_void_p), ("curvature", c_void_p), ("median_depth", c_void_p),
                ("distortion", c_void_p), ("median_pos", c_void_p), ("steps", c_void_p), ("step_count", c_void_p)]


def replay_words(capacity: int, tiles: int) -> int:
    """64-bit words of the backward replay bitmap for a list capacity and a tile count."""
    return 4 * ((capacity + 63) // 64 + tiles + 1)


class QgsImageGrads(ctypes.Structure):
    _fields_ = [("dcolor", c_void_p), ("ddepth", c_void_p), ("dnormal", c_void_p), ("dcurvature", c_void_p),
                ("dmedian_depth", c_void_p), ("ddistortion", c_void_p)]


class QgsSceneGrads(ctypes.Structure):
    _fields_ = [("center", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("curv", c_void_p),
                ("opacity", c_void_p), ("rgb", c_void_p), ("sh", c_void_p), ("screen_grad", c_void_p),
                ("visible", c_void_p)]


class QgsServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", c_int64), ("max_slots", c_int32), ("max_width", c_int32), ("max_height", c_int32),
                ("n_streams", c_int32), ("device", c_int32), ("opts", QgsRenderOpts), ("flags", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class QgsCompletion(ctypes.Structure):
    _fields_ = [("req_id", c_uint64), ("state", c_int32), ("status", c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("num_pairs", c_uint64)]


class QgsServeStats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("cancelled", c_uint64), ("failed", c_uint64),
                ("peak_pool_bytes", c_uint64), ("peak_in_flight", c_int32), ("pad", c_int32),
                ("graph_launches", c_uint64), ("graph_builds", c_uint64)]


QGS_SERVE_NO_GRAPHS = 1
QGS_REQ_DONE = 0
QGS_REQ_CANCELLED = 1
QGS_REQ_FAILED = 2


class QgsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().qgs_status_string(status).decode()
        if status == QGS_ERR_HIP:
            msg += f" (hipError {lib().qgs_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


_handle = None

# name -> (argtypes, restype)
_SIGS = {
    "qgs_status_string": ([c_int32], ctypes.c_char_p),
    "qgs_last_hip_error": ([], c_int32),
    "qgs_build_id": ([], ctypes.c_char_p),
    "qgs_default_opts": ([ctypes.POINTER(QgsRenderOpts)], None),
    "qgs_workspace_query": ([c_int64, ctypes.POINTER(QgsCamera), c_uint64, c_uint32,
                             ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], c_int32),
    "qgs_preprocess": ([ctypes.POINTER(QgsScene), ctypes.POINTER(QgsCamera), ctypes.POINTER(QgsRenderOpts),
                        ctypes.POINTER(QgsPrimBuf), c_void_p], c_int32),
    "qgs_bin_sort": ([ctypes.POINTER(QgsPrimBuf), ctypes.POINTER(QgsCamera), ctypes.POINTER(QgsRenderOpts),
                      ctypes.POINTER(QgsTileLists), c_void_p, ctypes.c_size_t, ctypes.POINTER(c_uint64),
                      c_void_p], c_int32),
    "qgs_render_fwd": ([ctypes.POINTER(QgsPrimBuf), ctypes.POINTER(QgsTileLists), ctypes.POINTER(QgsCamera),
                        ctypes.POINTER(QgsRenderOpts), ctypes.POINTER(QgsImages), c_void_p], c_int32),
    "qgs_render_bwd": ([ctypes.POINTER(QgsScene), ctypes.POINTER(QgsPrimBuf), ctypes.POINTER(QgsTileLists),
                        ctypes.POINTER(QgsCamera), ctypes.POINTER(QgsRenderOpts), ctypes.POINTER(QgsImages),
                        ctypes.POINTER(QgsImageGrads), ctypes.POINTER(QgsSceneGrads), c_void_p, ctypes.c_size_t,
                        c_void_p], c_int32),
    "qgs_render_bwd_static": ([ctypes.POINTER(QgsScene), ctypes.POINTER(QgsPrimBuf), ctypes.POINTER(QgsTileLists),
                               ctypes.POINTER(QgsCamera), ctypes.POINTER(QgsRenderOpts), ctypes.POINTER(QgsImages),
                               ctypes.POINTER(QgsImageGrads), ctypes.POINTER(QgsSceneGrads), c_void_p], c_int32),
    "qgs_serve_create": ([ctypes.POINTER(QgsScene), ctypes.POINTER(QgsServeConfig), ctypes.POINTER(c_void_p)],
                         c_int32),
    "qgs_serve_submit": ([c_void_p, ctypes.POINTER(QgsCamera), c_void_p, ctypes.POINTER(c_uint64)], c_int32),
    "qgs_serve_poll": ([c_void_p, ctypes.POINTER(QgsCompletion), c_int32, ctypes.POINTER(c_int32), c_int32],
                       c_int32),
    "qgs_serve_cancel": ([c_void_p, c_uint64], c_int32),
    "qgs_serve_stats_get": ([c_void_p, ctypes.POINTER(QgsServeStats)], c_int32),
    "qgs_serve_clock": ([c_void_p], ctypes.c_double),
    "qgs_serve_destroy": ([c_void_p], c_int32),
}


def verify_build(handle, expected: str | None = None) -> str:
    """Raises unless the library's build stamp equals the hash of the sources
    beside it (or `expected`); returns the stamp."""
    from paper_2411_16392_amd import build as _build
    want = expected if expected is not None else _build.source_hash()
    got = handle.qgs_build_id().decode()
    if got != want:
        raise RuntimeError(f"{LIB_PATH} was built from other sources (stamp {got[:16]}, sources {want[:16]}): "
                           "rebuild it with `python -m paper_2411_16392_amd.build`")
    return got


def lib():
    """The loaded libqgs.so; raises if it has not been built or was built from
    other sources than the ones beside it."""
    global _handle
    if _handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_16392_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        verify_build(L)
        _handle = L
    return _handle


def exported_symbols():
    return list(_SIGS.keys())


def _check(status: int, where: str):
    if status != QGS_OK:
        raise QgsError(status, where)


def qgs_default_opts() -> QgsRenderOpts:
    o = QgsRenderOpts()
    lib().qgs_default_opts(ctypes.byref(o))
    return o


def qgs_workspace_query(n: int, cam: QgsCamera, capacity: int, flags: int = 0):
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(lib().qgs_workspace_query(n, ctypes.byref(cam), capacity, flags, ctypes.byref(a), ctypes.byref(b)),
           "qgs_workspace_query")
    return a.value, b.value


def qgs_preprocess(scene: QgsScene, cam: QgsCamera, opts: QgsRenderOpts, out: QgsPrimBuf, stream=None):
    _check(lib().qgs_preprocess(ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(out),
                                stream), "qgs_preprocess")


def qgs_bin_sort(prims: QgsPrimBuf, cam: QgsCamera, opts: QgsRenderOpts, lists: QgsTileLists, ws: int,
                 ws_bytes: int, want_count: bool = True, stream=None, raise_on_capacity: bool = True):
    """Returns (status, num_pairs or None)."""
    cnt = c_uint64(0)
    st = lib().qgs_bin_sort(ctypes.byref(prims), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(lists), ws,
                            ws_bytes, ctypes.byref(cnt) if want_count else None, stream)
    if st == QGS_ERR_CAPACITY and not raise_on_capacity:
        return st, cnt.value
    _check(st, "qgs_bin_sort")
    return st, (cnt.value if want_count else None)


def qgs_render_fwd(prims: QgsPrimBuf, lists: QgsTileLists, cam: QgsCamera, opts: QgsRenderOpts, out: QgsImages,
                   stream=None):
    _check(lib().qgs_render_fwd(ctypes.byref(prims), ctypes.byref(lists), ctypes.byref(cam), ctypes.byref(opts),
                                ctypes.byref(out), stream), "qgs_render_fwd")


def qgs_render_bwd(scene: QgsScene, prims: QgsPrimBuf, lists: QgsTileLists, cam: QgsCamera, opts: QgsRenderOpts,
                   fwd: QgsImages, dL: QgsImageGrads, out: QgsSceneGrads, ws: int, ws_bytes: int, stream=None):
    _check(lib().qgs_render_bwd(ctypes.byref(scene), ctypes.byref(prims), ctypes.byref(lists), ctypes.byref(cam),
                                ctypes.byref(opts), ctypes.byref(fwd), ctypes.byref(dL), ctypes.byref(out), ws,
                                ws_bytes, stream), "qgs_render_bwd")


def qgs_render_bwd_static(scene: QgsScene, prims: QgsPrimBuf, lists: QgsTileLists, cam: QgsCamera,
                          opts: QgsRenderOpts, fwd: QgsImages, dL: QgsImageGrads, out: QgsSceneGrads, stream=None):
    """qgs_render_bwd with the library's static per-device workspace (no allocation)."""
    _check(lib().qgs_render_bwd_static(ctypes.byref(scene), ctypes.byref(prims), ctypes.byref(lists),
                                       ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(fwd), ctypes.byref(dL),
                                       ctypes.byref(out), stream), "qgs_render_bwd_static")


def qgs_serve_create(scene: QgsScene, cfg: QgsServeConfig) -> int:
    h = c_void_p(0)
    _check(lib().qgs_serve_create(ctypes.byref(scene), ctypes.byref(cfg), ctypes.byref(h)), "qgs_serve_create")
    return h.value


def qgs_serve_submit(srv: int, cam: QgsCamera, out_rgb: int) -> int:
    rid = c_uint64(0)
    _check(lib().qgs_serve_submit(srv, ctypes.byref(cam), out_rgb, ctypes.byref(rid)), "qgs_serve_submit")
    return rid.value


def qgs_serve_poll(srv: int, max_n: int = 64, timeout_us: int = 0):
    buf = (QgsCompletion * max_n)()
    n = c_int32(0)
    _check(lib().qgs_serve_poll(srv, buf, max_n, ctypes.byref(n), timeout_us), "qgs_serve_poll")
    return [buf[i] for i in range(n.value)]


def qgs_serve_cancel(srv: int, req_id: int) -> int:
    """Returns the status (QGS_OK, QGS_ERR_NOT_FOUND, QGS_ERR_STATE)."""
    return lib().qgs_serve_cancel(srv, req_id)


def qgs_serve_stats_get(srv: int) -> QgsServeStats:
    st = QgsServeStats()
    _check(lib().qgs_serve_stats_get(srv, ctypes.byref(st)), "qgs_serve_stats_get")
    return st


def qgs_serve_clock(srv: int) -> float:
    return lib().qgs_serve_clock(srv)


def qgs_serve_destroy(srv: int):
    _check(lib().qgs_serve_destroy(srv), "qgs_serve_destroy")
