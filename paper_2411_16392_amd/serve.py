"""Serving driver: a resident scene behind qgs_serve_*, a Poisson arrival
trace, and the one-view-at-a-time baseline on the same trace.

Device work and scheduling run in libqgs's scheduler thread; this module only
submits requests at their arrival times, owns the output buffers and reads
completions.
"""
from __future__ import annotations

import threading
import time

import numpy as np
import torch

from . import _lib as L
from . import render as R


class Server:
    def __init__(self, scene_t: dict, budget_bytes: int = 8 << 30, max_slots: int = 8, max_size=(1920, 1080),
                 n_streams: int = 4, opts: L.QgsRenderOpts | None = None, device: int = 0, graphs: bool = True):
        self.scene_t = scene_t  # keeps the resident arrays alive
        cfg = L.QgsServeConfig()
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.max_width, cfg.max_height = int(max_size[0]), int(max_size[1])
        cfg.n_streams = int(n_streams)
        cfg.device = int(device)
        cfg.opts = opts if opts is not None else R.make_opts()
        cfg.flags = 0 if graphs else L.QGS_SERVE_NO_GRAPHS
        self.handle = L.qgs_serve_create(R._scene_struct(scene_t), cfg)

    def submit(self, cam, out: torch.Tensor) -> int:
        return L.qgs_serve_submit(self.handle, R.make_camera(cam), out.data_ptr())

    def poll(self, max_n: int = 64, timeout_us: int = 0):
        return L.qgs_serve_poll(self.handle, max_n, timeout_us)

    def cancel(self, req_id: int) -> int:
        return L.qgs_serve_cancel(self.handle, req_id)

    def clock(self) -> float:
        return L.qgs_serve_clock(self.handle)

    def stats(self):
        return L.qgs_serve_stats_get(self.handle)

    def close(self):
        if self.handle:
            L.qgs_serve_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class OutputRing:
    """Reusable output images per resolution; a buffer is handed out again only
    after the request that used it has completed."""

    def __init__(self, device, per_size: int = 48):
        self.device = device
        self.per_size = per_size
        self.free = {}
        self.busy = {}

    def get(self, w, h):
        key = (w, h)
        lst = self.free.setdefault(key, [])
        if not lst:
            n_busy = sum(1 for v in self.busy.values() if v[0] == key)
            if n_busy >= self.per_size:
                return None
            lst.append(torch.empty((3, h, w), dtype=torch.float32, device=self.device))
        return lst.pop()

    def hold(self, rid, key, buf):
        self.busy[rid] = (key, buf)

    def release(self, rid):
        key, buf = self.busy.pop(rid)
        self.free.setdefault(key, []).append(buf)


def run_trace(server: Server, trace, per_size: int = 48, keep: set | None = None):
    """Submits trace[i] = (arrival_s, camera) at its arrival time (relative to
    now) and collects completions.  Returns a dict with per-request latencies,
    frames/s and the server's stats; outputs of request indices in `keep` are
    copied out."""
    dev = server.scene_t["center"].device
    ring = OutputRing(dev, per_size)
    rid_of = {}
    idx_of = {}
    lat = {}
    kept = {}
    done_evt = threading.Event()
    lock = threading.Lock()

    def collect(block_us):
        for c in server.poll(64, block_us):
            with lock:
                i = idx_of[c.req_id]
            lat[i] = (c.t_done - c.t_submit, c.state, c.status, c.num_pairs, c.t_submit, c.t_done)
            if keep is not None and i in keep and c.state == L.QGS_REQ_DONE:
                kept[i] = ring.busy[c.req_id][1].clone()
            ring.release(c.req_id)

    t0 = server.clock()
    for i, (arr, cam) in enumerate(trace):
        # wait for the arrival time, collecting completions meanwhile
        while True:
            now = server.clock() - t0
            if now >= arr:
                break
            collect(int(min(2000, (arr - now) * 1e6)))
        buf = ring.get(cam.width, cam.height)
        while buf is None:
            collect(1000)
            buf = ring.get(cam.width, cam.height)
        rid = server.submit(cam, buf)
        with lock:
            rid_of[i] = rid
            idx_of[rid] = i
        ring.hold(rid, (cam.width, cam.height), buf)
    while len(lat) < len(trace):
        collect(5000)
    done_evt.set()
    t_first = min(v[4] for v in lat.values())
    t_last = max(v[5] for v in lat.values())
    return dict(latency=np.array([lat[i][0] for i in range(len(trace))]),
                state=np.array([lat[i][1] for i in range(len(trace))]),
                pairs=np.array([lat[i][3] for i in range(len(trace))]),
                frames_per_s=len(trace) / (t_last - t_first), span_s=t_last - t_first,
                stats=server.stats(), kept=kept)


def run_sequential(scene_t: dict, trace, renderer: R.Renderer | None = None):
    """Same arrival trace, one view at a time with the plain forward (preprocess,
    exact-count bin/sort, forward) on one stream; latency includes queueing."""
    r = renderer or R.Renderer(device=scene_t["center"].device)
    stream = torch.cuda.current_stream()
    lat = []
    t0 = time.perf_counter()
    t_done_prev = 0.0
    for arr, cam in trace:
        now = time.perf_counter() - t0
        if now < arr:
            time.sleep(arr - now)
        start = time.perf_counter() - t0
        st = r.forward(scene_t, cam, exact=True)
        stream.synchronize()
        done = time.perf_counter() - t0
        lat.append(done - arr)
        t_done_prev = done
        del st
    lat = np.array(lat)
    span = t_done_prev - trace[0][0]
    return dict(latency=lat, frames_per_s=len(trace) / span, span_s=span)


def latency_summary(lat: np.ndarray) -> dict:
    return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), max_ms=float(lat.max() * 1e3))
