#!/usr/bin/env python3
"""Throughput of the quadric rasterizer's training step on one MI355X.

A step is one pass of the whole hot path over one view: preprocess, tile|depth
binning and sort, forward rasterization, backward rasterization and the
preprocess backward, with N(0,1) upstream gradients on colour, depth and
normal.  Workload: 500,000 quadrics on the noisy union surface of 8 ellipsoids,
64 ring views at 1600 x 1200 (f = 1600), one view per step, inputs resident in
HBM.  Prints one JSON line: Mpix/s = steps * W * H / elapsed, plus the
roofline of the dominant kernel and the FP64 CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd+bwd at 500K quadrics 1600x1200; serving frames/s + p99 ms"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3       # packed FP32 (two lanes per op)
PEAK_FP32_UNPACKED_TFLOPS = 78.6      # 256 CU x 64 FMA lanes x 2 flops x 2.4 GHz

# Algorithmic FP32 operations per unit of rasterizer work, counted from the
# method's formulas (each add, multiply, compare-select, square root,
# reciprocal, exponential or logarithm counts one; see the design notes):
#   per evaluated (pixel, primitive) pair: ray in the local frame, A, B, C,
#   discriminant and roots, candidate point, Q, rho, u, g(u), E and the test
FLOPS_EVAL = 69
#   extra per blended pair in the forward: G, alpha, transmittance, colour,
#   depth, normal (normalise, face the camera, rotate) and accumulation
FLOPS_BLEND_FWD = 38
#   per blended pair in the backward: T recovery, dX/dalpha over 7 channels,
#   suffix sums and the chain rule through normal, density, arc length, root,
#   frame and projection (re-evaluation of the pair counted by FLOPS_EVAL)
FLOPS_BLEND_BWD = 230

# Algorithmic HBM bytes of the memory-bound stages (what each kernel must move):
#   preprocess: 60 B of parameters read; 128 B record, 64 B conic, 16 B tile
#   rectangle, 4 B depth key and 4 B tile count written per primitive
BYTES_PRE_PRIM = 60 + 216
#   binning: depth-key init (16 B) and four 8-bit radix passes over (key, index)
#   (20 B each), the pair-offset scan (8 B) and the emission's per-primitive
#   reads (order, rectangle, conic, offset, count: 92 B) per primitive ...
BYTES_SORT_PRIM = 16 + 80 + 8 + 92
#   ... and per pair the emitted (tile, primitive) (8 B), two 8-bit radix passes
#   (20 B each) and the range scan (4 B)
BYTES_SORT_PAIR = 8 + 40 + 4
#   preprocess backward (inside the backward stage): record gradient 64 B,
#   parameters 60 B and tile count 4 B read, 60 B of gradients written
BYTES_PRE_BWD_PRIM = 64 + 60 + 4 + 60


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_render_500k_1600x1200.md")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's
    reading), or None when the rasterizer sources changed since the counters
    were taken."""
    import hashlib
    try:
        line = next(l for l in open(TRAFFIC_SUMMARY) if l.strip().startswith("traffic "))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.strip()[len("traffic "):])
    h = hashlib.sha256()
    for f in ("raster.hip", "qgs_device.hpp", "qgs_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2411_16392_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec.get("source"):
        return None
    return rec.get("bytes") if kernel == "render_bwd" else rec.get("fwd_bytes")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--views", type=int, default=None, help="views of the workload (default: 64 ring views for "
                    "workload 2, 4 views for workload 3)")
    ap.add_argument("--workload", type=int, choices=(2, 3), default=2,
                    help="2: 500K quadrics, 1600x1200 (headline); 3: 3M quadrics, shells + background ball, "
                         "1237x822 and 1600x1064 views from inside the scene")
    ap.add_argument("--loose-bound", action="store_true",
                    help="the k-sigma local box without the chord bound (QGS_TIGHT_BOUND off)")
    ap.add_argument("--cpu-rows", type=int, default=1200, help="rows of view 0 the CPU oracle renders (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-quick", action="store_true", help="only the all-thread oracle timing of view 0")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-no-graphs", action="store_true", help="serving with direct launches instead of graphs")
    ap.add_argument("--full-model", action="store_true",
                    help="the paper's full-model ordering (per-tile sort depth and the 8-entry resort buffer)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU design is described in DESIGN.md and not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_16392_amd import _lib as L
    from paper_2411_16392_amd import render as R
    from paper_2411_16392_amd import scenes

    L.lib()  # fails loudly without the HIP library
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    q = args.quiet

    if args.copy_probe:
        # known traffic: 256 MiB read + 256 MiB written per launch
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.time()
    cfg = scenes.make_config(args.workload, n_views=args.views)
    cams = cfg.cameras
    W, H = cams[0].width, cams[0].height
    sc_t = R.scene_to_device(cfg.scene, dev)
    log(f"[bench] scene {cfg.scene.n} quadrics, {len(cams)} views {W}x{H}, generated in {time.time() - t0:.1f}s", q)

    # size the pair capacity once, untimed, from exact counts of the views used
    steps_total = args.warmup + args.steps
    used = sorted({i % len(cams) for i in range(steps_total)})
    mode = (L.QGS_TILE_DEPTH | L.QGS_RESORT) if args.full_model else 0
    probe = R.Renderer(device=dev, opts=R.make_opts(flags=mode, tight_bound=not args.loose_bound))
    max_pairs = 0
    for v in used:
        st = probe.preprocess(sc_t, cams[v])
        probe.bin_sort(st, exact=True)
        max_pairs = max(max_pairs, st.num_pairs)
    capacity = int(max_pairs * 1.05) + 4096
    log(f"[bench] max pairs over used views {max_pairs}, capacity {capacity}", q)

    # evaluation counts (untimed): list entries processed and blended pairs
    cnt_r = R.Renderer(device=dev, capacity=capacity,
                       opts=R.make_opts(flags=L.QGS_COUNT_EVALS | mode, tight_bound=not args.loose_bound))
    evals_per_view = []
    for v in used[: min(8, len(used))]:
        st = cnt_r.forward(sc_t, cams[v], exact=False)
        torch.cuda.synchronize()
        evals_per_view.append(int(st.counters.cpu().numpy().view(np.uint32)[2]))
    evals_mean = float(np.mean(evals_per_view))

    rend = R.Renderer(device=dev, capacity=capacity, opts=R.make_opts(flags=mode, tight_bound=not args.loose_bound))
    gen = torch.Generator(device=dev)
    gen.manual_seed(2)
    dLs = {}
    for c in cams:
        if (c.height, c.width) not in dLs:
            h, w = c.height, c.width
            dLs[(h, w)] = [(torch.randn((3, h, w), generator=gen, device=dev),
                            torch.randn((h, w), generator=gen, device=dev),
                            torch.randn((3, h, w), generator=gen, device=dev)) for _ in range(4)]
    grads = {k: torch.empty_like(v) for k, v in sc_t.items()}
    stream = torch.cuda.current_stream()

    stage_names = ("preprocess", "bin_sort", "render_fwd", "render_bwd")
    n_ev = len(stage_names) + 1

    def kernel_events(pair):
        # the library records these around the rasterizer kernel alone
        rend.opts.kernel_events[0] = pair[0].cuda_event if pair else None
        rend.opts.kernel_events[1] = pair[1].cuda_event if pair else None

    def step(i, events=None, kev=None):
        cam = cams[i % len(cams)]
        dl = dLs[(cam.height, cam.width)][i % 4]
        if events is not None:
            events[0].record(stream)
        st = rend.preprocess(sc_t, cam)
        if events is not None:
            events[1].record(stream)
        rend.bin_sort(st, exact=False)
        if events is not None:
            events[2].record(stream)
        kernel_events(kev[0:2] if kev else None)
        rend.render_fwd(st)
        if events is not None:
            events[3].record(stream)
        kernel_events(kev[2:4] if kev else None)
        rend.backward(sc_t, st, dl[0], dl[1], dl[2], out=grads)
        kernel_events(None)
        if events is not None:
            events[4].record(stream)
        return st

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # timed region: exactly K steps, bracketed by device synchronisation
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(args.steps)]
    # per step: forward rasterizer begin/end, backward rasterizer begin/end;
    # torch creates an event at its first record, so record each once here
    kevs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for kv in kevs:
        for e in kv:
            e.record(stream)
    states = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        states.append(step(args.warmup + i, evs[i], kevs[i]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    overflow = any(int(s.counters[1].item()) != 0 for s in states)
    if overflow:
        print("pair capacity overflowed during the timed steps", file=sys.stderr)
        sys.exit(3)
    npairs = [int(s.counters[0].item()) & 0xFFFFFFFF for s in states]
    del states
    stage_ms = {}
    for k, name in enumerate(stage_names):
        stage_ms[name] = float(np.mean([evs[i][k].elapsed_time(evs[i][k + 1]) for i in range(args.steps)]))
    kernel_ms = {"render_fwd": float(np.mean([kevs[i][0].elapsed_time(kevs[i][1]) for i in range(args.steps)])),
                 "render_bwd": float(np.mean([kevs[i][2].elapsed_time(kevs[i][3]) for i in range(args.steps)]))}
    ms_per_step = elapsed * 1e3 / args.steps
    pixels = sum(cams[(args.warmup + i) % len(cams)].width * cams[(args.warmup + i) % len(cams)].height
                 for i in range(args.steps))
    mpix = pixels / elapsed / 1e6
    log(f"[bench] {ms_per_step:.3f} ms/step, {mpix:.1f} Mpix/s, stages {stage_ms}, kernels {kernel_ms}", q)

    # roofline of the dominant kernel: algorithmic FP32 operations per launch
    # from the forward's pair counts, divided by the kernel's own event time
    evald, blended, wrect, weval, wblend = [], [], [], [], []
    for v in used[: min(8, len(used))]:
        st = cnt_r.forward(sc_t, cams[v], exact=False)
        torch.cuda.synchronize()
        c = st.counters.cpu().numpy().view(np.uint32)
        evald.append(int(c[3]))
        blended.append(int(c[4]))
        wrect.append(int(c[5]))
        weval.append(int(c[6]))
        wblend.append(int(c[7]))
    ev = float(np.mean(evald))
    bl = float(np.mean(blended))
    # forward lane use: intersections evaluated per (wave, entry) step that evaluated any
    fwd_lane_use = ev / (64.0 * max(1.0, float(np.mean(weval))))
    kern = {"render_fwd": ev * FLOPS_EVAL + bl * FLOPS_BLEND_FWD,
            "render_bwd": bl * (FLOPS_EVAL + FLOPS_BLEND_BWD)}
    # the longer of the two rasterizer kernels, timed alone (kernel_events)
    dominant = max(kernel_ms, key=kernel_ms.get)
    achieved = kern[dominant] / (kernel_ms[dominant] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4), "traffic": measured_traffic(dominant),
                "launch_ms": round(kernel_ms[dominant], 4),
                "flops_per_launch": kern[dominant], "pairs_evaluated": ev, "pairs_blended": bl,
                "fwd_wave_steps_rect": float(np.mean(wrect)), "fwd_wave_steps_eval": float(np.mean(weval)),
                "fwd_wave_steps_blend": float(np.mean(wblend)),
                "fwd_lane_use": round(fwd_lane_use, 4)}

    # every stage against its own roofline (algorithmic work / stage time)
    n_p = cfg.scene.n
    pairs_mean = float(np.mean(npairs))
    stage_roofline = {
        "preprocess": {"bound": "hbm", "bytes": n_p * BYTES_PRE_PRIM},
        "bin_sort": {"bound": "hbm", "bytes": n_p * BYTES_SORT_PRIM + pairs_mean * BYTES_SORT_PAIR},
        "render_fwd": {"bound": "alu", "flops": kern["render_fwd"]},
        "render_bwd": {"bound": "alu", "flops": kern["render_bwd"],
                       "bytes_preprocess_bwd": n_p * BYTES_PRE_BWD_PRIM},
    }
    for k, v in stage_roofline.items():
        t = stage_ms[k] * 1e-3
        if v["bound"] == "hbm":
            v["GB/s"] = round(v["bytes"] / t / 1e9, 1)
            v["frac"] = round(v["bytes"] / t / 1e9 / PEAK_HBM_GBS, 4)
        else:
            v["TFLOP/s"] = round(v["flops"] / t / 1e12, 3)
            v["frac"] = round(v["flops"] / t / 1e12 / PEAK_FP32_UNPACKED_TFLOPS, 4)

    result = {
        "metric": METRIC,
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"500K quadrics on 8 noisy ellipsoids, 1600x1200 ring views ({len(cams)}), "
                                "fwd+bwd per view, N(0,1) upstream gradients") if args.workload == 2 else
                               (f"3M quadrics, 5 shells + background ball of radius 50, {len(cams)} views from "
                                "inside the scene at 1237x822 and 1600x1064, fwd+bwd per view, N(0,1) upstream "
                                "gradients"),
                   "n_prims": cfg.scene.n, "width": W, "height": H, "views": len(cams),
                   "ordering": "per-tile depth + 8-entry resort" if args.full_model else "centre depth",
                   "bound": "k-sigma box" if args.loose_bound else "chord bound"},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "kernels_ms": {k: round(v, 4) for k, v in kernel_ms.items()},
        "pairs_per_view": int(np.mean(npairs)),
        "evals_per_view": int(evals_mean),
        "evals_per_s": evals_mean / (kernel_ms["render_fwd"] * 1e-3),
        "roofline": roofline,
        "stages_roofline": stage_roofline,
    }

    if not args.no_cpu_baseline and args.cpu_rows > 0:
        result["cpu_baseline"], result["units_pin"] = cpu_baseline(args, cfg, cams, cnt_r, sc_t, mode, q)

    if not args.no_serve and args.serve_requests > 0:
        result["serving"] = bench_serving(args, dev, q)

    print(json.dumps(result), flush=True)


def oracle_entries_processed(oracle, ks, cam, stop_id):
    """E of one view from the oracle: per pixel, the entries of its tile's
    list (the key stage's sorted lists, bit-identical to the GPU's) up to and
    including the one it stopped at, or the whole list."""
    import numpy as np
    keys_, prims, ranges = oracle.bin_sort(ks, cam)
    n = len(ks["tiles"])
    tile = (keys_ >> np.uint64(32)).astype(np.int64)
    pos = np.arange(len(prims), dtype=np.int64) - ranges[tile, 0].astype(np.int64)
    combo = tile * n + prims.astype(np.int64)
    order = np.argsort(combo)
    combo_s = combo[order]
    H, W = stop_id.shape
    py, px = np.mgrid[0:H, 0:W]
    t = (py // 16) * cam.tiles_x + px // 16
    lens = (ranges[:, 1] - ranges[:, 0]).astype(np.int64)
    e = lens[t].copy()
    st = stop_id >= 0
    idx = np.searchsorted(combo_s, t[st] * n + stop_id[st])
    assert np.array_equal(combo_s[idx], t[st] * n + stop_id[st]), "stopping primitive not in its tile's list"
    e[st] = pos[order[idx]] + 1
    return int(e.sum())


def cpu_baseline(args, cfg, cams, cnt_r, sc_t, mode, q):
    """The FP64 oracle timed on the host (forward + backward of view 0, all
    threads), plus its work units pinned against the forward's counters on the
    same view: E (list entries processed up to and including each pixel's
    stop) and the pairs blended."""
    import numpy as np
    import torch

    import oracle
    from paper_2411_16392_amd import scenes

    cam = cams[0]
    W, H = cam.width, cam.height
    rows = min(args.cpu_rows, H)
    y0 = (H - rows) // 2
    win = (0, y0, W, rows)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = min(threads, os.cpu_count() or threads)
    dl = scenes.upstream_grads(0, H, W)
    oo = dict(resort=8, tile_depth=True) if mode else None
    t = time.perf_counter()
    # the key stage with the bound the GPU lists were built with (E counts list entries)
    ks = oracle.keys(cfg.scene, cam, tight=not args.loose_bound)
    o = oracle.render(cfg.scene, cam, opts=oo, window=win, key_stage=ks, nthreads=threads, dL=dl)
    dt = time.perf_counter() - t
    base = {"value": round(W * rows / dt / 1e6, 5), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"view 0, rows {y0}-{y0 + rows - 1} ({W}x{rows} px), key stage + FP64 forward + backward, "
                      f"{dt:.1f}s"}
    log(f"[bench] cpu oracle {base}", q)
    pin = None
    if rows == H and not mode:
        st = cnt_r.forward(sc_t, cam, exact=False)
        torch.cuda.synchronize()
        c = st.counters.cpu().numpy().view(np.uint32)
        e_gpu, bl_gpu = int(c[2]), int(c[4])
        e_or = oracle_entries_processed(oracle, ks, cam, o["stop_id"])
        bl_or = int(o["n_blend"].sum())
        near = int((o["margin"] < 1.0).sum())
        pin = {"view": 0, "E_gpu": e_gpu, "E_oracle": e_or, "blended_gpu": bl_gpu, "blended_oracle": bl_or,
               "E_ratio": round(e_gpu / max(e_or, 1), 7), "blended_ratio": round(bl_gpu / max(bl_or, 1), 7),
               "near_tied_pixels": near,
               "note": "the two may differ only on pixels with a near-tied decision"}
        log(f"[bench] units pinned against the oracle: {pin}", q)
    if not args.cpu_quick:
        # the oracle's throughput on one host thread (a band of rows of the
        # same view) and on the 100K-quadric sphere at 800 x 600 (full frame,
        # all threads, and a band on one thread)
        runs = []
        c1 = scenes.make_config(1)
        cam1 = c1.cameras[0]
        ks1 = oracle.keys(c1.scene, cam1, tight=not args.loose_bound)
        dl1 = scenes.upstream_grads(0, cam1.height, cam1.width)
        for label, sc, cm, kk, dd, nthr, nrows in (
                ("500K quadrics 1600x1200 view 0", cfg.scene, cam, ks, dl, 1, max(1, H // 16)),
                ("100K quadrics 800x600", c1.scene, cam1, ks1, dl1, threads, cam1.height),
                ("100K quadrics 800x600", c1.scene, cam1, ks1, dl1, 1, cam1.height // 16)):
            yy = (cm.height - nrows) // 2
            t = time.perf_counter()
            r = oracle.render(sc, cm, opts=oo, window=(0, yy, cm.width, nrows), key_stage=kk, nthreads=nthr,
                              dL=dd)
            d = time.perf_counter() - t
            runs.append({"workload": label, "threads": nthr, "rows": nrows, "s": round(d, 2),
                         "Mpix_s": round(cm.width * nrows / d / 1e6, 5), "evals_per_s": round(r["evals"] / d, 1)})
        base["more"] = runs
        log(f"[bench] cpu oracle, more: {runs}", q)
    return base, pin


def bench_serving(args, dev, q):
    """Config 4: a resident 1M-quadric scene, Poisson arrivals at 500/s of
    views at 256x256, 512x384, 1280x720 or 1920x1080; continuous batching
    under an 8 GiB tile-list budget vs one view at a time on the same trace."""
    import numpy as np
    import torch

    from paper_2411_16392_amd import render as R
    from paper_2411_16392_amd import scenes
    from paper_2411_16392_amd import serve

    cfg = scenes.make_config(4)
    sc_t = R.scene_to_device(cfg.scene, dev)
    n_req, n_warm = args.serve_requests, args.serve_warmup
    trace = scenes.serve_trace(n_req + n_warm, rate_hz=500.0, seed=4)
    budget = 8 << 30
    graphs = not args.serve_no_graphs
    with serve.Server(sc_t, budget_bytes=budget, max_slots=8, n_streams=4, graphs=graphs) as srv:
        res = serve.run_trace(srv, trace)
    ok = res["state"][n_warm:] == 0
    lat = res["latency"][n_warm:]
    st = res["stats"]
    s_b = serve.latency_summary(lat)
    log(f"[bench] serving: {res['frames_per_s']:.1f} frames/s, {s_b}, graphs {st.graph_launches} launched / "
        f"{st.graph_builds} built", q)
    seq = serve.run_sequential(sc_t, trace)
    s_s = serve.latency_summary(seq["latency"][n_warm:])
    log(f"[bench] one at a time: {seq['frames_per_s']:.1f} frames/s, {s_s}", q)
    # saturation: the same request mix with every request arriving at once
    # (the client keeps at most 48 output buffers per resolution in flight);
    # latency is arrival to completion, so it includes the queueing
    n2 = max(200, n_req // 2)
    trace2 = scenes.serve_trace(n2 + 50, rate_hz=1e7, seed=5)
    with serve.Server(sc_t, budget_bytes=budget, max_slots=8, n_streams=4, graphs=graphs) as srv:
        res2 = serve.run_trace(srv, trace2)
    seq2 = serve.run_sequential(sc_t, trace2)
    s2b = serve.latency_summary(res2["latency"][50:])
    s2s = serve.latency_summary(seq2["latency"][50:])
    log(f"[bench] saturated: batched {res2['frames_per_s']:.1f} frames/s {s2b}, one at a time "
        f"{seq2['frames_per_s']:.1f} frames/s {s2s}", q)
    # small views alone: does one request fill the chip?  Device time of one
    # view rendered alone (events around preprocess, count + sort and forward
    # on one stream) against the batched throughput of a saturated trace of
    # such views; fill = batched frames/s x device time per view, above 1 when
    # overlapping requests gets more out of the chip than one request does
    small = {}
    for wh in ((256, 256), (512, 384)):
        tr = scenes.serve_trace(400, rate_hz=1e7, seed=6, sizes=[wh])
        r1 = R.Renderer(device=dev)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for k, (_, cam) in enumerate(tr[:60]):
            ev0.record()
            r1.forward(sc_t, cam, exact=True)
            ev1.record()
            torch.cuda.synchronize()
            if k >= 10:
                times.append(ev0.elapsed_time(ev1))
        t_alone = float(np.median(times))
        with serve.Server(sc_t, budget_bytes=budget, max_slots=8, n_streams=4, graphs=graphs) as srv:
            rs = serve.run_trace(srv, tr)
        small[f"{wh[0]}x{wh[1]}"] = {"device_ms_alone": round(t_alone, 4),
                                     "batched_frames_per_s": round(rs["frames_per_s"], 1),
                                     "fill": round(rs["frames_per_s"] * t_alone * 1e-3, 3)}
    log(f"[bench] small views: {small}", q)
    torch.cuda.synchronize()
    return {"workload": "1M quadrics (shells + background ball), Poisson 500/s, views 256x256 / 512x384 / "
                        "1280x720 / 1920x1080, colour only",
            "requests": n_req, "warmup": n_warm, "rate_hz": 500.0,
            "frames_per_s": round(res["frames_per_s"], 2), "p50_ms": round(s_b["p50_ms"], 3),
            "p99_ms": round(s_b["p99_ms"], 3), "mean_ms": round(s_b["mean_ms"], 3),
            "all_done": bool(ok.all()), "budget_gib": budget / 2 ** 30,
            "peak_in_flight": int(st.peak_in_flight), "peak_pool_gib": round(st.peak_pool_bytes / 2 ** 30, 3),
            "graphs": graphs, "graph_launches": int(st.graph_launches), "graph_builds": int(st.graph_builds),
            "mean_pairs": float(np.mean(res["pairs"])),
            "one_at_a_time": {"frames_per_s": round(seq["frames_per_s"], 2), "p50_ms": round(s_s["p50_ms"], 3),
                              "p99_ms": round(s_s["p99_ms"], 3), "mean_ms": round(s_s["mean_ms"], 3)},
            "saturated": {"requests": n2 + 50, "frames_per_s": round(res2["frames_per_s"], 2),
                          "p50_ms": round(s2b["p50_ms"], 3), "p99_ms": round(s2b["p99_ms"], 3),
                          "one_at_a_time_frames_per_s": round(seq2["frames_per_s"], 2),
                          "one_at_a_time_p50_ms": round(s2s["p50_ms"], 3),
                          "one_at_a_time_p99_ms": round(s2s["p99_ms"], 3),
                          "all_done": bool((res2["state"] == 0).all())},
            "small_views": small}


if __name__ == "__main__":
    main()
