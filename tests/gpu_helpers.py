"""Shared helpers for the GPU parity tests (HIP path through the C ABI vs the
FP64 oracle on the same seeded inputs).

Every pixel is checked.  Where no decision of the oracle's per-pixel sequence
is near-tied (margin >= 1) the GPU must match the oracle's result; where one is
(reading R19: FP32 and FP64 may then decide differently, and both results are
correct) it must match one of the results the near-tied decisions allow, which
the oracle enumerates.  The gradient check then runs the oracle's backward
with each such pixel's decisions set to the ones of the result the GPU matched,
and leaves out (zero upstream gradient on both sides) only the pixels whose
derivative is ill-conditioned or ambiguous there (an accepted root at a
near-tangent ray, the alpha clamp, the small-|A| branch), whose share every
test reports and bounds.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2411_16392_amd import render as R

# tolerances (the benchmark spec): colour / normal 1e-4 absolute, depth 1e-4 relative to
# max(1, depth), gradients 1e-3 relative with a floor of 1e-2 of the largest
# entry of the tensor
TOL_COLOR = 1e-4
TOL_NORMAL = 1e-4
TOL_DEPTH = 1e-4
TOL_GRAD = 1e-3
GRAD_FLOOR = 1e-2

# compared channels, in the order of oracle.ALT_CHANNELS: (index, relative?)
_CH_BASE = [(0, False), (1, False), (2, False), (3, True), (4, False), (5, False), (6, False), (10, False)]
_CH_GEO = [(7, True), (8, True), (9, True)]
_CH_NAMES = dict(enumerate(oracle.ALT_CHANNELS))


def gpu_forward(scene, cam, renderer=None, exact=True, opts=None):
    r = renderer or R.Renderer(opts=R.make_opts(**(opts or {})))
    st = r.forward(R.scene_to_device(scene), cam, exact=exact)
    torch.cuda.synchronize()
    return r, st


def to_np(t):
    return t.detach().cpu().numpy()


def window_of(st, window, geometry=False):
    x0, y0, w, h = window
    sl = (slice(y0, y0 + h), slice(x0, x0 + w))
    out = dict(color=to_np(st.color)[:, sl[0], sl[1]], depth=to_np(st.depth)[sl],
               normal=to_np(st.normal)[:, sl[0], sl[1]], T_final=to_np(st.T_final)[sl],
               last=to_np(st.last)[sl])
    if geometry:
        out.update(curvature=to_np(st.curvature)[sl], median_depth=to_np(st.median_depth)[sl],
                   distortion=to_np(st.distortion)[sl])
    return out


def _stack(m, geometry):
    """[11, h, w] in oracle.ALT_CHANNELS order (maps a colour-only image lacks,
    and the geometry maps unless asked for, are zero)."""
    h, w = m["color"].shape[1:]
    z = np.zeros((h, w))
    if "depth" not in m:
        return np.stack([m["color"][0], m["color"][1], m["color"][2]] + [z] * 8).astype(np.float64)
    geo = [m.get("curvature", z), m.get("median_depth", z), m.get("distortion", z)] if geometry else [z, z, z]
    return np.stack([m["color"][0], m["color"][1], m["color"][2], m["depth"], m["normal"][0], m["normal"][1],
                     m["normal"][2], *geo, m["T_final"]]).astype(np.float64)


def _ratios(G, O, chans):
    """|G - O| / tolerance per compared channel (leading axis)."""
    out = []
    for c, rel in chans:
        tol = 1e-4 * np.maximum(1.0, np.abs(O[c])) if rel else 1e-4
        out.append(np.abs(G[c] - O[c]) / tol)
    return np.stack(out)


def check_forward(g, scene, cam, window=None, opts=None, ks=None, geometry=False, label="", nthreads=None,
                  max_excluded=None, color_only=False):
    """g: GPU maps of the window (window_of).  Checks every pixel as the module
    docstring says and returns (report, forced, oracle result): report holds
    the largest error per channel over all pixels (against the matched
    result), `excluded` (share of pixels with a near-tied decision),
    `alt_taken` (share matching a result other than the oracle's own),
    `unchecked` (pixels whose enumeration was cut short and matched none) and
    `unmatched`; forced = (pixels, paths, lengths) of the matched results.
    color_only: g holds only "color" (a served image), the one map compared."""
    win = window if window is not None else (0, 0, cam.width, cam.height)
    o = oracle.render(scene, cam, opts=opts, window=win, key_stage=ks, branch_median=geometry, nthreads=nthreads)
    chans = _CH_BASE[:3] if color_only else _CH_BASE + (_CH_GEO if geometry else [])
    G = _stack(g, geometry)
    O = _stack(o, geometry)
    C, h, w = G.shape
    err = _ratios(G, O, chans)                       # [c, h, w]
    low = o["margin"] < 1.0
    idx = np.flatnonzero(low.ravel())
    best_err = err.reshape(len(chans), -1).copy()    # per pixel: error against the result it is checked with
    forced = (idx, np.zeros((len(idx), oracle.PATH_MAX), np.uint8), np.zeros(len(idx), np.int32))
    unmatched = unchecked = 0
    alt_taken = 0
    if len(idx):
        a = oracle.alternatives(scene, cam, idx, opts=opts, window=win, key_stage=ks, branch_median=geometry,
                                nthreads=nthreads)
        Gp = G.reshape(C, -1)[:, idx]                # [C, k]
        V = np.moveaxis(a["vals"], 2, 0)             # [11, k, L]
        leaf_err = _ratios(Gp[:, :, None], V, chans).max(0)   # [k, L]
        L = V.shape[2]
        leaf_err[np.arange(L)[None, :] >= a["n"][:, None]] = np.inf
        best = leaf_err.argmin(1)
        ok = leaf_err[np.arange(len(idx)), best] <= 1.0
        unmatched = int((~ok).sum())
        unchecked = int(((~ok) & (a["overflow"] != 0)).sum())
        alt_taken = int((best > 0).sum())
        sel = V[:, np.arange(len(idx)), best]        # [11, k]
        best_err[:, idx] = _ratios(Gp, sel, chans)
        forced = (idx, a["paths"][np.arange(len(idx)), best], a["plen"][np.arange(len(idx)), best])
    worst = best_err.max(1) if best_err.size else np.zeros(len(chans))
    rep = dict(excluded=float(low.mean()), alt_taken=alt_taken / (h * w), unmatched=unmatched, unchecked=unchecked,
               pixels=h * w)
    if best_err.size:
        # where the largest error relative to its tolerance sits
        k = int(best_err.max(0).argmax())
        rep["worst_at"] = dict(x=int(win[0] + k % w), y=int(win[1] + k // w), ratio=float(best_err[:, k].max()),
                               margin=float(o["margin"].ravel()[k]), blended=int(o["n_blend"].ravel()[k]))
    for (c, rel), e in zip(chans, worst):
        rep[_CH_NAMES[c]] = float(e) * 1e-4
    bad_natural = int(((err.max(0) > 1.0) & ~low).sum())
    rep["bad"] = bad_natural
    assert bad_natural == 0 and unmatched == 0, (label, rep)
    if max_excluded is not None:
        assert rep["excluded"] <= max_excluded, (label, rep)
    return rep, forced, o


def grad_errors(g, o):
    """Per-tensor check |g - o| <= 1e-3 (|o| + 1e-2 max|o|); returns worst ratio."""
    worst = 0.0
    for k in R.SCENE_KEYS:
        a = np.asarray(g[k], np.float64).reshape(o[k].shape)
        b = o[k]
        scale = np.abs(b).max() + 1e-30
        tol = TOL_GRAD * (np.abs(b) + GRAD_FLOOR * scale)
        ratio = float((np.abs(a - b) / tol).max())
        worst = max(worst, ratio)
        assert ratio <= 1.0, (k, ratio, np.unravel_index(np.argmax(np.abs(a - b) / tol), b.shape))
    return worst


def oracle_backward(scene, cam, window, dL, forced, ks=None, opts=None, geometry=False, nthreads=None):
    """Oracle forward + backward of the window with the matched decisions and
    ill-conditioned pixels left out.  Returns (grads, dL zeroed outside the
    window and on those pixels, their share of the window)."""
    x0, y0, w, h = window
    ob = oracle.render(scene, cam, opts=opts, window=window, key_stage=ks, dL=dL, forced=forced,
                       branch_median=geometry, grad_skip=True, nthreads=nthreads)
    keep = np.zeros((cam.height, cam.width), bool)
    keep[y0:y0 + h, x0:x0 + w] = ob["gmargin"] >= 1.0
    dLm = tuple(np.ascontiguousarray(a * keep, np.float32) for a in dL)
    return ob["grads"], dLm, float((ob["gmargin"] < 1.0).mean())


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def backward_parity(scene, cam, window, dL, flags=0, oracle_opts=None, geometry=False, ks=None, label="",
                    max_excluded=None, max_grad_excluded=0.02, renderer=None, nthreads=None):
    """GPU forward + backward of one view against the oracle, every pixel of
    `window` checked forward and carrying its upstream gradient dL (full view:
    colour, depth, normal and with geometry also curvature, median depth,
    distortion) unless its derivative is ill-conditioned.  Returns (report,
    GPU gradients, oracle gradients)."""
    r = renderer or R.Renderer(opts=R.make_opts(flags=flags), geometry=geometry)
    sc_t = R.scene_to_device(scene)
    st = r.forward(sc_t, cam)
    torch.cuda.synchronize()
    rep, forced, _ = check_forward(window_of(st, window, geometry), scene, cam, window, opts=oracle_opts, ks=ks,
                                   geometry=geometry, label=label, max_excluded=max_excluded, nthreads=nthreads)
    og, dLm, gex = oracle_backward(scene, cam, window, dL, forced, ks=ks, opts=oracle_opts, geometry=geometry,
                                   nthreads=nthreads)
    d = [_dev(a) for a in dLm]
    if geometry:
        g = r.backward(sc_t, st, d[0], d[1], d[2], dcurvature=d[3], dmedian_depth=d[4], ddistortion=d[5])
    else:
        g = r.backward(sc_t, st, d[0], d[1], d[2])
    torch.cuda.synchronize()
    g = {k: to_np(v) for k, v in g.items()}
    rep["grad_excluded"] = gex
    rep["grad_worst"] = grad_errors(g, og)
    assert gex <= max_grad_excluded, (label, rep)
    return rep, g, og
