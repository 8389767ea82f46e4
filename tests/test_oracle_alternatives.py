"""Pins of the oracle's alternative results (reading R19: where a decision is
near-tied, FP32 and FP64 may fall on different sides of its boundary and both
results are correct).  The enumeration over near-tied decisions is checked
against sets of results written out here by brute force, per pixel, from the
compositing rules themselves (Eq. 1 with the alpha skip and the stop rule)."""
import itertools
import math

import numpy as np

import oracle
from paper_2411_16392_amd import scenes

from test_oracle_pins import _fd_scene, unit

# margin scales that make no decision near-tied ...
NEVER = dict(A=1e-30, D=1e-30, near=1e-30, E=1e-30, alpha_min=1e-30, T=1e-30, normal=1e-30, clamp=1e-30,
             median=1e-30, sort=1e-30, Dcond=1e-30)


def _setup():
    sc = _fd_scene(31, 7)
    cam = scenes.look_at((0.1, 0.05, -3.0), width=16, height=16, f=20)
    return sc, cam, oracle.keys(sc, cam)


def _hits(sc, cam, ks, px, py):
    """(alpha, rgb, t) of every primitive whose ray hit passes the 3-sigma test, in key order."""
    camv = oracle.cam_array(cam, np.float64)
    order = sorted([i for i in range(sc.n) if not ks["culled"][i]], key=lambda i: (int(ks["depth_bits"][i]), i))
    d = unit([((px + 0.5) - camv[14]) / camv[12], ((py + 0.5) - camv[15]) / camv[13], 1.0])
    amax = oracle.opts_array()[3]
    out = []
    for i in order:
        h = oracle.ray_hit(sc.center[i], sc.quat[i], sc.scale[i], sc.curv[i], camv, d)
        if h["ok"]:
            out.append((min(amax, float(sc.opacity[i]) * math.exp(-0.5 * h["E"])), sc.rgb[i].astype(float), h["t"]))
    return out


def _composite(entries, stop=True):
    teps = oracle.opts_array()[4]
    T, col, dep = 1.0, np.zeros(3), 0.0
    for al, rgb, t in entries:
        if stop and T * (1 - al) < teps:
            break
        col += al * T * rgb
        dep += al * T * t
        T *= 1 - al
    return np.concatenate([col, [dep, T]])


def _leaf_set(alts, k):
    v = alts["vals"][k, :alts["n"][k]]
    return v[:, [0, 1, 2, 3, 10]]  # colour, depth, T_final


def _same_sets(a, b, tol=1e-12):
    def covered(x, ys):
        return any(np.all(np.abs(x - y) <= tol * np.maximum(1.0, np.abs(y))) for y in ys)
    return all(covered(x, b) for x in a) and all(covered(y, a) for y in b)


def test_first_result_is_the_render():
    c = scenes.make_config(0)
    cam = c.cameras[0]
    r = oracle.render(c.scene, cam, nthreads=4)
    low = np.flatnonzero(r["margin"].ravel() < 1.0)
    assert len(low) > 0
    a = oracle.alternatives(c.scene, cam, low, nthreads=4)
    assert np.all(a["n"] >= 2) and not a["overflow"].any()
    flat = {k: r[k].reshape(r[k].shape[0], -1) if r[k].ndim == 3 else r[k].reshape(1, -1)
            for k in ("color", "depth", "normal", "T_final")}
    want = np.concatenate([flat["color"], flat["depth"], flat["normal"]], 0)[:, low].T
    assert np.array_equal(a["vals"][:, 0, :7], want)
    assert np.array_equal(a["vals"][:, 0, 10], flat["T_final"][0, low])
    # the other side of a near-tie changes the result of most of these pixels
    # (not of all: a flipped decision may lead to the same outcome, such as a
    # root rejected by the 3-sigma test either way)
    differs = [any(np.any(a["vals"][k, j] != a["vals"][k, 0]) for j in range(1, a["n"][k])) for k in range(len(low))]
    assert np.mean(differs) > 0.5


def test_alpha_skip_either_way_gives_every_subset():
    """With every alpha-vs-alpha_min decision near-tied, the results of a pixel
    are the composites of every subset of its hits (each hit blended or
    skipped), with the stop rule."""
    sc, cam, ks = _setup()
    delta = dict(NEVER, alpha_min=1e30)
    pix = np.arange(cam.width * cam.height)
    a = oracle.alternatives(sc, cam, pix, key_stage=ks, delta=delta, nthreads=2)
    checked = 0
    for k in pix:
        py, px = divmod(int(k), cam.width)
        hits = _hits(sc, cam, ks, px, py)
        if len(hits) > 6 or a["overflow"][k]:
            continue
        want = [_composite([h for h, keep in zip(hits, mask) if keep])
                for mask in itertools.product([0, 1], repeat=len(hits))]
        assert _same_sets(_leaf_set(a, k), want), (px, py, len(hits))
        checked += len(hits) >= 2
    assert checked > 50


def test_stop_either_way_gives_every_prefix():
    """With every stop decision near-tied, the results of a pixel are the
    composites of every prefix of its blended hits."""
    sc, cam, ks = _setup()
    delta = dict(NEVER, T=1e30)
    amin = oracle.opts_array()[2]
    pix = np.arange(cam.width * cam.height)
    a = oracle.alternatives(sc, cam, pix, key_stage=ks, delta=delta, nthreads=2)
    checked = 0
    for k in pix:
        py, px = divmod(int(k), cam.width)
        hits = [h for h in _hits(sc, cam, ks, px, py) if h[0] >= amin]
        want = [_composite(hits[:m], stop=False) for m in range(len(hits) + 1)]
        assert _same_sets(_leaf_set(a, k), want), (px, py)
        checked += len(hits) >= 2
    assert checked > 50


def test_forced_paths_reproduce_their_results():
    sc, cam, ks = _setup()
    delta = dict(NEVER, alpha_min=1e30)
    pix = np.arange(0, cam.width * cam.height, 3)
    a = oracle.alternatives(sc, cam, pix, key_stage=ks, delta=delta, nthreads=2)
    rng = np.random.default_rng(5)
    pick = np.array([rng.integers(0, n) for n in a["n"]])
    forced = (pix, a["paths"][np.arange(len(pix)), pick], a["plen"][np.arange(len(pix)), pick])
    r = oracle.render(sc, cam, key_stage=ks, delta=delta, forced=forced, nthreads=2)
    got = np.concatenate([r["color"].reshape(3, -1), r["depth"].reshape(1, -1), r["normal"].reshape(3, -1)], 0)
    want = a["vals"][np.arange(len(pix)), pick]
    assert np.array_equal(got[:, pix].T, want[:, :7])
    assert np.array_equal(r["T_final"].ravel()[pix], want[:, 10])
    assert np.any(pick > 0)


def test_gradient_skip_drops_ill_conditioned_pixels():
    sc, cam, ks = _setup()
    rng = np.random.default_rng(3)
    dL = (rng.standard_normal((3, 16, 16)), rng.standard_normal((16, 16)), rng.standard_normal((3, 16, 16)))
    # every accepted root counted as ill-conditioned and every |A| test as
    # near-tied: no pixel with a hit contributes
    r = oracle.render(sc, cam, key_stage=ks, dL=dL, delta=dict(Dcond=1e30, A=1e30), grad_skip=True, nthreads=2)
    assert np.all(r["gmargin"][r["n_blend"] > 0] < 1.0)
    for k, g in r["grads"].items():
        assert np.all(g == 0.0), k
    # with the default scales the same call equals the plain backward on the
    # pixels it keeps
    r1 = oracle.render(sc, cam, key_stage=ks, dL=dL, grad_skip=True, nthreads=2)
    keep = r1["gmargin"] >= 1.0
    dLk = tuple(x * keep for x in dL)
    r2 = oracle.render(sc, cam, key_stage=ks, dL=dLk, nthreads=2)
    for k in r1["grads"]:
        assert np.allclose(r1["grads"][k], r2["grads"][k], rtol=1e-13, atol=1e-15), k
