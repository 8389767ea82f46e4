"""The chord-bound local box (QGS_TIGHT_BOUND, a default flag) on the GPU.

Keys, rectangles, conics and sorted lists are bit-exact against the oracle's
key stage with the same box.  The box is conservative, so the rendered image
and, in the deterministic mode, the gradients are bit-identical to the default
box's; the FP64 renderer (which bins with its own bound) agrees within the
usual tolerances on strongly curved primitives, where the box is much smaller.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

from gpu_helpers import backward_parity, gpu_forward, to_np
from test_gpu_parity import check_keys, check_lists

pytestmark = pytest.mark.gpu

TB = L.QGS_TIGHT_BOUND
DET = L.QGS_DETERMINISTIC_BWD


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


_CACHE = {}


def curved_cfg0(lim=60.0, seed=5):
    """Workload 0 with curvatures U[-lim, lim] (10% planar) and opacity as drawn."""
    key = ("curved", lim, seed)
    if key not in _CACHE:
        c = scenes.make_config(0)
        rng = np.random.Generator(np.random.PCG64(seed))
        sc = scenes.Scene(*(a.copy() for a in c.scene.arrays()))
        l = rng.uniform(-lim, lim, (sc.n, 2)).astype(np.float32)
        l[rng.random(sc.n) < 0.1] = 0.0
        sc.curv = l
        _CACHE[key] = (sc, c.cameras[0])
    return _CACHE[key]


def cfg(i, **kw):
    key = (i, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = scenes.make_config(i, **kw)
    return _CACHE[key]


def cases():
    sc, cam = curved_cfg0()
    yield "curved", sc, cam
    c = cfg(0)
    yield "cfg0", c.scene, c.cameras[0]
    c = cfg(1)
    yield "cfg1", c.scene, c.cameras[0]
    c = cfg(3, n_override=300_000, n_views=2)
    for v, cam in enumerate(c.cameras):
        yield f"cfg3 v{v}", c.scene, cam


def test_tight_keys_and_lists_bitexact():
    for name, sc, cam in cases():
        print(name, flush=True)
        for det in (False, True):
            _, st = gpu_forward(sc, cam, opts=dict(flags=DET if det else 0))
            assert st.flags & TB
            ks = check_keys(sc, cam, st, tight=True)
            check_lists(ks, cam, st)


def test_tight_keys_headline_size():
    c = cfg(2, n_views=64)
    cam = c.cameras[13]
    _, st = gpu_forward(c.scene, cam)
    ks = check_keys(c.scene, cam, st, tight=True)
    assert check_lists(ks, cam, st) > 1_000_000


def _planes(st):
    return {k: to_np(getattr(st, k)) for k in ("color", "depth", "normal", "T_final")}


def test_tight_bound_same_image_and_deterministic_gradients():
    for name, sc, cam in cases():
        print(name, flush=True)
        dL = scenes.upstream_grads(3, cam.height, cam.width)
        dLt = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in dL]
        out = {}
        for flags in (DET, DET | TB):
            r = R.Renderer(opts=R.make_opts(flags=flags, tight_bound=bool(flags & TB)))
            sc_t = R.scene_to_device(sc)
            st = r.forward(sc_t, cam)
            g = r.backward(sc_t, st, *dLt)
            torch.cuda.synchronize()
            out[flags] = (_planes(st), {k: to_np(v) for k, v in g.items()}, st.num_pairs)
        (pa, ga, na), (pb, gb, nb) = out[DET], out[DET | TB]
        assert nb <= na, name
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (name, k)
        for k in ga:
            assert np.array_equal(ga[k], gb[k]), (name, k)
        print(name, "pairs default", na, "tight", nb)


def test_tight_bound_fewer_pairs_on_curved_primitives():
    sc, cam = curved_cfg0()
    _, a = gpu_forward(sc, cam, opts=dict(tight_bound=False))
    _, b = gpu_forward(sc, cam)
    assert b.num_pairs < 0.85 * a.num_pairs, (a.num_pairs, b.num_pairs)


def test_tight_bound_oracle_parity_curved():
    sc, cam = curved_cfg0()
    win = (0, 0, cam.width, cam.height)
    dL = scenes.upstream_grads(4, cam.height, cam.width)
    # strongly curved primitives put more pixels near a decision boundary
    # (grazing rays: discriminant near 0) than workload 0
    rep, _, _ = backward_parity(sc, cam, win, dL, label="curved", max_excluded=0.03, max_grad_excluded=0.05)
    print("curved", rep)
