"""The paper's full-model ordering on the GPU (per-tile sort depth and the
8-entry per-pixel resort buffer, with the front-to-back backward) against the
FP64 oracle with the same ordering, through the C ABI.  Same tolerances and
every-pixel check as the plain path; the buffer's choice between two close hit
depths is one of the near-tied decisions whose other side is also accepted."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

from gpu_helpers import backward_parity, check_forward, to_np, window_of

pytestmark = pytest.mark.gpu

FULL = L.QGS_TILE_DEPTH | L.QGS_RESORT
ORACLE_FULL = dict(resort=8, tile_depth=True)
_CFG = {}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def cfg(i, **kw):
    key = (i, tuple(sorted(kw.items())))
    if key not in _CFG:
        _CFG[key] = scenes.make_config(i, **kw)
    return _CFG[key]


def _fwd(scene, cam, flags=FULL, geometry=False):
    r = R.Renderer(opts=R.make_opts(flags=flags), geometry=geometry)
    sc_t = R.scene_to_device(scene)
    st = r.forward(sc_t, cam)
    torch.cuda.synchronize()
    return r, sc_t, st


@pytest.mark.parametrize("ci,flags,o_opts", [(0, FULL, ORACLE_FULL), (1, FULL, ORACLE_FULL),
                                              (1, L.QGS_RESORT, dict(resort=8)),
                                              (1, L.QGS_TILE_DEPTH, dict(tile_depth=True))])
def test_full_model_forward_full_frame(ci, flags, o_opts):
    c = cfg(ci)
    cam = c.cameras[0]
    _, _, st = _fwd(c.scene, cam, flags)
    # the sphere of config 1 puts many hits of one surface within a few 1e-6 of
    # each other in depth: the buffer's choice between them is often near-tied
    res, _, _ = check_forward(window_of(st, (0, 0, cam.width, cam.height)), c.scene, cam, opts=o_opts,
                              label=f"full cfg{ci}", max_excluded=0.05)
    print("full model", ci, flags, res)


def test_full_model_forward_headline_crops():
    c = cfg(2, n_views=64)
    cam = c.cameras[3]
    _, _, st = _fwd(c.scene, cam)
    ks = oracle.keys(c.scene, cam)
    for win in [(760, 560, 64, 64), (1100, 700, 48, 56)]:
        res, _, _ = check_forward(window_of(st, win), c.scene, cam, win, opts=ORACLE_FULL, ks=ks,
                                  label=f"full cfg2 {win}", max_excluded=0.5)
        print("full model cfg2", win, res)


def test_resort_changes_the_image():
    # the ordering options are not no-ops on these scenes
    c = cfg(1)
    cam = c.cameras[0]
    _, _, a = _fwd(c.scene, cam, 0)
    _, _, b = _fwd(c.scene, cam, FULL)
    assert float((a.color - b.color).abs().max()) > 1e-3


def _bwd_case(scene, cam, window, seed, flags=FULL, geometry=False):
    dL = scenes.upstream_grads(seed, cam.height, cam.width, crop=window)
    if geometry:
        dL = dL + scenes.upstream_geometry_grads(seed, cam.height, cam.width, crop=window)
    rep, g, o = backward_parity(scene, cam, window, dL, flags=flags, oracle_opts=ORACLE_FULL, geometry=geometry,
                                label=f"full bwd {window}", max_excluded=0.5, max_grad_excluded=0.04)
    print("full bwd", window, rep)
    return g, o


def test_full_model_backward_config0():
    c = cfg(0)
    _bwd_case(c.scene, c.cameras[0], (0, 0, 128, 128), 27)


def test_full_model_backward_config1_crop():
    c = cfg(1)
    _bwd_case(c.scene, c.cameras[0], (368, 268, 64, 64), 28)


def test_full_model_backward_with_geometry_maps():
    c = cfg(1)
    _bwd_case(c.scene, c.cameras[0], (368, 268, 64, 64), 29, geometry=True)


def test_full_model_deterministic_backward():
    c = cfg(1)
    cam = c.cameras[0]
    win = (368, 268, 64, 64)
    flags = FULL | L.QGS_DETERMINISTIC_BWD
    g1, o = _bwd_case(c.scene, cam, win, 28, flags=flags)
    g2, _ = _bwd_case(c.scene, cam, win, 28, flags=flags)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k


def test_full_model_geometry_forward():
    c = cfg(0)
    cam = c.cameras[0]
    _, _, st = _fwd(c.scene, cam, FULL, geometry=True)
    win = (0, 0, cam.width, cam.height)
    res, _, _ = check_forward(window_of(st, win, geometry=True), c.scene, cam, opts=ORACLE_FULL, geometry=True,
                              label="full geo cfg0", max_excluded=0.01)
    print("full model geometry", res)
