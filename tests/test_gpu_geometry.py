"""Parity of the geometry maps (curvature, median depth, depth distortion) and
their gradients: HIP path through the C ABI against the FP64 oracle.

Maps within 1e-4 relative to max(1, |value|), every pixel checked (the
median's choices are among the near-tied decisions whose other side is also
accepted); gradients to the same bar as the other outputs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

from gpu_helpers import backward_parity, check_forward, to_np, window_of

pytestmark = pytest.mark.gpu

TOL_GEO = 1e-4

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


def _geo_forward(scene, cam, flags=0):
    r = R.Renderer(opts=R.make_opts(flags=flags), geometry=True)
    sc_t = R.scene_to_device(scene)
    st = r.forward(sc_t, cam)
    torch.cuda.synchronize()
    return r, sc_t, st


def _compare_geo(st, scene, cam, window, label, ks=None):
    res, _, _ = check_forward(window_of(st, window, geometry=True), scene, cam, window, ks=ks, geometry=True,
                              label=label, max_excluded=0.03)
    x0, y0, w, h = window
    sl = (slice(y0, y0 + h), slice(x0, x0 + w))
    # the median is a hit depth of a blended entry; none means 0
    medp = to_np(st.median_pos)[sl]
    assert np.all((medp == 0) == (to_np(st.median_depth)[sl] == 0.0))
    assert np.all(medp <= to_np(st.last)[sl])
    return res


@pytest.mark.parametrize("ci", [0, 1])
def test_geometry_maps_full_frame(ci):
    c = cfg(ci)
    cam = c.cameras[0]
    _, _, st = _geo_forward(c.scene, cam)
    res = _compare_geo(st, c.scene, cam, (0, 0, cam.width, cam.height), f"cfg{ci}")
    assert res["excluded"] < 0.01
    print("geo", ci, res)


def test_geometry_maps_headline_crops():
    c = cfg(2, n_views=64)
    cam = c.cameras[21]
    _, _, st = _geo_forward(c.scene, cam)
    ks = oracle.keys(c.scene, cam)
    for win in [(760, 560, 64, 64), (1536, 1136, 64, 64)]:
        res = _compare_geo(st, c.scene, cam, win, f"cfg2 {win}", ks=ks)
        print("geo cfg2", win, res)


def test_geometry_off_leaves_outputs_unchanged():
    # the plain forward and the geometry forward write identical colour, depth,
    # normal, T_final and last
    c = cfg(1)
    cam = c.cameras[0]
    sc_t = R.scene_to_device(c.scene)
    a = R.Renderer().forward(sc_t, cam)
    _, _, b = _geo_forward(c.scene, cam)
    torch.cuda.synchronize()
    for k in ("color", "depth", "normal", "T_final", "last"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def _geo_bwd_case(scene, cam, window, seed, flags=0):
    dL = (scenes.upstream_grads(seed, cam.height, cam.width, crop=window) +
          scenes.upstream_geometry_grads(seed, cam.height, cam.width, crop=window))
    rep, g, o = backward_parity(scene, cam, window, dL, flags=flags, geometry=True, label=f"geo bwd {window}",
                                max_excluded=0.03, max_grad_excluded=0.04)
    print("geo bwd", window, rep)
    return g, o


def test_geometry_backward_config0():
    c = cfg(0)
    _geo_bwd_case(c.scene, c.cameras[0], (0, 0, 128, 128), 17)


def test_geometry_backward_config1_crop():
    c = cfg(1)
    _geo_bwd_case(c.scene, c.cameras[0], (368, 268, 64, 64), 18)


def test_geometry_backward_deterministic():
    c = cfg(1)
    cam = c.cameras[0]
    win = (368, 268, 64, 64)
    g1, o = _geo_bwd_case(c.scene, cam, win, 18, flags=L.QGS_DETERMINISTIC_BWD)
    g2, _ = _geo_bwd_case(c.scene, cam, win, 18, flags=L.QGS_DETERMINISTIC_BWD)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k


def test_geometry_autograd_matches_direct_backward():
    c = cfg(0)
    cam = c.cameras[0]
    sc_t = {k: v.clone().requires_grad_(True) for k, v in R.scene_to_device(c.scene).items()}
    rend = R.Renderer(geometry=True)
    outs = R.render(sc_t, cam, rend)
    assert len(outs) == 6
    rng = np.random.default_rng(5)
    w = [torch.from_numpy(rng.standard_normal(t.shape).astype(np.float32)).cuda() for t in outs]
    loss = sum((o_ * w_).sum() for o_, w_ in zip(outs, w))
    loss.backward()
    det = {k: v.detach() for k, v in sc_t.items()}
    st = rend.forward(det, cam)
    g = rend.backward(det, st, w[0], w[1], w[2], dcurvature=w[3], dmedian_depth=w[4], ddistortion=w[5])
    torch.cuda.synchronize()
    for k in R.SCENE_KEYS:
        a, b = to_np(sc_t[k].grad), to_np(g[k])
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * (np.abs(b).max() + 1e-12)), k


def test_geometry_argument_checks():
    c = cfg(0)
    cam = c.cameras[0]
    r = R.Renderer()
    sc_t = R.scene_to_device(c.scene)
    st = r.forward(sc_t, cam)
    # partial geometry outputs are rejected
    im = st.images()
    im.curvature = st.depth.data_ptr()
    with pytest.raises(L.QgsError) as e:
        L.qgs_render_fwd(st.prim_buf(), st.lists(), st.cam, r.opts, im)
    assert e.value.status == L.QGS_ERR_INVALID_ARG
    # geometry gradients without geometry maps are rejected, by the binding and by the C ABI
    with pytest.raises(ValueError):
        r.backward(sc_t, st, dcurvature=torch.zeros_like(st.depth))
    out = {k: torch.empty_like(v) for k, v in sc_t.items()}
    g = L.QgsSceneGrads()
    for k in R.SCENE_KEYS:
        setattr(g, k, out[k].data_ptr())
    dl = L.QgsImageGrads()
    dz = torch.zeros_like(st.depth)
    dl.ddistortion = dz.data_ptr()
    _, nbytes = L.qgs_workspace_query(st.n, st.cam, st.capacity, 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.QgsError) as e:
        L.qgs_render_bwd(R._scene_struct(sc_t), st.prim_buf(), st.lists(), st.cam, r.opts, st.images(), dl, g,
                         ws.data_ptr(), ws.numel())
    assert e.value.status == L.QGS_ERR_INVALID_ARG
