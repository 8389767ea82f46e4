"""Spherical-harmonics colour and the densification statistics on the GPU,
through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

from gpu_helpers import (check_forward, grad_errors, oracle_backward, to_np, window_of, TOL_GRAD,
                         GRAD_FLOOR)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def _sh_scene(ci, deg):
    c = scenes.make_config(ci)
    return c, scenes.with_sh(c.scene, deg, 70 + ci)


@pytest.mark.parametrize("ci,deg", [(0, 3), (1, 1)])
def test_sh_colour_forward(ci, deg):
    c, sc = _sh_scene(ci, deg)
    cam = c.cameras[0]
    r = R.Renderer()
    st = r.forward(R.scene_to_device(sc), cam)
    torch.cuda.synchronize()
    res, _, _ = check_forward(window_of(st, (0, 0, cam.width, cam.height)), sc, cam, label=f"sh cfg{ci}",
                              max_excluded=0.01)
    print("sh", ci, deg, res)


def test_sh_backward_and_densification_stats():
    c, sc = _sh_scene(0, 3)
    cam = c.cameras[0]
    win = (0, 0, cam.width, cam.height)
    dL = scenes.upstream_grads(31, cam.height, cam.width)
    ks = oracle.keys(sc, cam)
    r = R.Renderer()
    sc_t = R.scene_to_device(sc)
    st = r.forward(sc_t, cam)
    torch.cuda.synchronize()
    # every pixel checked forward and carrying its upstream gradient unless
    # its derivative is ill-conditioned (see gpu_helpers)
    rep, forced, _ = check_forward(window_of(st, win), sc, cam, ks=ks, label="sh fwd", max_excluded=0.01)
    og, dLm, gex = oracle_backward(sc, cam, win, dL, forced, ks=ks)
    assert gex <= 0.005, rep
    o = {"grads": og}
    stats = {"screen_grad": torch.zeros(sc.n, device="cuda"), "visible": torch.zeros(sc.n, device="cuda")}
    t = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in dLm]
    g = r.backward(sc_t, st, *t, stats=stats)
    gg = {k: to_np(v) for k, v in g.items()}
    r.backward(sc_t, st, *t, stats=stats)   # statistics add up over calls
    torch.cuda.synchronize()
    print("sh bwd", rep, "worst", grad_errors(gg, og), "grad excluded", gex)
    a, b = gg["sh"], o["grads"]["sh"]
    tol = TOL_GRAD * (np.abs(b) + GRAD_FLOOR * np.abs(b).max())
    assert np.all(np.abs(a - b) <= tol)
    # statistics from the oracle's centre gradient: |(W/2 z/fx g_x, H/2 z/fy g_y)| in camera axes
    camv = oracle.cam_array(cam, np.float64)
    Wr = camv[:9].reshape(3, 3)
    gcam = o["grads"]["center"] @ Wr.T
    z = (sc.center.astype(np.float64) @ Wr.T + camv[9:12])[:, 2]
    want = np.hypot(0.5 * cam.width * z / camv[12] * gcam[:, 0], 0.5 * cam.height * z / camv[13] * gcam[:, 1])
    vis = to_np(stats["visible"])
    live = oracle.keys(sc, cam, tight=bool(st.flags & L.QGS_TIGHT_BOUND))["tiles"] > 0
    assert np.array_equal(vis, 2.0 * live)
    got = to_np(stats["screen_grad"]) / 2.0
    assert np.all(np.abs(got - want) <= 2e-3 * (want + 1e-2 * want.max()))


def test_sh_autograd_matches_direct_backward():
    c, sc = _sh_scene(0, 2)
    cam = c.cameras[0]
    sc_t = {k: v.clone().requires_grad_(True) for k, v in R.scene_to_device(sc).items()}
    rend = R.Renderer()
    col, dep, nrm = R.render(sc_t, cam, rend)
    rng = np.random.default_rng(9)
    w = [torch.from_numpy(rng.standard_normal(t.shape).astype(np.float32)).cuda() for t in (col, dep, nrm)]
    ((col * w[0]).sum() + (dep * w[1]).sum() + (nrm * w[2]).sum()).backward()
    det = {k: v.detach() for k, v in sc_t.items()}
    st = rend.forward(det, cam)
    g = rend.backward(det, st, *w)
    torch.cuda.synchronize()
    assert sc_t["sh"].grad is not None
    for k in list(R.SCENE_KEYS) + ["sh"]:
        a, b = to_np(sc_t[k].grad), to_np(g[k])
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * (np.abs(b).max() + 1e-12)), k


def test_sh_argument_checks():
    c, sc = _sh_scene(0, 1)
    cam = c.cameras[0]
    sc_t = R.scene_to_device(sc)
    r = R.Renderer()
    st = r.forward(sc_t, cam)
    out = {k: torch.empty_like(v) for k, v in sc_t.items() if k != "sh"}
    g = L.QgsSceneGrads()
    for k in R.SCENE_KEYS:
        setattr(g, k, out[k].data_ptr())
    dl = L.QgsImageGrads()
    dc = torch.ones_like(st.color)
    dl.dcolor = dc.data_ptr()
    _, nbytes = L.qgs_workspace_query(st.n, st.cam, st.capacity, 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.QgsError) as e:   # SH scene without an sh gradient buffer
        L.qgs_render_bwd(R._scene_struct(sc_t), st.prim_buf(), st.lists(), st.cam, r.opts, st.images(), dl, g,
                         ws.data_ptr(), ws.numel())
    assert e.value.status == L.QGS_ERR_INVALID_ARG
    s = R._scene_struct(sc_t)
    s.sh_degree = 4
    with pytest.raises(L.QgsError) as e:
        L.qgs_preprocess(s, st.cam, r.opts, st.prim_buf())
    assert e.value.status == L.QGS_ERR_INVALID_ARG
