"""Serving: served images against the FP64 oracle; results in the mix equal
results alone; admission by memory; cancellation; budget refusal; a Poisson
trace completes."""
import numpy as np
import pytest
import torch

from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes
from paper_2411_16392_amd import serve

from gpu_helpers import check_forward

pytestmark = pytest.mark.gpu


_SCENE = {}


def _scene():
    if "s" not in _SCENE:
        _SCENE["s"] = scenes.scene_unbounded(200_000, 4)
    return _SCENE["s"]


@pytest.fixture(scope="module")
def scene_t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return R.scene_to_device(_scene())


def _views(n, seed):
    tr = scenes.serve_trace(n, rate_hz=500.0, seed=seed)
    return [cam for _, cam in tr]


def _alone(scene_t, cam):
    r = R.Renderer()
    st = r.forward(scene_t, cam)
    torch.cuda.synchronize()
    return st.color.clone(), st.num_pairs


def _drain(srv, n, timeout_s=60.0):
    got = {}
    import time
    t0 = time.time()
    while len(got) < n and time.time() - t0 < timeout_s:
        for c in srv.poll(64, 20000):
            got[c.req_id] = (c.state, c.status, c.num_pairs, c.t_submit, c.t_admit, c.t_done)
    assert len(got) == n, f"only {len(got)} of {n} completions"
    return got


def test_each_result_alone_equals_in_the_mix(scene_t):
    cams = _views(24, 11)
    outs = [torch.full((3, c.height, c.width), -1.0, device="cuda") for c in cams]
    with serve.Server(scene_t, budget_bytes=2 << 30, max_slots=6, n_streams=4) as srv:
        ids = [srv.submit(c, o) for c, o in zip(cams, outs)]   # burst: all overlap
        got = _drain(srv, len(ids))
        st = srv.stats()
    assert st.peak_in_flight > 1
    for rid, cam, out in zip(ids, cams, outs):
        state, status, pairs, *_ = got[rid]
        assert state == L.QGS_REQ_DONE and status == 0
        ref, npairs = _alone(scene_t, cam)
        assert pairs == npairs
        err = float((out - ref).abs().max())
        assert err <= 1e-6, (rid, err)


def test_graph_launches_match_direct_launches(scene_t):
    # the slots' persistent graphs (updated in place per request) against
    # plain stream launches: bit-identical images, and every pass went
    # through a graph
    cams = _views(16, 21)
    res = {}
    for graphs in (True, False):
        outs = [torch.full((3, c.height, c.width), -1.0, device="cuda") for c in cams]
        with serve.Server(scene_t, budget_bytes=2 << 30, max_slots=4, n_streams=2, graphs=graphs) as srv:
            ids = [srv.submit(c, o) for c, o in zip(cams, outs)]
            got = _drain(srv, len(ids))
            st = srv.stats()
        assert all(got[i][0] == L.QGS_REQ_DONE for i in ids)
        if graphs:
            assert st.graph_launches == 2 * len(cams)
            assert 1 <= st.graph_builds <= st.graph_launches
        else:
            assert st.graph_launches == 0
        res[graphs] = outs
    for a, b in zip(res[True], res[False]):
        assert torch.equal(a, b)


def test_admission_waits_for_list_memory(scene_t):
    cams = _views(12, 12)
    # the budget fits about one large request's lists at a time
    need = []
    for c in cams:
        _, n = _alone(scene_t, c)
        need.append(n)
    budget = int(max(need) * 16 * 1.6) + (4 << 20)
    outs = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    with serve.Server(scene_t, budget_bytes=budget, max_slots=8, n_streams=4) as srv:
        ids = [srv.submit(c, o) for c, o in zip(cams, outs)]
        got = _drain(srv, len(ids))
        st = srv.stats()
    assert all(got[i][0] == L.QGS_REQ_DONE for i in ids)
    assert st.peak_pool_bytes <= budget
    # admitted in arrival order
    admits = [got[i][4] for i in ids]
    assert all(a <= b for a, b in zip(admits, admits[1:]))
    for rid, cam, out in zip(ids, cams, outs):
        ref, _ = _alone(scene_t, cam)
        assert float((out - ref).abs().max()) <= 1e-6


def test_request_that_can_never_fit_is_refused(scene_t):
    cam = _views(1, 13)[0]
    out = torch.empty((3, cam.height, cam.width), device="cuda")
    with serve.Server(scene_t, budget_bytes=4096, max_slots=2, n_streams=1) as srv:
        rid = srv.submit(cam, out)
        got = _drain(srv, 1)
    assert got[rid][0] == L.QGS_REQ_FAILED and got[rid][1] == L.QGS_ERR_BUDGET


def test_cancel_queued_request(scene_t):
    cams = _views(10, 14)
    outs = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    with serve.Server(scene_t, budget_bytes=1 << 30, max_slots=1, n_streams=1) as srv:
        ids = [srv.submit(c, o) for c, o in zip(cams, outs)]
        assert srv.cancel(ids[-1]) == 0
        assert srv.cancel(987654321) == L.QGS_ERR_NOT_FOUND
        got = _drain(srv, len(ids))
    assert got[ids[-1]][0] == L.QGS_REQ_CANCELLED
    assert all(got[i][0] == L.QGS_REQ_DONE for i in ids[:-1])


def test_invalid_submissions(scene_t):
    with serve.Server(scene_t, budget_bytes=1 << 28, max_slots=2, max_size=(640, 480), n_streams=1) as srv:
        big = scenes.look_at((0, 0, -3), width=1280, height=720)
        out = torch.empty((3, 720, 1280), device="cuda")
        with pytest.raises(L.QgsError) as e:
            srv.submit(big, out)
        assert e.value.status == L.QGS_ERR_INVALID_ARG


def test_poisson_trace_completes(scene_t):
    trace = scenes.serve_trace(150, rate_hz=500.0, seed=15)
    with serve.Server(scene_t, budget_bytes=2 << 30, max_slots=8, n_streams=4) as srv:
        res = serve.run_trace(srv, trace, keep={0, 7, 100})
    assert np.all(res["state"] == L.QGS_REQ_DONE)
    assert np.all(res["latency"] > 0)
    for i, img in res["kept"].items():
        ref, _ = _alone(scene_t, trace[i][1])
        assert float((img - ref).abs().max()) <= 1e-6


def test_served_images_match_the_oracle(scene_t):
    # served colour against the FP64 oracle, every pixel of a 256 x 256 view
    # and crops of 1280 x 720 and 1920 x 1080 views (centre and a corner),
    # requests overlapping in the server
    sc = _scene()
    rng = np.random.default_rng(17)
    cams = []
    for (w, h) in ((256, 256), (1280, 720), (1920, 1080)):
        eye = scenes.unit_vectors(rng, 1)[0] * 3.0
        cams.append(scenes.look_at(eye, width=w, height=h, f=w))
    outs = [torch.full((3, c.height, c.width), -1.0, device="cuda") for c in cams]
    with serve.Server(scene_t, budget_bytes=2 << 30, max_slots=4, n_streams=4) as srv:
        ids = [srv.submit(c, o) for c, o in zip(cams, outs)]
        got = _drain(srv, len(ids))
    assert all(got[i][0] == L.QGS_REQ_DONE for i in ids)
    for cam, out in zip(cams, outs):
        img = out.cpu().numpy()
        if cam.width == 256:
            wins = [(0, 0, 256, 256)]
        else:
            wins = [(cam.width // 2 - 32, cam.height // 2 - 32, 64, 64), (cam.width - 48, cam.height - 40, 48, 40)]
        for win in wins:
            x0, y0, w, h = win
            g = dict(color=img[:, y0:y0 + h, x0:x0 + w])
            rep, _, _ = check_forward(g, sc, cam, win, color_only=True, label=f"served {cam.width}x{cam.height} {win}",
                                      max_excluded=0.02)
            print("served", cam.width, cam.height, win, rep)
