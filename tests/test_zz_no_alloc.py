"""The backward without a caller workspace (qgs_render_bwd_static) against
qgs_render_bwd through the C ABI: same gradients on two calls in a row, the
second on a smaller scene and view, so the static workspace holds the first
call's contents when the second starts."""
import numpy as np
import pytest
import torch

from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def _grads_both_ways(scene, cam, flags, seed):
    # a small starting capacity: the lists grow to 1.25 x the pair count, so
    # the deterministic mode's pair partials stay within the static workspace
    r = R.Renderer(opts=R.make_opts(flags=flags), capacity=1024)
    sc_t = R.scene_to_device(scene)
    st = r.forward(sc_t, cam)
    dL = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
          for a in scenes.upstream_grads(seed, cam.height, cam.width)]
    ref = {k: v.clone() for k, v in r.backward(sc_t, st, *dL).items()}
    out = {k: torch.full_like(sc_t[k], float("nan")) for k in R.SCENE_KEYS}
    g = L.QgsSceneGrads()
    for k in R.SCENE_KEYS:
        setattr(g, k, out[k].data_ptr())
    dl = L.QgsImageGrads()
    dl.dcolor, dl.ddepth, dl.dnormal = (t.data_ptr() for t in dL)
    opts = L.QgsRenderOpts.from_buffer_copy(r.opts)
    L.qgs_render_bwd_static(R._scene_struct(sc_t), st.prim_buf(), st.lists(), st.cam, opts, st.images(), dl, g,
                            R._stream())
    torch.cuda.synchronize()
    return {k: ref[k].cpu().numpy() for k in R.SCENE_KEYS}, {k: out[k].cpu().numpy() for k in R.SCENE_KEYS}


@pytest.mark.parametrize("flags", [L.QGS_DETERMINISTIC_BWD, 0])
def test_static_workspace_backward_matches(flags):
    if flags & L.QGS_DETERMINISTIC_BWD:
        # the pair partials take 256 bytes per pair: scenes of ~100K pairs
        first = (scenes.scene_uniform_cube(20_000, 10), scenes.look_at((0.0, 0.0, -3.0), width=400, height=300,
                                                                      f=400))
    else:
        c1 = scenes.make_config(1)
        first = (c1.scene, c1.cameras[0])
    second = (scenes.scene_uniform_cube(1500, 11), scenes.look_at((0.2, 0.1, -3.0), width=200, height=136, f=200))
    for (scene, cam), seed in ((first, 21), (second, 22)):
        ref, got = _grads_both_ways(scene, cam, flags, seed)
        for k in R.SCENE_KEYS:
            assert np.all(np.isfinite(got[k])), k
            if flags & L.QGS_DETERMINISTIC_BWD:
                # same kernels, same fixed summation order: bit-identical
                assert np.array_equal(got[k], ref[k]), k
            else:
                # atomic accumulation in arrival order: equal to rounding
                scale = np.abs(ref[k]).max() + 1e-30
                assert np.max(np.abs(got[k] - ref[k])) <= 1e-5 * scale, k


def test_static_workspace_rejects_oversized_calls():
    # 2M primitives need 128 MB of record gradients, beyond the static 64 MiB
    n = 2_000_000
    cam = R.make_camera(scenes.look_at((0, 0, -3), width=64, height=64, f=64))
    _, need = L.qgs_workspace_query(n, cam, 0, 0)
    assert need > L.QGS_BWD_STATIC_BYTES
    sc = scenes.scene_uniform_cube(n, 2)
    sc_t = R.scene_to_device(sc)
    r = R.Renderer()
    st = r.preprocess(sc_t, scenes.look_at((0, 0, -3), width=64, height=64, f=64))
    r._alloc_lists(st, 0)
    g = L.QgsSceneGrads()
    out = {k: torch.empty_like(sc_t[k]) for k in R.SCENE_KEYS}
    for k in R.SCENE_KEYS:
        setattr(g, k, out[k].data_ptr())
    dl = L.QgsImageGrads()
    with pytest.raises(L.QgsError) as e:
        L.qgs_render_bwd_static(R._scene_struct(sc_t), st.prim_buf(), st.lists(), st.cam, r.opts, st.images(), dl,
                                g, R._stream())
    assert e.value.status == L.QGS_ERR_WORKSPACE
