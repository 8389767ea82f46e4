"""CPU checks of the boundary: the library loads and exports every entry point
the header declares; host-only calls behave as documented."""
import re
import os

import pytest

from paper_2411_16392_amd import _lib as L
from paper_2411_16392_amd import render as R
from paper_2411_16392_amd import scenes

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qgs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qgs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("qgs_preprocess", "qgs_bin_sort", "qgs_render_fwd", "qgs_render_bwd"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(L.exported_symbols())


def test_binding_mirrors_every_header_constant():
    src = open(HEADER).read()
    consts = re.findall(r"#define\s+(QGS_[A-Z0-9_]+)\s+(-?\d+)u?\b", src)
    assert len(consts) >= 8
    for name, val in consts:
        assert hasattr(L, name), name
        assert getattr(L, name) == int(val), name


def test_status_strings_and_defaults():
    lib = L.lib()
    assert lib.qgs_status_string(L.QGS_ERR_CAPACITY) == b"tile list capacity exceeded"
    assert lib.qgs_status_string(12345) == b"unknown status"
    o = L.qgs_default_opts()
    assert o.tile == 16 and abs(o.near_plane - 0.2) < 1e-7 and abs(o.k_sigma - 3) < 1e-7
    assert abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.alpha_max - 0.99) < 1e-7
    assert abs(o.T_eps - 1e-4) < 1e-10 and abs(o.A_eps - 1e-6) < 1e-12


def test_workspace_query_host_only():
    cam = R.make_camera(scenes.look_at((0, 0, -3), width=1600, height=1200, f=1600))
    s0, b0 = L.qgs_workspace_query(500_000, cam, 10_000_000, 0)
    s1, b1 = L.qgs_workspace_query(500_000, cam, 20_000_000, L.QGS_DETERMINISTIC_BWD)
    assert s1 > s0 and b1 >= b0 + 20_000_000 * 64
    with pytest.raises(L.QgsError) as e:
        L.qgs_workspace_query(-1, cam, 10, 0)
    assert e.value.status == L.QGS_ERR_INVALID_ARG
    bad = R.make_camera(scenes.look_at((0, 0, -3), width=16, height=16, f=16))
    bad.width = 0
    with pytest.raises(L.QgsError):
        L.qgs_workspace_query(10, bad, 10, 0)


def test_invalid_arguments_rejected_before_launch():
    # null scene pointers with n > 0: rejected on the host, nothing launched
    cam = R.make_camera(scenes.look_at((0, 0, -3), width=16, height=16, f=16))
    sc = L.QgsScene()
    sc.n = 10
    pb = L.QgsPrimBuf()
    pb.n = 10
    with pytest.raises(L.QgsError) as e:
        L.qgs_preprocess(sc, cam, L.qgs_default_opts(), pb)
    assert e.value.status == L.QGS_ERR_INVALID_ARG
    o = L.qgs_default_opts()
    o.tile = 32
    sc.n = 0
    pb.n = 0
    with pytest.raises(L.QgsError):
        L.qgs_preprocess(sc, cam, o, pb)


def test_replay_bitmap_arguments_both_or_neither():
    # placeholder addresses that are never dereferenced: the call must fail
    # validation on the host before anything is launched
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check with placeholder pointers")
    cam = R.make_camera(scenes.look_at((0, 0, -3), width=16, height=16, f=16))
    pb = L.QgsPrimBuf()
    pb.n = 1
    pb.records = pb.depth_key = pb.rect = pb.tiles = pb.pair_offset = pb.conic = 0x1000
    lists = L.QgsTileLists()
    lists.pair_tile = lists.pair_prim = lists.ranges = lists.counters = lists.tile_order = 0x1000
    lists.capacity = 16
    im = L.QgsImages()
    im.color = im.depth = im.normal = im.T_final = im.last = 0x1000
    im.steps = 0x1000  # without step_count
    with pytest.raises(L.QgsError) as e:
        L.qgs_render_fwd(pb, lists, cam, L.qgs_default_opts(), im)
    assert e.value.status == L.QGS_ERR_INVALID_ARG
    sc = L.QgsScene()
    sc.n = 0
    dl = L.QgsImageGrads()
    g = L.QgsSceneGrads()
    pb.n = 0
    with pytest.raises(L.QgsError) as e:
        L.qgs_render_bwd(sc, pb, lists, cam, L.qgs_default_opts(), im, dl, g, 0x1000, 1 << 20)
    assert e.value.status == L.QGS_ERR_INVALID_ARG


def test_binding_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of the header's structs, as compiled by the
    C compiler, against the ctypes mirrors of the binding."""
    import ctypes
    import subprocess
    structs = {"qgs_scene": L.QgsScene, "qgs_camera": L.QgsCamera, "qgs_render_opts": L.QgsRenderOpts,
               "qgs_prim_buf": L.QgsPrimBuf, "qgs_tile_lists": L.QgsTileLists, "qgs_images": L.QgsImages,
               "qgs_image_grads": L.QgsImageGrads, "qgs_scene_grads": L.QgsSceneGrads,
               "qgs_serve_config": L.QgsServeConfig, "qgs_completion": L.QgsCompletion,
               "qgs_serve_stats": L.QgsServeStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qgs.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_library_stamp_matches_its_sources():
    # the binding loaded the library, so its stamp is the hash of the sources
    from paper_2411_16392_amd import build as B
    lib = L.lib()
    assert L.verify_build(lib) == B.source_hash()
    assert len(B.source_hash()) == 64


def test_stale_library_is_refused():
    # a library stamped from other sources is refused with a clear message
    lib = L.lib()
    with pytest.raises(RuntimeError, match="built from other sources"):
        L.verify_build(lib, expected="0" * 64)


def test_source_hash_follows_every_source(tmp_path, monkeypatch):
    # changing any stamped file changes the hash
    from paper_2411_16392_amd import build as B
    files = B.stamped_files()
    assert any(f.endswith("qgs.h") for f in files) and any(f.endswith(".hip") for f in files)
    copies = []
    for f in files:
        dst = tmp_path / os.path.basename(f)
        dst.write_bytes(open(f, "rb").read())
        copies.append(str(dst))
    monkeypatch.setattr(B, "stamped_files", lambda: copies)
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    h0 = B.source_hash()
    with open(copies[0], "ab") as fh:
        fh.write(b"\n// edit\n")
    assert B.source_hash() != h0


def test_device_code_has_no_packed_fp32_arithmetic():
    from paper_2411_16392_amd import build as B
    assert B.check_no_packed_fp32(L.LIB_PATH) > 10_000
