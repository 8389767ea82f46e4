"""The rasterizers' per-block filter (conic_meets_block) against the per-pixel
conic pre-test it stands for, brute force on the host: a block may be dropped
only if every one of its 64 pixels fails the pre-test.  Both functions are the
kernels' own code (host-callable), compiled here for the host only."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("cbc") / "conic_block_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2411_16392_amd", "csrc"),
           os.path.join(ROOT, "tests", "conic_block_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def test_block_filter_never_drops_a_block_with_a_passing_pixel(checker):
    r = subprocess.run([checker, "300000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    blocks, kept_pix, kept_filter, missed, far_blocks, far_rejected = map(int, r.stdout.split()[-6:])
    assert blocks == 1_200_000
    assert missed == 0, r.stdout
    # it filters: blocks it keeps are within 10% of the blocks some pixel
    # keeps, and nearly all blocks far from the conic are dropped
    assert kept_pix > 10_000
    assert kept_filter <= 1.1 * kept_pix
    assert far_rejected >= 0.95 * far_blocks
