"""Host logic of the serving scheduler, on the CPU: the first-fit pool that
reserves each request's tile-list memory (no overlap, refusal only when no
free range fits, full coalescing, exact accounting)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_allocator(tmp_path):
    exe = tmp_path / "pool_check"
    src = os.path.join(ROOT, "tests", "serve_pool_check.cpp")
    inc = os.path.join(ROOT, "paper_2411_16392_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined", "-I", inc, src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True)
    assert "pool ok" in out.stdout
