"""Host check of the tile-pass register and LDS layouts for every instantiated geometry
(no GPU): the check program compiles tile_layout.hpp, the header the kernels use, with g++."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_tile_geometry(tmp_path):
    exe = tmp_path / "layout_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1910_08020_amd", "csrc"),
                    os.path.join(ROOT, "tests", "layout_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    lines = r.stdout.strip().splitlines()
    assert r.returncode == 0, r.stdout
    assert lines[-1] == "failures: 0"
    assert sum(1 for ln in lines if ln.endswith(": ok")) == 29
