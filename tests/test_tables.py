"""Host check of the complex64 step tables (no GPU): tests/table_check.cpp compiles the
library's own schedule.cpp with g++ and checks, for long runs of small steps (the paper's
scans) and for the benchmark's steps, that pieced and whole rounding agree, that the phase
rows undo the link layers' norm gains to 5e-7 over 2 x 10^5 rows, that every row is of unit
magnitude or a gathered correction, and that the phase angles are kept."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")


def test_complex64_tables(tmp_path):
    exe = tmp_path / "table_check"
    csrc = os.path.join(ROOT, "paper_1910_08020_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", ROCM_INCLUDE, "-I", csrc, os.path.join(ROOT, "tests", "table_check.cpp"),
                    os.path.join(csrc, "schedule.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    lines = r.stdout.strip().splitlines()
    assert r.returncode == 0, r.stdout
    assert lines[-1] == "failures: 0"
    assert sum(1 for ln in lines if ln.endswith(": ok")) == 6
