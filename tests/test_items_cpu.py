"""The work-item planner of the X-stage kernels (host logic, no GPU): every
block of the lower triangle of every channel is computed exactly once, for
every path, tile, table, row-block count (1..24) and channel count (1..5).
The check is a small host program built from the planner's own source."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_8288_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "items_coverage")


def test_planner_covers_every_block_once():
    from paper_1401_8288_amd import build
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    # host code only; the HIP headers come with hipcc
    cmd = [build.hipcc(), "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "items_coverage.cpp"), os.path.join(CSRC, "xcorr_items.cpp"),
           "-o", OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([OUT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
