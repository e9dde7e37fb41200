"""The benchmark's command line on the CPU: it measures one GPU and says so for any other count,
and its roofline accounting adds up (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_step_bytes_are_the_sum_of_the_calls():
    from paper_2409_13055_amd import roofline as RF
    c = dict(N=1000, V=3, Pn=59, M=50_000, Nv=1200, Px=30_000, T=120, ckpt=True)
    b = RF.algorithmic_bytes(c)
    S = 3 * ((1000 + 63) // 64)
    assert b["project"] == 1000 * 4 * 59 + 3 * 1000 * 4 + 1200 * 64 + S * 4
    assert b["render_bwd"] == b["raster_bwd"] + b["project_bwd"]
    fused = ["project", "bin_sort", "render_fwd", "raster_bwd", "project_bwd_adam"]
    assert RF.step_bytes(b, fused) == sum(b[k] for k in fused)
    # the fused call moves less than the separate projection backward and Adam
    assert b["project_bwd_adam"] < b["project_bwd"] + b["adam"]
