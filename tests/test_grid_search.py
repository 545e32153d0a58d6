"""Host build of the window plan's grid search (a device function) checked
against std::lower_bound / std::upper_bound on uniform, jittered and ragged
grids (no GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2501_09308_amd", "csrc")
BUILD = os.path.join(HERE, "_build")


def test_grid_search_equals_std_bounds():
    exe = os.path.join(BUILD, "grid_search_test")
    os.makedirs(BUILD, exist_ok=True)
    subprocess.check_call(
        ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC,
         os.path.join(HERE, "native", "grid_search_test.cpp"), "-o", exe],
        stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert "0 mismatches" in out.stdout
