"""Host logic of the block-step plans (no GPU): the split partials a block
step of any size writes fit in the rows the integrator allocates, for both
precisions, with the launch constants the library is built with.  The check
is a small host program compiled against the library's internal header."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0707_0438_amd", "csrc")


@pytest.mark.timeout(300)
def test_block_plans_fit_the_partials(tmp_path):
    from paper_0707_0438_amd import build
    exe = str(tmp_path / "plan_bound")
    cmd = [build.hipcc(), "-O2", "-std=c++17", "-x", "hip", f"--offload-arch={build.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "plan_bound.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
