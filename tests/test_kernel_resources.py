"""Build-time checks of the HIP kernels (no GPU needed): the hot kernels use no scratch
(private) memory.  A kernel whose LDS pointer table is demoted to scratch turns every
LDS access into a flat access and runs about 40% slower, with identical results, so
only this check catches it."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_02036_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src", ["k_linearize.hip", "k_update.hip", "k_cost.hip", "k_solve.hip", "k_init.hip"])
def test_hot_kernels_use_no_scratch(src, tmp_path):
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-c",
           os.path.join(CSRC, src), "-o", str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stderr)]
    assert names and len(names) == len(scratch)
    bad = [(n, s) for n, s in zip(names, scratch) if s != 0]
    assert not bad, f"kernels with scratch memory: {bad}"
