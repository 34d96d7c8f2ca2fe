"""Resource checks of the gfx950 code objects, on the CPU (hipcc cross-compiles).

The step kernels must not use scratch memory (a private segment turns
register arrays into global-memory traffic and limits how many waves can be
resident), must not spill VGPRs, and must fit their LDS in one CU (160 KB).
A fused block runs an emulator and a writer wave on every SIMD, so the fused
kernels may use at most 256 of the SIMD's 512 registers per lane (VGPRs and
AGPRs together).
A fused block of IPW envs may use at most IPW/256 of the CU's LDS, so that
256 envs per CU (65,536 envs on 256 CUs) are resident at once at every block
size; a few hundred bytes over the line cost a whole second round of blocks.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01764_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _kernels(src):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
               "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
        subprocess.run(cmd, check=True, capture_output=True)
        text = open(out).read()
    meta = text[text.index("amdhsa.kernels:"):]
    kernels = []
    for block in re.split(r"\n  - ", meta)[1:]:
        fields = dict(re.findall(r"\.(\w+):\s+(\S+)", block))
        if "name" in fields:
            kernels.append(fields)
    return kernels


@pytest.mark.parametrize("src", ["step_fused.hip", "step_plain.hip", "step_schip.hip", "reset.hip", "calib.hip"])
def test_no_scratch_no_spills_lds_fits(src):
    ks = _kernels(src)
    assert ks, src
    for k in ks:
        assert int(k["private_segment_fixed_size"]) == 0, (k["name"], "uses scratch")
        assert int(k.get("vgpr_spill_count", 0)) == 0, (k["name"], "spills VGPRs")
        assert int(k["group_segment_fixed_size"]) <= 160 * 1024, (k["name"], "LDS above 160 KB")


def test_fused_blocks_keep_256_envs_per_cu_resident():
    for k in _kernels("step_fused.hip"):
        ipw = int(re.search(r"kernelILi(\d+)E", k["name"]).group(1))
        assert int(k["group_segment_fixed_size"]) <= 160 * 1024 * ipw // 256, (k["name"], k["group_segment_fixed_size"])
        assert int(k["vgpr_count"]) <= 256, (k["name"], "two waves per SIMD need at most 256 registers", k["vgpr_count"])
