"""The generated gfx950 code writes memory through vector stores only.

Compiles the kernels to AMDGPU assembly (CPU-only, needs hipcc) and checks that
no scalar-memory store, scalar atomic or scalar-cache write-back/discard
instruction appears.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FORBIDDEN = re.compile(r"^\s+s_(store|scratch_store|buffer_store|atomic|buffer_atomic|dcache_wb|dcache_discard)",
                       re.M)


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src,kernel", [("kernels.hip", "k_tile_pass_r"), ("adjoint.hip", "k_backward_r")])
def test_kernels_use_no_scalar_memory_writes(tmp_path, src, kernel):
    out = tmp_path / "k.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2604_11599_amd", "csrc"), "--cuda-device-only", "-S",
           os.path.join(ROOT, "paper_2604_11599_amd", "csrc", src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text()
    assert kernel in text
    assert not FORBIDDEN.findall(text)
