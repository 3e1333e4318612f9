"""The step kernel's compiled resources (CPU: a compile with the
compiler's resource remarks): no private (scratch) memory, which an
out-of-line call taking a pointer to a local array would need, at most 128
VGPRs and 4 wavefronts per SIMD, no VGPR spills, for every instantiation.
A launch of this kernel is short enough that a stack or spills show up in
every PCG iteration."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_kernel_uses_no_scratch_and_fits_four_waves(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    from paper_1309_5796_amd import build as B
    cmd = [hipcc if os.path.exists(hipcc) else "hipcc", *B.FLAGS, "-c",
           os.path.join(B.CSRC, "kernels.hip"), "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    blocks = re.split(r"remark: Function Name: ", r.stderr)[1:]
    steps = [b for b in blocks if b.startswith("_ZN4mmsd12_GLOBAL__N_16k_step")]
    assert len(steps) == 6, len(steps)   # double and float, 4, 8 and 16 lanes per magnet row
    for b in steps:
        name = b.split()[0]
        field = lambda key: int(re.search(key + r": (\d+)", b).group(1))
        assert field(r"ScratchSize \[bytes/lane\]") == 0, name
        assert field(r"VGPRs Spill") == 0, name
        assert field(r"VGPRs") <= 128, name
        assert field(r"Occupancy \[waves/SIMD\]") >= 4, name
