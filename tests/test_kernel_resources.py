"""The attempt kernels compile without scratch memory and within the register
budget of eight waves per SIMD (compiler resource remarks, no GPU)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2512_06715_amd import build as hipbuild


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
def test_attempt_kernels_spill_nothing(tmp_path):
    src = os.path.join(hipbuild.CSRC, "attempt.hip")
    cmd = [hipbuild._hipcc(), *hipbuild.HIPCC_FLAGS, "-c", src, "-o", str(tmp_path / "a.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)",
                      line)
        if m and name:
            kernels[name][m.group(1).split()[0]] = int(m.group(2))
    main = {k: v for k, v in kernels.items() if re.search(r"k_(primal|dual)I[df]Lb", k)}
    # 2 kernels x (FP32; FP64 on FP64 or FP32 values) x 16-bit/32-bit x 2 load policies
    assert len(main) == 24, sorted(kernels)
    for k, v in main.items():
        assert v["ScratchSize"] == 0, (k, v)
        assert v["VGPRs"] <= 64 and v["Occupancy"] == 8, (k, v)
