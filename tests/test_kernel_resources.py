"""Every kernel of the library compiles for gfx950 without private
(scratch) memory: a kernel that spills registers or indexes a private array
at run time would pay the latency of memory the register-resident design is
built to avoid, and the library refuses to launch FFT shapes that use it.
Compiles the device sources with the compiler's resource remarks."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_13628_amd", "csrc")


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_no_kernel_uses_scratch(tmp_path):
    worst = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        cmd = ["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "--offload-arch=gfx950", "--cuda-device-only", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", "-Rpass-analysis=kernel-resource-usage", "-c", src,
               "-o", str(tmp_path / "k.o")]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        name = None
        for line in r.stderr.splitlines():
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
            m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
            if m and int(m.group(1)) > 0:
                worst.append((os.path.basename(src), name, int(m.group(1))))
    assert not worst, worst
