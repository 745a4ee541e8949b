"""No kernel of the library spills registers or uses scratch memory: a
spill or a private array left in scratch turns register traffic into memory
traffic in the hot loops.  Compiles the device code (gfx950) with the
build's own flags and reads the compiler's resource report.  Host only."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1611_09379_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC),
                    reason="hipcc not available")
def test_no_spills_no_scratch(tmp_path):
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-c", "-o", str(tmp_path / "dev.o"),
           build.SRC, "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    kernels, cur = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        for key in ("ScratchSize [bytes/lane]", "VGPRs Spill", "SGPRs Spill"):
            m = re.search(re.escape(key) + r": (\d+)", line)
            if m and cur:
                kernels[cur][key] = int(m.group(1))
    assert len(kernels) > 50  # the report was read
    bad = {k: v for k, v in kernels.items() if any(v.get(x, 0) for x in v)}
    assert not bad, bad
