"""Every device kernel of the library compiles for gfx950 without scratch
memory (register spills or dynamically indexed private arrays): a kernel that
spills turns its register traffic into memory traffic and runs several times
slower, with no change in its results.  The resource report of the compiler
is read for each source file (device code only, no link)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2602_07853_amd import _build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# kernels allowed to use scratch: the dense export of the stored tangent
# (called by tests and field exports only, never inside a step)
ALLOWED = ("k_export_abar",)


def resource_report(src, tmp_path):
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared",)]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-c", "-I", os.path.join(_build.HERE, "..", "include"),
           "-Rpass-analysis=kernel-resource-usage", "-o", str(tmp_path / "k.o"), src]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True)
    kernels, name = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            kernels[name] = int(m.group(1))
    return kernels


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not found")
@pytest.mark.parametrize("src", _build.sources(), ids=os.path.basename)
def test_no_kernel_uses_scratch(src, tmp_path):
    kernels = resource_report(src, tmp_path)
    if "__global__" not in open(src).read():
        assert not kernels
        return
    assert kernels, "no kernel resource report"
    spills = {k: v for k, v in kernels.items() if v > 0 and not any(a in k for a in ALLOWED)}
    assert not spills, f"kernels with scratch (bytes/lane): {spills}"
