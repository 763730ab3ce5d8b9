"""The device code is built without gfx950's three-input bitwise
instruction: this compiler folded a three-input and/xor chain of the
directed split into one v_bitop3 with a wrong truth table.  The flag that
keeps it out is part of every HIP build (paper_1908_06418_amd/build.py);
this test compiles the search kernels to assembly with those flags and
checks that none is left."""
import os
import shutil
import subprocess

import pytest

from paper_1908_06418_amd import build

KERNELS = ["mcs_seg.hip", "mcs_search.hip"]


@pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
@pytest.mark.parametrize("src", KERNELS)
def test_search_kernels_have_no_bitop3(tmp_path, src):
    out = tmp_path / (src + ".s")
    cmd = [build.HIPCC] + [f for f in build.COMMON if f != "-fPIC"] + [
        "--cuda-device-only", "-S", "-o", str(out), os.path.join(build.CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    text = out.read_text()
    assert "mcs_" in text  # the kernels are there
    assert "v_bitop3" not in text
