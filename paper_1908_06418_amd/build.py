"""Compile the HIP search library (libmcs.so) in-tree for gfx950.

The library is the product: hand-written HIP kernels plus the host driver of
the C ABI in include/mcs.h.  It is built with hipcc, always from source."""
from __future__ import annotations

import os
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmcs.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instructions stay off in every HIP build of this project, and
# so does gfx950's three-input bitwise instruction (v_bitop3): this
# compiler folded a chain of and/xor over three inputs (x ^ (x & y), then
# its and with a third row, then the xor of the two) into one v_bitop3
# with a wrong truth table (three minterms for what is a single one), which
# made the directed split drop its parts.  Without the feature the same
# code is plain v_and/v_xor/v_bfi.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Xclang", "-target-feature", "-Xclang", "-bitop3-insts"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC] + DEVICE_FLAGS

SOURCES = ["mcs_search.hip", "mcs_seg.hip", "mcs_policy.hip", "mcs_static.hip", "mcs_host.cpp"]


def build(verbose: bool = False) -> str:
    """Compile every source and link libmcs.so (atomically replaced)."""
    from concurrent.futures import ThreadPoolExecutor
    with tempfile.TemporaryDirectory(prefix="mcs_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(src)[0] + ".o") for src in SOURCES]
        cmds = [[HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(min(4, len(cmds))) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        out = os.path.join(tmp, "libmcs.so")
        # No HIP runtime is linked in: the library binds to the runtime the
        # host process already has (torch's under Python, -lamdhip64 in C),
        # so one process never holds two HIP runtimes.
        _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-no-hip-rt", "-o", out] + objs,
             verbose)
        os.replace(out, LIB + ".tmp")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}")


if __name__ == "__main__":
    print(build(verbose=True))
