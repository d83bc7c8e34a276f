"""Builds the gfx950 HIP library ``libgoldi.so`` in-tree with hipcc.

``python -m paper_2506_09505_amd.build`` regenerates the constant tables
from the seeded instance and compiles ``csrc/goldi.hip`` for gfx950 only.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgoldi.so")
FB_LIB = os.path.join(HERE, "libgoldi_fieldbench.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code (they are not
# used by this integer code, and some of their forms are unreliable).
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def sources():
    return [os.path.join(CSRC, "goldi.hip"), os.path.join(CSRC, "server.hip")]


def build(verbose: bool = False) -> str:
    from . import gen_constants
    gen_constants.main()
    os.makedirs(os.path.join(HERE, "_special"), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # The Table-1 function library (device field operations, rates).
    tmp = FB_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                 os.path.join(CSRC, "fieldbench.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, FB_LIB)
    # Test-only libraries compiled against special instances with closed forms.
    for inc in gen_constants.write_specials():
        name = os.path.basename(inc)[len("special_"):-len(".inc")]
        out = special_lib(name)
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                     '-DGOLDI_CONSTANTS_INC="%s"' % os.path.basename(inc)] + sources() + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return LIB


def special_lib(name: str) -> str:
    return os.path.join(HERE, "_special", "libgoldi_%s.so" % name)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
