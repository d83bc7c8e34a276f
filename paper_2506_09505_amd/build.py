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
             "-Wall", "-Wno-unused-function", "-Werror=inline-asm"]


def sources():
    return [os.path.join(CSRC, "goldi.hip"), os.path.join(CSRC, "server.hip")]


def _jobs(gen_constants):
    """(output, sources, extra flags) of every library; the test-only ones go
    to _special/."""
    yield LIB, sources(), []
    # The Table-1 function library (device field operations, per-function
    # and per-opcode rates).
    yield FB_LIB, [os.path.join(CSRC, "fieldbench.hip"), os.path.join(CSRC, "rates.hip")], []
    # Test-only libraries compiled against special instances with closed forms.
    for inc in gen_constants.write_specials():
        name = os.path.basename(inc)[len("special_"):-len(".inc")]
        yield special_lib(name), sources(), ['-DGOLDI_CONSTANTS_INC="%s"' % os.path.basename(inc)]
    # Test-only: the seeded instance with the partial rounds in the sparse
    # form and in the dense form, so that both stay checked against the oracle.
    yield special_lib("sparse"), sources(), ["-DGOLDI_PARTIAL_FORM=1"]
    yield special_lib("dense"), sources(), ["-DGOLDI_PARTIAL_FORM=0"]
    # Test-only: the full-round matrix on 24-bit multipliers (22-bit limbs),
    # the alternative to the 32 x 32 -> 64-bit multiply-adds, kept checked
    # against the oracle and timed against them.
    yield special_lib("limb24"), sources(), ["-DGOLDI_MDS_LIMB24=1"]


def build(verbose: bool = False) -> str:
    """Compiles every library (hipcc runs in parallel, one process each)."""
    from . import count_valu, gen_constants, gen_field_asm
    gen_constants.main()
    gen_field_asm.main()
    os.makedirs(os.path.join(HERE, "_special"), exist_ok=True)
    running = []
    for out, srcs, extra in _jobs(gen_constants):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + extra + srcs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append((out, tmp, cmd, subprocess.Popen(cmd)))
    # The device assembly of the Table-1 functions, for their instruction counts.
    asm_tmp = count_valu.OUT + ".s%d" % os.getpid()
    asm_cmd = count_valu.asm_command(HIPCC, HIP_FLAGS, [os.path.join(ROOT, "include"), CSRC], asm_tmp)
    if verbose:
        print(" ".join(asm_cmd), flush=True)
    asm_proc = subprocess.Popen(asm_cmd)
    failed = [cmd for out, tmp, cmd, proc in running if proc.wait() != 0]
    if asm_proc.wait() != 0:
        failed.append(asm_cmd)
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    for out, tmp, cmd, proc in running:
        os.replace(tmp, out)
    count_valu.write(asm_tmp)
    os.remove(asm_tmp)
    return LIB


def special_lib(name: str) -> str:
    return os.path.join(HERE, "_special", "libgoldi_%s.so" % name)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
