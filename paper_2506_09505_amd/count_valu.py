"""VALU instructions per call of the Table-1 functions, counted in this
library's own gfx950 code object (a build step; ``build.py`` runs it).

``csrc/fieldbench.hip`` compiles each function into a chain kernel
``k_fb_chain<OP>`` whose only loop applies the function ``CALLS[op]`` times
per iteration (8 independent words for the one-word functions, one state for
the matrix products).  The device assembly of that file is generated with the
library's flags, each chain kernel's innermost loop is found (the block the
compiler marks as a loop header, up to the last branch back to it), and its
vector instructions are counted and divided by the calls per iteration.
Writes ``libgoldi_fieldbench_valu.json`` next to the library.
"""

from __future__ import annotations

import json
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "libgoldi_fieldbench_valu.json")
# Order of GOLDI_FB_* in include/goldi_fieldbench.h.
OPS = ("add", "sub", "reduce_128_64", "square_128", "mult_128", "mult_72", "sbox", "mmult_12x12_small",
       "mmult_12x12_full")
CALLS = (8, 8, 8, 8, 8, 8, 8, 1, 1)


def asm_command(hipcc: str, flags, include_dirs, out: str):
    cmd = [hipcc] + [f for f in flags if f not in ("-shared", "-fPIC")] + ["--cuda-device-only", "-S"]
    for d in include_dirs:
        cmd += ["-I", d]
    return cmd + [os.path.join(HERE, "csrc", "fieldbench.hip"), "-o", out]


def loop_valu(lines):
    """Vector instructions of the innermost loop of one function's assembly."""
    header = None
    for i, line in enumerate(lines):
        if "Inner Loop Header" in line:
            header = i
            label = line.split(":")[0].strip()
    if header is None:
        raise ValueError("no loop in the function")
    end = max(i for i, line in enumerate(lines) if re.search(r"s_cbranch_\w+\s+" + re.escape(label) + r"\b", line))
    return sum(1 for line in lines[header:end] if re.match(r"\s*v_\w+", line))


def counts_from_asm(text: str) -> dict:
    out = {}
    for op, name in enumerate(OPS):
        m = re.search(r"^(_Z\S*k_fb_chainILi%dEE\S*):" % op, text, re.M)
        if not m:
            raise ValueError("k_fb_chain<%d> not found" % op)
        start = m.end()
        end = text.index("s_endpgm", start)
        valu = loop_valu(text[start:end].splitlines())
        out[name] = round(valu / CALLS[op], 2)
    return out


def write(asm_path: str) -> dict:
    with open(asm_path) as f:
        counts = counts_from_asm(f.read())
    with open(OUT, "w") as f:
        json.dump({"valu_per_call": counts,
                   "source": "innermost loop of k_fb_chain<op> in the library's gfx950 assembly "
                             "(paper_2506_09505_amd/count_valu.py), per call"}, f, indent=1)
    return counts


def read() -> dict:
    with open(OUT) as f:
        return json.load(f)["valu_per_call"]


if __name__ == "__main__":
    import sys
    from . import build
    tmp = OUT + ".s"
    subprocess.check_call(asm_command(build.HIPCC, build.HIP_FLAGS, [os.path.join(build.ROOT, "include"), build.CSRC], tmp))
    print(write(tmp))
    os.remove(tmp)
    sys.exit(0)
