"""Writes ``csrc/field_asm.inc``: Goldilocks products as single inline-assembly
blocks that interleave one, two or three independent products.

Why: the compiler cannot see inside inline assembly, so after each asm
statement it pads conservatively with wait states (``s_nop``), and a VALU
instruction that writes a carry into an SGPR pair needs two wait states before
a VALU instruction reads it (gfx950).  One block per group of products lets
the products fill each other's wait states: with three products interleaved
every carry is read at least two instructions after it was written, so no
wait state is spent at all; with two or one, the generator inserts exactly the
``s_nop`` the hazard needs.

Each product is the one of ``field.hpp`` (Sec. 3.1, Eqs. 2-3: 2^64 = 2^32 - 1
mod p), its borrow fix-up riding in the final fold as a signed correction:

    p00 = a0 b0;  t = a1 b0 + hi(p00);  u + c 2^64 = a0 b1 + t;
    h = a1 b1 + hi(u);  y = r_l - hi(h) - c (borrow b);
    r1 + k 2^64 = lo(h) (2^32 - 1) + y;  d = k - b;  r = r1 + d 2^32 - d

The intermediate pairs live in fixed scratch VGPRs (the block must address
the halves of 64-bit values it computes itself, which operands cannot), which
the asm statement declares clobbered.  ``STEPS`` below is the single source
of the instruction sequence: the header is printed from it, and the CPU test
(tests/test_field_asm.py) replays it with exact integers, checks every hazard
distance and that only declared registers are touched.

Run: python -m paper_2506_09505_amd.gen_field_asm  (build.py runs it).
"""

from __future__ import annotations

import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "csrc", "field_asm.inc")

# First scratch VGPR: the kernels are compiled for at least four waves per
# SIMD (128 VGPRs each); the scratch takes the top of that budget.
VBASE = 110
MAX_WAYS = 3
# Blocks written into the header: three products serve the four-lanes-per-
# state layout (no wait state at all), one and two the one-word-per-lane
# layout, whose lone waves pay for every wait state.  (The one-lane layout
# keeps the statement-level product of field.hpp: its other waves hide the
# wait states, and the compiler interleaves the pieces with other work.)
HEADER_WAYS = (1, 2, 3)
REGS_PER_PRODUCT = 6

# One product as a list of instructions over symbolic registers:
#   P, Z, U   scratch pairs (P.lo/P.hi, ... their halves)
#   S, T      the product's SGPR pairs (carries and borrows)
#   AL AH BL BH   the 32-bit halves of the operands
#   R         the output pair
# Each step: (opcode, destination, carry destination, sources...).  Carry
# destination "vcc" means the carry is not used.  A last source "S" or "T"
# of a carry reader is a hazard read of that SGPR pair.
STEPS = [
    ("v_mad_u64_u32", "P", "vcc", "AL", "BL", "0"),        # p00 = a0 b0
    ("v_mov_b32", "Z.lo", None, "P.hi"),                    # Z = (hi(p00), 0)
    ("v_mov_b32", "Z.hi", None, "0"),
    ("v_mad_u64_u32", "U", "vcc", "AH", "BL", "Z"),        # t = a1 b0 + hi(p00)
    ("v_mad_u64_u32", "U", "S", "AL", "BH", "U"),          # u + c 2^64 = a0 b1 + t
    ("v_mov_b32", "Z.lo", None, "U.hi"),                    # Z = (hi(u), 0)
    ("v_mad_u64_u32", "Z", "vcc", "AH", "BH", "Z"),        # h = a1 b1 + hi(u)
    ("v_subb_co_u32", "P.lo", "S", "P.lo", "Z.hi", "S"),   # y0 = lo(p00) - hi(h) - c
    ("v_subb_co_u32", "P.hi", "S", "U.lo", "0", "S"),      # y1 = lo(u) - borrow; S = b
    ("v_mad_u64_u32", "U", "T", "Z.lo", "-1", "P"),        # r1 + k 2^64 = lo(h) (2^32 - 1) + y
    ("v_addc_co_u32", "Z.lo", "vcc", "0", "0", "T"),       # k
    ("v_subb_co_u32", "Z.lo", "vcc", "Z.lo", "0", "S"),    # d = k - b, in {-1, 0, 1}
    ("v_add_u32", "U.hi", None, "U.hi", "Z.lo"),            # r1 + d 2^32
    ("v_mad_i64_i32", "R", "vcc", "Z.lo", "-1", "U"),      # - d (signed)
]

# Instructions that read an SGPR pair (S or T) as a carry or borrow input.
CARRY_READERS = ("v_subb_co_u32", "v_addc_co_u32")
HAZARD_WAIT = 2   # wait states between a VALU write of an SGPR and a VALU read of it


def scratch(k: int, reg: str) -> str:
    """Physical register text of scratch `reg` ("P", "Z.lo", ...) of product k."""
    base = {"P": 0, "Z": 2, "U": 4}[reg[0]]
    v = VBASE + REGS_PER_PRODUCT * k + base
    if reg.endswith(".lo"):
        return "v%d" % v
    if reg.endswith(".hi"):
        return "v%d" % (v + 1)
    return "v[%d:%d]" % (v, v + 1)


def operand(k: int, name: str, square: bool) -> str:
    if name in ("P", "Z", "U") or name[:2] in ("P.", "Z.", "U."):
        return scratch(k, name)
    if name in ("S", "T"):
        return "%%[%s%d]" % (name.lower(), k)
    if name == "R":
        return "%%[r%d]" % k
    if name in ("AL", "AH"):
        return "%%[a%d%s]" % (k, "l" if name == "AL" else "h")
    if name in ("BL", "BH"):
        src = "a" if square else "b"
        return "%%[%s%d%s]" % (src, k, "l" if name == "BL" else "h")
    return name  # "0", "-1", "vcc"


def schedule(ways: int):
    """The interleaved instruction list for `ways` products, with the wait
    states each carry read needs: entries ("insn", k, step) and ("nop", n)
    (n wait states, printed as s_nop n-1)."""
    out = []
    pos = 0            # wait-state clock: an instruction is 1, "s_nop n-1" is n
    last_write = {}    # (product, pair) -> clock right after its last write
    for step in STEPS:
        for k in range(ways):
            src = step[-1]
            if step[0] in CARRY_READERS and src in ("S", "T") and (k, src) in last_write:
                have = pos - last_write[(k, src)]
                if have < HAZARD_WAIT:
                    out.append(("nop", HAZARD_WAIT - have))
                    pos += HAZARD_WAIT - have
            out.append(("insn", k, step))
            pos += 1
            if step[2] in ("S", "T"):
                last_write[(k, step[2])] = pos
    return out


def render(ways: int, square: bool) -> list:
    """Assembly text lines of one block."""
    lines = []
    for e in schedule(ways):
        if e[0] == "nop":
            lines.append("s_nop %d" % (e[1] - 1))
            continue
        k, step = e[1], e[2]
        op, dst, cdst = step[0], step[1], step[2]
        srcs = [operand(k, x, square) for x in step[3:]]
        d = operand(k, dst, square)
        if cdst is None:
            lines.append("%s %s, %s" % (op, d, ", ".join(srcs)))
        else:
            lines.append("%s %s, %s, %s" % (op, d, operand(k, cdst, square), ", ".join(srcs)))
    return lines


def clobbers(ways: int):
    regs = ['"v%d"' % (VBASE + i) for i in range(REGS_PER_PRODUCT * ways)]
    return ", ".join(regs + ['"vcc"'])


def function_text(ways: int, square: bool) -> str:
    name = "%s%d_asm" % ("sqr" if square else "mul", ways)
    pairs = ("s", "t")
    params = []
    for k in range(ways):
        params.append("u64 a%d" % k)
        if not square:
            params.append("u64 b%d" % k)
    params += ["u64 &r%d" % k for k in range(ways)]
    body = ["    u64 " + ", ".join("%s%d" % (x, k) for x in pairs for k in range(ways)) + ";"]
    lines = render(ways, square)
    asm = ["    asm volatile("]
    asm += ['        "%s\\n\\t"' % line for line in lines[:-1]]
    asm.append('        "%s"' % lines[-1])
    outs = ['[r%d] "=v"(r%d)' % (k, k) for k in range(ways)]
    outs += ['[%s%d] "=&s"(%s%d)' % (x, k, x, k) for x in pairs for k in range(ways)]
    ins = []
    for k in range(ways):
        ins += ['[a%dl] "v"(lo32(a%d))' % (k, k), '[a%dh] "v"(hi32(a%d))' % (k, k)]
        if not square:
            ins += ['[b%dl] "v"(lo32(b%d))' % (k, k), '[b%dh] "v"(hi32(b%d))' % (k, k)]
    asm.append("        : " + ", ".join(outs))
    asm.append("        : " + ", ".join(ins))
    asm.append("        : " + clobbers(ways) + ");")
    doc = "// %s: %s of %d independent pair%s, weak results (any 64-bit inputs).\n" % (
        name, "squares" if square else "products", ways, "s" if ways > 1 else "")
    return doc + "__device__ __forceinline__ void %s(%s) {\n%s\n}\n" % (name, ", ".join(params), "\n".join(body + asm))


HEADER = """// Generated by paper_2506_09505_amd/gen_field_asm.py -- do not edit.
//
// Goldilocks products as single inline-assembly blocks interleaving one, two
// or three independent products (see the generator for the sequences and
// why).
// Scratch VGPRs v%d..v%d are declared clobbered.
#pragma once

namespace goldi {

""" % (VBASE, VBASE + REGS_PER_PRODUCT * MAX_WAYS - 1)


def text() -> str:
    parts = [HEADER]
    for ways in HEADER_WAYS:
        for square in (False, True):
            parts.append(function_text(ways, square))
            parts.append("\n")
    parts.append("}  // namespace goldi\n")
    return "".join(parts)


def main(check: bool = False) -> str:
    t = text()
    if check:
        with open(OUT) as f:
            if f.read() != t:
                raise SystemExit("%s is stale: run python -m paper_2506_09505_amd.gen_field_asm" % OUT)
        return OUT
    with open(OUT, "w") as f:
        f.write(t)
    return OUT


if __name__ == "__main__":
    print(main())
