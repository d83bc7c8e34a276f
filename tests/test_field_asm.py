"""CPU checks of the generated product blocks (csrc/field_asm.inc, written by
paper_2506_09505_amd/gen_field_asm.py).  The block text is executed here by a small interpreter of its six opcodes with exact
integers, one lane at a time: every result must be congruent to the product
mod p (Sec. 3.1, Eqs. 2-3), every carry must be read at least two wait states
after the VALU instruction that wrote it, and the block may write only its
outputs, its SGPR temporaries, VCC and the scratch VGPRs it declares
clobbered."""

import random
import re

import pytest

from paper_2506_09505_amd import gen_field_asm as gen

P = 2**64 - 2**32 + 1
M32, M64 = 2**32 - 1, 2**64 - 1


class Lane:
    """One lane of the interpreted block: named 32-bit registers, carry bits
    of SGPR pairs, and a wait-state clock."""

    def __init__(self, inputs):
        self.v = dict(inputs)          # register name -> 32-bit value
        self.s = {}                    # SGPR pair / vcc -> carry bit
        self.s_written = {}            # pair -> clock after the write
        self.clock = 0
        self.written = set()

    def halves(self, text):
        m = re.fullmatch(r"v\[(\d+):(\d+)\]", text)
        if m:
            lo, hi = int(m.group(1)), int(m.group(2))
            assert hi == lo + 1 and lo % 2 == 0, "unaligned pair " + text
            return "v%d" % lo, "v%d" % hi
        m = re.fullmatch(r"%\[(r\d+)\]", text)
        if m:
            return m.group(1) + ".lo", m.group(1) + ".hi"
        raise AssertionError("not a pair: " + text)

    def read32(self, text):
        if text in ("0", "-1"):
            return int(text) & M32
        m = re.fullmatch(r"%\[(\w+)\]", text)
        name = m.group(1) if m else text
        return self.v[name]

    def read64(self, text):
        if text == "0":
            return 0
        lo, hi = self.halves(text)
        return self.v[lo] | (self.v[hi] << 32)

    def write32(self, text, value):
        m = re.fullmatch(r"%\[(\w+)\]", text)
        name = m.group(1) if m else text
        self.v[name] = value & M32
        self.written.add(name)

    def write64(self, text, value):
        lo, hi = self.halves(text)
        self.v[lo], self.v[hi] = value & M32, (value >> 32) & M32
        self.written.update((lo, hi))

    def sgpr(self, text):
        m = re.fullmatch(r"%\[([st]\d+)\]", text)
        assert m or text == "vcc", text
        return m.group(1) if m else "vcc"

    def write_carry(self, text, bit):
        name = self.sgpr(text)
        self.s[name] = bit
        self.s_written[name] = self.clock

    def read_carry(self, text):
        name = self.sgpr(text)
        assert name != "vcc", "a block never reads VCC"
        assert self.clock - self.s_written[name] >= gen.HAZARD_WAIT, "carry read too early"
        return self.s[name]

    def run(self, lines):
        for line in lines:
            op, _, rest = line.partition(" ")
            args = [a.strip() for a in rest.split(",")]
            if op == "s_nop":
                self.clock += int(args[0]) + 1
                continue
            self.clock += 1
            if op == "v_mad_u64_u32":
                d, sd, a, b, c = args
                val = self.read32(a) * self.read32(b) + self.read64(c)
                self.write64(d, val)
                self.write_carry(sd, val >> 64)
            elif op == "v_mad_i64_i32":
                d, sd, a, b, c = args
                def s32(x):
                    return x - (1 << 32) if x >> 31 else x
                cv = self.read64(c)
                cv = cv - (1 << 64) if cv >> 63 else cv
                self.write64(d, s32(self.read32(a)) * s32(self.read32(b)) + cv)
                self.write_carry(sd, 0)
            elif op == "v_add_u32":
                d, a, b = args
                self.write32(d, self.read32(a) + self.read32(b))
            elif op == "v_mov_b32":
                d, a = args
                self.write32(d, self.read32(a))
            elif op in ("v_subb_co_u32", "v_addc_co_u32"):
                d, sd, a, b, cin = args
                ci = self.read_carry(cin)
                if op == "v_subb_co_u32":
                    val = self.read32(a) - self.read32(b) - ci
                    self.write32(d, val)
                    self.write_carry(sd, 1 if val < 0 else 0)
                else:
                    val = self.read32(a) + self.read32(b) + ci
                    self.write32(d, val)
                    self.write_carry(sd, val >> 32)
            else:
                raise AssertionError("unexpected opcode " + op)


def run_block(ways, square, pairs):
    inputs = {}
    for k, (a, b) in enumerate(pairs):
        inputs["a%dl" % k], inputs["a%dh" % k] = a & M32, a >> 32
        if not square:
            inputs["b%dl" % k], inputs["b%dh" % k] = b & M32, b >> 32
    lane = Lane(inputs)
    lane.run(gen.render(ways, square))
    allowed = {"v%d" % (gen.VBASE + i) for i in range(gen.REGS_PER_PRODUCT * ways)}
    allowed |= {"r%d.lo" % k for k in range(ways)} | {"r%d.hi" % k for k in range(ways)}
    assert lane.written <= allowed, lane.written - allowed
    return [lane.v["r%d.lo" % k] | (lane.v["r%d.hi" % k] << 32) for k in range(ways)]


EDGE = [0, 1, 2, M32 - 1, M32, M32 + 1, 2**63, P - 2, P - 1, P, P + 1, M64 - 1, M64, 0xFFFFFFFE00000000,
        0xFFFFFFFF00000000, 0x00000001FFFFFFFF, 0xFFFFFFFEFFFFFFFF]


# Operands whose product has lo(h) = 0, the case where the correction d is
# -1 (a = s 2^48, b = t 2^48 with small s, t).
LOW_H = [s << 48 for s in (1, 2, 3, 0xFFFF, 0x8000)]


@pytest.mark.parametrize("ways", [1, 2, 3])
@pytest.mark.parametrize("square", [False, True])
def test_blocks_compute_products(ways, square):
    rnd = random.Random(ways * 7 + square)
    cases = [(a, b) for a in EDGE + LOW_H for b in EDGE + LOW_H]
    cases += [(rnd.getrandbits(64), rnd.getrandbits(64)) for _ in range(3000)]
    for i in range(0, len(cases) - ways + 1, ways):
        group = cases[i:i + ways]
        if square:
            group = [(a, a) for a, _ in group]
        got = run_block(ways, square, group)
        for (a, b), r in zip(group, got):
            assert 0 <= r <= M64 and r % P == a * b % P, (ways, square, a, b)


def test_blocks_take_the_negative_correction():
    # The d = -1 path (carry 0, borrow 1) must occur among the cases above.
    seen = False
    for a in LOW_H:
        for b in LOW_H:
            lane = Lane({"a0l": a & M32, "a0h": a >> 32, "b0l": b & M32, "b0h": b >> 32})
            lane.run(gen.render(1, False))
            d_reg = "v%d" % (gen.VBASE + 2)  # Z.lo holds d before the last fold
            seen |= lane.v[d_reg] == M32
    assert seen


def test_wait_states_per_block():
    assert not any(line.startswith("s_nop") for line in gen.render(3, False))
    assert sum(line.startswith("s_nop") for line in gen.render(2, False)) == 2
    assert sum(line.startswith("s_nop") for line in gen.render(1, False)) == 2


def test_a_planted_mistake_is_caught():
    # Reading a carry one wait state too early, or a dropped instruction, must
    # fail the checks above.
    lines = [l for l in gen.render(1, False) if l != "s_nop 1"]
    lane = Lane({"a0l": 5, "a0h": 7, "b0l": 9, "b0h": 11})
    with pytest.raises(AssertionError):
        lane.run(lines)
    lines = gen.render(1, False)
    target = "v_addc_co_u32 v112"
    assert sum(l.startswith(target) for l in lines) == 1
    dropped = [l for l in lines if not l.startswith(target)]
    a = b = M64
    lane = Lane({"a0l": a & M32, "a0h": a >> 32, "b0l": b & M32, "b0h": b >> 32})
    lane.run(dropped)
    r = lane.v.get("r0.lo", 0) | (lane.v.get("r0.hi", 0) << 32)
    assert r % P != a * b % P or "r0.lo" not in lane.v


def test_header_is_current():
    gen.main(check=True)
