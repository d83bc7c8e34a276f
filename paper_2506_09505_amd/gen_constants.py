"""Writes ``csrc/poseidon12_constants.inc`` from the seeded instance file.

The instance (round constants C[30][12] and the first row of the circulant
matrix M) lives in ``synth/poseidon12.json``; this script turns it into the
tables the kernels compile against:

* ``GOLDI_RC_SPLIT[31][12][2]``: C[r][i] split into its low and high 32-bit
  halves, each stored in a 64-bit word so that a scalar load yields a 64-bit
  SGPR pair that is directly the addend of a 32x32+64 multiply-add.  Row 30
  is all zero: no constant follows the last matrix product (the permutation's
  constants enter at the start of each round, Sec. 2.4).
* ``GOLDI_MDS[12][12]``: the small matrix entries (they fit 8 bits, as the
  paper's ``mult_72`` / ``mmult_4x12_8`` functions assume, Table 1).
* the constants of the sparse form of the partial rounds (Sec. 2.4, Alg. 1:
  a dense pre-matrix once, then per partial round a sparse matrix whose first
  row and first column are full and whose remainder is the identity), derived
  from C and M by ``sparse_form`` below.  Full-width entries that enter dot
  products are split into three 22-bit limbs (a 32 x 22-bit product is below
  2^54, so a dozen of them add up in 64 bits without carries).
* the constants of the partial rounds taken three at a time (``block_form``):
  the integer matrices (M P)^m and their columns, the first partial round
  folded into the last opening round's matrix, and per-block constants.

Apart from ``sparse_form``, ``block_form`` and ``cap0_constants`` the script
only reformats.
"""

from __future__ import annotations

import json
import math
import os

P = (1 << 64) - (1 << 32) + 1
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SPEC = os.path.join(ROOT, "synth", "poseidon12.json")
OUT = os.path.join(HERE, "csrc", "poseidon12_constants.inc")


def _mm(a, b):
    return [[sum(a[i][k] * b[k][j] for k in range(len(b))) % P for j in range(len(b[0]))] for i in range(len(a))]


def _mv(a, x):
    return [sum(a[i][k] * x[k] for k in range(len(x))) % P for i in range(len(a))]


def _identity(n):
    return [[int(i == j) for j in range(n)] for i in range(n)]


def _inverse(m):
    """Inverse of a square matrix mod p (Gauss-Jordan), or None if singular."""
    n = len(m)
    a = [[m[i][j] % P for j in range(n)] + _identity(n)[i] for i in range(n)]
    for c in range(n):
        piv = next((r for r in range(c, n) if a[r][c]), None)
        if piv is None:
            return None
        a[c], a[piv] = a[piv], a[c]
        inv = pow(a[c][c], P - 2, P)
        a[c] = [v * inv % P for v in a[c]]
        for r in range(n):
            if r != c and a[r][c]:
                f = a[r][c]
                a[r] = [(x - f * y) % P for x, y in zip(a[r], a[c])]
    return [row[n:] for row in a]


def _power(m, e):
    r = _identity(len(m))
    for _ in range(e):
        r = _mm(r, m)
    return r


def sparse_form(rc, mds, half_full: int = 4, partial: int = 22):
    """Constants of the partial rounds in sparse form (Sec. 2.4, Alg. 1).

    Write M = [[m00, w^T], [v, Mh]] with Mh the lower-right 11 x 11 block.
    With D_j = diag(1, Mh^(j - partial)) (j = 0..partial), the matrices
    D_j^-1 M D_(j-1) have the identity as lower-right block, first row
    (m00, w^T Mh^(j - 1 - partial)) and first column Mh^(partial - j) v; the
    state entering the partial rounds is multiplied once by
    D_0^-1 = diag(1, Mh^partial) and D_partial = I leaves nothing behind.
    Only word 0 passes the S-box in a partial round, so a round constant's
    words 1..11 can be moved through the matrix into the next round's
    constant; what is left before each S-box is a scalar k_r on word 0, and
    the carry after the last partial round joins the first constant of the
    closing full rounds.

    Returns None when Mh is singular (no sparse form exists), else a dict:
      k[j]   = k_(half_full + j), j = 0..partial-1 (scalar constants);
      c_end  = the 12-word constant added after the last partial round;
      row[j] = first-row entries 1..11 of partial round half_full + j;
      col[j] = first-column entries 1..11 of that round;
      pre    = Mh^partial (11 x 11);
      pre_m  = rows 1..11 of diag(1, Mh^partial) M (11 x 12): the pre-matrix
               folded into the matrix of the last opening full round."""
    w12 = len(mds)
    mh = [row[1:] for row in mds[1:]]
    mh_inv = _inverse(mh)
    if mh_inv is None:
        return None
    w = mds[0][1:]
    v = [mds[i][0] for i in range(1, w12)]
    row, col = [], []
    for j in range(1, partial + 1):
        back = _power(mh_inv, partial + 1 - j)          # Mh^(j - 1 - partial)
        row.append([sum(w[k] * back[k][i] for k in range(w12 - 1)) % P for i in range(w12 - 1)])
        col.append(_mv(_power(mh, partial - j), v))
    pre = _power(mh, partial)
    pre_m = _mm(pre, [r[:] for r in mds[1:]])
    carry = [0] * w12
    k = []
    for r in range(half_full, half_full + partial):
        d = [(rc[r][i] + carry[i]) % P for i in range(w12)]
        k.append(d[0])
        carry = _mv(mds, [0] + d[1:])
    c_end = [(rc[half_full + partial][i] + carry[i]) % P for i in range(w12)]
    # Partial rounds in groups: a later round's dot product can use the words
    # from the start of its group, plus lag[r][d] times the S-box output of
    # round r - 1 - d of the same group, lag[r][d] = <row of r, col of r-1-d>.
    lag = [[sum(row[r][i] * col[r - 1 - d][i] for i in range(w12 - 1)) % P if r - 1 - d >= 0 else 0
            for d in range(3)] for r in range(partial)]
    return {"k": k, "c_end": c_end, "row": row, "col": col, "pre": pre, "pre_m": pre_m, "lag": lag}


BLOCK = 3            # partial rounds per block
# Bound on a block row's coefficients (see block_form): a row adds products
# of 32-bit limbs and a 32-bit constant half into one accumulator, which the
# kernels' split reduction needs below 2^63: (2^31 - 2 + 1)(2^32 - 1) < 2^63.
BLOCK_ROW_SUM = (1 << 31) - 2


def block_form(rc, mds, k: int = BLOCK, half_full: int = 4, partial: int = 22):
    """Constants of the partial rounds taken k at a time.

    A partial round on a state b that already holds its round constant is
    b' = M P b + c0 S(b_0) + C[r+1], with P the projection that zeroes word 0
    and c0 the first column of M.  Over m consecutive rounds from b:
      b_(m) = A_m b + sum_(j<m) f_m[j] S_j + K_m,
    where A_m = (M P)^m, f_m[j] = A_(m-1-j) c0, S_j is the S-box output of
    round j of the block (its input is word 0 of b_(j)), and
    K_m = sum_(j=1..m) A_(m-j) C[r+j].  A_m and f_m are the same for every
    block and, for small matrix entries and small m, are integers far below
    2^32, so a block costs one dense product with 32-bit entries instead of
    m products.

    The first partial round is not in a block: it joins the matrix of the
    last opening full round (lead_b, lead_k below).

    Returns None unless every entry of A_m (m <= k), f_m and lead_b is below
    2^32 and every row's coefficients sum to at most BLOCK_ROW_SUM (so that a
    row's products of 32-bit limbs and its constant add up below 2^63), else a
    dict:
      a[m]    = A_m (12 x 12 integers, column 0 zero for m >= 1), m = 0..k;
      f[m]    = f_m as f[m][i][j] (12 x m integers), m = 1..k;
      lead_b  = M P M (12 x 12 integers);
      lead_k  = M P C[half_full] + C[half_full + 1] (mod p);
      starts  = first round of each block (half_full + 1, half_full + 1 + k, ...);
      tail    = the partial rounds after the last block (taken one by one);
      kc[b]   = block b's constants: K_1[0] .. K_(k-1)[0], then K_k[0..11]."""
    w12 = len(mds)
    mp = [[0 if j == 0 else mds[i][j] for j in range(w12)] for i in range(w12)]
    c0 = [mds[i][0] for i in range(w12)]
    a = [_identity(w12)]
    for _ in range(k):
        a.append([[sum(mp[i][t] * a[-1][t][j] for t in range(w12)) for j in range(w12)] for i in range(w12)])
    f = [None]
    for m in range(1, k + 1):
        f.append([[sum(a[m - 1 - j][i][t] * c0[t] for t in range(w12)) for j in range(m)] for i in range(w12)])
    # The first partial round joins the last opening full round's matrix:
    # from the S-box outputs y of that round, the state after the partial
    # round is (M P M) y + c0 S(row 0 of M y + C[h][0]) + M P C[h] + C[h+1]
    # (h = half_full).
    lead_b = [[sum(mp[i][t] * mds[t][j] for t in range(w12)) for j in range(w12)] for i in range(w12)]
    rows = [a[m][i][1:] + f[m][i] for m in range(1, k + 1) for i in range(w12)]
    rows += [lead_b[i] + [c0[i]] for i in range(w12)]
    if any(max(r) >= 1 << 32 or sum(r) > BLOCK_ROW_SUM for r in rows):
        return None
    h = half_full
    lead_k = [(x + y) % P for x, y in zip(_mv(mp, rc[h]), rc[h + 1])]
    n_blocks = (partial - 1) // k
    starts = [h + 1 + k * b for b in range(n_blocks)]
    tail = list(range(h + 1 + k * n_blocks, h + partial))
    kc = []
    for r in starts:
        ks = []
        for m in range(1, k + 1):
            km = [sum(_mv(a[m - j], rc[r + j])[i] for j in range(1, m + 1)) % P for i in range(w12)]
            ks.append(km)
        kc.append([ks[m - 1][0] for m in range(1, k)] + ks[k - 1])
    return {"a": a, "f": f, "starts": starts, "tail": tail, "kc": kc, "k": k, "lead_b": lead_b, "lead_k": lead_k}


def cap0_constants(rc, mds):
    """Row constants of round 0's matrix for a state whose words 8..11 are
    zero: those words enter the S-box as C[0][8..11], so their outputs and
    matrix terms are constants, folded into C[1]:
      C[1][i] + sum_k M[i][8+k] C[0][8+k]^7  (mod p)."""
    caps = [pow(rc[0][8 + k], 7, P) for k in range(4)]
    return [(rc[1][i] + sum(mds[i][8 + k] * caps[k] for k in range(4))) % P for i in range(12)]


def _limbs22(x: int):
    return [x & 0x3FFFFF, (x >> 22) & 0x3FFFFF, x >> 44]


def _c_array(name: str, ctype: str, dims, flat) -> str:
    """A nested brace initializer for an array of shape dims from row-major values."""
    flat = list(flat)
    assert len(flat) == math.prod(dims)

    def nest(vals, shape):
        if len(shape) == 1:
            return "{" + ", ".join("0x%xu" % v for v in vals) + "}"
        step = len(vals) // shape[0]
        return "{" + ", ".join(nest(vals[i * step:(i + 1) * step], shape[1:]) for i in range(shape[0])) + "}"

    return "#define %s_INIT %s  /* %s%s */" % (name, nest(flat, dims), ctype, "".join("[%d]" % d for d in dims))


def render_sparse(rc, mds) -> list:
    sp = sparse_form(rc, mds)
    lines = ["// Partial rounds in sparse form (see gen_constants.sparse_form)."]
    if sp is None:
        lines.append("#define GOLDI_SPARSE_OK 0  // the lower-right 11 x 11 block of M is singular")
        sp = {"k": [0] * 22, "c_end": [0] * 12, "row": [[0] * 11] * 22, "col": [[0] * 11] * 22,
              "pre_m": [[0] * 12] * 11, "lag": [[0] * 3] * 22}
    else:
        lines.append("#define GOLDI_SPARSE_OK 1")
    k = sp["k"] + [sp["c_end"][0]]
    lines.append("// GOLDI_SP_K[j]: 22-bit limbs of k_(4+j); j = 22: word 0 of the closing constant.")
    lines.append(_c_array("GOLDI_SP_K", "u32", [23, 3], [l for x in k for l in _limbs22(x)]))
    lines.append("// GOLDI_SP_CEND[i]: 32-bit halves of word i+1 of the closing constant.")
    lines.append(_c_array("GOLDI_SP_CEND", "u32", [11, 2], [h for x in sp["c_end"][1:] for h in (x & 0xFFFFFFFF, x >> 32)]))
    lines.append("// GOLDI_SP_ROW[j][i]: 22-bit limbs of first-row entry i+1 of partial round 4+j.")
    lines.append(_c_array("GOLDI_SP_ROW", "u32", [22, 11, 3], [l for r in sp["row"] for x in r for l in _limbs22(x)]))
    lines.append("// GOLDI_SP_COL22[j][i]: 22-bit limbs of first-column entry i+1 of partial round 4+j.")
    lines.append(_c_array("GOLDI_SP_COL22", "u32", [22, 11, 3], [l for r in sp["col"] for x in r for l in _limbs22(x)]))
    lines.append("// GOLDI_SP_LAG[j][d]: 22-bit limbs of <row of round 4+j, col of round 4+j-1-d>.")
    lines.append(_c_array("GOLDI_SP_LAG", "u32", [22, 3, 3], [l for r in sp["lag"] for x in r for l in _limbs22(x)]))
    lines.append("// GOLDI_SP_PRE_M[i][j]: 22-bit limbs of row i+1, column j of diag(1, Mh^22) M.")
    lines.append(_c_array("GOLDI_SP_PRE_M", "u32", [11, 12, 3], [l for r in sp["pre_m"] for x in r for l in _limbs22(x)]))
    k4 = sp["k"][0]
    lines.append("// GOLDI_SP_K4_SPLIT: k_4 as the {lo32, 0}, {hi32, 0} pair of a matrix row's addends.")
    lines.append("#define GOLDI_SP_K4_SPLIT {0x%08xull, 0x%08xull}" % (k4 & 0xFFFFFFFF, k4 >> 32))
    return lines


def render_blocks(rc, mds) -> list:
    bf = block_form(rc, mds)
    lines = ["// Partial rounds in blocks (see gen_constants.block_form)."]
    if bf is None:
        lines.append("#define GOLDI_BLOCK_OK 0  // block coefficients too large for 32-bit limbs")
        return lines
    k = bf["k"]
    lines.append("#define GOLDI_BLOCK_OK 1")
    lines.append("#define GOLDI_BLK %d  // partial rounds per block" % k)
    lines.append("#define GOLDI_BLK_N %d  // blocks; the partial rounds after them go one by one" % len(bf["starts"]))
    lines.append("#define GOLDI_BLK_FIRST_TAIL %d  // first partial round after the blocks" %
                 (bf["tail"][0] if bf["tail"] else bf["starts"][-1] + k))
    assert bf["starts"][0] == 5, "the lead round is partial round 4"
    lines.append("// GOLDI_BLK_A[m-1] = (M P)^m, m = 1..%d (P zeroes word 0): exact integers." % k)
    lines.append("static constexpr unsigned GOLDI_BLK_A[%d][12][12] = %s;" % (
        k, "{" + ", ".join("{" + ", ".join("{" + ", ".join("%du" % v for v in row) + "}" for row in bf["a"][m]) + "}"
                           for m in range(1, k + 1)) + "}"))
    lines.append("// GOLDI_BLK_F[m-1][i][j] = ((M P)^(m-1-j) c0)_i for j < m (c0 = column 0 of M), else 0.")
    lines.append("static constexpr unsigned GOLDI_BLK_F[%d][12][%d] = %s;" % (
        k, k, "{" + ", ".join("{" + ", ".join("{" + ", ".join("%du" % (bf["f"][m][i][j] if j < m else 0)
                                                                 for j in range(k)) + "}" for i in range(12)) + "}"
                              for m in range(1, k + 1)) + "}"))
    lines.append("// GOLDI_BLK_LEAD_B = M P M: the last opening round's matrix with the first partial round.")
    lines.append("static constexpr unsigned GOLDI_BLK_LEAD_B[12][12] = %s;" % (
        "{" + ", ".join("{" + ", ".join("%du" % v for v in row) + "}" for row in bf["lead_b"]) + "}"))
    lines.append("// GOLDI_BLK_LEAD_K = M P C[4] + C[5] (mod p), split as RC_SPLIT.")
    lines.append(_c_array("GOLDI_BLK_LEAD_K", "u64", [12, 2], [h for v in bf["lead_k"] for h in (v & 0xFFFFFFFF, v >> 32)]))
    lines.append("// GOLDI_BLK_K[b]: block b's constants K_1[0] .. K_%d[0], K_%d[0..11], split as RC_SPLIT." % (k - 1, k))
    cells = [h for blk in bf["kc"] for v in blk for h in (v & 0xFFFFFFFF, v >> 32)]
    lines.append(_c_array("GOLDI_BLK_K", "u64", [len(bf["kc"]), k - 1 + 12, 2], cells))
    return lines


def render(spec: dict, source: str = "synth/poseidon12.json") -> str:
    rc = [[int(v) for v in row] for row in spec["rc"]] + [[0] * 12]
    mds = spec["mds"]
    assert len(rc) == 31 and all(len(r) == 12 for r in rc)
    assert all(0 <= v < 2**64 - 2**32 + 1 for r in rc for v in r)
    assert all(0 <= m <= 64 for row in mds for m in row)
    assert all(mds[i][j] == mds[0][(j - i) % 12] for i in range(12) for j in range(12)), "circulant"
    lines = ["// Generated by paper_2506_09505_amd/gen_constants.py from %s." % source,
             "// Do not edit by hand.",
             "#pragma once",
             "#define GOLDI_SPEC_SEED %d" % spec["seed"],
             "static constexpr unsigned GOLDI_MDS[12][12] = {"]
    for row in mds:
        lines.append("    {%s}," % ", ".join("%du" % m for m in row))
    lines.append("};")
    lines.append("// GOLDI_RC_SPLIT[r][i] = {C[r][i] mod 2^32, C[r][i] >> 32}; row 30 = 0.")
    lines.append("#define GOLDI_RC_SPLIT_INIT { \\")
    for r, row in enumerate(rc):
        cells = ", ".join("{0x%08xull, 0x%08xull}" % (v & 0xFFFFFFFF, v >> 32) for v in row)
        lines.append("    {%s}, \\" % cells)
    lines.append("}")
    rc_int = [[int(v) for v in row] for row in spec["rc"]]
    mds_int = [[int(v) for v in row] for row in mds]
    r1 = cap0_constants(rc_int, mds_int)
    lines.append("// GOLDI_CAP0_RC1[i]: C[1][i] + sum_k M[i][8+k] C[0][8+k]^7 (mod p), split as above.")
    lines.append("#define GOLDI_CAP0_RC1_INIT {%s}" % ", ".join("{0x%08xull, 0x%08xull}" % (v & 0xFFFFFFFF, v >> 32)
                                                              for v in r1))
    lines.extend(render_sparse(rc_int, mds_int))
    lines.extend(render_blocks(rc_int, mds_int))
    return "\n".join(lines) + "\n"


def special_specs():
    """Instances with closed-form permutations, compiled into test-only
    libraries (the kernels of every layout run against a closed form, not
    against the oracle):
      identity  M = I, C = 0: word 0 ends as x0^(7^30), words 1..11 as x^(7^8);
      shift     M[i][j] = [j = i + 1 mod 12], C = 0: words move one place per
                round and pick up a factor 7 per S-box they pass through;
      const     M = I, C zero except C[5][0] = 3 and C[27][4] = 5."""
    zero = [["0"] * 12 for _ in range(30)]
    ident = [[int(i == j) for j in range(12)] for i in range(12)]
    shift = [[int(j == (i + 1) % 12) for j in range(12)] for i in range(12)]
    const = [row[:] for row in zero]
    const[5][0] = "3"
    const[27][4] = "5"
    return {"identity": {"seed": 0, "rc": zero, "mds": ident},
            "shift": {"seed": 0, "rc": zero, "mds": shift},
            "const": {"seed": 0, "rc": const, "mds": ident}}


def special_path(name: str) -> str:
    return os.path.join(HERE, "csrc", "special_%s.inc" % name)


def write_specials() -> list:
    out = []
    for name, spec in special_specs().items():
        path = special_path(name)
        text = render(spec, "the special instance '%s' (closed-form tests only)" % name)
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as f:
                f.write(text)
        out.append(path)
    return out


def main(check: bool = False) -> str:
    with open(SPEC) as f:
        text = render(json.load(f))
    if check:
        with open(OUT) as f:
            if f.read() != text:
                raise SystemExit("%s is stale: run python -m paper_2506_09505_amd.gen_constants" % OUT)
        return OUT
    old = open(OUT).read() if os.path.exists(OUT) else None
    if old != text:
        with open(OUT, "w") as f:
            f.write(text)
    return OUT


if __name__ == "__main__":
    print(main())
