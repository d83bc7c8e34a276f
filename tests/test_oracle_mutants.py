"""Planted mistakes in the oracle must fail its pins.

Each mutant is a copy of ``oracle/oracle.c`` with one plausible mistake (a
dropped term, a transposed operand, a shifted index, a wrong exponent, a
misplaced constant, a wrong sponge or tree rule).  It is compiled with gcc
into a temporary directory and swapped in for the real library while the pin
tests run; at least one pin must fail for every mutant.  CPU only.
"""

import ctypes
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_field as tf
from tests import test_oracle_perm as tp
from tests import test_oracle_tree as tt

MUTANTS = {
    "mds_drops_first_term": ("for (int j = 0; j < WIDTH; j++) acc", "for (int j = 1; j < WIDTH; j++) acc"),
    "mds_transposed": ("prm->mds[i][j], s[j]", "prm->mds[j][i], s[j]"),
    "rc_wrong_round": ("s[i] = oracle_fadd(s[i], prm->rc[r][i]);",
                       "s[i] = oracle_fadd(s[i], prm->rc[(r + 1) % ROUNDS][i]);"),
    "partial_sbox_word1": ("s[0] = sbox(s[0]);", "s[1] = sbox(s[1]);"),
    "sbox_x5": ("oracle_fpow(x, 7)", "oracle_fpow(x, 5)"),
    "three_full_rounds_each_side": ("#define HALF_FULL 4 ", "#define HALF_FULL 3 "),
    "rc_after_sbox": (
        "        for (int i = 0; i < WIDTH; i++) s[i] = oracle_fadd(s[i], prm->rc[r][i]);\n"
        "        if (full) {\n"
        "            for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);\n"
        "        } else {\n"
        "            s[0] = sbox(s[0]);\n"
        "        }\n",
        "        if (full) {\n"
        "            for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);\n"
        "        } else {\n"
        "            s[0] = sbox(s[0]);\n"
        "        }\n"
        "        for (int i = 0; i < WIDTH; i++) s[i] = oracle_fadd(s[i], prm->rc[r][i]);\n"),
    "fmul_no_reduction": ("return (uint64_t)(((u128)a * b) % ORACLE_P); }",
                          "return (uint64_t)((u128)a * b); }"),
    "fadd_wraps_2_64": ("return (uint64_t)(((u128)a + b) % ORACLE_P); }", "return a + b; }"),
    "sponge_overwrites": ("s[i] = oracle_fadd(s[i], words[k + i]);", "s[i] = words[k + i];"),
    "digest_from_capacity": ("memcpy(out, s, DIGEST * sizeof(uint64_t));",
                             "memcpy(out, s + 8, DIGEST * sizeof(uint64_t));"),
    "odd_node_hashed_alone": ("memcpy(x->parents + i * DIGEST, x->children + 2 * i * DIGEST, DIGEST * sizeof(uint64_t));",
                              "sponge(x->prm, x->children + 2 * i * DIGEST, DIGEST, x->parents + i * DIGEST);"),
    "children_swapped": ("sponge(x->prm, x->children + 2 * i * DIGEST, 2 * DIGEST, x->parents + i * DIGEST);",
                         "{ uint64_t t[8]; memcpy(t, x->children + (2*i+1)*DIGEST, 32); memcpy(t+4, x->children + 2*i*DIGEST, 32); sponge(x->prm, t, 8, x->parents + i * DIGEST); }"),
    "row_major_leaves": ("row[col] = x->leaves[col * x->n_rows + r];", "row[col] = x->leaves[r * x->n_cols + col];"),
}


def _pins(prm):
    """Every pin of the three oracle test modules, as zero-argument calls."""
    calls = [tf.test_random_pairs, tf.test_identities, tf.test_fermat_inverse_and_sbox_bijection,
             tf.test_reduce128_any_input,
             tp.test_identity_matrix_round_counts, tp.test_permutation_matrix_orientation,
             tp.test_all_ones_matrix_dense_sum, tp.test_inverse_round_trip_spec_constants,
             tp.test_bigint_implementation_agrees]
    calls += [lambda r=r, k=k: tp.test_single_round_constant_placement(r, k)
              for r, k in [(0, 0), (0, 5), (4, 0), (26, 9), (29, 11)]]
    calls += [lambda w=w: tt.test_sponge_single_chunk(prm, w) for w in (3, 8)]
    calls += [lambda w=w: tt.test_sponge_multi_chunk(prm, w) for w in (12, 16)]
    calls += [lambda n=n, w=w: tt.test_tree_vs_bigint_recursion(prm, n, w) for n, w in [(3, 1), (5, 9), (8, 16), (13, 7)]]
    calls += [lambda: tt.test_single_leaf_tree(prm), lambda: tt.test_one_leaf_flip_changes_one_path(prm, 21)]
    return calls


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert src.count(old) == 1, name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", str(mpath), "-o", str(so)])
    real = oracle.lib()
    m = ctypes.CDLL(str(so))
    for fn in ("oracle_fadd", "oracle_fsub", "oracle_fmul", "oracle_fpow", "oracle_reduce128",
               "oracle_permute", "oracle_leaf_hash", "oracle_merkle_level", "oracle_merkle_build",
               "oracle_merkle_num_nodes"):
        getattr(m, fn).restype = getattr(real, fn).restype
        getattr(m, fn).argtypes = getattr(real, fn).argtypes
    monkeypatch.setattr(oracle, "_lib", m)
    prm = oracle.spec_params()
    failed = []
    for call in _pins(prm):
        try:
            call()
        except AssertionError:
            failed.append(call)
    assert failed, "mutant %s passed every pin" % name
