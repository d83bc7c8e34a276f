"""CPU checks of the C ABI library: it exists, loads, exports every symbol
include/goldi.h declares, and answers the calls that need no GPU."""

import ctypes
import os
import re

import pytest

import oracle
import paper_2506_09505_amd as goldi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "goldi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(goldi_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("goldi_poseidon_permute", "goldi_merkle_build", "goldi_merkle_build_many"):
        assert s in syms
    assert sorted(goldi.EXPORTS) == syms


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(goldi.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_num_nodes_matches_oracle():
    for n in list(range(0, 70)) + [1 << 22, (1 << 21) + 1, 10**9]:
        assert goldi.goldi_merkle_num_nodes(n) == (oracle.num_nodes(n) if n else 0)


def test_rejections_without_device_work():
    L = goldi.lib()
    assert L.goldi_poseidon_permute(None, 0) == goldi.GOLDI_EINVAL
    assert L.goldi_poseidon_permute(None, 5) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build(None, 0, 8, None) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build(None, 8, 0, None) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build_many(None, 0) == goldi.GOLDI_EINVAL
    assert b"n" in L.goldi_last_error()
    assert L.goldi_strerror(goldi.GOLDI_EINVAL) == b"invalid argument"


def test_constants_table_is_current():
    from paper_2506_09505_amd import gen_constants
    gen_constants.main(check=True)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(goldi, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(goldi, "_lib", None)
    with pytest.raises(RuntimeError):
        goldi.lib()


def test_every_documented_knob_reads_back():
    for k in goldi.TUNE_KEYS:
        v = goldi.goldi_tune_get(k)
        goldi.goldi_tune_set(k, v)
        assert goldi.goldi_tune_get(k) == v


def test_split_knob_bounds():
    old = goldi.goldi_tune_get("split_parts")
    try:
        for parts in (0, 1, 2, 3, 4):
            goldi.goldi_tune_set("split_parts", parts)
            assert goldi.goldi_tune_get("split_parts") == parts
        with pytest.raises(goldi.GoldiError):
            goldi.goldi_tune_set("split_parts", 5)
        assert goldi.goldi_tune_get("split_parts") == 4
    finally:
        goldi.goldi_tune_set("split_parts", old)


@pytest.mark.parametrize("name,form", [(None, 2), ("sparse", 1), ("dense", 0)])
def test_partial_form_of_each_build(name, form):
    # The default library takes the partial rounds in blocks; the test-only
    # builds keep the sparse and the dense forms.  The key is read-only.
    from paper_2506_09505_amd import build
    L = ctypes.CDLL(goldi.LIB_PATH if name is None else build.special_lib(name))
    L.goldi_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]
    L.goldi_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    v = ctypes.c_size_t(99)
    assert L.goldi_tune_get(b"partial_form", ctypes.byref(v)) == 0
    assert v.value == form
    assert L.goldi_tune_set(b"partial_form", form) == goldi.GOLDI_EINVAL


def test_tune_knobs_cpu():
    old = goldi.goldi_tune_get("quad_max_rows")
    goldi.goldi_tune_set("quad_max_rows", 123)
    assert goldi.goldi_tune_get("quad_max_rows") == 123
    goldi.goldi_tune_set("quad_max_rows", old)
    with pytest.raises(goldi.GoldiError):
        goldi.goldi_tune_set("no_such_knob", 1)
    top = goldi.goldi_tune_get("top_max_parents")
    assert top == 16
    with pytest.raises(goldi.GoldiError):
        goldi.goldi_tune_set("top_max_parents", 65)
    assert goldi.goldi_tune_get("top_max_parents") == top
