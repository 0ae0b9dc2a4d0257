"""The C ABI library loads and exports every entry point that
include/itpp.h declares (CPU only: no compute call is made)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "itpp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(itpp_[a-z_]+)\s*\(", src)))


def test_header_declares_api():
    names = declared_functions()
    for n in ("itpp_create", "itpp_evolve", "itpp_expect", "itpp_export", "itpp_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2601_14400_amd", "libitpp.so")
    if not os.path.exists(lib_path):
        pytest.skip("libitpp.so not built (run __graft_entry__.build())")
    import paper_2601_14400_amd as P

    lib = P.load_library()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(P._native.EXPORTED)
    assert "gfx950" in P.version()


def test_create_without_gpu_fails_loudly():
    """No CPU fallback: without a gfx950 device, creating an engine raises."""
    lib_path = os.path.join(ROOT, "paper_2601_14400_amd", "libitpp.so")
    if not os.path.exists(lib_path):
        pytest.skip("libitpp.so not built")
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2601_14400_amd as P

    with pytest.raises(P.ItppError):
        P.Engine(8, 1e-14, 1 << 10)


def test_string_packing_roundtrip():
    import numpy as np

    from paper_2601_14400_amd import strings_to_words, words_to_strings

    strs = ["IXYZ" * 20, "Z" + "I" * 79, "Y" * 80]
    x, z = strings_to_words(strs, 80)
    assert x.shape == (3, 2)
    assert words_to_strings(x, z, 80) == strs
    assert int(x[0, 0]) & 0b0110 == 0b0110 and int(z[0, 0]) & 0b1100 == 0b1100


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: a missing shared library is an import error."""
    from paper_2601_14400_amd import _native

    with pytest.raises(ImportError):
        _native.load_library(str(tmp_path / "libitpp.so"))
