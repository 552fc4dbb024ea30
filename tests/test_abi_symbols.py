"""The C-ABI library loads and exports every function include/tmqcd.h declares
(no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmqcd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s+((?:tm|tsm)_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1211_0126_amd as tq
    if not os.path.exists(tq.LIB_PATH):
        from paper_1211_0126_amd.build import build
        build()
    return tq.load_library()


def test_header_parses():
    names = declared_functions()
    for must in ("tm_gauge_load", "tm_dslash", "tsm_solve_batch", "tsm_loops", "tm_create", "tm_destroy"):
        assert must in names


def test_every_declared_symbol_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        fn = getattr(lib, name)
        assert ctypes.cast(fn, ctypes.c_void_p).value


def test_binding_covers_header():
    import paper_1211_0126_amd as tq
    assert sorted(tq.EXPORTS) == declared_functions()


def test_abi_version(lib):
    assert lib.tm_abi_version() == 1


def test_product_path_has_no_oracle_dependency():
    # the package and its native sources never reference the oracle
    pkg = os.path.join(ROOT, "paper_1211_0126_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "tm_oracle" not in text and "orc_" not in text, f


def test_missing_library_fails_loudly(tmp_path):
    from paper_1211_0126_amd import binding
    saved = binding._lib
    binding._lib = None
    try:
        with pytest.raises(RuntimeError):
            binding.load_library(str(tmp_path / "libtmqcd.so"))
    finally:
        binding._lib = saved
