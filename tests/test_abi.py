"""The C ABI library loads and exports every function include/bpjd.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bpjd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bpjd_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bpjd_ctx_create", "bpjd_problem_create", "bpjd_problem_create_geom", "bpjd_solve",
                     "bpjd_apply_preconditioner", "bpjd_spmm", "bpjd_strerror", "bpjd_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2203_06327_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares the same set
    assert set(binding.EXPORTS) == set(declared_functions())


def test_error_strings_without_gpu():
    from paper_2203_06327_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    L = binding.lib()
    assert L.bpjd_strerror(-2) == b"malformed CSR matrix"
    assert L.bpjd_strerror(0) == b"ok"
