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


def _lib_or_skip():
    from paper_2203_06327_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    return binding, binding.lib()


def test_null_arguments_are_rejected_without_touching_a_device():
    binding, L = _lib_or_skip()
    h = ctypes.c_void_p()
    assert L.bpjd_ctx_create(0, None, None, None) == binding.ERR_ARG
    assert b"NULL" in L.bpjd_last_error(None)
    # an allocator with only one of its two callbacks
    half = binding.Allocator()
    half.alloc = binding.ALLOC_FN(lambda n, u: None)
    assert L.bpjd_ctx_create(0, ctypes.byref(half), None, ctypes.byref(h)) == binding.ERR_ARG
    assert b"allocator" in L.bpjd_last_error(None)
    assert L.bpjd_problem_create(None, None, None, None, None, ctypes.byref(h)) == binding.ERR_ARG
    assert L.bpjd_problem_create_geom(None, None, None, None, None, ctypes.byref(h)) == binding.ERR_ARG
    for call in (lambda: L.bpjd_solve(None, None, None, binding.MEM_HOST, None),
                 lambda: L.bpjd_setup(None),
                 lambda: L.bpjd_spmm(None, None, 1, None, None, binding.MEM_HOST),
                 lambda: L.bpjd_coarse_eigenvalues(None, None, binding.MEM_HOST),
                 lambda: L.bpjd_apply_preconditioner(None, None, None, None, binding.MEM_HOST),
                 lambda: L.bpjd_problem_set_values(None, None, None, binding.MEM_HOST),
                 lambda: L.bpjd_problem_footprint(None, None),
                 lambda: L.bpjd_server_create(None, 0, 4, ctypes.byref(h)),
                 lambda: L.bpjd_server_submit(None, None, None, None, None, None, None),
                 lambda: L.bpjd_server_poll(None, 1, None, None, None),
                 lambda: L.bpjd_server_get_info(None, None)):
        assert call() == binding.ERR_ARG
    L.bpjd_problem_destroy(None)             # no-ops on NULL
    L.bpjd_ctx_destroy(None)
    L.bpjd_server_destroy(None)


def test_bad_device_ordinal_is_an_error():
    binding, L = _lib_or_skip()
    h = ctypes.c_void_p()
    code = L.bpjd_ctx_create(-1, None, None, ctypes.byref(h))
    # no device at all (CPU host) or an ordinal out of range
    assert code in (binding.ERR_HIP, binding.ERR_ARG)
    assert L.bpjd_last_error(None) != b""
    assert not h.value


def test_every_error_code_has_a_message():
    binding, L = _lib_or_skip()
    codes = [binding.OK, binding.ERR_ARG, binding.ERR_CSR, binding.ERR_DD, binding.ERR_NOT_SPD, binding.ERR_NOCONV,
             binding.ERR_OOM, binding.ERR_HIP, binding.ERR_OVER_BUDGET, binding.ERR_STATE]
    msgs = [L.bpjd_strerror(c) for c in codes]
    assert all(msgs) and len(set(msgs)) == len(msgs)
    assert L.bpjd_strerror(-999) != b""


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_2203_06327_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libbpjd.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.LibraryNotBuilt):
        binding.lib()
