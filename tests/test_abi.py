"""The C ABI library loads and exports every entry point include/dfjk.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dfjk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(df_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_2601_08077_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return ctypes.CDLL(binding.LIB_PATH)


def test_header_declares_the_expected_surface():
    names = _declared()
    for required in ("df_build_jk", "df_slice", "df_set_precision", "df_create", "df_destroy",
                     "df_workspace_size", "df_set_workspace", "df_get_status", "df_last_error",
                     "df_b_exponents", "df_build_x", "df_debug_slice_gemm_i32"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2601_08077_amd import binding
    assert set(_declared()) <= set(binding.SIGNATURES)


def test_argument_checks_without_gpu_work():
    # calls that fail validation before touching the device
    from paper_2601_08077_amd import binding
    lib = binding.load()
    assert lib.df_set_precision(None, 3) == binding.DF_EINVAL
    assert lib.df_get_precision(None) == binding.DF_EINVAL
    n = ctypes.c_size_t()
    assert lib.df_workspace_size(None, 10, 10, 2, 0, ctypes.byref(n)) == binding.DF_EINVAL
