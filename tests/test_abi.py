"""The C-ABI library loads and exports every entry point include/sts.h
declares (no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:sts_status|char\s*\*|long long|void)\s*\**\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1610_01265_amd import _binding, build
    if not os.path.exists(_binding.LIB_PATH):
        build.build()
    return ctypes.CDLL(_binding.LIB_PATH)


def test_header_declares_the_hot_path():
    names = declared_functions()
    for required in ("sts_create", "sts_destroy", "sts_set_spitzer", "sts_set_isotropic",
                     "sts_dt_euler", "apply_F", "rkl2_step", "be_pcg_solve"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_1610_01265_amd import _binding
    assert set(declared_functions()) == set(_binding.exported_symbols())


def test_create_rejects_bad_arguments_without_gpu_work(lib):
    """Argument checks run before any device call."""
    import numpy as np
    lib.sts_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    f = np.array([1.0, 0.5, 2.0])  # not increasing
    pd = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    bc = (ctypes.c_int * 6)(0, 0, 0, 0, 2, 2)
    st = lib.sts_create(ctypes.byref(h), 0, 2, 2, 2, pd, pd, pd, bc, None)
    assert st == -1 and not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1610_01265_amd import _binding
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_binding, "_lib", None)
    with pytest.raises(RuntimeError):
        _binding.load()
