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


BAD_CREATE = [
    # (coord, n, bc, face arrays: "ok" | "dec" | "neg" | "pole"), each rejected on the host
    (0, (2048, 2048, 1024), (0, 0, 0, 0, 2, 2), "ok"),   # 4.3e9 cells: 32-bit indices overflow
    (0, (1024, 1024, 1024), (0, 0, 0, 0, 2, 2), "ok"),   # 2^30 cells: one past the limit
    (0, (0, 4, 4), (0, 0, 0, 0, 2, 2), "ok"),            # empty axis
    (0, (4, 4, 4), (0, 0, 0, 0, 2, 0), "ok"),            # periodic on one side only
    (0, (4, 4, 2), (0, 0, 0, 0, 2, 2), "ok"),            # periodic axis with < 3 cells
    (0, (4, 4, 4), (0, 0, 1, 0, 2, 2), "ok"),            # Dirichlet off axis 0
    (0, (4, 4, 4), (0, 0, 0, 0, 2, 7), "ok"),            # unknown boundary condition
    (5, (4, 4, 4), (0, 0, 0, 0, 2, 2), "ok"),            # unknown coordinate system
    (0, (4, 4, 4), (0, 0, 0, 0, 2, 2), "dec"),           # faces not increasing
    (0, (4, 4, 4), (0, 0, 0, 0, 2, 2), "neg"),           # non-positive radius
    (0, (4, 4, 4), (0, 0, 0, 0, 2, 2), "pole"),          # colatitude reaches pi
]


@pytest.mark.parametrize("coord,n,bc,faces", BAD_CREATE)
def test_create_rejects_each_bad_argument(lib, coord, n, bc, faces):
    """Each invalid grid, boundary set or coordinate array is STS_EINVAL with
    no handle, decided on the host (no GPU is needed to run this test)."""
    import math
    import numpy as np
    lib.sts_create.restype = ctypes.c_int
    m = max(n) + 1
    r = np.linspace(1.0, 2.0, m)
    th = np.linspace(0.1, 0.9 * math.pi, m)
    ph = np.linspace(0.0, 2 * math.pi, m)
    if faces == "dec":
        th = th[::-1].copy()
    elif faces == "neg":
        r = np.linspace(-1.0, 2.0, m)
    elif faces == "pole":
        th = np.linspace(0.1, math.pi, m)
    arrs = [np.ascontiguousarray(a) for a in (r, th, ph)]
    ptr = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
    h = ctypes.c_void_p()
    cbc = (ctypes.c_int * 6)(*bc)
    st = lib.sts_create(ctypes.byref(h), coord, n[0], n[1], n[2], *ptr, cbc, None)
    assert st == -1 and not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1610_01265_amd import _binding
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_binding, "_lib", None)
    with pytest.raises(RuntimeError):
        _binding.load()
