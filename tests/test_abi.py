"""Host-side checks of the C ABI library (no GPU needed).

* libbeadscf.so loads and exports every function include/beadscf.h declares.
* The host-built Boys table (Gauss-Legendre quadrature) matches mpmath.
* Without a GPU, context creation fails with an error code instead of crashing.
"""

import os
import re

import mpmath
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "beadscf.h")).read()
    decl = r"^\s*(?:bscf_status|double|const char\s*\*)\s*(bscf_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1601_02713_amd import beadscf
    import ctypes
    lib = ctypes.CDLL(beadscf.LIB_PATH)
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(beadscf.exported_symbols())


def test_host_boys_table_against_mpmath():
    from paper_1601_02713_amd import beadscf
    mpmath.mp.dps = 40
    for k in [0, 1, 37, 150, 299, 400]:
        T = mpmath.mpf(k) / 10
        for m in [0, 1, 5, 9, 16, 22]:
            if T == 0:
                ref = mpmath.mpf(1) / (2 * m + 1)
            else:
                ref = mpmath.gammainc(m + mpmath.mpf(1) / 2, 0, T) / (2 * T ** (m + mpmath.mpf(1) / 2))
            got = beadscf.boys_table_entry(m, k)
            assert abs(got - float(ref)) <= 4e-15 * float(ref), (m, k, got, float(ref))


def test_create_without_gpu_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1601_02713_amd import beadscf
    with pytest.raises(beadscf.BscfError):
        beadscf.Engine(0)
