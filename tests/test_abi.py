"""The C-ABI library loads on a machine without a GPU and exports every
function that include/cpm.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cpm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[A-Za-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libcpm():
    from paper_2111_06704_amd import build, cpm
    if not os.path.exists(cpm.LIB_PATH):
        build.build()
    return ctypes.CDLL(cpm.LIB_PATH)


def test_every_declared_symbol_is_exported(libcpm):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(libcpm, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2111_06704_amd import cpm
    assert sorted(cpm.EXPORTS) == _declared()


def test_status_strings(libcpm):
    libcpm.cpm_status_str.restype = ctypes.c_char_p
    assert libcpm.cpm_status_str(-4) == b"CPM_ENOTSPD"
    assert libcpm.cpm_status_str(0) == b"CPM_OK"


def test_build_rejects_bad_arguments_before_touching_the_device(libcpm):
    """Host-side validation runs before any HIP call: these fail with
    CPM_EINVAL on a machine without a GPU."""
    from paper_2111_06704_amd import cpm
    L = cpm.lib()
    import numpy as np
    p = cpm.Params(gauss_inv_width=1.979, ewald_split=0.3, rcut=12.0, kspace_eps=1e-6)
    out = ctypes.c_void_p()
    pos = np.zeros((2, 3))
    box = np.array([10.0, 10.0, 10.0])
    assert L.cpm_build_E(pos.ctypes.data, 2, box.ctypes.data, ctypes.byref(p), None, ctypes.byref(out)) == cpm.CPM_EINVAL
    assert b"coincide" in L.cpm_last_error()
    pos = np.array([[0, 0, 0], [1, 1, 1.0]])
    box_bad = np.array([10.0, -1.0, 10.0])
    assert L.cpm_build_E(pos.ctypes.data, 2, box_bad.ctypes.data, ctypes.byref(p), None, ctypes.byref(out)) == cpm.CPM_EINVAL
    p.ewald_split = 0.0
    assert L.cpm_build_E(pos.ctypes.data, 2, box.ctypes.data, ctypes.byref(p), None, ctypes.byref(out)) == cpm.CPM_EINVAL
    p.ewald_split = 0.3
    p.kspace_eps = 2.0
    assert L.cpm_build_E(pos.ctypes.data, 2, box.ctypes.data, ctypes.byref(p), None, ctypes.byref(out)) == cpm.CPM_EINVAL
    assert not out.value
    assert L.cpm_solve(None, None, None, 1, None, None, None) == cpm.CPM_EINVAL
    assert L.cpm_gcd_build(None, None, 2, None, None, None, None, None) == cpm.CPM_EINVAL
    assert L.cpm_gcd_solve(None, None, None, 1, None, None, None, None) == cpm.CPM_EINVAL
