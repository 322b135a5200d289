"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every function include/cpm.h declares, and
parameter validation in cpm_create must reject bad input before any device
call is made.
"""
import ctypes
import os
import re

import pytest

from paper_2203_15461_amd import cpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[a-z_]+)\s*\(", src)))


def test_library_exports_header():
    L = cpm.lib()
    names = header_functions()
    assert "cpm_build_elastance" in names and "cpm_solve_charges" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(cpm.EXPORTS) == names


def _create(**over):
    p = cpm.Params(14.757, 25.56, 30.0)
    for k, v in over.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    cp = p.to_c()
    st = cpm.lib().cpm_create(ctypes.byref(cp), None, ctypes.byref(h))
    assert not h.value  # rejected before anything was allocated
    return st


@pytest.mark.parametrize("over,status", [
    (dict(Lx=-1.0), cpm.EINVAL),
    (dict(h=float("nan")), cpm.EINVAL),
    (dict(slab_factor=1.0), cpm.EINVAL),
    (dict(slab_factor=1.2), cpm.EINVAL),          # (f - 1) h = 6 A < r_c
    (dict(eta=0.0), cpm.EINVAL),
    (dict(alpha=float("inf")), cpm.EINVAL),
    (dict(kspace_eps=0.0), cpm.EINVAL),
    (dict(kspace_eps=2.0), cpm.EINVAL),
    (dict(geometry=1), cpm.EUNSUPPORTED),
])
def test_create_validation(over, status):
    assert _create(**over) == status


def test_null_arguments():
    L = cpm.lib()
    assert L.cpm_create(None, None, None) == cpm.EINVAL
    assert L.cpm_set_electrolyte(None, 0, None) == cpm.EINVAL
    assert L.cpm_invert(None, 1) == cpm.EINVAL
    assert L.cpm_solve_charges(None, 1, None, 0, 0, None, None) == cpm.EINVAL
    assert L.cpm_last_error(None) == b"no context"
    L.cpm_destroy(None)
