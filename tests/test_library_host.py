"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every function declared in
  include/dm.h;
* the library's own cut fractions (C++ host code, computed independently of
  the oracle) agree with the oracle's to 1e-13 absolute;
* argument errors come back as documented codes, and building without a
  device reports DM_ENODEVICE instead of falling back to anything.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import geometry as geo
import layout as lay

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "dm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def dm():
    from paper_1301_3794_amd import dm as mod
    mod.lib()
    return mod


def test_exports_every_declared_symbol(dm):
    names = header_functions()
    assert len(names) >= 19
    L = ctypes.CDLL(dm.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert set(dm.EXPORTS) <= set(names)


@pytest.mark.parametrize("name", ["sphere16", "ellipsoid_ragged", "box"])
def test_library_fractions_match_oracle(dm, name):
    if name == "sphere16":
        n, h = (16, 16, 16), 1.0 / 16
        og, pg = geo.sphere((0.5, 0.5, 0.5), 0.45), dm.sphere((0.5, 0.5, 0.5), 0.45)
    elif name == "ellipsoid_ragged":
        n, h = (12, 10, 14), 1.0 / 14
        c, s = (0.45, 0.36, 0.5), (0.38, 0.31, 0.42)
        og, pg = geo.Ellipsoid(c, s), dm.ellipsoid(c, s)
    else:
        n, h = (6, 5, 7), 0.2
        og, pg = geo.Box(), dm.box()
    ref = lay.fractions_to_padded(geo.fractions(og, n, h), n)
    got = dm.compute_fractions(pg, n, h)
    assert got.shape == ref.shape
    assert np.max(abs(got - ref)) <= 1e-13
    assert np.array_equal(got > 0, ref > 0)


def test_face_neglect_in_library(dm):
    from oracle import operators as ops
    n, h = (8, 8, 8), 1.0 / 8
    ref = ops.apply_face_neglect(geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h), 0.1)
    got = dm.compute_fractions(dm.sphere((0.5, 0.5, 0.5), 0.45, a_min=0.1), n, h)
    assert np.max(abs(got - lay.fractions_to_padded(ref, n))) <= 1e-13


def test_error_codes_without_device(dm):
    L = dm.lib()
    g = dm.sphere()
    out = np.zeros(7 * lay.padded_size((4, 4, 4)))
    bad = (ctypes.c_int * 3)(1, 4, 4)
    rc = L.dm_compute_fractions(ctypes.byref(g), bad, 0.25, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == dm.DM_EINVAL
    assert b"dims" in L.dm_last_error_message()
    g2 = dm.sphere()
    g2.bc_lo[0] = 7
    dims = (ctypes.c_int * 3)(4, 4, 4)
    rc = L.dm_compute_fractions(ctypes.byref(g2), dims, 0.25, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == dm.DM_EINVAL
    assert L.dm_strerror(dm.DM_ESINGULAR).startswith(b"coarsest")


def test_build_without_device_fails_loudly(dm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(dm.DMError) as e:
        dm.Operator(dm.sphere(), (8, 8, 8), 1.0 / 8, 5.0)
    assert e.value.code in (dm.DM_ENODEVICE, dm.DM_EHIP)
