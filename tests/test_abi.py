"""The C-ABI library loads and exports every symbol include/chefsi.h declares (CPU only, no compute)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2302_09708_amd import chefsi as cs
from paper_2302_09708_amd.inputs import small_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chefsi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chefsi_[a-z0-9_]+)\s*\(", text)))


def test_library_is_built():
    assert os.path.exists(cs.LIB_PATH), "run python -m paper_2302_09708_amd.build"


def test_exports_every_declared_symbol():
    lib = cs.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in chefsi.h but not exported"
    assert sorted(cs.EXPORTS) == names


def test_strerror_and_version():
    lib = cs.load()
    assert lib.chefsi_version() >= 100
    for st in range(0, 9):
        assert len(cs.strerror(st)) > 0
    assert cs.strerror(4) == "overlap matrix not positive definite"


def _create(prob, precision=0, max_ns=4, mutate=None):
    lib = cs.load()
    g = cs.Grid()
    for d in range(3):
        g.n[d], g.h[d], g.bc[d] = prob.n[d], prob.h[d], prob.bc[d]
    g.fd_order = prob.fd_order
    if mutate:
        mutate(g)
    veff = np.ascontiguousarray(prob.veff, dtype=np.float64)
    arrs = [np.ascontiguousarray(prob.supp_ptr, np.int64), np.ascontiguousarray(prob.supp_idx, np.int32),
            np.ascontiguousarray(prob.nproj, np.int32), np.ascontiguousarray(prob.chi, np.float64),
            np.ascontiguousarray(prob.gamma, np.float64)]
    nl = cs.Nonlocal()
    nl.n_atoms = len(prob.nproj)
    nl.supp_ptr = arrs[0].ctypes.data_as(C.POINTER(C.c_int64))
    nl.supp_idx = arrs[1].ctypes.data_as(C.POINTER(C.c_int32))
    nl.nproj = arrs[2].ctypes.data_as(C.POINTER(C.c_int32))
    nl.chi = arrs[3].ctypes.data_as(C.POINTER(C.c_double))
    nl.gamma = arrs[4].ctypes.data_as(C.POINTER(C.c_double))
    h = C.c_void_p()
    st = lib.chefsi_create(C.byref(g), veff.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nl), precision,
                           max_ns, C.byref(h))
    if st == 0:
        lib.chefsi_destroy(h)
    return st


@pytest.mark.parametrize("mutate", [
    lambda g: setattr(g, "fd_order", 7),
    lambda g: setattr(g, "fd_order", 14),
    lambda g: g.n.__setitem__(0, 0),
    lambda g: g.n.__setitem__(1, 3),        # periodic n < r = 6
    lambda g: g.h.__setitem__(2, 0.0),
    lambda g: g.bc.__setitem__(0, 2),
])
def test_create_rejects_bad_grid_before_touching_the_device(mutate):
    prob = small_problem(n=(12, 10, 14), n_atoms=2, seed=1)
    assert _create(prob, mutate=mutate) == cs.ERR_INVALID_ARG


def test_create_rejects_bad_projectors_and_sizes():
    prob = small_problem(n=(12, 10, 14), n_atoms=2, seed=1)
    bad = small_problem(n=(12, 10, 14), n_atoms=2, seed=1)
    bad.supp_idx = bad.supp_idx.copy()
    bad.supp_idx[0] = prob.nd            # outside the grid
    assert _create(bad) == cs.ERR_INVALID_ARG
    bad2 = small_problem(n=(12, 10, 14), n_atoms=2, seed=1)
    bad2.supp_idx = bad2.supp_idx.copy()
    bad2.supp_idx[1] = bad2.supp_idx[0]  # not strictly increasing
    assert _create(bad2) == cs.ERR_INVALID_ARG
    assert _create(prob, precision=5) == cs.ERR_INVALID_ARG
    assert _create(prob, max_ns=0) == cs.ERR_INVALID_ARG
    assert _create(prob, max_ns=prob.nd + 1) == cs.ERR_INVALID_ARG
    nanv = small_problem(n=(12, 10, 14), n_atoms=2, seed=1)
    nanv.veff = nanv.veff.copy()
    nanv.veff[3] = np.nan
    assert _create(nanv) == cs.ERR_INVALID_ARG


def test_null_handle_calls_fail_cleanly():
    lib = cs.load()
    b = C.c_size_t()
    assert lib.chefsi_workspace_bytes(None, 4, C.byref(b)) == cs.ERR_INVALID_ARG
    assert lib.chefsi_last_error(None) == b""
    lib.chefsi_destroy(None)
