"""Host-only checks of the C ABI: the library loads, exports every declared
entry point, and rejects malformed hierarchies before any device call."""
import copy
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stv.h")


@pytest.fixture(scope="module")
def stv():
    import paper_2107_10561_amd as m
    return m


@pytest.fixture(scope="module")
def c1_levels():
    from stgen.problem import make_problem
    p = make_problem(2, (16, 4), 2, 1, 0.01, 1e-3, 1001)
    return p


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(stv_\w+)\(", txt, re.M)))


def test_header_declares_the_api():
    names = _declared()
    for n in ["stv_create", "stv_destroy", "stv_set_hierarchy", "stv_build_cell_inverses",
              "stv_vanka_sweep", "stv_vcycle", "stv_gmres_solve", "stv_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(stv):
    out = subprocess.run(["nm", "-D", "--defined-only", stv.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(stv_\w+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(stv.library(), n)
    assert set(stv.EXPORTED) == set(_declared())


def test_valid_hierarchy_passes(stv, c1_levels):
    rc, msg = stv.validate_hierarchy(c1_levels.levels, 2, 1)
    assert rc == stv.STV_OK, msg


def _mutable(levels):
    out = []
    for L in levels:
        d = dict(n_sdofs=L.n_sdofs, rowptr=L.rowptr.astype(np.int32).copy(), col=L.col.copy(),
                 val=L.val.copy(), cell_sdofs=L.cell_sdofs.copy(),
                 P=None if L.P is None else tuple(a.copy() for a in L.P))
        out.append(d)
    return out


def _expect(stv, levels, dim, k, needle):
    rc, msg = stv.validate_hierarchy(levels, dim, k)
    assert rc == stv.STV_EINVAL and needle in msg, msg


def test_rejects_unsorted_columns(stv, c1_levels):
    lv = _mutable(c1_levels.levels)
    r0 = lv[1]["rowptr"][5]
    lv[1]["col"][r0], lv[1]["col"][r0 + 1] = lv[1]["col"][r0 + 1], lv[1]["col"][r0]
    _expect(stv, lv, 2, 1, "strictly increasing")


def test_rejects_out_of_range_cell_dof(stv, c1_levels):
    lv = _mutable(c1_levels.levels)
    lv[1]["cell_sdofs"][3, 4] = lv[1]["n_sdofs"] + 7
    _expect(stv, lv, 2, 1, "cell_sdofs out of range")


def test_accepts_missing_cell_pair(stv, c1_levels):
    """An absent pair of a cell is a zero block, not an error."""
    lv = _mutable(c1_levels.levels)
    L = lv[1]
    s = int(L["cell_sdofs"][10, 0])
    t = int(L["cell_sdofs"][10, 20])
    lo, hi = int(L["rowptr"][s]), int(L["rowptr"][s + 1])
    q = lo + int(np.searchsorted(L["col"][lo:hi], t))
    L["col"] = np.delete(L["col"], q)
    L["val"] = np.delete(L["val"], q, axis=0)
    L["rowptr"][s + 1:] -= 1
    rc, msg = stv.validate_hierarchy(lv, 2, 1)
    assert rc == stv.STV_OK, msg


def test_rejects_repeated_dof_in_cell(stv, c1_levels):
    lv = _mutable(c1_levels.levels)
    lv[1]["cell_sdofs"][2, 1] = lv[1]["cell_sdofs"][2, 0]
    _expect(stv, lv, 2, 1, "repeated DoF in cell 2")


def test_rejects_wrong_dimension_and_degree(stv, c1_levels):
    _expect(stv, _mutable(c1_levels.levels), 3, 1, "n_ls")
    rc, msg = stv.validate_hierarchy(_mutable(c1_levels.levels), 2, 7)
    assert rc == stv.STV_EINVAL and "k must be" in msg


def test_rejects_bad_prolongation(stv, c1_levels):
    lv = _mutable(c1_levels.levels)
    lv[1]["P"][1][0] = lv[0]["n_sdofs"] + 1
    _expect(stv, lv, 2, 1, "P_col out of range")
    lv = _mutable(c1_levels.levels)
    lv[1]["P"] = None
    _expect(stv, lv, 2, 1, "must not be NULL")


def test_rejects_orphan_dof(stv, c1_levels):
    lv = _mutable(c1_levels.levels)
    lv[0]["n_sdofs"] += 1
    rp = lv[0]["rowptr"]
    lv[0]["rowptr"] = np.concatenate([rp, rp[-1:]])
    _expect(stv, lv, 2, 1, "belongs to no cell")


def test_rejects_bad_level_count(stv):
    import ctypes
    buf = ctypes.create_string_buffer(256)
    rc = stv.library().stv_validate_hierarchy(0, 2, 1, None, buf, 256)
    assert rc == stv.STV_EINVAL and b"n_levels" in buf.value


def test_null_context_calls_are_rejected(stv):
    lib = stv.library()
    assert lib.stv_set_hierarchy(None, 1, 2, 1, None) == stv.STV_EINVAL
    assert lib.stv_build_cell_inverses(None, 0, None, None) == stv.STV_EINVAL
    assert lib.stv_vanka_sweep(None, 1, None, None, 1, 0.7, 0) == stv.STV_EINVAL
    assert lib.stv_gmres_solve(None, None, None, None, None) == stv.STV_EINVAL
    lib.stv_destroy(None)


def test_create_without_gpu_reports_hip_error(stv):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes
    h = ctypes.c_void_p()
    rc = stv.library().stv_create(ctypes.byref(h), 0, None)
    assert rc == stv.STV_EHIP
    assert b"device" in stv.library().stv_last_error(None)
