"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and argument validation that happens before any device work reports errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1910_11239_amd as fts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fts_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fts_setup_1d_eigs", "fts_apply_operator", "fts_schwarz_smooth", "fts_vcycle"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = fts.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(fts._SIGS)


def test_version_and_error_buffer():
    assert b"fts" in fts.lib().fts_version()
    assert fts.lib().fts_last_error(None, 0) == -1


def _desc(dim=3, k=4, m=(4, 4, 4), gamma=1.0, h=None):
    ws = [np.full(mm, 1.0 / mm) for mm in m]
    if h is not None:
        ws = h
    d, keep = fts._desc(dim, k, ws, gamma)
    d.ncells[0] = m[0]
    return d, keep


@pytest.mark.parametrize("field,value,code", [("dim", 4, -4), ("dim", 1, -4), ("degree", 0, -4),
                                              ("degree", 10, -4), ("penalty_factor", 0.0, -1),
                                              ("penalty_factor", -1.0, -1)])
def test_level_create_validates(field, value, code):
    d, keep = _desc()
    setattr(d, field, value)
    h = ctypes.c_void_p()
    assert fts.lib().fts_level_create(ctypes.byref(d), ctypes.byref(h)) == code
    assert h.value is None
    assert fts.last_error()


def test_level_create_rejects_bad_widths():
    d, keep = _desc(h=[np.array([0.5, -0.5, 0.5, 0.5]), np.full(4, .25), np.full(4, .25)])
    h = ctypes.c_void_p()
    assert fts.lib().fts_level_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d, keep = _desc(h=[np.array([0.5, np.nan, 0.5, 0.5]), np.full(4, .25), np.full(4, .25)])
    assert fts.lib().fts_level_create(ctypes.byref(d), ctypes.byref(h)) == -1


def test_null_arguments():
    lib = fts.lib()
    assert lib.fts_level_create(None, None) == -1
    assert lib.fts_apply_operator(None, None, None, None) == -1
    assert lib.fts_residual(None, None, None, None, None) == -1
    assert lib.fts_schwarz_smooth(None, None, 1.0, 0, None, None, 1, None, 0, None) == -1
    assert lib.fts_vcycle(None, 0, None, None, None) == -1
    assert lib.fts_setup_1d_eigs(None, 0, None) == -1
    assert lib.fts_level_destroy(None) == 0
    assert lib.fts_eigs_destroy(None) == 0
    assert lib.fts_hierarchy_destroy(None) == 0
    assert lib.fts_level_ndofs(None) == -1


def test_hierarchy_validates_before_allocating():
    d, keep = _desc(m=(3, 4, 4), h=[np.full(3, 1 / 3), np.full(4, .25), np.full(4, .25)])
    om = np.full(2, 0.5)
    h = ctypes.c_void_p()
    # 3 cells cannot be coarsened
    assert fts.lib().fts_hierarchy_create(ctypes.byref(d), 2, 1, om.ctypes.data, None, 1, 1, ctypes.byref(h)) == -1
    assert fts.lib().fts_hierarchy_create(ctypes.byref(d), 0, 1, om.ctypes.data, None, 1, 1, ctypes.byref(h)) == -1


def test_library_sources_never_call_hipmalloc():
    """Ownership: every device allocation goes through the allocator the caller
    registers (fts_set_allocator); the sources call no hipMalloc / hipFree."""
    import glob
    import re
    csrc = os.path.join(ROOT, "paper_1910_11239_amd", "csrc")
    for f in glob.glob(os.path.join(csrc, "*.cpp")) + glob.glob(os.path.join(csrc, "*.hip")) + \
            glob.glob(os.path.join(csrc, "*.h")):
        text = re.sub(r"//[^\n]*", "", open(f).read())
        assert not re.search(r"(?<!Host)hipMalloc\w*\(|(?<!Host)hipFree\(", text), f


def test_allocator_must_be_given_in_pairs():
    lib = fts.lib()
    assert lib.fts_set_allocator(fts._ALLOC_CB, ctypes.cast(None, fts._FREE_T), None) == -1


def test_mapped_hierarchy_validates_before_allocating():
    """fts_mapped_hierarchy_create checks the level list (count, dimension,
    degree, twice the cells per axis from one level to the next) before any
    device work; the setters check their handle and value."""
    lib = fts.lib()
    verts = [np.zeros(((2 * 2 ** l + 1) ** 2, 2)) for l in range(2)]
    descs = (fts.MappedDesc * 2)()
    for l in range(2):
        descs[l].dim, descs[l].degree, descs[l].penalty_factor = 2, 2, 4.0
        for a in range(3):
            descs[l].ncells[a] = 2 * 2 ** l if a < 2 else 1
        descs[l].vertices = verts[l].ctypes.data
    descs[1].ncells[0] = 3  # not twice the coarse count
    om = np.array([0.0, 0.5])
    h = ctypes.c_void_p()
    assert lib.fts_mapped_hierarchy_create(descs, 2, om.ctypes.data, 1, 1, ctypes.byref(h)) == -1
    assert "twice" in fts.last_error()
    descs[1].ncells[0] = 4
    descs[1].degree = 3  # another degree
    assert lib.fts_mapped_hierarchy_create(descs, 2, om.ctypes.data, 1, 1, ctypes.byref(h)) == -1
    assert lib.fts_mapped_hierarchy_create(descs, 0, om.ctypes.data, 1, 1, ctypes.byref(h)) == -1
    assert lib.fts_mapped_hierarchy_create(descs, 2, om.ctypes.data, -1, 1, ctypes.byref(h)) == -1
    assert lib.fts_mapped_hierarchy_set_smoother(None, 0) == -1
    assert lib.fts_mapped_hierarchy_set_local_solver(None, 0) == -1
    assert lib.fts_mapped_hierarchy_destroy(None) == 0
    assert lib.fts_mapped_hierarchy_ndofs(None) == -1
    assert lib.fts_hierarchy_set_smoother(None, 2) == -1
