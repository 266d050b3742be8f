"""Host-side checks of the C interface (no GPU): the library loads, exports
every declared entry point, and rejects bad meshes before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2411_14315_amd as hbl
from hbinputs.meshes import cube_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hbl.LIB_PATH):
        from paper_2411_14315_amd import build
        build.build(verbose=False)
    return hbl.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "hb.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(hb_\w+)\s*\(", hdr, re.M))
    assert {"hb_mesh_create", "hb_residual", "hb_jvp", "hb_newton_solve"} <= names
    for n in names:
        assert hasattr(lib, n), n


def _create(lib, m, tets=None, kinds=None):
    tets = np.ascontiguousarray(m.tets if tets is None else tets, np.int32)
    kinds = np.ascontiguousarray(m.group_kind if kinds is None else kinds, np.int32)
    xyz = np.ascontiguousarray(m.xyz)
    faces = np.ascontiguousarray(m.faces, np.int32)
    grp = np.ascontiguousarray(m.face_group, np.int32)
    h = C.c_void_p()
    st = lib.hb_mesh_create(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                            faces.shape[0], faces.ctypes.data, grp.ctypes.data, kinds.shape[0],
                            kinds.ctypes.data, C.byref(h))
    if st == 0:
        lib.hb_mesh_destroy(h)
    return st


def test_rejects_bad_meshes_on_host(lib):
    m = cube_mesh(2)
    bad = m.tets.copy()
    bad[3, 1] = m.n_nodes + 5
    assert _create(lib, m, tets=bad) == hbl.HB_ERR_MESH
    assert b"out of range" in lib.hb_last_error()
    deg = m.tets.copy()
    deg[0, 3] = deg[0, 2]
    assert _create(lib, m, tets=deg) == hbl.HB_ERR_MESH
    assert b"degenerate" in lib.hb_last_error()
    assert _create(lib, m, kinds=np.zeros_like(m.group_kind)) == hbl.HB_ERR_ARG
    assert b"outlet" in lib.hb_last_error()


def test_null_arguments(lib):
    h = C.c_void_p()
    assert lib.hb_mesh_create(0, None, 0, None, 0, None, None, 0, None, C.byref(h)) == hbl.HB_ERR_ARG
    assert lib.hb_residual(None, None, None, None, None, None) == hbl.HB_ERR_ARG
    assert lib.hb_jvp(None, None, None, None, None, None, 0, None) == hbl.HB_ERR_ARG
    assert lib.hb_newton_solve(None, None, None, None, None, None, None) == hbl.HB_ERR_ARG


class _FakeMesh:
    """Stands in for a mesh handle: the binding checks its arguments against
    these sizes before it calls into the library."""
    n_nodes = 10
    n_outlets = 1
    _h = None


def test_binding_rejects_bad_tensors_before_launch():
    torch = pytest.importorskip("torch")
    m = _FakeMesh()
    prm = hbl.Params(K=2)
    bc = hbl.BC(torch.zeros((3, 5, 10), dtype=torch.float64), np.zeros((1, 5)), None)
    cases = [
        (lambda: hbl.residual(m, prm, bc, torch.zeros((4, 5, 10), dtype=torch.float32)), "dtype"),
        (lambda: hbl.residual(m, prm, bc, torch.zeros((4, 3, 10), dtype=torch.float64)), "shape"),
        (lambda: hbl.jvp(m, prm, bc, torch.zeros((4, 5, 9), dtype=torch.float64),
                         torch.zeros((4, 5, 10), dtype=torch.float64)), "shape"),
        (lambda: hbl.jvp(m, prm, bc, torch.zeros((4, 5, 10), dtype=torch.float32),
                         torch.zeros((4, 5, 10), dtype=torch.float32)), "dtype"),
        (lambda: hbl.newton_solve(m, hbl.Params(K=3), bc,
                                  torch.zeros((4, 5, 10), dtype=torch.float64)), "shape"),
        (lambda: hbl.jacobi(m, prm, bc, torch.zeros((4, 5, 10), dtype=torch.float16)), "dtype"),
        (lambda: hbl.tm_residual(m, prm, None, torch.zeros((4, 11), dtype=torch.float64)), "shape"),
        (lambda: hbl.precond_apply(m, prm, bc, torch.zeros((4, 5, 10), dtype=torch.float32),
                                   torch.zeros((4, 5, 10), dtype=torch.float64)), "dtype"),
        (lambda: hbl.residual(m, prm, bc, torch.zeros((4, 5, 10), dtype=torch.float64)),
         "device"),
    ]
    for fn, what in cases:
        with pytest.raises(hbl.HBError) as e:
            fn()
        assert e.value.status == hbl.HB_ERR_ARG and what in str(e.value), str(e.value)
    # host boundary arrays are checked against the mesh and N as well
    bad_h = hbl.BC(torch.zeros((3, 5, 10), dtype=torch.float64), np.zeros((2, 5)), None)
    with pytest.raises(hbl.HBError) as e:
        bad_h._c(m, 5)
    assert "outlet_h" in str(e.value)
