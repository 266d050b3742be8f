"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): a sanitized build (paper_2411_14315_amd/build.py --sanitize; host
code only) is loaded into a child process with the ASan runtime preloaded,
and the entry points that do their work on the host are driven through
their normal and error paths: the symmetric eigensolver at several sizes
(including repeated eigenvalues and n = 1), mesh creation with out-of-range
indices, degenerate tetrahedra, a missing outlet group and NULL arrays, and
NULL or out-of-range arguments to the solver, preconditioner, POD and
network entry points, and the multigrid hierarchy's graph code (matching,
aggregation, colouring) on a cube mesh.  Any sanitizer report fails the
test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r"""
    import ctypes as C, sys
    import numpy as np
    sys.path.insert(0, sys.argv[2])
    from hbinputs.meshes import cube_mesh
    lib = C.CDLL(sys.argv[1])
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.hb_last_error.restype = C.c_char_p
    lib.hb_sym_eig.argtypes = [i32, vp, vp, vp]
    rng = np.random.default_rng(0)
    mats = [rng.normal(size=(n, n)) for n in (1, 2, 3, 17, 70)]
    mats = [a + a.T for a in mats] + [np.diag([2.0, 1.0, 2.0, 1.0]), np.eye(6)]
    for A in mats:
        A = np.ascontiguousarray(A)
        n = A.shape[0]
        w, V = np.zeros(n), np.zeros((n, n))
        assert lib.hb_sym_eig(n, A.ctypes.data, w.ctypes.data, V.ctypes.data) == 0
        assert np.linalg.norm(A @ V - V * w) <= 1e-12 * n * max(np.abs(w).max(), 1.0)
    bad = np.array([[1.0, 2.0], [3.0, 1.0]])
    w, V = np.zeros(2), np.zeros((2, 2))
    assert lib.hb_sym_eig(2, bad.ctypes.data, w.ctypes.data, V.ctypes.data) == -1
    assert lib.hb_sym_eig(0, None, None, None) == -1

    lib.hb_mesh_create.argtypes = [i64, vp, i64, vp, i64, vp, vp, i32, vp, C.POINTER(vp)]
    m = cube_mesh(2)
    def create(tets=None, kinds=None, xyz=None):
        t = np.ascontiguousarray(m.tets if tets is None else tets, np.int32)
        k = np.ascontiguousarray(m.group_kind if kinds is None else kinds, np.int32)
        x = np.ascontiguousarray(m.xyz if xyz is None else xyz)
        f = np.ascontiguousarray(m.faces, np.int32)
        g = np.ascontiguousarray(m.face_group, np.int32)
        h = vp()
        return lib.hb_mesh_create(x.shape[0], x.ctypes.data, t.shape[0], t.ctypes.data,
                                  f.shape[0], f.ctypes.data, g.ctypes.data, k.shape[0],
                                  k.ctypes.data, C.byref(h))
    t = m.tets.copy(); t[3, 1] = m.n_nodes + 5
    assert create(tets=t) == -2
    t = m.tets.copy(); t[0, 3] = t[0, 2]
    assert create(tets=t) == -2
    t = m.tets.copy(); t[2, 0] = -1
    assert create(tets=t) == -2
    assert create(kinds=np.zeros_like(m.group_kind)) == -1
    h = vp()
    assert lib.hb_mesh_create(0, None, 0, None, 0, None, None, 0, None, C.byref(h)) == -1

    assert lib.hb_residual(None, None, None, None, None, None) == -1
    assert lib.hb_jvp(None, None, None, None, None, None, 0, None) == -1
    assert lib.hb_newton_solve(None, None, None, None, None, None, None) == -1
    assert lib.hb_precond_apply(None, None, None, None, dbl(0.0), None, 0, None, None,
                                None) == -1
    lib.hb_pod_fit.argtypes = [vp, vp, i64, i64, i32, dbl, vp, vp, vp, vp, vp, vp]
    assert lib.hb_pod_fit(None, None, 0, 0, 0, 0.0, None, None, None, None, None, None) == -1
    lib.hb_mlp_create.argtypes = [i32, vp, vp, C.c_uint64, C.POINTER(vp)]
    widths = np.array([4, 0, 2], np.int32)
    assert lib.hb_mlp_create(2, widths.ctypes.data, None, 0, C.byref(h)) == -1
    assert lib.hb_mlp_create(0, None, None, 0, C.byref(h)) == -1
    lib.hb_pod_expand.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp]
    assert lib.hb_pod_expand(0, 0, None, None, None, None, None, None) == -1
    assert len(lib.hb_last_error()) > 0
    lib.hb_precond_hierarchy.argtypes = [i64, i64, vp, i32, i32, i32, vp, C.POINTER(i32), vp, vp]
    mc = cube_mesh(4)
    tets = np.ascontiguousarray(mc.tets, np.int32)
    for aggr in (0, 1):
        sizes = np.zeros(8, np.int64); nl = i32()
        agg = np.zeros(mc.n_nodes, np.int32); col = np.zeros(mc.n_nodes, np.int32)
        assert lib.hb_precond_hierarchy(mc.n_nodes, tets.shape[0], tets.ctypes.data, 8, aggr, 8,
                                        sizes.ctypes.data, C.byref(nl), agg.ctypes.data,
                                        col.ctypes.data) == 0
        assert nl.value >= 2 and sizes[0] == mc.n_nodes
    bad = tets.copy(); bad[1, 2] = mc.n_nodes
    assert lib.hb_precond_hierarchy(mc.n_nodes, bad.shape[0], bad.ctypes.data, 8, 0, 8,
                                    sizes.ctypes.data, C.byref(nl), None, None) == -1
    print("host entry points clean", flush=True)
""")


@pytest.fixture(scope="module")
def san_lib():
    from paper_2411_14315_amd import build
    try:
        rt = build.asan_runtime()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("no clang to locate the AddressSanitizer runtime")
    if not os.path.exists(rt):
        pytest.skip("AddressSanitizer runtime not installed")
    srcs = [os.path.join(build.CSRC, f) for f in build.SOURCES]
    srcs += [os.path.join(build.CSRC, "hb_internal.h"), os.path.join(ROOT, "include", "hb.h")]
    if (not os.path.exists(build.SAN_LIB) or
            max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(build.SAN_LIB)):
        build.build_sanitized(verbose=False)
    return build.SAN_LIB, rt


def test_host_entry_points_under_sanitizers(san_lib):
    lib, rt = san_lib
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-c", CHILD, lib, ROOT], env=env, capture_output=True,
                       text=True, timeout=300)
    report = p.stdout + p.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert p.returncode == 0, report[-4000:]
    assert "host entry points clean" in p.stdout
