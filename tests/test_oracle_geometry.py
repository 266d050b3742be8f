"""Pins of the oracle's P1 geometry and quadrature against closed forms."""
from math import factorial

import numpy as np

from hbinputs.meshes import boundary_faces, cube_mesh, cylinder_mesh
from oracle import fem


def test_shape_function_gradients():
    m = cube_mesh(3, jitter=0.2, seed=3)
    om = fem.from_mesh(m)
    assert np.allclose(om.grad.sum(axis=1), 0.0, atol=1e-12)
    # N_A is linear with N_A(x_B) = delta_AB
    x = om.xyz[om.tets]                                   # (e, 4, 3)
    dN = np.einsum("eai,ebi->eab", om.grad, x - x[:, :1])  # N_A(x_B) - N_A(x_0)
    ref = np.eye(4)[None] - np.eye(4)[:, :1][None]
    assert np.allclose(dN, ref, atol=1e-12)


def test_volumes():
    om = fem.from_mesh(cube_mesh(4, jitter=0.25, seed=1))
    assert np.all(om.vol > 0)
    assert abs(om.vol.sum() - 1.0) < 1e-13
    c = cylinder_mesh(1.0, 6.0, 4, 8, reorder=False)
    om = fem.from_mesh(c)
    nring = 24                                           # outer ring polygon
    area = 0.5 * nring * np.sin(2 * np.pi / nring)
    assert abs(om.vol.sum() - 6.0 * area) < 1e-12


def test_reorientation_counts():
    m = cube_mesh(2)
    t = m.tets.copy()
    t[::3, 2], t[::3, 3] = m.tets[::3, 3], m.tets[::3, 2]
    om = fem.prepare(m.xyz, t, m.faces, m.face_group, m.group_kind)
    assert om.n_reoriented == len(range(0, t.shape[0], 3))
    assert np.all(om.vol > 0)


def test_metric_rotation_invariance():
    rng = np.random.default_rng(0)
    m = cube_mesh(2, jitter=0.2, seed=5)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    a = fem.from_mesh(m)
    b = fem.prepare(m.xyz @ Q.T, m.tets, m.faces, m.face_group, m.group_kind)
    assert np.allclose(a.xixi, b.xixi, rtol=1e-12)
    u = rng.normal(size=(a.ne, 3))
    qa = np.einsum("ei,eij,ej->e", u, a.xi, u)
    qb = np.einsum("ei,eij,ej->e", u @ Q.T, b.xi, u @ Q.T)
    assert np.allclose(qa, qb, rtol=1e-11)
    # unit right reference tetrahedron: xi = identity
    ref = fem.tet_geometry(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]),
                           np.array([[0, 1, 2, 3]]))
    assert np.allclose(ref[2][0], np.eye(3))


def _mono_exact(p, dim):
    return factorial(dim) * np.prod([factorial(k) for k in p]) / factorial(dim + sum(p))


def test_tet_rule_is_degree_two():
    for p in [(0, 0, 0, 0), (1, 0, 0, 0), (2, 0, 0, 0), (1, 1, 0, 0), (0, 1, 0, 1)]:
        val = np.sum(fem.TET_QW * np.prod(fem.TET_QP ** np.array(p), axis=1))
        assert abs(val - _mono_exact(p, 3)) < 1e-15
    # degree 3 is not exact (so the rule really is the degree-2 one)
    val = np.sum(fem.TET_QW * fem.TET_QP[:, 0] ** 3)
    assert abs(val - _mono_exact((3, 0, 0, 0), 3)) > 1e-4


def test_triangle_rule_is_degree_two():
    for p in [(0, 0, 0), (1, 0, 0), (2, 0, 0), (1, 1, 0)]:
        val = np.sum(fem.TRI_QW * np.prod(fem.TRI_QP ** np.array(p), axis=1))
        assert abs(val - _mono_exact(p, 2)) < 1e-15


def test_outlet_normals():
    m = cylinder_mesh(1.0, 6.0, 4, 8)
    om = fem.from_mesh(m)
    assert np.allclose(om.onormal, [0, 0, 1], atol=1e-14)
    nring = 24
    assert abs(om.oarea.sum() - 0.5 * nring * np.sin(2 * np.pi / nring)) < 1e-13
    # independent boundary extraction agrees on the outward direction
    bf = boundary_faces(m.xyz, m.tets)
    n = np.cross(m.xyz[bf[:, 1]] - m.xyz[bf[:, 0]], m.xyz[bf[:, 2]] - m.xyz[bf[:, 0]])
    assert np.allclose(0.5 * n.sum(axis=0), 0.0, atol=1e-12)   # closed surface
