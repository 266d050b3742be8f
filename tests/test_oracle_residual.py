"""Pins of the oracle's HB-GLS residual (Section 2.3, eq. Rmc) against
identities and closed forms that any correct implementation satisfies."""
from dataclasses import replace

import numpy as np
import pytest

from hbinputs.meshes import boundary_faces, cube_mesh, cylinder_mesh
from hbinputs.problems import Params, c1_womersley, seeded_state
from oracle import api, fem, spectral
from oracle import residual as res


def _c1(K=2):
    P = c1_womersley(K=K)
    return P, fem.from_mesh(P.mesh)


def _samples(P, om, seed):
    return api.samples_of(om, P.params, seeded_state(P, seed), P.dirichlet)


def _r(om, prm, y, hs, R=None, **kw):
    return res.residual_samples(om, prm, y, hs, R, api.H_of(prm), res.Options(**kw))


def test_continuity_rows_sum_to_boundary_flux():
    """sum_A r^c_A = int_Gamma u.n at every sample, for any state: the
    shape functions sum to one and their gradients to zero."""
    P, om = _c1()
    y = _samples(P, om, 0)
    r = _r(om, P.params, y, api.h_samples(P.params, P.outlet_h))
    bf = boundary_faces(P.mesh.xyz, P.mesh.tets)
    x = P.mesh.xyz
    nA = 0.5 * np.cross(x[bf[:, 1]] - x[bf[:, 0]], x[bf[:, 2]] - x[bf[:, 0]])  # area * n
    ubar = y[:3][:, :, bf].mean(axis=3)                  # (3, N, F)
    flux = np.einsum("inf,fi->n", ubar, nA)
    assert np.allclose(r[3].sum(axis=1), flux, rtol=1e-12, atol=1e-13 * np.abs(flux).max())


def test_uniform_flow_leaves_interior_rows_zero():
    m = cube_mesh(4, jitter=0.2, seed=2)
    om = fem.from_mesh(m)
    prm = Params(K=2)
    N = prm.N
    y = np.zeros((4, N, om.n))
    y[0], y[1], y[2], y[3] = 0.7, -0.3, 0.45, 2.0
    r = _r(om, prm, y, np.zeros((om.n_outlets, N)))
    inner = np.ones(om.n, bool)
    inner[boundary_faces(m.xyz, m.tets).ravel()] = False
    assert inner.sum() > 0
    assert np.abs(r[:, :, inner]).max() < 1e-13


def test_dirichlet_rows():
    P, om = _c1()
    y = _samples(P, om, 1)
    r = _r(om, P.params, y, api.h_samples(P.params, P.outlet_h))
    assert np.all(r[:3][:, :, om.dirichlet] == 0.0)
    assert np.abs(r[3][:, om.dirichlet]).min() > 0.0          # continuity kept everywhere


def test_similarity_scaling():
    """(u, p, mu, omega, g, h, R) -> (l u, l^2 p, l mu, l omega, l g, l^2 h, l R)
    maps r^m -> l^2 r^m and r^c -> l r^c (every term of the HB-GLS form,
    tau included, scales this way)."""
    P, om = _c1()
    lam = 2.7
    rng = np.random.default_rng(3)
    y = _samples(P, om, 2)
    hs = rng.normal(size=(om.n_outlets, P.params.N))
    R = np.array([1.3])
    r1 = _r(om, P.params, y, hs, R)
    p2 = replace(P.params, mu=lam * P.params.mu, period=P.params.period / lam)
    y2 = y.copy()
    y2[:3] *= lam
    y2[3] *= lam ** 2
    r2 = _r(om, p2, y2, lam ** 2 * hs, lam * R)
    assert np.allclose(r2[:3], lam ** 2 * r1[:3], rtol=1e-11, atol=1e-12 * np.abs(r2[:3]).max())
    assert np.allclose(r2[3], lam * r1[3], rtol=1e-11, atol=1e-12 * np.abs(r2[3]).max())


def test_time_shift_equivariance():
    """H is circulant, everything else pointwise in time: a cyclic shift of
    the samples (and of the boundary data) shifts the residual."""
    P, om = _c1()
    y = _samples(P, om, 4)
    hs = np.random.default_rng(0).normal(size=(1, P.params.N))
    r = _r(om, P.params, y, hs, np.array([0.7]))
    rs = _r(om, P.params, np.roll(y, 1, axis=1), np.roll(hs, 1, axis=1), np.array([0.7]))
    assert np.allclose(rs, np.roll(r, 1, axis=1), rtol=1e-12, atol=1e-13 * np.abs(r).max())


def test_rotation_equivariance():
    P, om = _c1()
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    y = _samples(P, om, 5)
    hs = rng.normal(size=(1, P.params.N))
    r = _r(om, P.params, y, hs, np.array([0.4]))
    m = P.mesh
    om2 = fem.prepare(m.xyz @ Q.T, m.tets, m.faces, m.face_group, m.group_kind)
    y2 = y.copy()
    y2[:3] = np.einsum("ij,jna->ina", Q, y[:3])
    r2 = _r(om2, P.params, y2, hs, np.array([0.4]))
    scale = np.abs(r).max()
    assert np.allclose(r2[:3], np.einsum("ij,jna->ina", Q, r[:3]), atol=1e-12 * scale)
    assert np.allclose(r2[3], r[3], atol=1e-12 * scale)


def _mms_fields(x, t, k, w):
    """Divergence-free u* = phi(t) (sin ky, sin kz, sin kx), p* = P(t) cos kx cos ky,
    with phi, P trigonometric polynomials of degree <= 2 in w t, and the
    body acceleration f = du/dt + u.grad u + grad p/rho - nu lap u."""
    phi = 1.0 + 0.5 * np.sin(w * t) + 0.3 * np.cos(2 * w * t)
    dphi = 0.5 * w * np.cos(w * t) - 0.6 * w * np.sin(2 * w * t)
    Pt = 0.5 + 0.2 * np.cos(w * t)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    s = np.stack([np.sin(k * Y), np.sin(k * Z), np.sin(k * X)])          # (3, n)
    conv = np.stack([np.sin(k * Z) * k * np.cos(k * Y),
                     np.sin(k * X) * k * np.cos(k * Z),
                     np.sin(k * Y) * k * np.cos(k * X)])
    gp = np.stack([-k * np.sin(k * X) * np.cos(k * Y), -k * np.cos(k * X) * np.sin(k * Y),
                   np.zeros_like(X)])
    u = phi[:, None, None] * s[None]
    p = Pt[:, None] * (np.cos(k * X) * np.cos(k * Y))[None]
    return u, p, s, conv, gp, phi, dphi, Pt


def test_manufactured_solution_consistency():
    """Interior residual rows of the interpolated exact solution of a forced
    time-periodic NS problem vanish as h -> 0 (consistency of every volume
    term: a wrong sign, index or coefficient leaves an O(1) defect)."""
    prm = Params(K=2, period=1.0)
    rho, nu = prm.rho, prm.mu / prm.rho
    w = 2 * np.pi / prm.period
    k = np.pi
    t = spectral.sample_times(prm.K, prm.period)
    errs, errc = [], []
    for n in (4, 8, 16):
        m = cube_mesh(n)
        om = fem.from_mesh(m)
        u, p, s, conv, gp, phi, dphi, Pt = _mms_fields(m.xyz, t, k, w)
        y = np.zeros((4, prm.N, om.n))
        y[:3] = u.transpose(1, 0, 2)
        y[3] = p
        f = (dphi[:, None, None] * s[None] + (phi ** 2)[:, None, None] * conv[None]
             + Pt[:, None, None] * gp[None] / rho + nu * k * k * phi[:, None, None] * s[None])
        f = f.transpose(1, 0, 2)
        r = res.residual_samples(om, prm, y, np.zeros((om.n_outlets, prm.N)), None,
                                 api.H_of(prm), res.Options(body_force=f, backflow=False))
        inner = np.ones(om.n, bool)
        inner[boundary_faces(m.xyz, m.tets).ravel()] = False
        VA = np.zeros(om.n)
        np.add.at(VA, om.tets.ravel(), np.repeat(om.vol / 4.0, 4))
        scale_m = rho * np.sqrt(np.mean(f ** 2))
        errs.append(np.sqrt(np.mean((r[:3][:, :, inner] / VA[inner]) ** 2)) / scale_m)
        errc.append(np.sqrt(np.mean((r[3][:, inner] / VA[inner]) ** 2)) / (k * np.abs(u).max()))
    rate_m = np.log2(errs[1] / errs[2])
    rate_c = np.log2(errc[1] / errc[2])
    assert rate_m > 0.9 and errs[2] < 0.05, (errs, rate_m)
    assert rate_c > 0.9 and errc[2] < 0.05, (errc, rate_c)


def test_backflow_is_dissipative():
    P, om = _c1()
    prm = P.params
    y = _samples(P, om, 6)
    hs = np.zeros((1, prm.N))
    d = _r(om, prm, y, hs, backflow=True) - _r(om, prm, y, hs, backflow=False)
    work = np.einsum("ina,ina->n", y[:3], d[:3])
    assert np.all(work >= -1e-14) and work.max() > 0
    # pure outflow: no backflow contribution
    y2 = y.copy()
    y2[2][:, ~om.dirichlet] = np.abs(y2[2][:, ~om.dirichlet]) + 10.0
    d2 = _r(om, prm, y2, hs, backflow=True) - _r(om, prm, y2, hs, backflow=False)
    assert np.abs(d2).max() == 0.0


def test_resistance_power_identity():
    """With h = -R Q the outlet term does work R Q^2 at every sample."""
    P, om = _c1()
    prm = P.params
    y = _samples(P, om, 7)
    hs = np.zeros((1, prm.N))
    Rv = np.array([2.5])
    d = _r(om, prm, y, hs, Rv, backflow=False) - _r(om, prm, y, hs, None, backflow=False)
    work = np.einsum("ina,ina->n", y[:3], d[:3])
    x = P.mesh.xyz
    of = om.ofaces
    nA = 0.5 * np.cross(x[of[:, 1]] - x[of[:, 0]], x[of[:, 2]] - x[of[:, 0]])
    Q = np.einsum("inf,fi->n", y[:3][:, :, of].mean(axis=3), nA)
    assert np.allclose(work, Rv[0] * Q ** 2, rtol=1e-12, atol=1e-14)


def test_steady_state_has_no_time_coupling():
    """Time-independent samples: H y = 0, so every sample's residual equals
    the K = 0 residual of the same field."""
    P, om = _c1()
    y1 = _samples(P, om, 8)[:, :1]
    yN = np.repeat(y1, P.params.N, axis=1)
    p0 = replace(P.params, K=0)
    r0 = _r(om, p0, y1, np.zeros((1, 1)))
    rN = _r(om, P.params, yN, np.zeros((1, P.params.N)))
    assert np.allclose(rN, np.repeat(r0, P.params.N, axis=1), atol=1e-13 * np.abs(r0).max())
