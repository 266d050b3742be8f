"""Pins of the oracle's Jacobian-vector products and Jacobi diagonal."""
import numpy as np
import pytest

from hbinputs.meshes import cylinder_mesh
from hbinputs.problems import Params, c1_womersley, poiseuille_dirichlet, seeded_state, womersley_like_flow
from oracle import api, fem, spectral, tangent
from oracle import residual as res


def _setup(K=2, R=None, small=False):
    if small:
        from hbinputs.problems import Problem
        m = cylinder_mesh(1.0, 6.0, 2, 4)
        prm = Params(K=K)
        P = Problem("tiny", m, prm, poiseuille_dirichlet(m, K, [womersley_like_flow(K)]),
                    np.zeros((1, prm.N)), R, u_ref=2 / np.pi)
    else:
        P = c1_womersley(K=K)
        P.outlet_R = R
    om = fem.from_mesh(P.mesh)
    return P, om


def _yv(P, om, s=0):
    y = api.samples_of(om, P.params, seeded_state(P, s), P.dirichlet)
    v = spectral.to_samples(seeded_state(P, s + 100), P.params.K)
    v[:3][:, :, om.dirichlet] = 0.0
    return y, v


@pytest.mark.parametrize("R", [None, np.array([3.0])])
def test_exact_jvp_matches_complex_step(R):
    P, om = _setup(R=R)
    prm = P.params
    y, v = _yv(P, om)
    hs = np.random.default_rng(1).normal(size=(1, prm.N))
    H = api.H_of(prm)
    jv = res.jvp_samples(om, prm, y, v, hs, R, H)
    eps = 1e-30
    cs = res.residual_samples(om, prm, y + 1j * eps * v, hs, R, H).imag / eps
    assert np.linalg.norm(cs - jv) <= 1e-13 * np.linalg.norm(jv)


def test_exact_jvp_matches_central_difference():
    P, om = _setup(R=np.array([1.0]))
    prm = P.params
    y, v = _yv(P, om, 3)
    hs = np.zeros((1, prm.N))
    H = api.H_of(prm)
    jv = res.jvp_samples(om, prm, y, v, hs, P.outlet_R, H)
    eps = 1e-6 * np.linalg.norm(y) / np.linalg.norm(v)
    rp = res.residual_samples(om, prm, y + eps * v, hs, P.outlet_R, H)
    rm = res.residual_samples(om, prm, y - eps * v, hs, P.outlet_R, H)
    fd = (rp - rm) / (2 * eps)
    assert np.linalg.norm(fd - jv) <= 1e-7 * np.linalg.norm(jv)


def test_backflow_branch_exercised():
    """The seeded state has inflow through part of the outlet, so the kink
    of min(u.n, 0) is on both sides across the outlet faces."""
    P, om = _setup()
    y, _ = _yv(P, om)
    un = np.einsum("inf,fi->nf", y[:3][:, :, om.ofaces].mean(axis=3), om.onormal)
    assert (un < 0).any() and (un > 0).any()


def test_shift_is_consistent_mass():
    P, om = _setup()
    prm = P.params
    y, v = _yv(P, om, 5)
    H = api.H_of(prm)
    hs = np.zeros((1, prm.N))
    a = res.jvp_samples(om, prm, y, v, hs, None, H, shift=2.0)
    b = res.jvp_samples(om, prm, y, v, hs, None, H)
    # int N_A N_B assembled independently: row sums give int N_A = V/4 per element
    d = (a - b)[:3] / 2.0
    ones = np.zeros_like(v)
    ones[:3][:, :, ~om.dirichlet] = 1.0
    e = res.jvp_samples(om, prm, y, ones, hs, None, H, shift=1.0) - res.jvp_samples(
        om, prm, y, ones, hs, None, H)
    VA = np.zeros(om.n)
    np.add.at(VA, om.tets.ravel(), np.repeat(om.vol / 4.0, 4))
    # interior nodes whose neighbours are all free: lumped row sum = int N_A
    free_nb = np.ones(om.n, bool)
    bad = om.tets[om.dirichlet[om.tets].any(axis=1)].ravel()
    free_nb[bad] = False
    assert free_nb.sum() > 0
    assert np.allclose(e[0][:, free_nb], VA[free_nb][None], rtol=1e-12)
    assert np.allclose(d[:, :, om.dirichlet], 0.0)


def test_paper_tangent_is_picard_derivative():
    """(C + P) v equals the complex-step derivative of the residual with the
    advecting velocity and tau frozen at y and the stabilisation's time
    terms removed (eq. K_mat and eq. ctangent)."""
    P, om = _setup(small=True)
    prm = P.params
    y, v = _yv(P, om, 7)
    H = api.H_of(prm)
    hs = np.zeros((1, prm.N))
    pj = api.paper_jvp_samples(om, prm, y, v)
    eps = 1e-30
    opt = res.Options(stab_time_terms=False, backflow=False, frozen_u=y[:3].copy())
    cs = res.residual_samples(om, prm, y + 1j * eps * v, hs, None, H, opt).imag / eps
    assert np.linalg.norm(cs - pj) <= 1e-13 * np.linalg.norm(pj)


def test_paper_equals_exact_at_rest_without_time_stabilisation():
    P, om = _setup(small=True)
    prm = P.params
    y = np.zeros((4, prm.N, om.n))
    _, v = _yv(P, om, 9)
    H = api.H_of(prm)
    opt = res.Options(stab_time_terms=False, backflow=False)
    ex = res.jvp_samples(om, prm, y, v, np.zeros((1, prm.N)), None, H, opt)
    pj = api.paper_jvp_samples(om, prm, y, v)
    assert np.linalg.norm(ex - pj) <= 1e-13 * np.linalg.norm(ex)


def test_jacobi_diagonal_by_probing():
    """diag(P + shift M_v) probed entry by entry with unit vectors through
    the frozen-residual derivative."""
    P, om = _setup(small=True)
    prm = P.params
    y, _ = _yv(P, om, 11)
    H = api.H_of(prm)
    shift = 3.0
    dg = tangent.jacobi_diagonal(om, prm, y, shift)
    opt = res.Options(stab_time_terms=False, backflow=False, frozen_u=y[:3].copy())
    rng = np.random.default_rng(0)
    free = np.nonzero(~om.dirichlet)[0]
    M = fem.consistent_mass_local(om.vol)
    for trial in range(12):
        f = int(rng.integers(0, 4))
        s = int(rng.integers(0, prm.N))
        a = int(rng.choice(free))
        e = np.zeros((4, prm.N, om.n))
        e[f, s, a] = 1.0
        col = res.residual_samples(om, prm, y + 1j * 1e-30 * e, np.zeros((1, prm.N)), None, H,
                                   opt).imag / 1e-30
        val = col[f, s, a]
        if f < 3:
            mass = sum(M[t, list(om.tets[t]).index(a), list(om.tets[t]).index(a)]
                       for t in np.nonzero((om.tets == a).any(axis=1))[0])
            # the time-diagonal part excludes F = H int rho N N, whose diagonal is 0
            assert abs(val + shift * mass - dg[0, s, a]) <= 1e-12 * abs(dg[0, s, a])
        else:
            assert abs(val - dg[1, s, a]) <= 1e-12 * abs(dg[1, s, a])
    assert np.all(dg[0][:, om.dirichlet] == 1.0)
