"""Pins of the oracle's HB solution: per-mode frequency-domain solves in
the linear limit, brute-force time marching, Womersley's closed form and
the steady limit."""
from dataclasses import replace

import numpy as np
import pytest

import pinlib
from hbinputs.meshes import cylinder_mesh
from hbinputs.problems import Params, poiseuille_dirichlet, seeded_state
from hbinputs.problems import Problem
from oracle import api, fem, solve, spectral
from oracle import residual as res

LINEAR = dict(convection=False, backflow=False)


def _pipe(n_rings, n_z, K, flows, period=1.0, h=None):
    m = cylinder_mesh(1.0, 6.0, n_rings, n_z)
    prm = Params(K=K, period=period)
    d = poiseuille_dirichlet(m, K, [np.asarray(flows, float)])
    oh = np.zeros((1, prm.N)) if h is None else np.asarray(h, float)[None]
    return Problem("pipe", m, prm, d, oh, None, u_ref=2 / np.pi), fem.from_mesh(m)


def _complex_mode(a, m):
    return a[..., 0, :] + 0j if m == 0 else 0.5 * (a[..., 2 * m - 1, :] - 1j * a[..., 2 * m, :])


def test_linear_limit_matches_per_mode_frequency_solves():
    K = 2
    P, om = _pipe(3, 6, K, [1.0, 0.3, 0.5, -0.2, 0.1], period=2.0,
                  h=[0.5, 0.1, -0.2, 0.05, 0.3])
    prm = P.params
    # linear problem: one undamped Newton step solves it to the GMRES tolerance
    Y, rep = solve.newton_solve(om, prm, np.zeros((4, prm.N, om.n)), P.dirichlet, P.outlet_h,
                                rtol=1e-11, eta=1e-11, max_gmres=4000, cfl=1e12,
                                opt=res.Options(**LINEAR))
    assert rep.converged
    blocks = pinlib.stokes_blocks(P.mesh.xyz, om.tets, prm.mu, prm.rho, prm.C_I)
    load = pinlib.outlet_load(P.mesh.xyz, om.ofaces, om.onormal, om.n)
    w = 2 * np.pi / prm.period
    ref = np.zeros_like(Y)
    for m in range(K + 1):
        g = _complex_mode(P.dirichlet, m) * om.dirichlet[None]
        h = complex(_complex_mode(P.outlet_h[0][:, None], m)[0])
        x = pinlib.solve_mode(blocks, 1j * m * w, prm.mu, prm.rho, om.dirichlet, g, h, load)
        if m == 0:
            ref[:, 0] = x.real
        else:
            ref[:, 2 * m - 1] = 2 * x.real
            ref[:, 2 * m] = -2 * x.imag
    for f in range(4):
        err = np.linalg.norm(Y[f] - ref[f]) / np.linalg.norm(ref[f])
        assert err < 1e-9, (f, err)


def test_time_marching_reproduces_hb_orbit():
    """Linear limit with the stabilisation's time terms off: the HB samples
    are the exact periodic orbit of a linear index-1 DAE; BDF2 marching
    from that orbit stays on it to O(dt^2)."""
    K = 2
    P, om = _pipe(2, 4, K, [1.0, 0.4, 0.6, 0.0, -0.3], h=[0.2, 0.0, 0.1, -0.1, 0.0])
    prm = P.params
    opt = res.Options(stab_time_terms=False, **LINEAR)
    Y, rep = solve.newton_solve(om, prm, np.zeros((4, prm.N, om.n)), P.dirichlet, P.outlet_h,
                                rtol=1e-12, eta=1e-12, max_gmres=4000, opt=opt)
    assert rep.converged
    w = 2 * np.pi / prm.period
    blocks = pinlib.stokes_blocks(P.mesh.xyz, om.tets, prm.mu, prm.rho, prm.C_I)
    load = pinlib.outlet_load(P.mesh.xyz, om.ofaces, om.onormal, om.n)

    def series(a, t):
        out = a[..., 0, :].copy()
        for m in range(1, K + 1):
            out = out + a[..., 2 * m - 1, :] * np.cos(m * w * t) + a[..., 2 * m, :] * np.sin(m * w * t)
        return out

    def g_of_t(t):
        return series(P.dirichlet, t) * om.dirichlet[None]

    def h_of_t(t):
        return float(series(P.outlet_h[0][:, None], t)[0])

    ysamp = spectral.to_samples(Y, K)
    errs = []
    for per in (100, 200):
        nst = prm.N * per
        dt = prm.period / nst
        traj = pinlib.march_bdf2(blocks, prm.mu, prm.rho, om.dirichlet, g_of_t, h_of_t, load,
                                 series(Y, 0.0), series(Y, dt), dt, nst)
        got = np.stack([traj[s * per] for s in range(prm.N)], axis=1)     # (4, N, n)
        errs.append(np.linalg.norm(got[:3] - ysamp[:3]) / np.linalg.norm(ysamp[:3]))
    assert errs[1] < 1e-4, errs
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


@pytest.mark.slow
def test_womersley_convergence():
    """alpha = 4 pipe (T = 2 pi rho/(16 mu)), exact Womersley inflow, zero
    traction, no slip: the nodal velocity error of the full HB-GLS solution
    falls at order >= 1.5 under mesh refinement, and its divergence (P-div)
    falls at order >= 0.9 relative to the velocity gradient."""
    K = 1
    rho, mu = 1.06, 0.04
    omega = 16.0 * mu / rho                 # alpha = R sqrt(omega/nu) = 4
    period = 2 * np.pi / omega
    q = np.array([1.0, 0.0, 0.5])           # Q = 1 + 0.5 sin(w t)
    errs, hs, divs = [], [], []
    for nr, nz in ((2, 4), (4, 8), (8, 16)):
        m = cylinder_mesh(1.0, 6.0, nr, nz)
        prm = Params(K=K, period=period, rho=rho, mu=mu)
        om = fem.from_mesh(m)
        uz, p = pinlib.womersley_modal(m.xyz, K, 1.0, 6.0, omega, mu, rho, q)
        d = np.zeros((3, prm.N, om.n))
        d[2] = uz * om.dirichlet[None]
        d[2][:, om.dirichlet & ~om.inlet] = 0.0
        Y, rep = solve.newton_solve(om, prm, np.zeros((4, prm.N, om.n)), d, np.zeros((1, prm.N)),
                                    rtol=1e-9, eta=1e-3, cfl=50.0)
        assert rep.converged
        ex = np.zeros((3, prm.N, om.n))
        ex[2] = uz
        errs.append(np.linalg.norm(Y[:3] - ex) / np.linalg.norm(ex))
        hs.append(1.0 / nr)
        # P-div: the discrete divergence (constant per tet for P1 velocity,
        # gradients from face normals) in the volume-weighted L2 norm over
        # the modes, relative to the velocity gradient's norm
        G, V = pinlib._tet_grads(m.xyz, m.tets)
        U = Y[:3][:, :, m.tets]                          # (3, N, E, 4)
        div = np.einsum("eai,inea->ne", G, U)
        grad = np.einsum("eai,jnea->neij", G, U)
        divs.append(np.sqrt(np.sum(V * div ** 2) / np.sum(V[None, :, None, None] * grad ** 2)))
    rates = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(2.0)
    assert rates[-1] >= 1.5, (errs, rates)
    assert errs[-1] < 0.05, errs
    # the PSPG-stabilised P1-P1 velocity is not pointwise divergence free; its
    # divergence falls with h (at least first order relative to the gradient)
    drates = np.log(np.array(divs[:-1]) / np.array(divs[1:])) / np.log(2.0)
    print("velocity error", errs, "divergence", divs, "rates", rates, drates)
    assert np.all(drates >= 0.9), (divs, drates)


def test_steady_boundary_data_give_time_independent_solution():
    """K > 0 with mode-0-only boundary data: the HB root has identical
    samples, equal to the K = 0 (steady) root."""
    K = 2
    P, om = _pipe(2, 4, K, [1.0, 0, 0, 0, 0])
    prm = P.params
    Y0 = seeded_state(P, 3, noise=0.05)
    Y, rep = solve.newton_solve(om, prm, Y0, P.dirichlet, P.outlet_h, rtol=1e-12, eta=1e-6)
    assert rep.converged
    p0 = replace(prm, K=0)
    Ys, rep0 = solve.newton_solve(om, p0, np.zeros((4, 1, om.n)), P.dirichlet[:, :1],
                                  P.outlet_h[:, :1], rtol=1e-12, eta=1e-6)
    assert rep0.converged
    scale = np.abs(Ys).max()
    assert np.abs(Y[:, 1:]).max() < 1e-9 * scale
    assert np.abs(Y[:, 0] - Ys[:, 0]).max() < 1e-9 * scale


def test_newton_converges_fast_near_root():
    K = 1
    P, om = _pipe(2, 4, K, [1.0, 0.2, 0.5])
    prm = P.params
    Y, rep = solve.newton_solve(om, prm, np.zeros((4, prm.N, om.n)), P.dirichlet, P.outlet_h,
                                rtol=1e-12, eta=1e-10, cfl=1e6)
    assert rep.converged and rep.newton_iters <= 8, rep.history
    r = api.residual_modal(om, prm, Y, P.dirichlet, P.outlet_h)
    assert api.sample_norm(r, K) <= 1e-12 * rep.r0


def test_k0_matches_independent_steady_solver():
    """K = 0: the oracle's HB solve is the steady GLS Navier-Stokes solve.
    It matches an independently written steady solver (face-normal basis
    gradients, its own assembly, finite-difference Jacobian, sparse direct
    Newton) at Re ~ 50 with a traction outlet."""
    P, om = _pipe(2, 5, 0, [1.6], h=[300.0])
    prm = P.params
    Y, rep = solve.newton_solve(om, prm, np.zeros((4, 1, om.n)), P.dirichlet, P.outlet_h,
                                rtol=1e-12, eta=1e-8, max_gmres=4000)
    assert rep.converged
    g = P.dirichlet[:, 0].T
    u, p, hist = pinlib.steady_gls_solve(P.mesh.xyz, om.tets, prm.mu, prm.rho, prm.C_I,
                                         om.dirichlet, g, om.ofaces, om.onormal, om.oarea,
                                         float(P.outlet_h[0, 0]), prm.beta_bf)
    assert hist[-1] <= 1e-11 * hist[0], hist
    ref = np.concatenate([u.T, p[None]])
    got = Y[:, 0]
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
    # a real convective case: the Stokes answer differs
    assert np.abs(u[:, 2]).max() > 0.5
