"""Pins of the oracle's GLS time-marching solver (the paper's comparison
solver of Section 3): the steady limit, second-order convergence of the
marched periodic orbit to the HB orbit of the same semi-discrete system,
the exact step tangent by complex step, and the omega-hat norms."""
import numpy as np
import pytest

from hbinputs.meshes import cylinder_mesh
from hbinputs.problems import Params, poiseuille_dirichlet, womersley_like_flow
from oracle import fem, march, solve, spectral
from oracle import residual as res


@pytest.fixture(scope="module")
def pipe():
    m = cylinder_mesh(1.0, 6.0, 3, 6)
    return m, fem.from_mesh(m)


def test_march_steady_limit(pipe):
    """Constant boundary data: marching from rest ends at the root of the
    steady (K = 0) residual, and omega-hat falls to zero with the
    acceleration."""
    m, om = pipe
    prm = Params(K=0, rho=1.0, mu=1.0)
    d = poiseuille_dirichlet(m, 0, [np.array([1.0])])
    Ys, rep = solve.newton_solve(om, prm, np.zeros((4, 1, om.n)), d, np.zeros((1, 1)), rtol=1e-12)
    assert rep.converged
    ys, a, r = march.march(om, prm, np.zeros((4, om.n)), np.zeros((3, om.n)), 0.2, 30,
                           lambda t: d[:, 0], lambda t: np.zeros(1))
    assert r.omega_hats[0] == 0.0 and r.omega_hats[1] > 1.0
    assert r.omega_hats[-1] < 1e-6
    for f in range(4):
        err = np.linalg.norm(ys[-1][f] - Ys[f, 0]) / np.linalg.norm(Ys[f, 0])
        assert err < 1e-8, (f, err)


def test_marched_orbit_converges_to_hb_orbit_at_second_order(pipe):
    """With omega-hat held at zero and the HB solver's -H N_A test term
    off, both solvers discretise the same semi-discrete system: the
    periodic orbit marched by generalized-alpha (rho_inf = 0, second
    order) must approach the HB orbit as dt^2.  A dropped history term or
    a wrong alpha_m gives first order (ratio 2) or no convergence."""
    m, om = pipe
    K = 2
    prm = Params(K=K, rho=1.0, mu=1.0, period=1.0)
    w = 2 * np.pi / prm.period
    d = poiseuille_dirichlet(m, K, [womersley_like_flow(K)])
    oh = np.zeros((1, prm.N))
    opt = res.Options(stab_test_time=False)
    Y0, _ = solve.plain_start(om, prm, d, oh, rtol=1e-12)
    Y, rep = solve.newton_solve(om, prm, Y0, d, oh, rtol=1e-12, opt=opt)
    assert rep.converged
    errs = []
    for spp in (10, 20):
        dt = prm.period / spp
        ys, _, r = march.march(om, prm, Y0[:, 0].copy(), np.zeros((3, om.n)), dt, 2 * spp,
                               lambda t: march.modal_at(d, K, w, t), lambda t: np.zeros(1),
                               what=0.0, rtol=1e-9, atol=1e-11, eta=1e-5)
        assert r.max_step_residual < 1e-7
        hb = np.stack([march.modal_at(Y, K, w, k * dt) for k in range(spp + 1)])
        last = ys[spp:]                       # second period: the first has washed out
        errs.append(np.array([np.linalg.norm(last[:, f] - hb[:, f]) / np.linalg.norm(hb[:, f])
                              for f in range(4)]))
    ratio = errs[0] / errs[1]
    assert np.all(errs[1] < 2e-2), errs
    assert np.all((ratio > 3.3) & (ratio < 4.7)), ratio


def test_step_tangent_by_complex_step(pipe):
    """tm_jvp is the exact derivative of tm_residual (convection, backflow,
    tau-hat with omega-hat > 0)."""
    m, om = pipe
    prm = Params(K=0, rho=1.06, mu=0.04)
    rng = np.random.default_rng(7)
    d = poiseuille_dirichlet(m, 0, [np.array([3.0])])
    y = rng.standard_normal((4, om.n))
    y[:3][:, om.dirichlet] = d[:, 0][:, om.dirichlet]
    y[2] += 1.0
    u_old = y[:3] + 0.1 * rng.standard_normal((3, om.n))
    a_old = rng.standard_normal((3, om.n))
    v = rng.standard_normal((4, om.n))
    v[:3][:, om.dirichlet] = 0.0
    dt, what, h = 0.05, 2.5, np.array([0.3])
    eps = 1e-30
    rc = march.tm_residual(om, prm, y + 1j * eps * v, u_old, a_old, dt, what, h)
    ref = rc.imag / eps
    jv = march.tm_jvp(om, prm, y, v, u_old, a_old, dt, what)
    err = np.linalg.norm(jv - ref) / np.linalg.norm(ref)
    assert err < 1e-12, err


def test_omega_hat_norms(pipe):
    """Lumped weights sum to the volume; omega-hat of a = c u is |c|, and
    it is zero for a fluid at rest."""
    m, om = pipe
    w = march.nodal_weights(om)
    assert abs(w.sum() - om.vol.sum()) < 1e-12 * om.vol.sum()
    u = np.random.default_rng(3).standard_normal((3, om.n))
    assert abs(march.omega_hat(om, u, -2.5 * u) - 2.5) < 1e-13
    assert march.omega_hat(om, np.zeros((3, om.n)), u) == 0.0


def test_modal_evaluation_matches_inverse_dft():
    """modal_at at the sample times t_n = nT/N equals the oracle's inverse
    real DFT."""
    K = 3
    N = 2 * K + 1
    Y = np.random.default_rng(5).standard_normal((2, N, 4))
    s = spectral.to_samples(Y, K)
    T = 2.0
    for n in range(N):
        q = march.modal_at(Y, K, 2 * np.pi / T, n * T / N)
        assert np.allclose(q, s[:, n], atol=1e-13)
