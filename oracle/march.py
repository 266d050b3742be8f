"""GLS time marching of the same semi-discrete equations (the paper's
comparison solver).  Test infrastructure: only tests and the benchmark's
CPU leg use this module.

Section 3 compares the HB solver with a time-stepping solver that keeps the
same Galerkin/least-squares terms and replaces tau by tau-hat of eq. tauhat,
whose extra omega-hat^2 = (||du/dt|| / ||u||)^2 accounts for the
acceleration.  The time derivative is integrated by the generalized-alpha
method for first-order systems (Jansen, Whiting and Hulbert, cited in
Section 2.3 for the pseudo-time term) with rho_inf = 0: alpha_m = 3/2,
alpha_f = 1, gamma = 1, so the tangent carries c1 rho/dt int N_A N_B with
c1 = alpha_m/gamma = 1.5 as in Section 2.3.  One step solves r = 0 for
(u_{n+1}, p_{n+1}) with the acceleration

    a := (c1/dt) (u_{n+1} - u_n) + (1 - c1) a_n

in place of H u, then sets a_{n+1} = (u_{n+1} - u_n)/(gamma dt)
- ((1 - gamma)/gamma) a_n.

Readings where the paper is silent:
* the semi-discrete test functions do not depend on time, so the momentum
  stabilisation test operator is u.grad N_A alone (the HB solver's -H N_A
  has no analogue); the acceleration stays inside the strong residual L;
* omega-hat is taken from the state at the start of each step and held
  fixed during its Newton iterations; the norms are lumped-mass L2 norms of
  the velocity (nodal weight = sum of V/4 over the node's tetrahedra), and
  omega-hat = 0 when ||u|| = 0;
* the boundary data and the outlet traction are taken at t_{n+1}
  (alpha_f = 1); Dirichlet nodes follow the same update as the interior.

The residual is the HB oracle's residual_samples at N = 1 with
H = [[c1/dt]] and the step's history c1/dt u_n + (c1 - 1) a_n passed as a
nodal body force, so every spatial term is the one the HB oracle pins.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import residual as res
from . import tangent
from .fem import OMesh

ALPHA_M = 1.5
GAMMA = 1.0
C1 = ALPHA_M / GAMMA


def nodal_weights(om: OMesh) -> np.ndarray:
    """Lumped mass: sum over the node's tetrahedra of V/4."""
    return np.bincount(om.tets.ravel(), weights=np.repeat(om.vol / 4.0, 4), minlength=om.n)


def omega_hat(om: OMesh, u3: np.ndarray, a3: np.ndarray) -> float:
    """||a|| / ||u|| with lumped-mass L2 norms of the velocity (eq. tauhat)."""
    w = nodal_weights(om)
    nu = float(np.sum(w * np.sum(u3 ** 2, axis=0)))
    na = float(np.sum(w * np.sum(a3 ** 2, axis=0)))
    return 0.0 if nu <= 0.0 else float(np.sqrt(na / nu))


def modal_at(coef: np.ndarray, K: int, omega: float, t: float) -> np.ndarray:
    """q(t) = a0 + sum_m a_m cos(m w t) + b_m sin(m w t); modes on axis -2
    in the order [a0, a1, b1, ..., aK, bK]."""
    b = np.ones(2 * K + 1)
    for m in range(1, K + 1):
        b[2 * m - 1] = np.cos(m * omega * t)
        b[2 * m] = np.sin(m * omega * t)
    return np.tensordot(coef, b, axes=([coef.ndim - 2], [0]))


def _options(dt: float, what: float, body=None) -> res.Options:
    return res.Options(stab_test_time=False, tau_add=what * what, body_force=body)


def tm_residual(om: OMesh, prm, y_new: np.ndarray, u_old: np.ndarray, a_old: np.ndarray,
                dt: float, what: float, h: np.ndarray, outlet_R=None) -> np.ndarray:
    """Residual (4, n) of one step at the candidate (u_{n+1}, p_{n+1}) = y_new
    (4, n), which must already carry the Dirichlet values of t_{n+1}.
    ``h`` is the outlet traction at t_{n+1} (n_outlets,)."""
    H = np.array([[C1 / dt]])
    hist = (C1 / dt) * u_old + (C1 - 1.0) * a_old
    r = res.residual_samples(om, prm, y_new[:, None, :], np.asarray(h, float)[:, None],
                             outlet_R, H, _options(dt, what, hist[:, None, :]))
    return r[:, 0]


def tm_jvp(om: OMesh, prm, y_new: np.ndarray, v: np.ndarray, u_old: np.ndarray,
           a_old: np.ndarray, dt: float, what: float, outlet_R=None) -> np.ndarray:
    """Exact derivative of tm_residual at y_new along v (4, n); v's Dirichlet
    velocity entries are treated as zero."""
    H = np.array([[C1 / dt]])
    hist = (C1 / dt) * u_old + (C1 - 1.0) * a_old
    out = res.jvp_samples(om, prm, y_new[:, None, :], v[:, None, :], np.zeros((om.n_outlets, 1)),
                          outlet_R, H, _options(dt, what, hist[:, None, :]))
    return out[:, 0]


@dataclass
class MarchReport:
    steps: int = 0
    newton_iters: int = 0
    gmres_iters: int = 0
    max_step_residual: float = 0.0
    omega_hats: list = field(default_factory=list)


def tm_step(om: OMesh, prm, y_old: np.ndarray, a_old: np.ndarray, dt: float, what: float,
            g_new: np.ndarray, h_new: np.ndarray, outlet_R=None, *, atol=1e-10, rtol=1e-10,
            eta=1e-6, max_newton=20, report: MarchReport | None = None):
    """One generalized-alpha step: returns (y_{n+1}, a_{n+1}).  Newton on the
    step residual (exact tangent, GMRES preconditioned by a sparse LU of the
    paper's tangent P + C + c1 rho/dt M) from the previous state, until
    ||r|| <= max(atol, rtol ||r_0||)."""
    mask = om.dirichlet
    y = np.array(y_old, dtype=float, copy=True)
    y[:3][:, mask] = g_new[:, mask]
    u_old = y_old[:3]

    def R(yy):
        return tm_residual(om, prm, yy, u_old, a_old, dt, what, h_new, outlet_R)

    mflat = tangent.dirichlet_masks(om, 1).ravel()
    r = R(y)
    r0 = rn = float(np.linalg.norm(r))
    for it in range(max_newton):
        if rn <= max(atol, rtol * r0):
            break

        def mv(v, y=y):
            out = tm_jvp(om, prm, y, v.reshape(y.shape), u_old, a_old, dt, what,
                         outlet_R).ravel()
            out[mflat] = v[mflat]
            return out

        A = spla.LinearOperator((y.size, y.size), matvec=mv, dtype=float)
        P = tangent.masked(tangent.assemble_paper_tangent(om, prm, y[:, None, :],
                                                          np.zeros((1, 1)),
                                                          prm.rho * C1 / dt),
                           mflat, True)
        lu = spla.splu(P.tocsc())
        M = spla.LinearOperator((y.size, y.size), matvec=lu.solve, dtype=float)
        b = -r.ravel()
        b[mflat] = 0.0
        count = [0]

        def cb(_x):
            count[0] += 1
        dx, _ = spla.gmres(A, b, rtol=eta, restart=50, maxiter=500, M=M, callback=cb,
                           callback_type="pr_norm")
        y = y + dx.reshape(y.shape)
        r = R(y)
        rn = float(np.linalg.norm(r))
        if report is not None:
            report.newton_iters += 1
            report.gmres_iters += count[0]
    if report is not None:
        report.steps += 1
        report.max_step_residual = max(report.max_step_residual, rn)
    a_new = (y[:3] - u_old) / (GAMMA * dt) - ((1.0 - GAMMA) / GAMMA) * a_old
    return y, a_new


def march(om: OMesh, prm, y0: np.ndarray, a0: np.ndarray, dt: float, n_steps: int,
          g_of_t, h_of_t, outlet_R=None, *, t0: float = 0.0, what=None, **kw):
    """March n_steps from (y0, a0) at t0.  ``g_of_t(t)`` gives the Dirichlet
    velocity (3, n), ``h_of_t(t)`` the outlet traction (n_outlets,).
    ``what`` = None takes omega-hat from each step's starting state; a number
    holds it fixed.  Returns (states (n_steps+1, 4, n), final a, report)."""
    rep = MarchReport()
    ys = [np.array(y0, dtype=float)]
    y, a = ys[0], np.array(a0, dtype=float)
    for k in range(n_steps):
        t1 = t0 + (k + 1) * dt
        w = omega_hat(om, y[:3], a) if what is None else float(what)
        rep.omega_hats.append(w)
        y, a = tm_step(om, prm, y, a, dt, w, g_of_t(t1), h_of_t(t1), outlet_R, report=rep, **kw)
        ys.append(y)
    return np.stack(ys), a, rep
