"""Newton-Raphson with pseudo-time continuation and GMRES, time-sample form.

Section 2.3, eq. NR: y <- y - L^{-1} r.  The linear systems are solved by
GMRES (Saad and Schultz) to a relative tolerance of 0.03 (Section 3); the
pseudo-time term c1 rho/dt int N_A N_B (c1 = 1.5 for rho_inf = 0) is added
to the velocity block of the tangent only, so the converged root is the
root of the HB residual.  The pseudo step starts from the CFL rule
dt = CFL h_c/u_c with h_c the edge of the regular tetrahedron of mean
element volume and u_c the mean inlet speed at peak flow, and grows by
switched evolution relaxation dt <- dt ||r_old||/||r_new||.

The oracle takes the exact tangent-linear for the Krylov operator and
preconditions GMRES with a sparse LU factorisation of the assembled paper
tangent C + P + shift M (of its time-diagonal part P + shift M alone on
large systems); the preconditioner changes the iteration count, not the
root.  Convergence: ||r||_2 <= rtol * r_ref with the time-sample 2-norm.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import residual as res
from . import spectral, tangent
from .api import H_of, apply_dirichlet_modal, h_samples
from .fem import OMesh


@dataclass
class SolveReport:
    newton_iters: int = 0
    gmres_iters: int = 0
    r0: float = 0.0
    r_final: float = 0.0
    history: list = field(default_factory=list)
    converged: bool = False


def pseudo_dt0(om: OMesh, prm, dirichlet, cfl: float) -> float:
    vbar = float(np.mean(om.vol))
    hc = (6.0 * np.sqrt(2.0) * vbar) ** (1.0 / 3.0)
    sel = om.inlet & ~_wall_nodes(om)
    if not np.any(sel):
        return cfl * hc
    g = spectral.to_samples(dirichlet[:, :, sel], prm.K)        # (3, N, m)
    speed = np.sqrt(np.sum(g ** 2, axis=0)).mean(axis=1)          # (N,)
    uc = max(float(speed.max()), 1e-30)
    return cfl * hc / uc


def _wall_nodes(om: OMesh) -> np.ndarray:
    return om.dirichlet & ~om.inlet


def newton_solve(om: OMesh, prm, Y0, dirichlet, outlet_h, outlet_R=None, *, rtol=1e-8,
                 r_ref: float | None = None, eta=0.03, restart=50, cfl=1.0, c1=1.5,
                 max_newton=60, max_gmres=2000, opt: res.Options | None = None,
                 verbose: bool = False, full_lu_max: int = 24000):
    """Returns (Y_modal, report)."""
    K, N, n = prm.K, prm.N, om.n
    H = H_of(prm)
    hs = h_samples(prm, outlet_h)
    y = spectral.to_samples(apply_dirichlet_modal(om, Y0, dirichlet), K)
    mask = tangent.dirichlet_masks(om, N).ravel()
    shape = y.shape

    def R(yy):
        return res.residual_samples(om, prm, yy, hs, outlet_R, H, opt)

    r = R(y)
    rn = float(np.linalg.norm(r))
    rep = SolveReport(r0=rn)
    ref = rn if r_ref is None else float(r_ref)
    dt = pseudo_dt0(om, prm, dirichlet, cfl)
    dt0 = dt
    rep.history.append(rn)
    for it in range(max_newton):
        if rn <= rtol * ref:
            rep.converged = True
            break
        shift = c1 * prm.rho / dt

        def mv(v, y=y, shift=shift):
            vv = v.reshape(shape)
            out = res.jvp_samples(om, prm, y, vv, hs, outlet_R, H, opt, shift=shift).ravel()
            out[mask] = v[mask]
            return out

        A = spla.LinearOperator((y.size, y.size), matvec=mv, dtype=float)
        P = tangent.masked(tangent.assemble_paper_tangent(om, prm, y, H, shift,
                                                          include_C=y.size <= full_lu_max),
                           mask, True)
        lu = spla.splu(P.tocsc())
        M = spla.LinearOperator((y.size, y.size), matvec=lu.solve, dtype=float)
        b = -r.ravel()
        b[mask] = 0.0
        count = [0]

        def cb(_x):
            count[0] += 1
        dx, info = spla.gmres(A, b, rtol=eta, restart=restart, maxiter=max_gmres, M=M,
                              callback=cb, callback_type="pr_norm")
        rep.gmres_iters += count[0]
        y = y + dx.reshape(shape)
        r = R(y)
        rn_new = float(np.linalg.norm(r))
        dt = min(dt * rn / max(rn_new, 1e-300), 1e6 * dt0)
        rn = rn_new
        rep.newton_iters = it + 1
        rep.history.append(rn)
        if verbose:
            print(f"  newton {it + 1}: |r| = {rn:.3e} gmres {count[0]} dt {dt:.3e}", flush=True)
    else:
        rep.converged = rn <= rtol * ref
    rep.r_final = rn
    return spectral.to_modal(y, K), rep


def plain_start(om: OMesh, prm, dirichlet, outlet_h, outlet_R=None, **kw):
    """Steady (K = 0) solve with the mode-0 boundary data, broadcast to all
    harmonics as the mean mode (the plain initial guess)."""
    from dataclasses import replace
    p0 = replace(prm, K=0)
    d0 = dirichlet[:, :1]
    h0 = np.asarray(outlet_h)[:, :1]
    Y0 = np.zeros((4, 1, om.n))
    Ys, rep = newton_solve(om, p0, Y0, d0, h0, outlet_R, **kw)
    Y = np.zeros((4, prm.N, om.n))
    Y[:, 0] = Ys[:, 0]
    return Y, rep
