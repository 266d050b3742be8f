"""HB-GLS residual and its exact directional derivative, time-sample form.

Follows Section 2.3, eq. Rmc, with the GLS operator of Section 2.2
(eq. NS-weak) and tau of eq. tau:

  momentum, A not on the Dirichlet boundary, i = 1..3:
    r^m_Ai = int N_A rho (H u_i + u_j d_j u_i) - d_i N_A p + mu d_j N_A d_j u_i
             - int_{Gamma_h} N_A h n_i
             + sum_el int (-H N_A + u_j d_j N_A) tau L_i
  continuity, every node A:
    r^c_A  = int N_A d_i u_i + sum_el int (1/rho) d_i N_A tau L_i
  with L_i = rho H u_i + rho u_j d_j u_i + d_i p  (the viscous part vanishes
  for linear elements, Section 2.3) and
    tau_n = (u_n . xi u_n + C_I nu^2 xi:xi)^(-1/2)  at every sample n.

H is constant in space, so the stabilisation's -H N_A factor is applied per
node after assembly: the element loop accumulates z_Ai = int N_A tau L_i and
the momentum rows receive -H z_Ai (H is skew-symmetric, Section 2.3).

The backflow term of Section 2.3 adds (w, rho/2 beta |u.n|_- u) to the right
hand side, i.e. the residual receives -int N_A (rho beta/2) min(u.n, 0) u_i
on outlets.  Resistance outlets (outside the paper's scope) use the
time-local h_n = h_given,n - R Q_n with Q_n the outlet flux.

Arrays: y is (4, N, n) samples [u1, u2, u3, p]; the same shape is returned.
Complex input is accepted so that a complex-step derivative can be taken;
the only branch (the sign of u.n) is decided on the real part.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fem import TET_QP, TRI_QP, OMesh

CHUNK = 8192


@dataclass
class Options:
    convection: bool = True       # rho u.grad u, u inside tau, u.grad N_A in the test
    stab_time_terms: bool = True  # rho H u inside L and the -H N_A test term
    backflow: bool = True
    frozen_u: np.ndarray | None = None     # (3, N, n) advecting velocity (Picard-frozen form)
    body_force: np.ndarray | None = None   # (3, N, n) nodal samples of f (manufactured tests)
    stab_test_time: bool = True   # the -H N_A part of the momentum test operator (HB only)
    tau_add: float = 0.0          # added inside tau's bracket (omega-hat^2 of eq. tauhat)


def _scatter(target: np.ndarray, idx: np.ndarray, vals: np.ndarray):
    """target.ravel()[idx] += vals with repeated indices summed."""
    t = target.reshape(-1)
    idx = idx.ravel()
    vals = vals.ravel()
    size = t.size
    if np.iscomplexobj(t):
        t += np.bincount(idx, weights=vals.real, minlength=size)
        t += 1j * np.bincount(idx, weights=vals.imag, minlength=size)
    else:
        t += np.bincount(idx, weights=vals, minlength=size)


def _gather(y3: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """(3, N, n) at element nodes idx (E, k) -> (E, N, k, 3)."""
    return y3[:, :, idx].transpose(2, 1, 3, 0)


def _scatter_vec(target3: np.ndarray, idx: np.ndarray, loc: np.ndarray):
    """target3 (3, N, n) += loc (E, N, k, 3) at nodes idx (E, k)."""
    _, N, n = target3.shape
    i = np.arange(3)[None, None, None, :]
    s = np.arange(N)[None, :, None, None]
    flat = (i * N + s) * n + idx[:, None, :, None]
    _scatter(target3, np.broadcast_to(flat, loc.shape), loc)


def _scatter_scalar(target: np.ndarray, idx: np.ndarray, loc: np.ndarray):
    """target (N, n) += loc (E, N, k) at nodes idx (E, k)."""
    N, n = target.shape
    s = np.arange(N)[None, :, None]
    flat = s * n + idx[:, None, :]
    _scatter(target, np.broadcast_to(flat, loc.shape), loc)


def _select_elements(om: OMesh, rows: np.ndarray | None):
    if rows is None:
        return np.arange(om.ne), np.arange(om.ofaces.shape[0])
    mark = np.zeros(om.n, bool)
    mark[rows] = True
    el = np.nonzero(mark[om.tets].any(axis=1))[0]
    fa = np.nonzero(mark[om.ofaces].any(axis=1))[0] if om.ofaces.size else np.zeros(0, int)
    return el, fa


def outlet_flux(om: OMesh, u3: np.ndarray) -> np.ndarray:
    """Q_k,n = int_{outlet k} u_n . n dGamma (exact for linear u)."""
    N = u3.shape[1]
    Q = np.zeros((om.n_outlets, N), dtype=u3.dtype)
    if om.ofaces.shape[0] == 0:
        return Q
    uf = _gather(u3, om.ofaces).mean(axis=2)                     # (F, N, 3)
    qf = np.einsum("fni,fi->fn", uf, om.onormal) * om.oarea[:, None]
    for n in range(N):
        if np.iscomplexobj(qf):
            Q[:, n] = (np.bincount(om.oid, weights=qf[:, n].real, minlength=om.n_outlets)
                       + 1j * np.bincount(om.oid, weights=qf[:, n].imag, minlength=om.n_outlets))
        else:
            Q[:, n] = np.bincount(om.oid, weights=qf[:, n], minlength=om.n_outlets)
    return Q


def residual_samples(om: OMesh, prm, y: np.ndarray, h_samples: np.ndarray,
                     outlet_R: np.ndarray | None, H: np.ndarray,
                     opt: Options | None = None, rows: np.ndarray | None = None) -> np.ndarray:
    """HB residual r(y) in time samples.  ``y`` must already carry the
    Dirichlet samples.  ``h_samples`` is (n_outlets, N).  If ``rows`` is given,
    only the rows of those nodes are valid in the result."""
    opt = opt or Options()
    rho, mu = prm.rho, prm.mu
    nu = mu / rho
    N, n = y.shape[1], y.shape[2]
    dt = np.result_type(y.dtype, np.float64)
    u3 = y[:3]
    Hu = np.einsum("nk,ika->ina", H, u3)
    adv_u = opt.frozen_u if opt.frozen_u is not None else u3
    rm = np.zeros((3, N, n), dtype=dt)
    rc = np.zeros((N, n), dtype=dt)
    z = np.zeros((3, N, n), dtype=dt)
    el, fa = _select_elements(om, rows)

    for c0 in range(0, el.size, CHUNK):
        e = el[c0:c0 + CHUNK]
        idx = om.tets[e]
        gr, vol, xi, xixi = om.grad[e], om.vol[e], om.xi[e], om.xixi[e]
        U = _gather(u3, idx)                                     # (E,N,4,3)
        UB = _gather(adv_u, idx)
        HU = _gather(Hu, idx)
        P = y[3][:, idx].transpose(1, 0, 2)                      # (E,N,4)
        FB = _gather(opt.body_force, idx) if opt.body_force is not None else None
        G = np.einsum("enai,eaj->enij", U, gr)                   # G_ij = sum_A u_Ai d_j N_A
        g = np.einsum("ena,eai->eni", P, gr)                     # grad p
        d = np.einsum("enii->en", G)
        pbar = P.mean(axis=2)
        lrm = np.zeros(U.shape, dtype=dt)
        lz = np.zeros(U.shape, dtype=dt)
        S = np.zeros(U.shape[:2] + (3,), dtype=dt)
        w = 0.25 * vol[:, None, None]
        for q in range(4):
            Nq = TET_QP[q]
            uq = np.einsum("a,enai->eni", Nq, UB)
            hq = np.einsum("a,enai->eni", Nq, HU)
            fq = np.einsum("a,enai->eni", Nq, FB) if FB is not None else 0.0
            kap = prm.C_I * nu * nu * xixi[:, None] + opt.tau_add
            if opt.convection:
                adv = np.einsum("enj,enij->eni", uq, G)
                kap = kap + np.einsum("eni,eij,enj->en", uq, xi, uq)
                cA = np.einsum("eni,eai->ena", uq, gr)
            else:
                adv = 0.0
                cA = None
            tau = kap ** -0.5
            gal = rho * (hq + adv - fq)
            L = rho * ((hq if opt.stab_time_terms else 0.0) + adv - fq) + g
            s = tau[:, :, None] * L
            lrm += w[..., None] * Nq[None, None, :, None] * gal[:, :, None, :]
            if cA is not None:
                lrm += w[..., None] * cA[..., None] * s[:, :, None, :]
            lz += w[..., None] * Nq[None, None, :, None] * s[:, :, None, :]
            S += w * s
        V = vol[:, None, None, None]
        lrm += V * (mu * np.einsum("eaj,enij->enai", gr, G)
                    - gr[:, None, :, :] * pbar[:, :, None, None])
        lrc = 0.25 * vol[:, None, None] * d[:, :, None] + np.einsum("eai,eni->ena", gr, S) / rho
        _scatter_vec(rm, idx, lrm)
        _scatter_vec(z, idx, lz)
        _scatter_scalar(rc, idx, lrc)

    if om.ofaces.shape[0]:
        h = np.asarray(h_samples, dtype=dt).copy()
        if outlet_R is not None:
            h = h - np.asarray(outlet_R)[:, None] * outlet_flux(om, u3)
        of = om.ofaces[fa]
        nrm, area, oid = om.onormal[fa], om.oarea[fa], om.oid[fa]
        # Neumann: -int N_A h n_i, h constant per outlet and sample
        neu = -(h[oid][:, :, None, None] * nrm[:, None, None, :]
                * (area / 3.0)[:, None, None, None]) * np.ones((1, 1, 3, 1))
        _scatter_vec(rm, of, neu)
        if opt.backflow and opt.convection:
            Uf = _gather(adv_u if opt.frozen_u is not None else u3, of)  # (F,N,3,3)
            bf = np.zeros(Uf.shape, dtype=dt)
            for q in range(3):
                Nq = TRI_QP[q]
                uq = np.einsum("a,fnai->fni", Nq, Uf)
                un = np.einsum("fni,fi->fn", uq, nrm)
                mneg = np.where(un.real < 0, un, 0.0)
                coef = -(area / 3.0)[:, None] * 0.5 * rho * prm.beta_bf * mneg
                bf += coef[:, :, None, None] * Nq[None, None, :, None] * uq[:, :, None, :]
            _scatter_vec(rm, of, bf)

    if opt.stab_time_terms and opt.stab_test_time:
        rm -= np.einsum("nk,ika->ina", H, z)
    rm[:, :, om.dirichlet] = 0.0
    out = np.empty((4, N, n), dtype=dt)
    out[:3] = rm
    out[3] = rc
    return out


def jvp_samples(om: OMesh, prm, y: np.ndarray, v: np.ndarray, h_samples: np.ndarray,
                outlet_R: np.ndarray | None, H: np.ndarray, opt: Options | None = None,
                shift: float = 0.0, rows: np.ndarray | None = None) -> np.ndarray:
    """Exact directional derivative d r(y)[v] written out term by term
    (tangent-linear of residual_samples).  v's Dirichlet velocity samples are
    treated as zero.  ``shift`` adds shift * int N_A N_B v_B,i on velocity
    rows (the pseudo-time term of Section 2.3).  A body force is constant in
    y: it enters only through the strong residual L that d tau and the
    perturbed advective test function multiply."""
    opt = opt or Options()
    if opt.frozen_u is not None:
        raise ValueError("jvp_samples takes the plain residual only")
    rho, mu = prm.rho, prm.mu
    nu = mu / rho
    N, n = y.shape[1], y.shape[2]
    v = np.array(v, dtype=np.float64, copy=True)
    v[:3][:, :, om.dirichlet] = 0.0
    u3, du3 = y[:3], v[:3]
    Hu = np.einsum("nk,ika->ina", H, u3)
    dHu = np.einsum("nk,ika->ina", H, du3)
    rm = np.zeros((3, N, n))
    rc = np.zeros((N, n))
    z = np.zeros((3, N, n))
    el, fa = _select_elements(om, rows)

    for c0 in range(0, el.size, CHUNK):
        e = el[c0:c0 + CHUNK]
        idx = om.tets[e]
        gr, vol, xi, xixi = om.grad[e], om.vol[e], om.xi[e], om.xixi[e]
        U, dU = _gather(u3, idx), _gather(du3, idx)
        HU, dHU = _gather(Hu, idx), _gather(dHu, idx)
        P = y[3][:, idx].transpose(1, 0, 2)
        dP = v[3][:, idx].transpose(1, 0, 2)
        FB = _gather(opt.body_force, idx) if opt.body_force is not None else None
        G = np.einsum("enai,eaj->enij", U, gr)
        dG = np.einsum("enai,eaj->enij", dU, gr)
        g = np.einsum("ena,eai->eni", P, gr)
        dg = np.einsum("ena,eai->eni", dP, gr)
        dd = np.einsum("enii->en", dG)
        dpbar = dP.mean(axis=2)
        lrm = np.zeros(U.shape)
        lz = np.zeros(U.shape)
        dS = np.zeros(U.shape[:2] + (3,))
        w = 0.25 * vol[:, None, None]
        st = 1.0 if opt.stab_time_terms else 0.0
        for q in range(4):
            Nq = TET_QP[q]
            uq = np.einsum("a,enai->eni", Nq, U)
            duq = np.einsum("a,enai->eni", Nq, dU)
            hq = np.einsum("a,enai->eni", Nq, HU)
            dhq = np.einsum("a,enai->eni", Nq, dHU)
            fq = np.einsum("a,enai->eni", Nq, FB) if FB is not None else 0.0
            kap = prm.C_I * nu * nu * xixi[:, None] + opt.tau_add
            if opt.convection:
                adv = np.einsum("enj,enij->eni", uq, G)
                dadv = np.einsum("enj,enij->eni", duq, G) + np.einsum("enj,enij->eni", uq, dG)
                xu = np.einsum("eij,enj->eni", xi, uq)
                kap = kap + np.einsum("eni,eni->en", uq, xu)
                dkap_half = np.einsum("eni,eni->en", xu, duq)       # u . xi du
                cA = np.einsum("eni,eai->ena", uq, gr)
                dcA = np.einsum("eni,eai->ena", duq, gr)
            else:
                adv = dadv = 0.0
                dkap_half = 0.0
                cA = dcA = None
            tau = kap ** -0.5
            dtau = -tau ** 3 * dkap_half
            L = rho * (st * hq + adv - fq) + g
            dL = rho * (st * dhq + dadv) + dg
            s = tau[:, :, None] * L
            ds = (dtau[:, :, None] * L if opt.convection else 0.0) + tau[:, :, None] * dL
            dgal = rho * (dhq + dadv)
            lrm += w[..., None] * Nq[None, None, :, None] * dgal[:, :, None, :]
            if cA is not None:
                lrm += w[..., None] * (dcA[..., None] * s[:, :, None, :]
                                       + cA[..., None] * ds[:, :, None, :])
            lz += w[..., None] * Nq[None, None, :, None] * ds[:, :, None, :]
            dS += w * ds
        V = vol[:, None, None, None]
        lrm += V * (mu * np.einsum("eaj,enij->enai", gr, dG)
                    - gr[:, None, :, :] * dpbar[:, :, None, None])
        if shift != 0.0:
            M = vol[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0
            lrm += shift * np.einsum("eab,enbi->enai", M, dU)
        lrc = 0.25 * vol[:, None, None] * dd[:, :, None] + np.einsum("eai,eni->ena", gr, dS) / rho
        _scatter_vec(rm, idx, lrm)
        _scatter_vec(z, idx, lz)
        _scatter_scalar(rc, idx, lrc)

    if om.ofaces.shape[0]:
        of = om.ofaces[fa]
        nrm, area, oid = om.onormal[fa], om.oarea[fa], om.oid[fa]
        if outlet_R is not None:
            dh = -np.asarray(outlet_R)[:, None] * outlet_flux(om, du3)
            neu = -(dh[oid][:, :, None, None] * nrm[:, None, None, :]
                    * (area / 3.0)[:, None, None, None]) * np.ones((1, 1, 3, 1))
            _scatter_vec(rm, of, neu)
        if opt.backflow and opt.convection:
            Uf, dUf = _gather(u3, of), _gather(du3, of)
            bf = np.zeros(Uf.shape)
            for q in range(3):
                Nq = TRI_QP[q]
                uq = np.einsum("a,fnai->fni", Nq, Uf)
                duq = np.einsum("a,fnai->fni", Nq, dUf)
                un = np.einsum("fni,fi->fn", uq, nrm)
                dun = np.einsum("fni,fi->fn", duq, nrm)
                neg = un < 0
                dterm = (np.where(neg, dun, 0.0)[:, :, None] * uq
                         + np.where(neg, un, 0.0)[:, :, None] * duq)
                coef = -(area / 3.0)[:, None, None] * 0.5 * rho * prm.beta_bf
                bf += (coef * dterm)[:, :, None, :] * Nq[None, None, :, None]
            _scatter_vec(rm, of, bf)

    if opt.stab_time_terms and opt.stab_test_time:
        rm -= np.einsum("nk,ika->ina", H, z)
    rm[:, :, om.dirichlet] = 0.0
    out = np.empty((4, N, n))
    out[:3] = rm
    out[3] = rc
    return out
