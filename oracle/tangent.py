"""The paper's approximate tangent L = C + P and its Jacobi diagonal,
assembled as a sparse matrix over the time-sample unknowns.

Section 2.3, eq. splitK/ptangent/K_mat: P holds, for every sample n, the
blocks (frozen advecting velocity u and frozen tau)
  K_AB   = int rho N_A u.grad N_B + mu grad N_A . grad N_B
           + sum_el int (u.grad N_A) rho tau (u.grad N_B)
  G_AB,i = -int d_i N_A N_B + sum_el int (u.grad N_A) tau d_i N_B
  D_AB,j =  int N_A d_j N_B + sum_el int d_j N_A tau (u.grad N_B)
  L_AB   =  sum_el int (1/rho) d_k N_A tau d_k N_B
all diagonal in time.  Eq. ctangent/F_mat: C = diag(F, F, F, 0) with
F_AB = H int rho N_A N_B (stabilisation contributions to C are dropped).
The pseudo-time term adds c1 rho/dt int N_A N_B to K (given here as
``shift``).  The preconditioner is diag(P) (Section 2.3: C has a zero
diagonal).

Unknown ordering: flat index (f N + n) n_nodes + A, f in (u1, u2, u3, p).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import TET_QP, OMesh
from .residual import _gather

CHUNK = 4096


def _local_blocks(om: OMesh, prm, e, ub3):
    """Per element and sample: K (E,N,4,4), G (E,N,4,4,3), D (E,N,4,4,3),
    L (E,N,4,4), with ub3 the (3, N, n) advecting velocity."""
    rho, mu = prm.rho, prm.mu
    nu = mu / rho
    idx = om.tets[e]
    gr, vol, xi, xixi = om.grad[e], om.vol[e], om.xi[e], om.xixi[e]
    UB = _gather(ub3, idx)                                       # (E,N,4,3)
    E, N = UB.shape[:2]
    w = 0.25 * vol[:, None]
    K = np.zeros((E, N, 4, 4))
    G = np.zeros((E, N, 4, 4, 3))
    D = np.zeros((E, N, 4, 4, 3))
    L = np.zeros((E, N, 4, 4))
    gg = np.einsum("eai,ebi->eab", gr, gr)
    for q in range(4):
        Nq = TET_QP[q]
        uq = np.einsum("a,enai->eni", Nq, UB)
        kap = np.einsum("eni,eij,enj->en", uq, xi, uq) + prm.C_I * nu * nu * xixi[:, None]
        tau = kap ** -0.5
        c = np.einsum("eni,eai->ena", uq, gr)                    # u.grad N_A
        wq = w[:, :, None, None]
        K += wq * (rho * Nq[None, None, :, None] * c[:, :, None, :]
                   + rho * tau[:, :, None, None] * c[:, :, :, None] * c[:, :, None, :])
        G += wq[..., None] * (-gr[:, None, :, None, :] * Nq[None, None, None, :, None]
                              + tau[:, :, None, None, None] * c[:, :, :, None, None]
                              * gr[:, None, None, :, :])
        D += wq[..., None] * (Nq[None, None, :, None, None] * gr[:, None, None, :, :]
                              + tau[:, :, None, None, None] * gr[:, None, :, None, :]
                              * c[:, :, None, :, None])
        L += wq * tau[:, :, None, None] * gg[:, None, :, :] / rho
    K += mu * vol[:, None, None, None] * gg[:, None, :, :]
    return idx, K, G, D, L


def assemble_paper_tangent(om: OMesh, prm, y: np.ndarray, H: np.ndarray,
                           shift: float = 0.0, include_C: bool = True) -> sp.csr_matrix:
    """(C + P + shift M_v) at the state y (4, N, n), without Dirichlet masking.
    With include_C=False only the time-diagonal part P + shift M_v."""
    N, n = y.shape[1], y.shape[2]
    rows, cols, vals = [], [], []

    def flat(f, s, a):
        return (f * N + s) * n + a

    sN = np.arange(N)
    for c0 in range(0, om.ne, CHUNK):
        e = np.arange(c0, min(om.ne, c0 + CHUNK))
        idx, K, G, D, L = _local_blocks(om, prm, e, y[:3])
        vol = om.vol[e]
        M = vol[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0
        A = idx[:, None, :, None]
        B = idx[:, None, None, :]
        s = sN[None, :, None, None]
        shp = K.shape
        for i in range(3):
            rows.append(np.broadcast_to(flat(i, s, A), shp).ravel())
            cols.append(np.broadcast_to(flat(i, s, B), shp).ravel())
            vals.append((K + shift * M[:, None]).ravel())
            rows.append(np.broadcast_to(flat(i, s, A), shp).ravel())
            cols.append(np.broadcast_to(flat(3, s, B), shp).ravel())
            vals.append(G[..., i].ravel())
            rows.append(np.broadcast_to(flat(3, s, A), shp).ravel())
            cols.append(np.broadcast_to(flat(i, s, B), shp).ravel())
            vals.append(D[..., i].ravel())
        rows.append(np.broadcast_to(flat(3, s, A), shp).ravel())
        cols.append(np.broadcast_to(flat(3, s, B), shp).ravel())
        vals.append(L.ravel())
        if not include_C:
            continue
        # F = H (x) int rho N_A N_B on each velocity component
        sk = sN[:, None]
        kk = sN[None, :]
        A5 = idx[:, None, None, :, None]
        B5 = idx[:, None, None, None, :]
        Fv = (H[None, :, :, None, None] * prm.rho * M[:, None, None, :, :])
        shp5 = Fv.shape
        for i in range(3):
            rows.append(np.broadcast_to(flat(i, sk[None, :, :, None, None], A5), shp5).ravel())
            cols.append(np.broadcast_to(flat(i, kk[None, :, :, None, None], B5), shp5).ravel())
            vals.append(Fv.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    m = 4 * N * n
    return sp.csr_matrix((v, (r, c)), shape=(m, m))


def dirichlet_masks(om: OMesh, N: int) -> np.ndarray:
    """Boolean (4, N, n): True on Dirichlet velocity unknowns."""
    mk = np.zeros((4, N, om.n), bool)
    mk[:3][:, :, om.dirichlet] = True
    return mk


def masked(Amat: sp.csr_matrix, mask_flat: np.ndarray, identity: bool) -> sp.csr_matrix:
    """Zero the rows and columns of the Dirichlet unknowns; put ones on their
    diagonal if ``identity``."""
    keep = sp.diags((~mask_flat).astype(float))
    out = keep @ Amat @ keep
    if identity:
        out = out + sp.diags(mask_flat.astype(float))
    return out.tocsr()


def jacobi_diagonal(om: OMesh, prm, y: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """(2, N, n): diag of K (+ shift int N_A^2) and diag of L, per node and
    sample.  Dirichlet velocity rows are set to one."""
    N, n = y.shape[1], y.shape[2]
    out = np.zeros((2, N, n))
    for c0 in range(0, om.ne, CHUNK):
        e = np.arange(c0, min(om.ne, c0 + CHUNK))
        idx, K, G, D, L = _local_blocks(om, prm, e, y[:3])
        kd = np.einsum("enaa->ena", K) + shift * (om.vol[e] / 10.0)[:, None, None]
        ld = np.einsum("enaa->ena", L)
        s = np.arange(N)[None, :, None]
        np.add.at(out[0], (np.broadcast_to(s, kd.shape), np.broadcast_to(idx[:, None, :], kd.shape)), kd)
        np.add.at(out[1], (np.broadcast_to(s, ld.shape), np.broadcast_to(idx[:, None, :], ld.shape)), ld)
    out[0][:, om.dirichlet] = 1.0
    return out


def frozen_tangent_apply(om: OMesh, prm, y: np.ndarray, v: np.ndarray, shift: float = 0.0,
                         H: np.ndarray | None = None) -> np.ndarray:
    """Tangent of eq. Rmc with advection and tau frozen at the state y, no
    outlet terms, applied to v (time samples, (4, N, n)).  With the
    advecting velocity and tau held at y the residual is linear in its
    argument, so this is the residual of v itself (v's Dirichlet velocity
    samples set to zero, traction and backflow off), plus shift * int N_A N_B
    on the velocity rows.  It is the paper's P of eq. K_mat with the
    Galerkin time term C of eq. ctangent and the stabilisation's time terms.
    """
    from .residual import Options, residual_samples
    N = y.shape[1]
    H = H_of_prm(prm) if H is None else H
    vv = np.array(v, dtype=np.float64, copy=True)
    vv[:3][:, :, om.dirichlet] = 0.0
    out = residual_samples(om, prm, vv, np.zeros((om.n_outlets, N)), None, H,
                           Options(frozen_u=np.asarray(y[:3], dtype=np.float64), backflow=False))
    if shift != 0.0:
        M = om.vol[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0
        mv = np.zeros((3, N, om.n))
        idx = om.tets
        for i in range(3):
            loc = np.einsum("eab,nbe->nae", M, vv[i][:, idx].transpose(0, 2, 1))
            for A in range(4):
                np.add.at(mv[i], (slice(None), idx[:, A]), loc[:, A, :])
        mv[:, :, om.dirichlet] = 0.0
        out[:3] += shift * mv
    return out


def meanflow_apply(om: OMesh, prm, y: np.ndarray, v: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """The frozen-coefficient tangent averaged over cyclic time shifts,
        A v = (1/N) sum_k S^-k J_f(y) S^k v,   (S^k v)_s = v_(s+k mod N),
    i.e. its circulant projection in time: every coefficient that varies
    over the samples is replaced by its sample mean, while H (already
    circulant) is kept.  The result commutes with time shifts and so maps
    each harmonic to itself.  This defines the operator that the solver's
    mean-flow preconditioner approximates (it changes iteration counts, not
    the root)."""
    N = y.shape[1]
    H = H_of_prm(prm)
    acc = np.zeros_like(np.asarray(v, dtype=np.float64))
    for k in range(N):
        w = frozen_tangent_apply(om, prm, y, np.roll(v, -k, axis=1), shift, H)
        acc += np.roll(w, k, axis=1)
    return acc / N


def H_of_prm(prm) -> np.ndarray:
    from .spectral import hb_matrix
    return hb_matrix(prm.K, 2.0 * np.pi / prm.period)
