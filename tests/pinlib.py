"""Independent reference results used to pin the oracle (CPU only).

* Womersley's closed form for oscillatory pipe flow (Womersley 1955).
* Per-mode frequency-domain GLS-Stokes solves: the linear limit of eq.
  NS-spec (Section 2.1) with the convolution matrix A = 0, where every
  Fourier mode decouples and H becomes multiplication by i m omega.  The
  element matrices are written here from the frequency-domain weak form,
  with closed-form P1 integrals (no quadrature loop), independently of
  the oracle's time-sample assembly.
* Brute-force BDF2 time marching of the same linear semi-discrete system
  (stabilisation time terms off), whose periodic orbit the HB samples
  must reproduce.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import jv

# ----------------------------------------------------------------- Womersley


def womersley_profile(r, R, omega, nu, rho, Qhat):
    """Complex velocity amplitude u_z(r) for flow amplitude Qhat at omega."""
    alpha = R * np.sqrt(omega / nu)
    lam = (1j ** 1.5) * alpha
    fac = 1.0 - 2.0 * jv(1, lam) / (lam * jv(0, lam))
    G = Qhat * 1j * omega * rho / (np.pi * R ** 2 * fac)
    return G / (1j * omega * rho) * (1.0 - jv(0, lam * r / R) / jv(0, lam)), G


def womersley_modal(xyz, K, R, L, omega, mu, rho, q_modal):
    """Exact (u_z, p) as real modal coefficients (N, n) for the flow rate
    with real modal coefficients q_modal: mode 0 Poiseuille, mode m
    Womersley at m omega."""
    N = 2 * K + 1
    r = np.sqrt(xyz[:, 0] ** 2 + xyz[:, 1] ** 2)
    z = xyz[:, 2]
    nu = mu / rho
    uz = np.zeros((N, xyz.shape[0]))
    p = np.zeros((N, xyz.shape[0]))
    Q0 = q_modal[0]
    uz[0] = 2.0 * Q0 / (np.pi * R ** 2) * (1.0 - r ** 2 / R ** 2)
    p[0] = 8.0 * mu * Q0 / (np.pi * R ** 4) * (L - z)
    for m in range(1, K + 1):
        Qh = 0.5 * (q_modal[2 * m - 1] - 1j * q_modal[2 * m])   # complex amplitude of e^{i m w t}
        if Qh == 0:
            continue
        prof, G = womersley_profile(r, R, m * omega, nu, rho, Qh)
        # real signal: 2 Re(c e^{imwt}) -> a = 2 Re c, b = -2 Im c
        uz[2 * m - 1] = 2.0 * prof.real
        uz[2 * m] = -2.0 * prof.imag
        p[2 * m - 1] = 2.0 * G.real * (L - z)
        p[2 * m] = -2.0 * G.imag * (L - z)
    return uz, p


# ------------------------------------------------------- P1 element algebra


def p1_elements(xyz, tets):
    x0 = xyz[tets[:, 0]]
    J = np.stack([xyz[tets[:, 1]] - x0, xyz[tets[:, 2]] - x0, xyz[tets[:, 3]] - x0], axis=2)
    V = np.linalg.det(J) / 6.0
    assert np.all(V > 0)
    Ji = np.linalg.inv(J)
    g = np.concatenate([-Ji.sum(axis=1, keepdims=True), Ji], axis=1)   # (e, 4, 3)
    xi = np.einsum("eki,ekj->eij", Ji, Ji)
    return g, V, np.einsum("eij,eij->e", xi, xi)


def _coo(rows, cols, vals, n):
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def stokes_blocks(xyz, tets, mu, rho, C_I):
    """Global P1 matrices of the linear GLS-Stokes operator:
    M_AB = int N_A N_B, A_AB = int grad N_A . grad N_B, B_i[A,B] = int N_A d_i N_B
    (so int d_i N_A N_B = B_i^T), plus the tau-weighted Laplacian and
    tau-weighted versions of M and B (tau constant per element)."""
    g, V, xixi = p1_elements(xyz, tets)
    nu = mu / rho
    tau = (C_I * nu * nu * xixi) ** -0.5
    n = xyz.shape[0]
    Ml = V[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0
    Al = V[:, None, None] * np.einsum("eai,ebi->eab", g, g)
    Bl = [V[:, None, None] / 4.0 * np.broadcast_to(g[:, None, :, i], (tets.shape[0], 4, 4))
          for i in range(3)]
    r = np.repeat(tets, 4, axis=1).ravel()
    c = np.tile(tets, (1, 4)).ravel()

    def glob(loc):
        return sp.csr_matrix((loc.ravel(), (r, c)), shape=(n, n))
    return dict(M=glob(Ml), A=glob(Al), B=[glob(b) for b in Bl],
                tM=glob(tau[:, None, None] * Ml), tA=glob(tau[:, None, None] * Al),
                tB=[glob(tau[:, None, None] * b) for b in Bl])


def outlet_load(xyz, faces, normals, n):
    """int_f N_A n_i over outlet faces, (3, n): area/3 per node."""
    a = 0.5 * np.linalg.norm(np.cross(xyz[faces[:, 1]] - xyz[faces[:, 0]],
                                      xyz[faces[:, 2]] - xyz[faces[:, 0]]), axis=1)
    out = np.zeros((3, n))
    for i in range(3):
        for k in range(3):
            np.add.at(out[i], faces[:, k], a / 3.0 * normals[:, i])
    return out


def solve_mode(blocks, sigma, mu, rho, dir_mask, g_hat, h_hat, load):
    """Frequency-domain GLS-Stokes for one harmonic sigma = i m omega:
       momentum: (rho sigma M + mu A - rho sigma^2 tM) u_i
                 + (-B_i^T - sigma tB_i) p - h load_i = 0
       continuity: sum_j (B_j + sigma tB_j^T) u_j + (1/rho) tA p = 0
    with u = g_hat on Dirichlet nodes.  (B_i[A,B] = int N_A d_i N_B.)"""
    M, A, B, tM, tA, tB = (blocks[k] for k in ("M", "A", "B", "tM", "tA", "tB"))
    n = M.shape[0]
    Kuu = rho * sigma * M + mu * A - rho * sigma * sigma * tM
    blocks_rows = []
    for i in range(3):
        row = [None] * 4
        row[i] = Kuu
        row[3] = -B[i].T - sigma * tB[i]
        blocks_rows.append(row)
    blocks_rows.append([B[j] + sigma * tB[j].T for j in range(3)] + [tA / rho])
    Aglob = sp.bmat(blocks_rows, format="csr").astype(complex)
    rhs = np.zeros(4 * n, complex)
    rhs[:3 * n] = (h_hat * load).ravel()
    mask = np.zeros(4 * n, bool)
    mask[:3 * n] = np.tile(dir_mask, 3)
    x_d = np.zeros(4 * n, complex)
    x_d[:3 * n] = g_hat.ravel()
    rhs = rhs - Aglob @ x_d
    free = ~mask
    Aff = Aglob[free][:, free]
    x = x_d.copy()
    x[free] = spla.spsolve(Aff.tocsc(), rhs[free])
    return x.reshape(4, n)


# ----------------------------------------------------------- time marching


def march_bdf2(blocks, mu, rho, dir_mask, g_of_t, h_of_t, load, x0, x1, dt, n_steps):
    """BDF2 for rho M du/dt + mu A u - B^T p = h load, sum_j B_j u_j +
    (1/rho) tA p = 0 (stabilisation time terms off), Dirichlet u = g(t).
    x0, x1: (4, n) states at t = 0 and t = dt.  Returns states at each step."""
    M, A, B, tA = blocks["M"], blocks["A"], blocks["B"], blocks["tA"]
    n = M.shape[0]
    Kuu = 1.5 * rho / dt * M + mu * A
    rows = []
    for i in range(3):
        row = [None] * 4
        row[i] = Kuu
        row[3] = -B[i].T
        rows.append(row)
    rows.append([B[j] for j in range(3)] + [tA / rho])
    Aglob = sp.bmat(rows, format="csr")
    mask = np.zeros(4 * n, bool)
    mask[:3 * n] = np.tile(dir_mask, 3)
    free = ~mask
    lu = spla.splu(Aglob[free][:, free].tocsc())
    Mv = sp.block_diag([M, M, M, sp.csr_matrix((n, n))], format="csr")
    xm, xc = x0.ravel().copy(), x1.ravel().copy()
    out = [x0.copy(), x1.copy()]
    for k in range(2, n_steps + 1):
        t = k * dt
        rhs = np.zeros(4 * n)
        rhs[:3 * n] = (h_of_t(t) * load).ravel()
        rhs += rho / dt * (Mv @ (2.0 * xc - 0.5 * xm))
        xd = np.zeros(4 * n)
        xd[:3 * n] = g_of_t(t).ravel()
        rhs -= Aglob @ xd
        xn = xd.copy()
        xn[free] = lu.solve(rhs[free])
        xm, xc = xc, xn
        out.append(xn.reshape(4, n))
    return out


# ------------------------------------------- independent steady GLS solver


_QA4 = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_QB4 = (5.0 - np.sqrt(5.0)) / 20.0


def _tet_grads(xyz, tets):
    """Gradients of the P1 basis from face normals: grad N_A = -n_A |f_A| /
    (3 V), n_A the outward unit normal of the face opposite node A; and the
    volume V.  Written from the cross-product identity, not from J^-1."""
    X = xyz[tets]                                        # (E, 4, 3)
    V = np.einsum("ei,ei->e", X[:, 1] - X[:, 0],
                  np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])) / 6.0
    if np.any(V <= 0):
        raise ValueError("tetrahedra must be positively oriented")
    G = np.empty((tets.shape[0], 4, 3))
    for A in range(4):
        o = [k for k in range(4) if k != A]
        a, b, c = X[:, o[0]], X[:, o[1]], X[:, o[2]]
        nA = np.cross(b - a, c - a)                      # |nA| = 2 |f_A|
        nA *= np.sign(np.einsum("ei,ei->e", nA, a - X[:, A]))[:, None]   # outward from A
        G[:, A] = -nA / (6.0 * V[:, None])
    return G, V


def steady_gls_residual(xyz, tets, u, p, mu, rho, C_I, ofaces, onormal, oarea, h_out, beta):
    """Steady GLS Navier-Stokes residual (Section 2.2/2.3 with H = 0):
    momentum rows int N_A rho u.grad u_i + mu grad N_A . grad u_i - d_i N_A p
    + (u.grad N_A) tau (rho u.grad u_i + d_i p), outlet -int N_A h n_i and
    backflow -int N_A rho beta/2 min(u.n, 0) u_i; continuity rows
    int N_A div u + (1/rho) d_i N_A tau (rho u.grad u_i + d_i p); tau from the
    4-point rule with xi = sum_k grad N_k grad N_k^T (k = 1..3).
    u (n, 3), p (n,); returns (rm (n, 3), rc (n,))."""
    nu = mu / rho
    G, V = _tet_grads(xyz, tets)
    xi = np.einsum("eki,ekj->eij", G[:, 1:], G[:, 1:])
    xx = np.einsum("eij,eij->e", xi, xi)
    ue = u[tets]                                         # (E, 4, 3)
    pe = p[tets]                                         # (E, 4)
    gu = np.einsum("eai,eaj->eij", ue, G)                # d_j u_i
    gp = np.einsum("ea,eaj->ej", pe, G)
    div = np.einsum("eii->e", gu)
    rm = np.zeros((xyz.shape[0], 3))
    rc = np.zeros(xyz.shape[0])
    lm = np.zeros((tets.shape[0], 4, 3))
    lc = np.zeros((tets.shape[0], 4))
    for q in range(4):
        w = np.full(4, _QB4)
        w[q] = _QA4
        uq = np.einsum("a,eai->ei", w, ue)
        pq = np.einsum("a,ea->e", w, pe)
        conv = np.einsum("ej,eij->ei", uq, gu)
        tau = 1.0 / np.sqrt(np.einsum("ei,eij,ej->e", uq, xi, uq) + C_I * nu * nu * xx)
        Ls = rho * conv + gp                             # strong residual (viscous part 0)
        ugN = np.einsum("ei,eai->ea", uq, G)
        wq = V / 4.0
        lm += wq[:, None, None] * (w[None, :, None] * rho * conv[:, None, :]
                                   - G * pq[:, None, None]
                                   + ugN[:, :, None] * tau[:, None, None] * Ls[:, None, :])
        lc += wq[:, None] * (w[None, :] * div[:, None]
                             + np.einsum("eai,ei->ea", G, tau[:, None] * Ls) / rho)
    lm += mu * V[:, None, None] * np.einsum("eaj,eij->eai", G, gu)
    for A in range(4):
        np.add.at(rm, tets[:, A], lm[:, A])
        np.add.at(rc, tets[:, A], lc[:, A])
    # outlet: traction and backflow on the 3-point rule
    uf = u[ofaces]                                       # (F, 3, 3)
    for q in range(3):
        w = np.full(3, 1.0 / 6.0)
        w[q] = 2.0 / 3.0
        uq = np.einsum("a,fai->fi", w, uf)
        un = np.einsum("fi,fi->f", uq, onormal)
        t = -(h_out * onormal + 0.5 * rho * beta * np.minimum(un, 0.0)[:, None] * uq)
        for A in range(3):
            np.add.at(rm, ofaces[:, A], (oarea / 3.0)[:, None] * w[A] * t)
    return rm, rc


def steady_gls_solve(xyz, tets, mu, rho, C_I, dir_mask, g, ofaces, onormal, oarea, h_out, beta,
                     tol=1e-12, max_it=30):
    """Newton's method on steady_gls_residual with a finite-difference
    Jacobian (columns grouped by a distance-2 colouring of the node graph)
    and a sparse direct solve.  Dirichlet velocities are fixed to g."""
    n = xyz.shape[0]
    u = np.zeros((n, 3))
    u[dir_mask] = g[dir_mask]
    p = np.zeros(n)
    free_u = ~dir_mask
    # distance-2 colouring: nodes sharing an element get different colours
    nbr = [set() for _ in range(n)]
    for t in tets:
        for a in t:
            nbr[a].update(t.tolist())
    col = -np.ones(n, int)
    for i in range(n):
        used = set()
        for j in nbr[i]:
            for k in nbr[j]:
                if col[k] >= 0:
                    used.add(col[k])
        c = 0
        while c in used:
            c += 1
        col[i] = c

    def R(u, p):
        rm, rc = steady_gls_residual(xyz, tets, u, p, mu, rho, C_I, ofaces, onormal, oarea,
                                     h_out, beta)
        rm[dir_mask] = 0.0
        return np.concatenate([rm[:, 0], rm[:, 1], rm[:, 2], rc])

    # unknown vector: u_x, u_y, u_z at free nodes (kept full, Dirichlet rows identity), p
    hist = []
    for _ in range(max_it):
        r = R(u, p)
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= tol * max(hist[0], 1e-300):
            break
        rows, cols, vals = [], [], []
        for c in range(col.max() + 1):
            sel = np.nonzero(col == c)[0]
            for f in range(4):
                eps = 1e-7 * (1.0 + (np.abs(u).max() if f < 3 else np.abs(p).max()))
                du, dp = u.copy(), p.copy()
                if f < 3:
                    du[sel, f] += eps
                else:
                    dp[sel] += eps
                d = (R(du, dp) - r) / eps
                for i in sel:
                    nb = np.fromiter(nbr[i], int)
                    for ff in range(4):
                        rr = ff * n + nb
                        rows.append(rr)
                        cols.append(np.full(nb.size, f * n + i))
                        vals.append(d[rr])
        J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(4 * n, 4 * n))
        # Dirichlet velocity unknowns: identity rows and columns
        dmask = np.concatenate([dir_mask, dir_mask, dir_mask, np.zeros(n, bool)])
        keep = sp.diags((~dmask).astype(float))
        J = (keep @ J @ keep + sp.diags(dmask.astype(float))).tocsc()
        x = spla.spsolve(J, -r)
        u[free_u] += np.stack([x[:n], x[n:2 * n], x[2 * n:3 * n]], axis=1)[free_u]
        p += x[3 * n:]
    return u, p, hist
