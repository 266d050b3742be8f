"""Seeded synthetic workloads: meshes plus Fourier boundary data plus fluid
parameters, in the modal layout of the C interface.

Modal layout (per field, per node): index 0 holds the mean a_0, index 2m-1
the cosine coefficient a_m and index 2m the sine coefficient b_m, so that a
quantity equals a_0 + sum_m a_m cos(m w t) + b_m sin(m w t).

Nothing here evaluates the harmonic-balance operator.  Random numbers that
the workloads need are drawn here and handed to both implementations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .meshes import (INLET, OUTLET, WALL, Mesh, branching_artery_mesh, cylinder_mesh,
                     stenosed_pipe_mesh, tjunction_mesh)

RHO = 1.06   # g/cm^3, whole blood
MU = 0.04    # poise (4 mPa s)


@dataclass
class Params:
    rho: float = RHO
    mu: float = MU
    period: float = 1.0
    K: int = 2
    C_I: float = 3.0
    beta_bf: float = 0.2

    @property
    def N(self) -> int:
        return 2 * self.K + 1


@dataclass
class Problem:
    name: str
    mesh: Mesh
    params: Params
    dirichlet: np.ndarray   # (3, N, n) modal coefficients; only Dirichlet nodes matter
    outlet_h: np.ndarray    # (n_outlets, N) modal coefficients of the normal traction h
    outlet_R: np.ndarray | None  # (n_outlets,) resistance, or None
    u_ref: float = 1.0      # velocity scale used by seeded states


def n_outlets(mesh: Mesh) -> int:
    return int(np.sum(mesh.group_kind == OUTLET))


def dirichlet_nodes(mesh: Mesh) -> np.ndarray:
    return np.union1d(mesh.group_nodes(WALL), mesh.group_nodes(INLET))


def poiseuille_dirichlet(mesh: Mesh, K: int, flows: list[np.ndarray]) -> np.ndarray:
    """Parabolic inflow on every inlet listed in mesh.info['inlets'] with the
    modal flow-rate coefficients ``flows[j]`` (length 2K+1); zero on walls."""
    N = 2 * K + 1
    n = mesh.n_nodes
    out = np.zeros((3, N, n))
    wall = np.zeros(n, bool)
    wall[mesh.group_nodes(WALL)] = True
    for inl, Qm in zip(mesh.info["inlets"], flows):
        sel = mesh.faces[mesh.face_group == inl["group"]].ravel()
        nodes = np.unique(sel)
        nodes = nodes[~wall[nodes]]
        c = np.asarray(inl["center"], float)
        e = np.asarray(inl["normal"], float)
        R = float(inl["radius"])
        d = mesh.xyz[nodes] - c
        r2 = np.sum((d - (d @ e)[:, None] * e) ** 2, axis=1)
        prof = np.maximum(0.0, 1.0 - r2 / R ** 2) * 2.0 / (np.pi * R ** 2)
        for i in range(3):
            out[i][:, nodes] = e[i] * np.outer(np.asarray(Qm, float), prof)
    return out


def womersley_like_flow(K: int) -> np.ndarray:
    """Q(t) = 1 + 0.5 sin(w t) as modal coefficients."""
    q = np.zeros(2 * K + 1)
    q[0] = 1.0
    if K >= 1:
        q[2] = 0.5
    return q


def c1_womersley(K: int = 2, period: float = 1.0, n_rings: int = 5, n_z: int = 20) -> Problem:
    """Straight rigid pipe R=1, L=6, Poiseuille inflow with Q = 1 + 0.5 sin(wt),
    zero-traction outlet, no-slip wall."""
    mesh = cylinder_mesh(1.0, 6.0, n_rings, n_z)
    prm = Params(period=period, K=K)
    dirv = poiseuille_dirichlet(mesh, K, [womersley_like_flow(K)])
    return Problem("c1_womersley_pipe", mesh, prm, dirv,
                   np.zeros((n_outlets(mesh), prm.N)), None, u_ref=2.0 / np.pi)


def seeded_waveform(K: int, qbar: float, seed: int, n_coef: int = 10, amp: float = 0.3) -> np.ndarray:
    """Q(t) = qbar [1 + amp sum_{k<=n_coef} k^-1.5 (alpha_k cos + beta_k sin)],
    alpha, beta ~ N(0, 1/2); truncated to the K retained harmonics."""
    rng = np.random.default_rng(seed)
    ab = rng.normal(0.0, np.sqrt(0.5), size=(n_coef, 2))
    q = np.zeros(2 * K + 1)
    q[0] = qbar
    for k in range(1, min(K, n_coef) + 1):
        q[2 * k - 1] = qbar * amp * k ** -1.5 * ab[k - 1, 0]
        q[2 * k] = qbar * amp * k ** -1.5 * ab[k - 1, 1]
    return q


def c2_tjunction(K: int = 10, h: float = 3.0 / 70.0, reynolds: float = 500.0,
                 resistance: bool = True, p_ref: float = 1.0e4) -> Problem:
    """Glenn-like T-junction: two inlets r=0.5 meeting head-on, outlet r=0.6,
    seeded inflow waveforms (seeds 11, 12), one resistance outlet."""
    mesh = tjunction_mesh(h=h)
    prm = Params(period=1.0, K=K)
    d_in = 2.0 * mesh.info["r_in"]
    ubar = reynolds * prm.mu / (prm.rho * d_in)
    qbar = ubar * np.pi * mesh.info["r_in"] ** 2
    flows = [seeded_waveform(K, qbar, 11), seeded_waveform(K, qbar, 12)]
    dirv = poiseuille_dirichlet(mesh, K, flows)
    nout = n_outlets(mesh)
    R = np.full(nout, p_ref * nout / (2.0 * qbar)) if resistance else None
    return Problem("c2_tjunction", mesh, prm, dirv, np.zeros((nout, prm.N)), R, u_ref=ubar)


def c3_branching(K: int = 10, h: float = 0.062, reynolds: float = 500.0,
                 p_ref: float = 1.0e4) -> Problem:
    """Curved branching artery: three bifurcation generations (radii 2.0,
    1.26, 0.79, 0.50, segment length 6 r, seeded arc curvature, seed 7),
    root inflow built like the T-junction's (seed 13, Re on the root
    diameter), eight resistance outlets R = 8 p_ref / Q (each outlet takes
    Q / 8 at pressure p_ref)."""
    mesh = branching_artery_mesh(h=h)
    prm = Params(period=1.0, K=K)
    r0 = mesh.info["r_root"]
    ubar = reynolds * prm.mu / (prm.rho * 2.0 * r0)
    qbar = ubar * np.pi * r0 ** 2
    dirv = poiseuille_dirichlet(mesh, K, [seeded_waveform(K, qbar, 13)])
    nout = n_outlets(mesh)
    R = np.full(nout, p_ref * nout / qbar)
    return Problem("c3_branching_artery", mesh, prm, dirv, np.zeros((nout, prm.N)), R,
                   u_ref=ubar)


def c4_stenosis_params(n: int, seed: int, K: int = 10, reynolds: float = 100.0,
                       max_severity: float = 0.7):
    """Parameter draws of the stenosed-pipe family: severity, position and
    the 2K+1 inflow coefficients (23 values for K = 10)."""
    rng = np.random.default_rng(seed)
    ubar = reynolds * MU / (RHO * 2.0)
    qref = ubar * np.pi
    out = np.zeros((n, 2 + 2 * K + 1))
    out[:, 0] = rng.uniform(0.0, max_severity, n)
    out[:, 1] = rng.uniform(2.0, 4.0, n)
    a0 = rng.uniform(0.5, 1.5, n) * qref
    out[:, 2] = a0
    for k in range(1, K + 1):
        sd = 0.3 * k ** -1.5 * a0
        out[:, 2 * k + 1] = rng.normal(0.0, 1.0, n) * sd
        out[:, 2 * k + 2] = rng.normal(0.0, 1.0, n) * sd
    return out


def c4_stenosed(theta: np.ndarray, K: int = 10, n_rings: int = 12, n_z: int = 90,
                period: float = 1.0) -> Problem:
    mesh = stenosed_pipe_mesh(float(theta[0]), float(theta[1]), n_rings, n_z)
    prm = Params(period=period, K=K)
    dirv = poiseuille_dirichlet(mesh, K, [np.asarray(theta[2:], float)])
    return Problem("c4_stenosed_pipe", mesh, prm, dirv,
                   np.zeros((n_outlets(mesh), prm.N)), None, u_ref=float(theta[2]) / np.pi)


def seeded_state(prob: Problem, seed: int, noise: float = 0.1) -> np.ndarray:
    """A seeded modal state Y (4, N, n): smooth spatial patterns with mode
    amplitudes decaying like (1+m)^-1.5 plus Gaussian noise.  Velocity scales
    with prob.u_ref, pressure with rho u_ref^2."""
    rng = np.random.default_rng(seed)
    m = prob.mesh
    N = prob.params.N
    x = m.xyz
    L = np.ptp(x, axis=0).max()
    Y = np.zeros((4, N, m.n_nodes))
    for f in range(4):
        scale = prob.u_ref if f < 3 else prob.params.rho * prob.u_ref ** 2
        for j in range(N):
            k = rng.normal(0.0, 2.0 * np.pi / L, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            decay = (1.0 + (j + 1) // 2) ** -1.5
            Y[f, j] = scale * decay * (np.sin(x @ k + ph) + noise * rng.normal(size=m.n_nodes))
    return Y


def stack(problems: list[Problem]) -> Problem:
    """Disjoint union of problems with zero-traction outlets and no
    resistance: one mesh whose connected components are the given meshes
    (node blocks in the given order), with one wall, one inlet and one outlet
    group.  The harmonic-balance equations of disconnected components do not
    couple, so one solve on the union solves every member."""
    K = problems[0].params.K
    if any(p.params != problems[0].params for p in problems):
        raise ValueError("stacked problems must share their fluid and time parameters")
    if any(p.outlet_R is not None or np.any(p.outlet_h != 0) for p in problems):
        raise ValueError("stacking needs zero-traction outlets without resistance")
    xyz, tets, faces, fgrp, dirv = [], [], [], [], []
    off = 0
    for p in problems:
        m = p.mesh
        xyz.append(m.xyz)
        tets.append(m.tets + off)
        faces.append(m.faces + off)
        fgrp.append(m.group_kind[m.face_group])
        dirv.append(p.dirichlet)
        off += m.n_nodes
    kinds = np.array([WALL, INLET, OUTLET], np.int32)
    kind_to_group = {int(k): g for g, k in enumerate(kinds)}
    grp = np.array([kind_to_group[int(k)] for k in np.concatenate(fgrp)], np.int32)
    mesh = Mesh(np.concatenate(xyz), np.concatenate(tets).astype(np.int32),
                np.concatenate(faces).astype(np.int32), grp, kinds,
                dict(kind="union", sizes=[p.mesh.n_nodes for p in problems]))
    return Problem("stack", mesh, problems[0].params, np.concatenate(dirv, axis=2),
                   np.zeros((1, 2 * K + 1)), None, u_ref=max(p.u_ref for p in problems))
