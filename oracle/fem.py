"""P1 tetrahedral geometry, quadrature and boundary data for the oracle.

Section 2.2-2.3: linear shape functions N_A on tetrahedra; the GLS
parameter uses the covariant metric xi of the physical-to-parent map
(eq. tau); the discrete residual of eq. Rmc integrates over elements and
over the Neumann boundary.  The paper does not state a quadrature rule; the
oracle uses the 4-point degree-2 tetrahedron rule and the 3-point degree-2
triangle rule, and the metric xi = J^{-T} J^{-1} for the unit right
reference tetrahedron (readings recorded with the design notes).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

WALL, INLET, OUTLET = 0, 1, 2

# 4-point rule, barycentric (a, b, b, b) and permutations, weight V/4 each
_QA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_QB = (5.0 - np.sqrt(5.0)) / 20.0
TET_QP = np.full((4, 4), _QB)
np.fill_diagonal(TET_QP, _QA)
TET_QW = np.full(4, 0.25)
# 3-point triangle rule at (2/3, 1/6, 1/6) and permutations, weight |f|/3
TRI_QP = np.full((3, 3), 1.0 / 6.0)
np.fill_diagonal(TRI_QP, 2.0 / 3.0)
TRI_QW = np.full(3, 1.0 / 3.0)


@dataclass
class OMesh:
    xyz: np.ndarray
    tets: np.ndarray          # positively oriented
    grad: np.ndarray          # (n_e, 4, 3) physical gradients of N_A
    vol: np.ndarray           # (n_e,)
    xi: np.ndarray            # (n_e, 3, 3)
    xixi: np.ndarray          # (n_e,)  xi : xi
    dirichlet: np.ndarray     # (n,) bool, nodes on wall or inlet faces
    inlet: np.ndarray         # (n,) bool, nodes on inlet faces
    ofaces: np.ndarray        # (n_of, 3) outlet triangles
    onormal: np.ndarray       # (n_of, 3) unit outward normal
    oarea: np.ndarray         # (n_of,)
    oid: np.ndarray           # (n_of,) outlet index 0..n_outlets-1
    n_outlets: int
    n_reoriented: int

    @property
    def n(self) -> int:
        return self.xyz.shape[0]

    @property
    def ne(self) -> int:
        return self.tets.shape[0]


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Jacobian J = [x1-x0, x2-x0, x3-x0]; gradients of the barycentric
    coordinates are the rows of J^{-1}; xi = J^{-T} J^{-1}."""
    x0 = xyz[tets[:, 0]]
    J = np.stack([xyz[tets[:, 1]] - x0, xyz[tets[:, 2]] - x0, xyz[tets[:, 3]] - x0], axis=2)
    vol = np.linalg.det(J) / 6.0
    Jinv = np.linalg.inv(J)                      # (e, 3, 3): row k = grad xi_k
    grad = np.empty((tets.shape[0], 4, 3))
    grad[:, 1:, :] = Jinv
    grad[:, 0, :] = -Jinv.sum(axis=1)
    xi = np.einsum("eki,ekj->eij", Jinv, Jinv)
    xixi = np.einsum("eij,eij->e", xi, xi)
    return grad, vol, xi, xixi


def prepare(xyz, tets, faces, face_group, group_kind) -> OMesh:
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.array(tets, dtype=np.int64, copy=True)
    faces = np.asarray(faces, dtype=np.int64)
    face_group = np.asarray(face_group, dtype=np.int64)
    group_kind = np.asarray(group_kind, dtype=np.int64)
    n = xyz.shape[0]

    _, vol, _, _ = tet_geometry(xyz, tets)
    neg = vol < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    grad, vol, xi, xixi = tet_geometry(xyz, tets)

    kind = group_kind[face_group]
    dirichlet = np.zeros(n, bool)
    dirichlet[faces[(kind == WALL) | (kind == INLET)].ravel()] = True
    inlet = np.zeros(n, bool)
    inlet[faces[kind == INLET].ravel()] = True

    outlet_groups = np.nonzero(group_kind == OUTLET)[0]
    gid2out = -np.ones(group_kind.size, np.int64)
    gid2out[outlet_groups] = np.arange(outlet_groups.size)
    osel = kind == OUTLET
    of = faces[osel]
    oid = gid2out[face_group[osel]]

    # outward normal: away from the fourth node of the tetrahedron owning the face
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])   # face opposite node lf
    keys = np.sort(of, axis=1)
    qk = keys[:, 0] * (n * n) + keys[:, 1] * n + keys[:, 2]
    order = np.argsort(qk)
    opp = np.full(of.shape[0], -1, np.int64)
    for lf in range(4):
        if of.shape[0] == 0:
            break
        tri = np.sort(tets[:, loc[lf]], axis=1)
        kk = tri[:, 0] * (n * n) + tri[:, 1] * n + tri[:, 2]
        pos = np.clip(np.searchsorted(qk[order], kk), 0, qk.size - 1)
        hit = qk[order][pos] == kk
        opp[order[pos[hit]]] = tets[hit, lf]
    if np.any(opp < 0):
        raise ValueError("outlet face not found among element faces")
    a = xyz[of[:, 1]] - xyz[of[:, 0]]
    b = xyz[of[:, 2]] - xyz[of[:, 0]]
    nrm = np.cross(a, b)
    s = np.einsum("ij,ij->i", nrm, xyz[opp] - xyz[of[:, 0]])
    nrm[s > 0] *= -1.0
    area2 = np.linalg.norm(nrm, axis=1)
    onormal = nrm / area2[:, None]
    return OMesh(xyz, tets, grad, vol, xi, xixi, dirichlet, inlet, of, onormal,
                 0.5 * area2, oid, int(outlet_groups.size), int(neg.sum()))


def from_mesh(mesh) -> OMesh:
    return prepare(mesh.xyz, mesh.tets, mesh.faces, mesh.face_group, mesh.group_kind)


def consistent_mass_local(vol: np.ndarray) -> np.ndarray:
    """int N_A N_B over a tetrahedron = V (1 + delta_AB) / 20."""
    return vol[:, None, None] * (np.ones((4, 4)) + np.eye(4)) / 20.0
