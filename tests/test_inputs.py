"""Synthetic input generators: the branching-artery mesh and the stacking
of problems (host only)."""
import numpy as np

from hbinputs.meshes import INLET, OUTLET, WALL, branching_artery_mesh


def test_branching_artery_mesh_is_valid():
    m = branching_artery_mesh(h=0.25)
    x, t = m.xyz, m.tets
    a, b, c = x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]], x[t[:, 3]] - x[t[:, 0]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    assert np.all(vol > 0)
    # closed, outward-oriented boundary: divergence theorem for x gives 3 V
    f = x[m.faces]
    nrm = np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0]) / 2.0
    flux = np.einsum("ij,ij->", nrm, f.mean(axis=1))
    assert abs(flux / 3.0 - vol.sum()) <= 1e-9 * vol.sum()
    # one wall, one planar root inlet at z = 0, eight non-empty leaf outlets
    kinds = m.group_kind
    assert list(kinds[:2]) == [WALL, INLET] and np.all(kinds[2:] == OUTLET) and kinds.size == 10
    counts = np.bincount(m.face_group, minlength=kinds.size)
    assert np.all(counts > 0)
    assert np.all(np.abs(f[m.face_group == 1][:, :, 2]) < 1e-12)
    # the boundary surface is closed: every edge is shared by an even number
    # of faces (two, or four where lattice carving leaves two parts of the
    # domain touching along an edge)
    e = np.sort(np.concatenate([m.faces[:, [0, 1]], m.faces[:, [1, 2]], m.faces[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert np.all(cnt % 2 == 0) and np.mean(cnt == 2) > 0.99
