"""Seeded synthetic tetrahedral meshes (input generation only).

Nothing here evaluates the harmonic-balance method: these routines build
node coordinates, P1 tetrahedra, boundary triangles and their groups.  Both
the CPU oracle and the HIP library consume the same meshes as plain arrays.

Group kinds follow the C interface: 0 = wall (no-slip Dirichlet),
1 = inlet (Dirichlet), 2 = outlet (Neumann traction / resistance).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, reverse_cuthill_mckee

WALL, INLET, OUTLET = 0, 1, 2


@dataclass
class Mesh:
    xyz: np.ndarray          # (n, 3) float64
    tets: np.ndarray         # (n_e, 4) int32, 0-based
    faces: np.ndarray        # (n_f, 3) int32 boundary triangles
    face_group: np.ndarray   # (n_f,) int32
    group_kind: np.ndarray   # (n_groups,) int32
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def group_nodes(self, kind: int) -> np.ndarray:
        groups = np.nonzero(self.group_kind == kind)[0]
        sel = np.isin(self.face_group, groups)
        return np.unique(self.faces[sel].ravel())


# ---------------------------------------------------------------- utilities

def _signed_volumes(xyz, tets):
    x0 = xyz[tets[:, 0]]
    a = xyz[tets[:, 1]] - x0
    b = xyz[tets[:, 2]] - x0
    c = xyz[tets[:, 3]] - x0
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def orient_positive(xyz, tets):
    """Swap local nodes 2 and 3 of every negatively oriented tetrahedron."""
    tets = np.array(tets, dtype=np.int32, copy=True)
    neg = _signed_volumes(xyz, tets) < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def boundary_faces(xyz, tets):
    """Triangles that belong to exactly one tetrahedron, ordered so that the
    right-hand normal points out of the domain."""
    loc = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
    opp = np.array([0, 1, 2, 3])
    f = tets[:, loc].reshape(-1, 3)
    other = tets[:, opp].reshape(-1)
    key = _face_keys(np.sort(f, axis=1))
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    keep = cnt[inv] == 1
    f = f[keep]
    other = other[keep]
    # orient: normal must point away from the opposite node
    n = np.cross(xyz[f[:, 1]] - xyz[f[:, 0]], xyz[f[:, 2]] - xyz[f[:, 0]])
    s = np.einsum("ij,ij->i", n, xyz[other] - xyz[f[:, 0]])
    flip = s > 0
    f[flip, 1], f[flip, 2] = f[flip, 2].copy(), f[flip, 1].copy()
    return f.astype(np.int32)


def _face_keys(sorted_faces):
    """One int64 per sorted node triple when node ids fit in 21 bits (fast
    1-D sorting); the triples themselves otherwise."""
    f = np.asarray(sorted_faces, dtype=np.int64)
    if f.size == 0 or f.max() < (1 << 21):
        return (f[:, 0] << 42) | (f[:, 1] << 21) | f[:, 2]
    return f


def compact(xyz, tets):
    """Drop unused nodes and renumber."""
    used = np.unique(tets.ravel())
    remap = -np.ones(xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return xyz[used].copy(), remap[tets].astype(np.int32)


def largest_component(xyz, tets):
    """Keep the face-connected component with the most tetrahedra."""
    loc = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
    ne = tets.shape[0]
    key = _face_keys(np.sort(tets[:, loc].reshape(-1, 3), axis=1))
    owner = np.repeat(np.arange(ne), 4)
    if key.ndim == 1:
        order = np.argsort(key, kind="stable")
        ks = key[order]
        same = ks[1:] == ks[:-1]
    else:
        order = np.lexsort(key.T[::-1])
        ks = key[order]
        same = np.all(ks[1:] == ks[:-1], axis=1)
    i = order[:-1][same]
    j = order[1:][same]
    g = sp.coo_matrix((np.ones(i.size), (owner[i], owner[j])), shape=(ne, ne))
    ncomp, lab = connected_components(g, directed=False)
    if ncomp == 1:
        return xyz, tets
    big = np.argmax(np.bincount(lab))
    return compact(xyz, tets[lab == big])


def rcm_reorder(mesh: Mesh, seed: int | None = None) -> Mesh:
    """Optionally shuffle node numbers with a seeded permutation, then apply
    reverse Cuthill-McKee so that node numbers follow mesh adjacency."""
    n = mesh.n_nodes
    xyz, tets, faces = mesh.xyz, mesh.tets, mesh.faces
    if seed is not None:
        perm = np.random.default_rng(seed).permutation(n)
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        xyz, tets, faces = xyz[perm], inv[tets], inv[faces]
    r = np.repeat(tets, 4, axis=1).ravel()
    c = np.tile(tets, (1, 4)).ravel()
    g = sp.csr_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(n, n))
    order = reverse_cuthill_mckee(g, symmetric_mode=True)
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    tets = inv[tets].astype(np.int32)
    faces = inv[faces].astype(np.int32)
    # elements sorted by their smallest node id: neighbouring elements share nodes
    eo = np.lexsort((tets.max(axis=1), tets.min(axis=1)))
    return Mesh(xyz[order].copy(), tets[eo].copy(), faces, mesh.face_group.copy(),
                mesh.group_kind.copy(), dict(mesh.info))


# ------------------------------------------------------------- structured

def _ring_disk(n_rings: int, radius: float):
    """Triangulated disk: centre node plus rings of 6k nodes."""
    pts = [(0.0, 0.0)]
    rings = [[0]]
    for k in range(1, n_rings + 1):
        m = 6 * k
        th = 2.0 * np.pi * np.arange(m) / m
        r = radius * k / n_rings
        ids = list(range(len(pts), len(pts) + m))
        pts.extend(zip(r * np.cos(th), r * np.sin(th)))
        rings.append(ids)
    pts = np.array(pts)
    tris = []
    for k in range(1, n_rings + 1):
        A, B = rings[k - 1], rings[k]
        na, nb = len(A), len(B)
        if na == 1:
            for j in range(nb):
                tris.append((A[0], B[j], B[(j + 1) % nb]))
            continue
        i = j = 0
        while i < na or j < nb:
            ta = 2 * np.pi * (i + 1) / na
            tb = 2 * np.pi * (j + 1) / nb
            if i < na and (j == nb or ta <= tb):
                tris.append((A[i], A[(i + 1) % na], B[j % nb]))
                i += 1
            else:
                tris.append((A[i % na], B[j], B[(j + 1) % nb]))
                j += 1
    return pts, np.array(tris, dtype=np.int64)


def _extrude(pts2, tris, zs):
    n2 = pts2.shape[0]
    ns = len(zs)
    xyz = np.zeros((n2 * ns, 3))
    for s, z in enumerate(zs):
        xyz[s * n2:(s + 1) * n2, :2] = pts2
        xyz[s * n2:(s + 1) * n2, 2] = z
    t = np.sort(tris, axis=1)
    out = []
    for s in range(ns - 1):
        b = t + s * n2
        u = b + n2
        v0, v1, v2 = b[:, 0], b[:, 1], b[:, 2]
        w0, w1, w2 = u[:, 0], u[:, 1], u[:, 2]
        # conforming prism split: each quad diagonal joins the lower-numbered
        # bottom vertex to the higher-numbered top vertex
        out.append(np.stack([v0, v1, v2, w2], 1))
        out.append(np.stack([v0, v1, w1, w2], 1))
        out.append(np.stack([v0, w0, w1, w2], 1))
    tets = np.concatenate(out).astype(np.int32)
    return xyz, orient_positive(xyz, tets)


def cylinder_mesh(radius=1.0, length=6.0, n_rings=5, n_z=20, reorder=True) -> Mesh:
    """Straight pipe along +z; inlet disk at z=0, outlet disk at z=length."""
    pts2, tris = _ring_disk(n_rings, radius)
    zs = np.linspace(0.0, length, n_z + 1)
    xyz, tets = _extrude(pts2, tris, zs)
    faces = boundary_faces(xyz, tets)
    cz = xyz[faces].mean(axis=1)[:, 2]
    tol = 1e-9 * length
    grp = np.where(cz < tol, 1, np.where(cz > length - tol, 2, 0)).astype(np.int32)
    m = Mesh(xyz, tets, faces, grp, np.array([WALL, INLET, OUTLET], np.int32),
             dict(kind="cylinder", radius=radius, length=length, axis=2,
                  inlets=[dict(group=1, center=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0),
                               radius=radius)]))
    return rcm_reorder(m) if reorder else m


def cube_mesh(n: int, jitter: float = 0.0, seed: int = 0, size: float = 1.0) -> Mesh:
    """Unit cube split into n^3 cubes of 6 Kuhn tetrahedra each.  Interior
    nodes are displaced by up to ``jitter`` cell widths.  All boundary faces
    form one wall group and one outlet group (the face x = size)."""
    g = np.linspace(0.0, size, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)

    def nid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    off = np.eye(3, dtype=np.int64)
    tets = []
    for p in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        c = np.zeros((i.size, 3), np.int64)
        vs = [nid(i, j, k)]
        for ax in p:
            c = c + off[ax]
            vs.append(nid(i + c[:, 0], j + c[:, 1], k + c[:, 2]))
        tets.append(np.stack(vs, 1))
    tets = np.concatenate(tets).astype(np.int32)
    h = size / n
    if jitter > 0:
        rng = np.random.default_rng(seed)
        inner = np.all((xyz > 1e-12) & (xyz < size - 1e-12), axis=1)
        xyz[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    tets = orient_positive(xyz, tets)
    faces = boundary_faces(xyz, tets)
    cx = xyz[faces].mean(axis=1)[:, 0]
    grp = np.where(cx > size - 1e-9, 1, 0).astype(np.int32)
    return Mesh(xyz, tets, faces, grp, np.array([WALL, OUTLET], np.int32),
                dict(kind="cube", n=n, h=h, size=size))


# ------------------------------------------------------------ carved lattices

def _kuhn_lattice(lo, counts, h):
    nx, ny, nz = counts
    gx = lo[0] + h * np.arange(nx + 1)
    gy = lo[1] + h * np.arange(ny + 1)
    gz = lo[2] + h * np.arange(nz + 1)

    def nid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    off = np.eye(3, dtype=np.int64)
    tets = []
    for p in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        c = np.zeros((i.size, 3), np.int64)
        vs = [nid(i, j, k)]
        for ax in p:
            c = c + off[ax]
            vs.append(nid(i + c[:, 0], j + c[:, 1], k + c[:, 2]))
        tets.append(np.stack(vs, 1))
    tets = np.concatenate(tets)
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    return xyz, tets


def _inside_tube(p, a, b, r):
    """Points p inside the finite cylinder with axis a->b and radius r."""
    ab = np.asarray(b, float) - np.asarray(a, float)
    L = np.linalg.norm(ab)
    e = ab / L
    d = p - np.asarray(a, float)
    s = d @ e
    rad = np.linalg.norm(d - s[:, None] * e, axis=1)
    return (s >= 0) & (s <= L) & (rad <= r)


def carve(lo, counts, h, inside, jitter, seed, plane_groups):
    """Keep lattice tetrahedra whose centroid satisfies ``inside``; jitter
    interior nodes; classify boundary faces lying on the given planes.

    plane_groups: list of (axis, value, group_id); remaining boundary faces
    go to group 0 (wall)."""
    xyz, tets = _kuhn_lattice(lo, counts, h)
    cen = xyz[tets].mean(axis=1)
    keep = np.zeros(tets.shape[0], bool)
    chunk = 1 << 20
    for s in range(0, tets.shape[0], chunk):
        keep[s:s + chunk] = inside(cen[s:s + chunk])
    xyz, tets = compact(xyz, tets[keep])
    xyz, tets = largest_component(xyz, tets)
    tets = orient_positive(xyz, tets)
    faces = boundary_faces(xyz, tets)
    bnd = np.zeros(xyz.shape[0], bool)
    bnd[faces.ravel()] = True
    if jitter > 0:
        rng = np.random.default_rng(seed)
        inner = ~bnd
        xyz = xyz.copy()
        xyz[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    grp = np.zeros(faces.shape[0], np.int32)
    fx = xyz[faces]
    for axis, val, gid in plane_groups:
        on = np.all(np.abs(fx[:, :, axis] - val) < 1e-6 * h, axis=1)
        grp[on] = gid
    return xyz, tets, faces, grp


def tjunction_mesh(h: float = 3.0 / 70.0, jitter: float = 0.15, seed: int = 1234,
                   r_in: float = 0.5, l_in: float = 3.0, r_out: float = 0.6,
                   l_out: float = 6.0, reorder_seed: int | None = 1234) -> Mesh:
    """Two inlet tubes (radius r_in, length l_in) along x meeting head-on at
    the origin, and an outlet tube (radius r_out, length l_out) along +y.
    Inlet planes x = -l_in and x = +l_in; outlet plane y = l_out."""
    lo = np.array([-l_in, -r_out, -r_out])
    hi = np.array([l_in, l_out, r_out])
    counts = np.rint((hi - lo) / h).astype(int)
    if np.any(np.abs(counts * h - (hi - lo)) > 1e-9):
        raise ValueError("h must divide the bounding box")

    def inside(p):
        return (_inside_tube(p, (-l_in, 0, 0), (0, 0, 0), r_in)
                | _inside_tube(p, (l_in, 0, 0), (0, 0, 0), r_in)
                | _inside_tube(p, (0, 0, 0), (0, l_out, 0), r_out))

    xyz, tets, faces, grp = carve(lo, counts, h, inside, jitter, seed,
                                  [(0, -l_in, 1), (0, l_in, 2), (1, l_out, 3)])
    m = Mesh(xyz, tets, faces, grp,
             np.array([WALL, INLET, INLET, OUTLET], np.int32),
             dict(kind="tjunction", h=h, r_in=r_in, r_out=r_out, l_in=l_in, l_out=l_out,
                  inlets=[dict(group=1, center=(-l_in, 0.0, 0.0), normal=(1.0, 0.0, 0.0),
                               radius=r_in),
                          dict(group=2, center=(l_in, 0.0, 0.0), normal=(-1.0, 0.0, 0.0),
                               radius=r_in)]))
    return rcm_reorder(m, seed=reorder_seed)


def stenosed_pipe_mesh(severity: float, z_s: float, n_rings: int = 12, n_z: int = 90,
                       radius: float = 1.0, length: float = 6.0, ell: float = 1.0) -> Mesh:
    """The straight pipe of cylinder_mesh, radially morphed by
    r(z) = 1 - s/2 (1 + cos(pi (z - z_s)/ell)) for |z - z_s| < ell.  The
    topology (connectivity, node order) is independent of the parameters."""
    base = cylinder_mesh(radius, length, n_rings, n_z, reorder=False)
    xyz = base.xyz.copy()
    dz = xyz[:, 2] - z_s
    f = np.where(np.abs(dz) < ell, 1.0 - severity * 0.5 * (1.0 + np.cos(np.pi * dz / ell)), 1.0)
    xyz[:, :2] *= f[:, None]
    m = Mesh(xyz, base.tets, base.faces, base.face_group, base.group_kind,
             dict(base.info, kind="stenosed", severity=severity, z_s=z_s))
    return m


# ------------------------------------------------------- branching artery

def _arc_frame(d0, rng):
    """A unit vector normal to d0, seeded."""
    t = rng.normal(size=3)
    t -= (t @ d0) * d0
    return t / np.linalg.norm(t)


def artery_tree(seed: int = 7, radii=(2.0, 1.26, 0.79, 0.50), length_factor: float = 6.0,
                branch_angle: float = 0.5, max_turn: float = 0.35):
    """Segments of a symmetric bifurcating tree: the root along +z from the
    origin, each parent splitting into two children (radius ratio 0.63) at
    +-branch_angle about a seeded axis; every segment is a circular arc of
    length 6 r whose total turn is drawn from U[0, max_turn] about a seeded
    normal.  Returns a list of dicts (p0, d0, n, kappa, L, r, level, end,
    d_end)."""
    rng = np.random.default_rng(seed)
    segs = []

    def add(p0, d0, level):
        r = radii[level]
        L = length_factor * r
        n = _arc_frame(d0, rng)
        turn = rng.uniform(0.0, max_turn)
        kappa = max(turn / L, 1e-6)
        ph = kappa * L
        end = p0 + np.sin(ph) / kappa * d0 + (1.0 - np.cos(ph)) / kappa * n
        d_end = np.cos(ph) * d0 + np.sin(ph) * n
        segs.append(dict(p0=p0, d0=d0, n=n, kappa=kappa, L=L, r=r, level=level, end=end,
                         d_end=d_end))
        if level + 1 < len(radii):
            ax = _arc_frame(d_end, rng)
            for sgn in (1.0, -1.0):
                dc = np.cos(branch_angle) * d_end + sgn * np.sin(branch_angle) * ax
                add(end, dc / np.linalg.norm(dc), level + 1)

    add(np.zeros(3), np.array([0.0, 0.0, 1.0]), 0)
    return segs


def _inside_arc(p, sg):
    """Points within distance r of the arc (arclength in [0, L]), and the
    arclength parameter of the nearest arc point."""
    d = p - sg["p0"]
    b = np.cross(sg["d0"], sg["n"])
    u, v, w = d @ sg["d0"], d @ sg["n"], d @ b
    k = sg["kappa"]
    phi = np.arctan2(u * k, 1.0 - v * k)
    ok = (phi >= 0.0) & (phi <= k * sg["L"])
    du = u - np.sin(phi) / k
    dv = v - (1.0 - np.cos(phi)) / k
    return ok & (du * du + dv * dv + w * w <= sg["r"] ** 2)


def branching_artery_mesh(h: float = 0.062, seed: int = 7, jitter: float = 0.15,
                          jitter_seed: int = 1234, reorder_seed: int | None = 1234) -> Mesh:
    """Carve a Kuhn lattice of spacing h to the union of the tree's arc tubes
    and a ball of the parent radius at each branch point.  Only lattice
    cells near each segment are generated.  Groups: 0 wall, 1 root inlet
    (the plane z = 0), 2..9 the leaf outlets (faces within h of a leaf's end
    plane and inside its radius)."""
    segs = artery_tree(seed)
    balls = [(sg["end"], sg["r"]) for sg in segs if sg["level"] + 1 < 4]
    off = np.eye(3, dtype=np.int64)
    perms = ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0])
    kept = []
    for si, sg in enumerate(segs):
        # bounding box of the arc (sampled) plus radius
        tt = np.linspace(0.0, sg["L"], 64)
        ph = sg["kappa"] * tt
        pts = (sg["p0"] + np.outer(np.sin(ph) / sg["kappa"], sg["d0"])
               + np.outer((1.0 - np.cos(ph)) / sg["kappa"], sg["n"]))
        pad = sg["r"] * (1.0 if sg["level"] + 1 == 4 else 1.0) + 2 * h
        if sg["level"] + 1 < 4:
            pts = np.vstack([pts, sg["end"] + sg["r"], sg["end"] - sg["r"]])
        lo = np.floor((pts.min(0) - pad) / h).astype(np.int64)
        hi = np.ceil((pts.max(0) + pad) / h).astype(np.int64)
        lo[2] = max(lo[2], 0)               # nothing below the inlet plane z = 0
        gi = [np.arange(lo[a], hi[a]) for a in range(3)]
        I, J, K = np.meshgrid(*gi, indexing="ij")
        cells = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
        cen = (cells + 0.5) * h
        near = _inside_arc(cen, dict(sg, r=sg["r"] + h))
        for (c, r) in balls:
            near |= np.sum((cen - c) ** 2, axis=1) <= (r + h) ** 2
        cells = cells[near]
        for t, p in enumerate(perms):
            c = np.zeros_like(cells)
            vs = [cells.copy()]
            for ax in p:
                c = c + off[ax]
                vs.append(cells + c)
            v = np.stack(vs, 1)                         # (m, 4, 3) lattice points
            cen_t = v.mean(axis=1) * h
            ins = _inside_arc(cen_t, sg)
            if sg["level"] + 1 < 4:
                ins |= np.sum((cen_t - sg["end"]) ** 2, axis=1) <= sg["r"] ** 2
            kept.append((v[ins], cells[ins], t))
    # de-duplicate tetrahedra generated by more than one segment: key = (cell, type)
    V = np.concatenate([k[0] for k in kept])
    C = np.concatenate([k[1] for k in kept])
    T = np.concatenate([np.full(k[1].shape[0], k[2]) for k in kept])
    base = C.min(0)
    span = C.max(0) - base + 2
    lin = ((C[:, 0] - base[0]) * span[1] + (C[:, 1] - base[1])) * span[2] + (C[:, 2] - base[2])
    _, first = np.unique(lin * 6 + T, return_index=True)
    V = V[first]
    vb = V.reshape(-1, 3) - base
    vid = (vb[:, 0] * span[1] + vb[:, 1]) * span[2] + vb[:, 2]
    uniq, inv = np.unique(vid, return_inverse=True)
    tets = inv.reshape(-1, 4)
    iz = uniq % span[2]
    iy = (uniq // span[2]) % span[1]
    ix = uniq // (span[1] * span[2])
    xyz = (np.stack([ix, iy, iz], 1) + base) * h
    xyz, tets = largest_component(xyz, tets.astype(np.int64))
    tets = orient_positive(xyz, tets)
    faces = boundary_faces(xyz, tets)
    bnd = np.zeros(xyz.shape[0], bool)
    bnd[faces.ravel()] = True
    if jitter > 0:
        rng = np.random.default_rng(jitter_seed)
        inner = ~bnd
        xyz = xyz.copy()
        xyz[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    grp = np.zeros(faces.shape[0], np.int32)
    fc = xyz[faces].mean(axis=1)
    fz = xyz[faces][:, :, 2]
    grp[np.all(np.abs(fz) < 1e-9, axis=1)] = 1
    leaves = [sg for sg in segs if sg["level"] == 3]
    for li, sg in enumerate(leaves):
        d = fc - sg["end"]
        ax = d @ sg["d_end"]
        lat = np.linalg.norm(d - np.outer(ax, sg["d_end"]), axis=1)
        grp[(grp == 0) & (np.abs(ax) < h) & (lat < sg["r"] - 0.25 * h)] = 2 + li
    kinds = np.array([WALL, INLET] + [OUTLET] * len(leaves), np.int32)
    m = Mesh(xyz, tets.astype(np.int32), faces, grp, kinds,
             dict(kind="branching_artery", h=h, seed=seed, r_root=2.0, n_leaves=len(leaves),
                  inlets=[dict(group=1, center=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0),
                               radius=2.0)]))
    return rcm_reorder(m, seed=reorder_seed)
