"""Seeded synthetic mesh generators: the shared *input* producer.

This module builds the unstructured-mesh description that the finite-volume
solver consumes (Section 3.1 of the paper states the problem: N polyhedral
cells with flat faces, each face shared by two cells or on the boundary,
unknowns at cell centroids).  It produces only inputs -- topology
(owner/neighbour), geometry (face area vectors Sf, face centres Cf, cell
centres C, cell volumes V) and patch ranges -- and holds none of the solver's
arithmetic (no interpolation weights, no coefficients, no Krylov).  Both the
FP64 oracle and the HIP path consume the arrays built here.

Geometry follows the usual polyhedral-mesh construction: a face's area vector
and centre come from the triangle fan about the mean of its vertices, and a
cell's volume and centre from the pyramid decomposition about the mean of its
vertices.  For a closed cell the outward area vectors therefore sum to zero up
to rounding, also for jittered (non-planar) faces.

Cell numbering, face canonical order and patch grouping:
  * cells start lexicographic (i fastest), optionally renumbered by a seeded
    random permutation and/or reverse Cuthill-McKee;
  * internal faces are canonical: owner < neighbour, Sf pointing out of the
    owner, sorted by (owner, neighbour);
  * boundary faces follow, grouped by patch (xmin, xmax, ymin, ymax, zmin,
    zmax), each patch sorted by its cells.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SIDES = ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax")


@dataclass
class Mesh:
    """A polyhedral mesh in face-addressed form (all arrays host numpy)."""

    owner: np.ndarray          # int32 [n_faces]
    neighbour: np.ndarray      # int32 [n_internal]
    Sf: np.ndarray             # float64 [n_faces, 3], out of the owner
    Cf: np.ndarray             # float64 [n_faces, 3]
    C: np.ndarray              # float64 [n_cells, 3]
    V: np.ndarray              # float64 [n_cells]
    patch_names: List[str]
    patch_start: np.ndarray    # int32 [n_patches]
    patch_size: np.ndarray     # int32 [n_patches]
    shape: Tuple[int, int, int] = (0, 0, 0)
    lengths: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    # lexicographic index of each cell (identity before renumbering)
    lex_of_cell: Optional[np.ndarray] = None

    @property
    def n_cells(self) -> int:
        return int(self.V.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])

    @property
    def n_internal(self) -> int:
        return int(self.neighbour.shape[0])

    def patch(self, name: str) -> Tuple[int, int]:
        i = self.patch_names.index(name)
        return int(self.patch_start[i]), int(self.patch_size[i])


def _axis_points(n: int, length: float, origin: float, grading: Optional[Sequence[float]]) -> np.ndarray:
    if grading is None:
        return origin + length * np.arange(n + 1, dtype=np.float64) / n
    g = np.asarray(grading, dtype=np.float64)
    assert g.shape == (n,) and np.all(g > 0)
    x = np.concatenate([[0.0], np.cumsum(g)])
    return origin + length * x / x[-1]


def _fan_geometry(P: np.ndarray, quads: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Area vector and centre of each quad (vertex ids [F,4]) by the triangle
    fan about the vertex mean."""
    v = P[quads]                                   # [F,4,3]
    m = v.mean(axis=1)                             # [F,3]
    Sf = np.zeros_like(m)
    acc = np.zeros_like(m)
    wsum = np.zeros(m.shape[0])
    for t in range(4):
        a = v[:, t] - m
        b = v[:, (t + 1) % 4] - m
        at = 0.5 * np.cross(a, b)
        ct = (v[:, t] + v[:, (t + 1) % 4] + m) / 3.0
        mag = np.linalg.norm(at, axis=1)
        Sf += at
        acc += mag[:, None] * ct
        wsum += mag
    Cf = acc / wsum[:, None]
    return Sf, Cf


def _uniform_box(nx, ny, nz, lengths, origin, owner, own_i, nei_i, b_own, p_start, p_size, I, J, K) -> "Mesh":
    """Closed-form geometry of a uniform, axis-aligned box mesh (the same
    quantities the triangle-fan / pyramid construction gives, without the
    per-vertex work)."""
    h = np.array([lengths[0] / nx, lengths[1] / ny, lengths[2] / nz])
    org = np.asarray(origin, dtype=np.float64)
    N = nx * ny * nz
    ijk = np.stack([I, J, K], axis=1).astype(np.float64)
    C = org + (ijk + 0.5) * h
    V = np.full(N, h[0] * h[1] * h[2])
    area = np.array([h[1] * h[2], h[0] * h[2], h[0] * h[1]])
    Fi = own_i.shape[0]
    d = nei_i - own_i
    axis = np.where(d == 1, 0, np.where(d == nx, 1, 2))
    if nx == 1:
        axis = np.where(d == nx * ny, 2, 1) if ny > 1 else np.full(Fi, 2)
    if nx > 1 and ny == 1:
        axis = np.where(d == 1, 0, 2)
    Sf_i = np.zeros((Fi, 3))
    Sf_i[np.arange(Fi), axis] = area[axis]
    Cf_i = C[own_i].copy()
    Cf_i[np.arange(Fi), axis] += 0.5 * h[axis]
    Sf_b, Cf_b = [], []
    for side, cells in zip(SIDES, b_own):
        ax = "xyz".index(side[0])
        sgn = -1.0 if side.endswith("min") else 1.0
        S = np.zeros((cells.shape[0], 3)); S[:, ax] = sgn * area[ax]
        Cf = C[cells].copy(); Cf[:, ax] += sgn * 0.5 * h[ax]
        Sf_b.append(S); Cf_b.append(Cf)
    return Mesh(owner=owner, neighbour=nei_i.astype(np.int32), Sf=np.concatenate([Sf_i] + Sf_b),
                Cf=np.concatenate([Cf_i] + Cf_b), C=C, V=V, patch_names=list(SIDES),
                patch_start=np.array(p_start, np.int32), patch_size=np.array(p_size, np.int32),
                shape=(nx, ny, nz), lengths=tuple(float(x) for x in lengths), lex_of_cell=np.arange(N, dtype=np.int64))


def box_mesh(nx: int, ny: int, nz: int,
             lengths: Tuple[float, float, float] = (1.0, 1.0, 1.0),
             origin: Tuple[float, float, float] = (0.0, 0.0, 0.0),
             jitter: float = 0.0, seed: Optional[int] = None,
             grading: Optional[Tuple[Optional[Sequence[float]], ...]] = None) -> Mesh:
    """Hexahedral box mesh of nx*ny*nz cells.

    jitter: interior vertices move by a uniform random offset in
    [-jitter*h, +jitter*h] per component (h = cell size along that axis),
    drawn from numpy.random.default_rng(seed).  For nz == 1 (a 2-D slab) only
    x/y move and both z-layers move together, so the front/back faces stay
    planar.
    grading: optional per-axis positive spacing ratios (non-uniform but
    orthogonal meshes).
    """
    assert nx >= 1 and ny >= 1 and nz >= 1
    gr = grading or (None, None, None)
    xs = _axis_points(nx, lengths[0], origin[0], gr[0])
    ys = _axis_points(ny, lengths[1], origin[1], gr[1])
    zs = _axis_points(nz, lengths[2], origin[2], gr[2])
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")          # [nx+1, ny+1, nz+1]
    P = np.stack([X, Y, Z], axis=-1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        h = np.array([lengths[0] / nx, lengths[1] / ny, lengths[2] / nz])
        if nz == 1:
            d = rng.uniform(-jitter, jitter, size=(nx + 1, ny + 1, 2)) * h[:2]
            inner = np.zeros((nx + 1, ny + 1), dtype=bool)
            inner[1:nx, 1:ny] = True
            d[~inner] = 0.0
            P[..., :2] += d[:, :, None, :]
        else:
            d = rng.uniform(-jitter, jitter, size=P.shape) * h
            inner = np.zeros(P.shape[:3], dtype=bool)
            inner[1:nx, 1:ny, 1:nz] = True
            d[~inner] = 0.0
            P = P + d
    # flatten points: id = i + (nx+1)*(j + (ny+1)*k)
    Pf = P.transpose(2, 1, 0, 3).reshape(-1, 3)

    def pid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    def cid(i, j, k):
        return i + nx * (j + ny * k)

    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I = I.transpose(2, 1, 0).ravel()
    J = J.transpose(2, 1, 0).ravel()
    K = K.transpose(2, 1, 0).ravel()
    N = nx * ny * nz
    cells = cid(I, J, K)
    assert np.array_equal(cells, np.arange(N))

    # quads whose right-hand normal points along +x, +y, +z at the lower-index
    # corner (i, j, k) of the plane x=i, y=j, z=k respectively
    def quad_x(i, j, k):
        return np.stack([pid(i, j, k), pid(i, j + 1, k), pid(i, j + 1, k + 1), pid(i, j, k + 1)], axis=-1)

    def quad_y(i, j, k):
        return np.stack([pid(i, j, k), pid(i, j, k + 1), pid(i + 1, j, k + 1), pid(i + 1, j, k)], axis=-1)

    def quad_z(i, j, k):
        return np.stack([pid(i, j, k), pid(i + 1, j, k), pid(i + 1, j + 1, k), pid(i, j + 1, k)], axis=-1)

    own_l, nei_l, quad_l = [], [], []
    m = I < nx - 1
    own_l.append(cells[m]); nei_l.append(cells[m] + 1); quad_l.append(quad_x(I[m] + 1, J[m], K[m]))
    m = J < ny - 1
    own_l.append(cells[m]); nei_l.append(cells[m] + nx); quad_l.append(quad_y(I[m], J[m] + 1, K[m]))
    m = K < nz - 1
    own_l.append(cells[m]); nei_l.append(cells[m] + nx * ny); quad_l.append(quad_z(I[m], J[m], K[m] + 1))
    own_i = np.concatenate(own_l)
    nei_i = np.concatenate(nei_l)
    quad_i = np.concatenate(quad_l)
    order = np.lexsort((nei_i, own_i))
    own_i, nei_i, quad_i = own_i[order], nei_i[order], quad_i[order]

    b_own, b_quad, p_start, p_size = [], [], [], []
    start = own_i.shape[0]
    for side in SIDES:
        if side == "xmin":
            m = I == 0; q = quad_x(I[m], J[m], K[m])[:, ::-1]
        elif side == "xmax":
            m = I == nx - 1; q = quad_x(I[m] + 1, J[m], K[m])
        elif side == "ymin":
            m = J == 0; q = quad_y(I[m], J[m], K[m])[:, ::-1]
        elif side == "ymax":
            m = J == ny - 1; q = quad_y(I[m], J[m] + 1, K[m])
        elif side == "zmin":
            m = K == 0; q = quad_z(I[m], J[m], K[m])[:, ::-1]
        else:
            m = K == nz - 1; q = quad_z(I[m], J[m], K[m] + 1)
        b_own.append(cells[m]); b_quad.append(q)
        p_start.append(start); p_size.append(int(m.sum())); start += int(m.sum())

    owner = np.concatenate([own_i] + b_own).astype(np.int32)
    quads = np.concatenate([quad_i] + b_quad)
    if jitter == 0.0 and grading is None:
        return _uniform_box(nx, ny, nz, lengths, origin, owner, own_i, nei_i, b_own, p_start, p_size, I, J, K)
    Sf, Cf = _fan_geometry(Pf, quads)

    # cell geometry: pyramids on each face about the cell vertex mean
    corner = np.stack([pid(I + a, J + b, K + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], axis=-1)
    mc = Pf[corner].mean(axis=1)
    Fi = own_i.shape[0]
    V = np.zeros(N)
    Cacc = np.zeros((N, 3))
    nb = np.concatenate([nei_i, np.full(owner.shape[0] - Fi, -1)])
    for sgn, cellsel in ((1.0, owner), (-1.0, nb)):
        sel = cellsel >= 0
        cc = cellsel[sel]
        S = sgn * Sf[sel]
        dC = Cf[sel] - mc[cc]
        pv = np.einsum("ij,ij->i", S, dC) / 3.0
        pc = mc[cc] + 0.75 * dC
        V += np.bincount(cc, weights=pv, minlength=N)
        for k in range(3):
            Cacc[:, k] += np.bincount(cc, weights=pv * pc[:, k], minlength=N)
    C = Cacc / V[:, None]
    return Mesh(owner=owner, neighbour=nei_i.astype(np.int32), Sf=Sf, Cf=Cf, C=C, V=V,
                patch_names=list(SIDES), patch_start=np.array(p_start, np.int32),
                patch_size=np.array(p_size, np.int32), shape=(nx, ny, nz),
                lengths=tuple(float(x) for x in lengths), lex_of_cell=np.arange(N, dtype=np.int64))


def renumber(mesh: Mesh, new_of_old: np.ndarray) -> Mesh:
    """Renumber cells (new id = new_of_old[old id]) and re-canonicalise the
    internal faces (owner < neighbour, sorted by (owner, neighbour)); each
    boundary patch is re-sorted by its (new) cell ids."""
    new_of_old = np.asarray(new_of_old, dtype=np.int64)
    N = mesh.n_cells
    assert np.array_equal(np.sort(new_of_old), np.arange(N))
    Fi = mesh.n_internal
    o = new_of_old[mesh.owner[:Fi]]
    n = new_of_old[mesh.neighbour]
    flip = o > n
    lo = np.where(flip, n, o)
    hi = np.where(flip, o, n)
    Sf_i = np.where(flip[:, None], -mesh.Sf[:Fi], mesh.Sf[:Fi])
    order = np.lexsort((hi, lo))
    owner_i, nei, Sf_i, Cf_i = lo[order], hi[order], Sf_i[order], mesh.Cf[:Fi][order]
    b_owner = new_of_old[mesh.owner[Fi:]]
    b_Sf, b_Cf = mesh.Sf[Fi:], mesh.Cf[Fi:]
    b_perm = []
    for s, z in zip(mesh.patch_start, mesh.patch_size):
        idx = np.arange(s - Fi, s - Fi + z)
        b_perm.append(idx[np.argsort(b_owner[idx], kind="stable")])
    b_perm = np.concatenate(b_perm) if b_perm else np.zeros(0, np.int64)
    C = np.empty_like(mesh.C); C[new_of_old] = mesh.C
    V = np.empty_like(mesh.V); V[new_of_old] = mesh.V
    lex = np.empty(N, np.int64); lex[new_of_old] = mesh.lex_of_cell
    return Mesh(owner=np.concatenate([owner_i, b_owner[b_perm]]).astype(np.int32),
                neighbour=nei.astype(np.int32),
                Sf=np.concatenate([Sf_i, b_Sf[b_perm]]), Cf=np.concatenate([Cf_i, b_Cf[b_perm]]),
                C=C, V=V, patch_names=list(mesh.patch_names), patch_start=mesh.patch_start.copy(),
                patch_size=mesh.patch_size.copy(), shape=mesh.shape, lengths=mesh.lengths, lex_of_cell=lex)


def random_permutation(mesh: Mesh, seed: int) -> Mesh:
    """new id = perm[old id], perm = default_rng(seed).permutation(N)."""
    perm = np.random.default_rng(seed).permutation(mesh.n_cells)
    return renumber(mesh, perm)


def rcm(mesh: Mesh) -> Mesh:
    """Reverse Cuthill-McKee renumbering of the cell adjacency graph."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    N = mesh.n_cells
    o = mesh.owner[: mesh.n_internal].astype(np.int64)
    n = mesh.neighbour.astype(np.int64)
    A = coo_matrix((np.ones(2 * o.size), (np.concatenate([o, n]), np.concatenate([n, o]))), shape=(N, N)).tocsr()
    order = reverse_cuthill_mckee(A, symmetric_mode=True)    # new k <- old order[k]
    new_of_old = np.empty(N, np.int64)
    new_of_old[order] = np.arange(N)
    return renumber(mesh, new_of_old)


def shuffle_faces(mesh: Mesh, seed: int, flip_fraction: float = 0.5) -> Mesh:
    """Scramble the internal face order and flip a random subset of internal
    faces (owner <-> neighbour, Sf negated).  The result is a valid but
    non-canonical face list, used to test a consumer's canonicalisation."""
    rng = np.random.default_rng(seed)
    Fi = mesh.n_internal
    order = rng.permutation(Fi)
    flip = rng.random(Fi) < flip_fraction
    o = mesh.owner[:Fi][order].copy(); n = mesh.neighbour[order].copy()
    Sf_i = mesh.Sf[:Fi][order].copy(); Cf_i = mesh.Cf[:Fi][order]
    o2 = np.where(flip, n, o); n2 = np.where(flip, o, n)
    Sf_i[flip] *= -1.0
    return Mesh(owner=np.concatenate([o2, mesh.owner[Fi:]]).astype(np.int32), neighbour=n2.astype(np.int32),
                Sf=np.concatenate([Sf_i, mesh.Sf[Fi:]]), Cf=np.concatenate([Cf_i, mesh.Cf[Fi:]]),
                C=mesh.C.copy(), V=mesh.V.copy(), patch_names=list(mesh.patch_names),
                patch_start=mesh.patch_start.copy(), patch_size=mesh.patch_size.copy(),
                shape=mesh.shape, lengths=mesh.lengths,
                lex_of_cell=None if mesh.lex_of_cell is None else mesh.lex_of_cell.copy())
