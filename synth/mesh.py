"""Structured simplex meshes of the unit square / unit cube.

The paper's 2D convergence meshes (Table 1) are N x N squares with every
cell cut into two triangles: (N+1)^2 vertices, 2 N^2 triangles and
3 N^2 + 2 N edges (its "dual elements").  The 3D workloads use the Kuhn
split of each cube cell into six tetrahedra, which is conforming and has
(n+1)^3 vertices and 6 n^3 tetrahedra.

Numbering (all integer, fixed):
  * lattice node (i, j[, k]) has id  i + (n+1) * (j + (n+1) * k);
  * 2D cell (i, j) has id i + n*j and yields triangles 2*cell + t,
      t = 0: [v(i,j), v(i+1,j), v(i+1,j+1)],
      t = 1: [v(i,j), v(i+1,j+1), v(i,j+1)]      (both counter-clockwise);
  * 3D cell (i, j, k) has id i + n*(j + n*k) and yields tetrahedra
    6*cell + s for the axis permutations s in lexicographic order
    (012, 021, 102, 120, 201, 210); the tetrahedron of permutation
    (a, b, c) is [v0, v0 + e_a, v0 + e_a + e_b, v0 + (1,1,1)], and for the
    odd permutations (021, 102, 210) vertices 1 and 2 are swapped so that
    every tetrahedron has positive orientation (decided from the parity of
    the permutation, not from floating point).

Coordinates: interior nodes (no lattice index equal to 0 or n) are moved by
a seeded jitter of up to ``jitter`` * h per axis,
    x = (i + jitter * (2u - 1)) / n,  u = uniform(seed, 1, 3*id + axis),
evaluated in that order; boundary nodes stay on the lattice so the domain
is exactly the unit square/cube.  Every boundary node is a Dirichlet
pressure node.
"""

from dataclasses import dataclass

import numpy as np

from .rng import STREAM_JITTER, uniform


@dataclass
class Mesh:
    dim: int
    n: int                    # cells per axis
    coords: np.ndarray        # float64 [n_nodes, dim]
    elems: np.ndarray         # int32  [n_elems, dim+1]
    dirichlet: np.ndarray     # uint8  [n_nodes]
    lattice: np.ndarray       # int32  [n_nodes, dim]
    period: object = None     # float64 [dim] (0 = open axis) for a periodic mesh, else None
    unmerged: object = None   # periodic mesh: the same mesh before its images were merged
    rep: object = None        # periodic mesh: merged node of each unmerged node

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_elems(self):
        return self.elems.shape[0]

    @property
    def h(self):
        return 1.0 / self.n


# Kuhn permutations in lexicographic order and their parity (1 = odd).
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
KUHN_ODD = (0, 1, 1, 0, 0, 1)


def table1_counts(N):
    """Vertices, triangles and edges of the N x N two-triangle split."""
    return (N + 1) ** 2, 2 * N * N, 3 * N * N + 2 * N


def _lattice(dim, n):
    m = n + 1
    ids = np.arange(m ** dim, dtype=np.int64)
    lat = np.empty((m ** dim, dim), dtype=np.int32)
    rem = ids
    for ax in range(dim):
        lat[:, ax] = rem % m
        rem = rem // m
    return lat


def _elements_2d(n):
    m = n + 1
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i = i.ravel().astype(np.int64)
    j = j.ravel().astype(np.int64)
    v00 = i + m * j
    v10 = v00 + 1
    v11 = v00 + 1 + m
    v01 = v00 + m
    el = np.empty((n * n, 2, 3), dtype=np.int64)
    el[:, 0] = np.stack([v00, v10, v11], axis=1)
    el[:, 1] = np.stack([v00, v11, v01], axis=1)
    return el.reshape(-1, 3).astype(np.int32)


def _elements_3d(n):
    m = n + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i = i.ravel().astype(np.int64)
    j = j.ravel().astype(np.int64)
    k = k.ravel().astype(np.int64)
    v0 = i + m * (j + m * k)
    step = (1, m, m * m)
    el = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for s, (a, b, _c) in enumerate(KUHN_PERMS):
        w1 = v0 + step[a]
        w2 = w1 + step[b]
        w3 = v0 + step[0] + step[1] + step[2]
        if KUHN_ODD[s]:
            el[:, s] = np.stack([v0, w2, w1, w3], axis=1)
        else:
            el[:, s] = np.stack([v0, w1, w2, w3], axis=1)
    return el.reshape(-1, 4).astype(np.int32)


def structured_mesh(dim, n, jitter=0.0, seed=0):
    """Unit square (dim 2) or cube (dim 3) with n cells per axis."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1:
        raise ValueError("n must be >= 1")
    lat = _lattice(dim, n)
    interior = np.all((lat > 0) & (lat < n), axis=1)
    coords = lat.astype(np.float64)
    if jitter != 0.0:
        ids = np.nonzero(interior)[0].astype(np.uint64)
        for ax in range(dim):
            u = uniform(seed, STREAM_JITTER, np.uint64(3) * ids + np.uint64(ax))
            coords[ids.astype(np.int64), ax] = lat[ids.astype(np.int64), ax] + jitter * (2.0 * u - 1.0)
    coords = coords / float(n)
    elems = _elements_2d(n) if dim == 2 else _elements_3d(n)
    dirichlet = (~interior).astype(np.uint8)
    return Mesh(dim=dim, n=n, coords=np.ascontiguousarray(coords), elems=elems,
                dirichlet=dirichlet, lattice=lat)


def fan_mesh(k=80):
    """An unstructured 2D mesh with one high-degree node: the centre of a
    disk joined to a ring of k nodes at radius 1 (k triangles meet there),
    and a second ring of k nodes at radius 2 joined to the first by 2k
    triangles.  The outer ring is Dirichlet.  Counter-clockwise triangles;
    no lattice (Morton keys come from the coordinates)."""
    ang = 2.0 * np.pi * np.arange(k) / k
    ring1 = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    ring2 = 2.0 * np.stack([np.cos(ang + np.pi / k), np.sin(ang + np.pi / k)], axis=1)
    coords = np.concatenate([np.zeros((1, 2)), ring1, ring2]).astype(np.float64)
    a = 1 + np.arange(k)
    b = 1 + (np.arange(k) + 1) % k
    c = 1 + k + np.arange(k)
    tri = [np.stack([np.zeros(k, dtype=np.int64), a, b], axis=1),
           np.stack([a, c, b], axis=1),
           np.stack([b, c, 1 + k + (np.arange(k) + 1) % k], axis=1)]
    elems = np.concatenate(tri).astype(np.int32)
    dirichlet = np.zeros(coords.shape[0], dtype=np.uint8)
    dirichlet[1 + k:] = 1
    return Mesh(2, 0, coords, elems, dirichlet, None)


def periodic_mesh(dim, n, periodic_axes, jitter=0.0, seed=0):
    """The unit square/cube with n cells per axis, periodic along
    ``periodic_axes`` (Sec. 3.6: the mesh is periodic and the matching
    boundary vertices are merged, so there are fewer pressure unknowns).

    Merged nodes have lattice indices i_ax in [0, n) on a periodic axis and
    [0, n] on an open one, numbered i0 + m0 (i1 + m1 i2) with m_ax the count
    per axis.  Node coordinates are (i + jitter (2u - 1)) / n with
    u = uniform(seed, 1, 3 id + axis); nodes on an open boundary stay on the
    lattice, every other node (also those on a periodic boundary, which may
    then leave [0, 1)) is jittered.  Elements are those of
    structured_mesh(dim, n) with each vertex replaced by its merged node.
    The nodes on the open boundaries are Dirichlet nodes.

    The returned mesh carries ``period`` (1 on the periodic axes, 0 on the
    open ones), ``unmerged`` (the structured mesh of (n+1)^dim nodes in which
    every image has its own coordinates: those of its merged node plus one
    period per wrapped axis) and ``rep`` (the merged node of each unmerged
    node)."""
    axes = sorted(set(int(a) for a in periodic_axes))
    if dim not in (2, 3) or not axes or any(a < 0 or a >= dim for a in axes):
        raise ValueError("bad dim or periodic axes")
    if n < 3:
        raise ValueError("a periodic axis needs at least 3 cells")
    per = np.zeros(dim)
    per[axes] = 1.0
    cnt = [n if per[ax] > 0 else n + 1 for ax in range(dim)]
    nm = int(np.prod(cnt))
    ids = np.arange(nm, dtype=np.int64)
    lat = np.empty((nm, dim), dtype=np.int32)
    rem = ids
    for ax in range(dim):
        lat[:, ax] = rem % cnt[ax]
        rem = rem // cnt[ax]
    on_open = np.zeros(nm, dtype=bool)
    for ax in range(dim):
        if per[ax] == 0:
            on_open |= (lat[:, ax] == 0) | (lat[:, ax] == n)
    coords = lat.astype(np.float64)
    if jitter != 0.0:
        moved = np.nonzero(~on_open)[0].astype(np.uint64)
        for ax in range(dim):
            u = uniform(seed, STREAM_JITTER, np.uint64(3) * moved + np.uint64(ax))
            coords[moved.astype(np.int64), ax] = lat[moved.astype(np.int64), ax] + jitter * (2.0 * u - 1.0)
    coords = coords / float(n)
    # unmerged lattice and the merge map
    ulat = _lattice(dim, n)
    rep = np.zeros(ulat.shape[0], dtype=np.int64)
    stride = 1
    for ax in range(dim):
        q = ulat[:, ax] % n if per[ax] > 0 else ulat[:, ax]
        rep += stride * q
        stride *= cnt[ax]
    ucoords = coords[rep] + (ulat // n) * per[None, :]
    uel = _elements_2d(n) if dim == 2 else _elements_3d(n)
    udir = np.zeros(ulat.shape[0], dtype=np.uint8)
    udir[:] = on_open[rep]
    unmerged = Mesh(dim=dim, n=n, coords=np.ascontiguousarray(ucoords), elems=uel, dirichlet=udir, lattice=ulat)
    elems = rep[uel].astype(np.int32)
    return Mesh(dim=dim, n=n, coords=np.ascontiguousarray(coords), elems=elems,
                dirichlet=on_open.astype(np.uint8), lattice=lat, period=per, unmerged=unmerged,
                rep=rep.astype(np.int32))
