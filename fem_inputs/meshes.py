"""Simplicial meshes and Lagrange cell-to-node Maps (inputs only).

Conventions (part of the library's ABI, restated here because the Maps built
below must follow them):

* Cell-to-vertex Map: local vertices 0..d in the order stored in ``cells``.
  Generated cells are positively oriented (the Jacobian whose columns are
  x_m - x_0 has a positive determinant); this is done combinatorially.
* Local node order of a degree-k Lagrange cell: vertices first; then edges in
  lexicographic order of their local vertex pairs ((0,1),(0,2),(0,3),(1,2),
  (1,3),(2,3) on a tetrahedron, (0,1),(0,2),(1,2) on a triangle), the two P3
  nodes of an edge ordered from its lower local vertex; then the P3 face nodes
  of a tetrahedron ((0,1,2),(0,1,3),(0,2,3),(1,2,3)) or the single interior P3
  node of a triangle.  A node is identified by its integer barycentric weights
  (summing to k) with respect to the cell's vertices.
* The unit square is split into n*n squares, each cut along its (x,y) to
  (x+1,y+1) diagonal into (v00,v10,v11) and (v00,v11,v01); vertex id is
  j*(n+1)+i, cell id 2*(j*n+i)+{0,1}.
* The unit cube is split into n^3 cubes, each into the 6 Kuhn (Freudenthal)
  tetrahedra along its (0,0,0)-(1,1,1) diagonal: for each axis permutation p
  the path origin, +e_p0, +e_p0+e_p1, +(1,1,1); odd permutations swap the last
  two vertices to keep a positive orientation.  Vertex id (k*(n+1)+j)*(n+1)+i,
  cell id 6*((k*n+j)*n+i)+permutation index.

The paper's Poisson and Cahn-Hilliard benchmarks run on the unit cube and unit
square (experiments section); its meshes are unstructured and RCM-renumbered,
which the permutation helpers below emulate by seeded shuffles that the
library's own renumbering then undoes.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field as dc_field

import numpy as np


@dataclass
class Mesh:
    dim: int
    coords: np.ndarray            # float64 [V][dim]
    cells: np.ndarray             # int32 [C][dim+1]  cell -> vertex Map
    n: int = 0                    # lattice divisions (0: not a lattice mesh)
    vlat: np.ndarray | None = None  # int64 [V][dim] lattice coordinates
    meta: dict = dc_field(default_factory=dict)

    @property
    def nverts(self) -> int:
        return int(self.coords.shape[0])

    @property
    def ncells(self) -> int:
        return int(self.cells.shape[0])


def unit_square(n: int) -> Mesh:
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    vlat = np.stack([i.ravel(), j.ravel()], 1).astype(np.int64)
    coords = vlat.astype(np.float64) / n
    vid = lambda a, b: b * (n + 1) + a
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii = ii.ravel(); jj = jj.ravel()
    v00 = vid(ii, jj); v10 = vid(ii + 1, jj); v11 = vid(ii + 1, jj + 1); v01 = vid(ii, jj + 1)
    cells = np.empty((2 * n * n, 3), dtype=np.int32)
    cells[0::2] = np.stack([v00, v10, v11], 1)
    cells[1::2] = np.stack([v00, v11, v01], 1)
    return Mesh(2, coords, cells, n, vlat, {"kind": "square"})


def _perm_parity(p) -> int:
    p = list(p); s = 0
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            s += p[a] > p[b]
    return s & 1


def unit_cube(n: int) -> Mesh:
    r = np.arange(n + 1)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    vlat = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.int64)
    coords = vlat.astype(np.float64) / n
    rc = np.arange(n)
    kk, jj, ii = np.meshgrid(rc, rc, rc, indexing="ij")
    origin = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
    vid = lambda x: (x[:, 2] * (n + 1) + x[:, 1]) * (n + 1) + x[:, 0]
    perms = list(itertools.permutations(range(3)))
    cells = np.empty((6 * n ** 3, 4), dtype=np.int32)
    for t, p in enumerate(perms):
        path = [origin.copy()]
        cur = origin.copy()
        for a in p:
            cur = cur.copy(); cur[:, a] += 1
            path.append(cur)
        ids = [vid(x) for x in path]
        if _perm_parity(p):
            ids[2], ids[3] = ids[3], ids[2]
        cells[t::6] = np.stack(ids, 1)
    return Mesh(3, coords, cells, n, vlat, {"kind": "cube"})


def two_triangles() -> Mesh:
    coords = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)
    cells = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return Mesh(2, coords, cells, 0, None, {"kind": "two_triangles"})


def two_tets() -> Mesh:
    coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]],
                      dtype=np.float64)
    cells = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int32)
    return Mesh(3, coords, cells, 0, None, {"kind": "two_tets"})


def jitter_interior(mesh: Mesh, amplitude: float, rng: np.random.Generator) -> Mesh:
    """Move every interior vertex by iid U[-a*h, a*h] per coordinate (h = 1/n).

    Boundary vertices stay on the unit square/cube, so the domain measure is
    exactly 1.
    """
    assert mesh.n > 0, "jitter needs a lattice mesh"
    h = 1.0 / mesh.n
    delta = rng.uniform(-amplitude * h, amplitude * h, size=mesh.coords.shape)
    interior = np.all((mesh.vlat > 0) & (mesh.vlat < mesh.n), axis=1)
    coords = mesh.coords.copy()
    coords[interior] += delta[interior]
    return Mesh(mesh.dim, coords, mesh.cells, mesh.n, mesh.vlat,
                dict(mesh.meta, jitter=amplitude))


def dg_coordinates(mesh: Mesh) -> np.ndarray:
    """Per-cell (discontinuous) copy of the vertex coordinates, float64
    [C][d+1][d]: coordinates as an ordinary field on its own cell-to-node Map
    (the mesh abstraction treats them so), which lets single cells be
    reshaped without moving their neighbours."""
    return np.ascontiguousarray(mesh.coords[mesh.cells])


def flatten_cells(xdg: np.ndarray, fraction: float, rng: np.random.Generator, ratio: float = 1e3):
    """Flatten round(fraction * C) tetrahedra of a per-cell coordinate field.

    The cells are the first ones of a seeded permutation (returned sorted).  In
    each, vertex 3 moves along the normal of the face (v0, v1, v2), staying on
    its side, to the height (longest edge of that face) / ratio above the
    face's plane; the aspect ratio becomes about ``ratio`` and the orientation
    is kept.  Returns (new coordinates, chosen cell ids).
    """
    C = xdg.shape[0]
    k = int(round(fraction * C))
    chosen = np.sort(rng.permutation(C)[:k])
    x = xdg.copy()
    v0, v1, v2, v3 = (x[chosen, m] for m in range(4))
    nrm = np.cross(v1 - v0, v2 - v0)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    h = np.einsum("ij,ij->i", v3 - v0, nrm)
    L = np.maximum(np.maximum(np.linalg.norm(v1 - v0, axis=1), np.linalg.norm(v2 - v0, axis=1)),
                   np.linalg.norm(v2 - v1, axis=1))
    foot = v3 - h[:, None] * nrm
    x[chosen, 3] = foot + (np.sign(h) * L / ratio)[:, None] * nrm
    return np.ascontiguousarray(x), chosen


def boundary_nodes(mesh: Mesh, cell_node: np.ndarray, degree: int) -> np.ndarray:
    """uint8 mask over the nodes of a degree-k space on the unit square or
    cube: 1 for nodes on the boundary (a coordinate equal to 0 or 1; jitter
    moves interior vertices only, so boundary nodes stay exactly on it)."""
    W = local_node_barycentrics(mesh.dim, degree) / degree
    N = int(cell_node.max()) + 1
    pos = np.zeros((N, mesh.dim))
    pos[cell_node] = np.einsum("ln,cnd->cld", W, mesh.coords[mesh.cells])
    return np.any((pos <= 1e-12) | (pos >= 1 - 1e-12), axis=1).astype(np.uint8)


def exterior_facets(mesh: Mesh, cell_node: np.ndarray, degree: int):
    """Exterior facets of a unit square or cube mesh and their Maps.

    A facet (the cell's vertices but one) is exterior when all its vertices
    share a coordinate equal to 0 or 1 (jitter leaves the boundary alone).
    Returns (facet_vertex int32 [F][d], facet_node int32 [F][nloc of the
    degree-k (d-1)-simplex]): the facet's vertices in the cell's local order,
    and its nodes in the facet's own local order (vertices, edges with the
    two P3 nodes from the lower vertex, the P3 triangle's face node), taken
    from the cell's nodes with the same barycentric weights.  Facets come in
    (cell, opposite local vertex) order.
    """
    d = mesh.dim
    W = local_node_barycentrics(d, degree)
    Wf = local_node_barycentrics(d - 1, degree)
    key = {tuple(r): i for i, r in enumerate(W.tolist())}
    X = mesh.coords
    fvs, fns, order = [], [], []
    for o in range(d + 1):
        loc = [m for m in range(d + 1) if m != o]
        P = X[mesh.cells[:, loc]]                                  # [C][d][d]
        on = np.zeros(mesh.ncells, dtype=bool)
        for a in range(d):
            for v in (0.0, 1.0):
                on |= np.all(np.abs(P[:, :, a] - v) <= 1e-12, axis=1)
        cid = np.nonzero(on)[0]
        # local node of the cell for every facet node (same weights, facet vertices -> loc)
        sel = []
        for wf in Wf.tolist():
            w = [0] * (d + 1)
            for j, m in enumerate(loc):
                w[m] = wf[j]
            sel.append(key[tuple(w)])
        fvs.append(mesh.cells[cid][:, loc])
        fns.append(cell_node[cid][:, sel])
        order.append(cid * (d + 1) + o)
    order = np.concatenate(order)
    perm = np.argsort(order, kind="stable")
    fv = np.concatenate(fvs)[perm]
    fn = np.concatenate(fns)[perm]
    return (np.ascontiguousarray(fv.astype(np.int32)), np.ascontiguousarray(fn.astype(np.int32)))


def local_node_barycentrics(dim: int, degree: int) -> np.ndarray:
    """Integer barycentric weights (rows sum to ``degree``) of the local nodes."""
    nv = dim + 1
    rows = []
    for v in range(nv):
        e = [0] * nv; e[v] = degree; rows.append(e)
    edges = list(itertools.combinations(range(nv), 2))
    if degree == 2:
        for a, b in edges:
            e = [0] * nv; e[a] = 1; e[b] = 1; rows.append(e)
    elif degree == 3:
        for a, b in edges:
            e = [0] * nv; e[a] = 2; e[b] = 1; rows.append(e)
            e = [0] * nv; e[a] = 1; e[b] = 2; rows.append(e)
        for f in itertools.combinations(range(nv), 3):
            e = [0] * nv
            for a in f:
                e[a] = 1
            rows.append(e)
    elif degree != 1:
        raise ValueError("degree must be 1, 2 or 3")
    return np.array(rows, dtype=np.int64)


def node_map(mesh: Mesh, degree: int, numbering: str = "auto"):
    """Cell-to-node Map of the degree-k Lagrange space on ``mesh``.

    Returns ``(cell_node int32 [C][nloc], nnodes)``.  With ``numbering`` =
    "lattice" (the default for lattice meshes) a node's id is its index in the
    refined (k*n+1)^d lattice, x fastest; with "first_touch" nodes are numbered
    in the order cells first reach them.
    """
    W = local_node_barycentrics(mesh.dim, degree)          # [nloc][d+1]
    cells = mesh.cells.astype(np.int64)
    if degree == 1:
        return mesh.cells.astype(np.int32).copy(), mesh.nverts
    if numbering == "auto":
        numbering = "lattice" if mesh.vlat is not None else "first_touch"
    if numbering == "lattice":
        m = degree * mesh.n + 1
        lat = np.einsum("lv,cvd->cld", W, mesh.vlat[cells])  # [C][nloc][d]
        idx = np.zeros(lat.shape[:2], dtype=np.int64)
        for d in reversed(range(mesh.dim)):
            idx = idx * m + lat[:, :, d]
        return idx.astype(np.int32), m ** mesh.dim
    # first_touch: key each node by its sorted (vertex, weight) pairs
    ids = {}
    out = np.empty((cells.shape[0], W.shape[0]), dtype=np.int64)
    for c in range(cells.shape[0]):
        for l in range(W.shape[0]):
            key = tuple(sorted((int(cells[c, v]), int(W[l, v]))
                               for v in range(W.shape[1]) if W[l, v]))
            if key not in ids:
                ids[key] = len(ids)
            out[c, l] = ids[key]
    return out.astype(np.int32), len(ids)


def permute_cells(perm: np.ndarray, *cell_arrays):
    """New cell c is old cell perm[c] (applies to every per-cell array)."""
    return tuple(np.ascontiguousarray(a[perm]) for a in cell_arrays)


def permute_nodes(cell_node: np.ndarray, perm: np.ndarray):
    """Renumber nodes so that new node id of old node o is ``inv[o]`` where
    new node i is old node perm[i]."""
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size, dtype=perm.dtype)
    return inv[cell_node].astype(np.int32)


def permute_vertices(mesh: Mesh, perm: np.ndarray) -> Mesh:
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size, dtype=perm.dtype)
    vlat = None if mesh.vlat is None else mesh.vlat[perm]
    return Mesh(mesh.dim, mesh.coords[perm].copy(), inv[mesh.cells].astype(np.int32),
                mesh.n, vlat, dict(mesh.meta))
