"""Icosahedral geodesic grid generator (seeded-input side, shared by both
the oracle and the HIP library).

The grid is the one of Sec. 2 (grid paragraph): the icosahedron's 20
triangles are bisected recursively ``level`` times and every new vertex is
projected onto the sphere, giving N_g = 10 * 4**level + 2 nodes.  Each node is
the centre of one control volume, the Voronoi region of that node.  No mesh
optimisation is applied (the paper only cites one).

Outputs (all on the UNIT sphere; the radius is a model parameter):

* ``xyz``      (N, 3) float64 -- node positions, unit vectors.
* ``deg``      (N,)   int32   -- 5 for the 12 pentagons, else 6.
* ``nbr``      (N, 6) int32   -- neighbours in counter-clockwise order seen
  from outside the sphere; a pentagon's slot 5 holds the cell itself.
* ``corners``  (N, 6, 3) float64 -- corner s of cell i is the Voronoi vertex
  shared by cells i, nbr[i,s], nbr[i,s+1 mod deg], i.e. the circumcentre of
  that Delaunay triangle.  Each Voronoi vertex is computed once per triangle
  and copied, so every cell sees bitwise the same corner coordinates.  A
  pentagon's slot 5 is zero.

Cells are numbered along the triangle quadtree of the subdivision (a
Z-order curve on each icosahedron face), so consecutive cell indices form
compact patches on the sphere.

This module holds mesh construction only: no finite-volume operator, no
model arithmetic.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

_ICO_V = np.array([
    (-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
    (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
    (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1)], dtype=np.float64)

_ICO_F = np.array([
    (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
    (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
    (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
    (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], dtype=np.int64)


def n_cells(level):
    return 10 * 4 ** level + 2


def _normalize(v):
    return v / np.sqrt(np.einsum("ij,ij->i", v, v))[:, None]


def _subdivide(xyz, tri):
    """One bisection: each triangle (a,b,c) -> 4 children, in quadtree order."""
    nv = xyz.shape[0]
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    e = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)])
    key = np.minimum(e[:, 0], e[:, 1]) * nv + np.maximum(e[:, 0], e[:, 1])
    ukey, inv = np.unique(key, return_inverse=True)
    lo, hi = ukey // nv, ukey % nv
    mid = _normalize(xyz[lo] + xyz[hi])
    xyz = np.concatenate([xyz, mid])
    t = tri.shape[0]
    ab, bc, ca = nv + inv[:t], nv + inv[t:2 * t], nv + inv[2 * t:]
    ch = np.stack([
        np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
        np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], 1)
    return xyz, ch.reshape(-1, 3)


def _orient(xyz, tri):
    """Make every triangle counter-clockwise seen from outside."""
    p, q, r = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(q - p, r - p), p)
    tri = tri.copy()
    flip = s < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def build_mesh(level):
    """Return dict(xyz, deg, nbr, corners, tri, level) for grid ``level``."""
    xyz = _normalize(_ICO_V.copy())
    tri = _orient(xyz, _ICO_F)
    for _ in range(level):
        xyz, tri = _subdivide(xyz, tri)
    nv, nt = xyz.shape[0], tri.shape[0]
    assert nv == n_cells(level) and nt == 20 * 4 ** level

    # Renumber vertices along the triangle quadtree: a vertex is owned by the
    # first triangle (in quadtree order) that has it as a corner.
    owner = np.full(nv, 3 * nt, dtype=np.int64)
    occ = np.arange(3 * nt, dtype=np.int64)       # occurrence id = 3*t + k
    np.minimum.at(owner, tri.reshape(-1), occ)
    perm = np.argsort(owner, kind="stable")      # new -> old
    newid = np.empty(nv, dtype=np.int64)
    newid[perm] = np.arange(nv)
    xyz = xyz[perm]
    tri = newid[tri]

    # Counter-clockwise rings: triangle (a,b,c) says "after b comes c" around a.
    a = tri.reshape(-1)
    b = np.roll(tri, -1, axis=1).reshape(-1)
    c = np.roll(tri, -2, axis=1).reshape(-1)
    tid = np.repeat(np.arange(nt), 3)
    key = a * nv + b
    order = np.argsort(key)
    skey, snext, stri = key[order], c[order], tid[order]

    deg = np.bincount(a, minlength=nv).astype(np.int64)
    assert set(np.unique(deg)) <= {5, 6}
    # start each ring at the smallest-index neighbour
    first = np.full(nv, nv, dtype=np.int64)
    np.minimum.at(first, a, b)
    nbr = np.empty((nv, 6), dtype=np.int64)
    ctri = np.full((nv, 6), -1, dtype=np.int64)
    cur = first
    ids = np.arange(nv)
    for s in range(6):
        nbr[:, s] = cur
        pos = np.searchsorted(skey, ids * nv + cur)
        assert np.all(skey[pos] == ids * nv + cur)
        ctri[:, s] = stri[pos]
        cur = snext[pos]
    pent = deg == 5
    assert np.all(nbr[~pent, 0] == cur[~pent])          # hexagon ring closes after 6
    assert np.all(nbr[pent, 0] == nbr[pent, 5])          # pentagon ring closes after 5
    nbr[pent, 5] = ids[pent]
    ctri[pent, 5] = -1

    # Voronoi vertices: one circumcentre per triangle, copied into each cell.
    p, q, r = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cc = _normalize(np.cross(q - p, r - p))
    corners = np.zeros((nv, 6, 3), dtype=np.float64)
    valid = ctri >= 0
    corners[valid] = cc[ctri[valid]]

    return dict(level=level, xyz=np.ascontiguousarray(xyz),
                deg=deg.astype(np.int32), nbr=nbr.astype(np.int32),
                corners=corners, tri=tri.astype(np.int32))


_CACHE = {}


def get_mesh(level):
    """Memoised ``build_mesh`` (mesh construction is deterministic)."""
    if level not in _CACHE:
        _CACHE[level] = build_mesh(level)
    return _CACHE[level]
