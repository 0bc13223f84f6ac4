"""Test-side helpers written from the documented cell-id convention.

These decode canonical ids into vertex sets and enumerate the Freudenthal
(Kuhn) complex of a small grid directly from its definition: a set of grid
vertices is a simplex iff, ordered by vertex id, consecutive members differ
by adding unit-cube corners that form a chain 0 < c1 < ... <= (1,1,1).
Nothing here is shared with the oracle or the GPU library.
"""
from __future__ import annotations

import itertools

import numpy as np

EDGE = [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (0, 6), (0, 7)]
TRI = [(0, 1, 3), (0, 2, 3), (0, 1, 5), (0, 4, 5), (0, 2, 6), (0, 4, 6),
       (0, 1, 7), (0, 2, 7), (0, 3, 7), (0, 4, 7), (0, 5, 7), (0, 6, 7)]
TET = [(0, 1, 3, 7), (0, 1, 5, 7), (0, 2, 3, 7), (0, 2, 6, 7), (0, 4, 5, 7), (0, 4, 6, 7)]
CHAINS = {0: [(0,)], 1: EDGE, 2: TRI, 3: TET}


def corner(m):
    return (m & 1, (m >> 1) & 1, (m >> 2) & 1)


def vid(dims, x, y, z):
    return x + dims[0] * (y + dims[1] * z)


def xyz(dims, v):
    return (v % dims[0], (v // dims[0]) % dims[1], v // (dims[0] * dims[1]))


def cell_vertices(dims, dim, cid):
    """Vertex ids of canonical cell (dim, cid), or None if invalid."""
    K = len(CHAINS[dim])
    u, t = divmod(int(cid), K)
    if u >= dims[0] * dims[1] * dims[2]:
        return None
    ux, uy, uz = xyz(dims, u)
    out = []
    for m in CHAINS[dim][t]:
        ox, oy, oz = corner(m)
        x, y, z = ux + ox, uy + oy, uz + oz
        if x >= dims[0] or y >= dims[1] or z >= dims[2]:
            return None
        out.append(vid(dims, x, y, z))
    return tuple(out)


def all_simplices(dims):
    """Every simplex of the triangulated grid as (dim, sorted vertex tuple),
    enumerated from the chain definition (not from the id tables)."""
    lx, ly, lz = dims
    out = set()
    for z, y, x in itertools.product(range(lz), range(ly), range(lx)):
        out.add((0, (vid(dims, x, y, z),)))
        # all chains of corners starting at 0
        for k in (1, 2, 3):
            for masks in itertools.permutations(range(1, 8), k):
                ok = all((masks[i] & masks[i + 1]) == masks[i] and masks[i] != masks[i + 1]
                         for i in range(k - 1))
                if not ok:
                    continue
                verts = [vid(dims, x, y, z)]
                good = True
                for m in masks:
                    ox, oy, oz = corner(m)
                    if x + ox >= lx or y + oy >= ly or z + oz >= lz:
                        good = False
                        break
                    verts.append(vid(dims, x + ox, y + oy, z + oz))
                if good:
                    out.add((k, tuple(sorted(verts))))
    return sorted(out)


def count_formula(dims):
    """Closed-form cell counts of the Freudenthal triangulation of a grid."""
    lx, ly, lz = dims
    a, b, c = lx - 1, ly - 1, lz - 1
    V = lx * ly * lz
    E = a * ly * lz + lx * b * lz + lx * ly * c + a * b * lz + a * ly * c + lx * b * c + a * b * c
    T = 2 * (a * b * lz + a * ly * c + lx * b * c) + 6 * a * b * c
    Q = 6 * a * b * c
    return V, E, T, Q


def gf2_rank(M):
    """Rank over Z/2 of a 0/1 matrix."""
    A = (np.array(M, dtype=np.uint8) & 1).copy()
    r = 0
    rows, cols = A.shape
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if A[i, c]:
                piv = i
                break
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == rows:
            break
    return r
