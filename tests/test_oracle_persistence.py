"""Pins of the oracle's persistence computation against the definition.

Sec. 2.2 defines the pairs through the lexicographic filtration and the
elder rule.  The oracle's full boundary reduction is pinned here against the
pairing lemma (the pairs are read off ranks of lower-left submatrices of the
boundary matrix, independently of any reduction), and its discrete-gradient
pairing (Sec. 4.2) is pinned against the full reduction, against textbook
union-find (dims 0 and 2) and against hand-built fields with known diagrams.
"""
import itertools
import math

import numpy as np
import pytest

from tests import kuhn


def _nz(P):
    """Multiset of (dim, v_birth, v_death) of non-zero-persistence pairs and the
    essential class (the diagram, Sec. 2.2)."""
    return sorted((int(p["dim"]), int(p["v_birth"]), int(p["v_death"]), int(p["essential"]))
                  for p in P if p["essential"] or p["v_birth"] != p["v_death"])


def _simplex_set(P):
    return {(int(p["dim"]), int(p["birth_cell"]), int(p["death_cell"])) for p in P}


def _field_from_order(dims, perm):
    lx, ly, lz = dims
    return np.asarray(perm, dtype=np.float32).reshape(lz, ly, lx)


# ---------------------------------------------------------------- definition


def _filtration(dims, f):
    """Simplices in lexicographic filtration order (Sec. 2.2) and boundary
    columns as Python-int bitmasks over positions."""
    flat = f.ravel()
    order = sorted(range(flat.size), key=lambda v: (float(flat[v]), v))
    rank = {v: i for i, v in enumerate(order)}
    simp = kuhn.all_simplices(dims)
    key = {s: tuple(sorted((rank[v] for v in s[1]), reverse=True)) for s in simp}
    filt = sorted(simp, key=lambda s: key[s])
    pos = {s: i for i, s in enumerate(filt)}
    cols = []
    for d, vs in filt:
        m = 0
        if d > 0:
            for drop in range(d + 1):
                face = (d - 1, tuple(v for k, v in enumerate(vs) if k != drop))
                m |= 1 << pos[face]
        cols.append(m)
    return filt, pos, cols, rank


def _rank_lower_left(cols, i, j):
    """Z2 rank of the boundary submatrix with rows >= i and columns <= j."""
    mask = ~((1 << i) - 1)
    piv = {}
    r = 0
    for c in cols[: j + 1]:
        c &= mask
        while c:
            h = c.bit_length() - 1
            if h in piv:
                c ^= piv[h]
            else:
                piv[h] = c
                r += 1
                break
    return r


def _check_against_pairing_lemma(dims, f, P):
    filt, pos, cols, rank = _filtration(dims, f)
    total = _rank_lower_left(cols, 0, len(cols) - 1)
    finite = [p for p in P if not p["essential"]]
    assert len(finite) == total
    for p in finite:
        d = int(p["dim"])
        b = (d, tuple(sorted(kuhn.cell_vertices(dims, d, p["birth_cell"]))))
        e = (d + 1, tuple(sorted(kuhn.cell_vertices(dims, d + 1, p["death_cell"]))))
        i, j = pos[b], pos[e]
        ind = (_rank_lower_left(cols, i, j) - _rank_lower_left(cols, i + 1, j)
               - _rank_lower_left(cols, i, j - 1) + _rank_lower_left(cols, i + 1, j - 1))
        assert ind == 1, (p, i, j)
    ess = [p for p in P if p["essential"]]
    assert len(ess) == 1 and rank[int(ess[0]["birth_cell"])] == 0


@pytest.mark.parametrize("dims,seed", [((2, 2, 2), s) for s in range(6)] +
                         [((3, 2, 2), 0), ((2, 3, 2), 1), ((2, 2, 3), 2)])
def test_full_reduction_matches_pairing_lemma(orc, dims, seed):
    rng = np.random.default_rng(seed)
    f = rng.permutation(int(np.prod(dims))).astype(np.float32).reshape(dims[::-1])
    P = orc.pairs(f, method=1)
    _check_against_pairing_lemma(dims, f, P)


def test_complex_counts_match_closed_form(orc):
    # Cell counts of the oracle's complex against the closed form and the
    # chain-definition enumeration.
    for dims in [(2, 2, 2), (3, 4, 2), (5, 3, 4)]:
        f = np.arange(int(np.prod(dims)), dtype=np.float32).reshape(dims[::-1])
        vup, eup, tup = orc.gradient(f)
        V, E, T, Q = kuhn.count_formula(dims)
        assert (eup != -2).sum() == E and (tup != -2).sum() == T
        enum = kuhn.all_simplices(dims)
        assert [sum(1 for s in enum if s[0] == d) for d in range(4)] == [V, E, T, Q]
        assert V - E + T - Q == 1


# --------------------------------------------------- exhaustive 2x2x2 orders


def test_all_orders_2x2x2(orc):
    """All 8! = 40,320 vertex orders of the 2x2x2 grid (51 simplices): the
    discrete-gradient pairing equals the full reduction at the simplex level,
    and union-find equals it for dims 0 and 2."""
    dims = (2, 2, 2)
    mismatches = 0
    for perm in itertools.permutations(range(8)):
        f = _field_from_order(dims, perm)
        full = orc.pairs(f, method=1)
        dms = orc.pairs(f, method=0)
        krus = orc.pairs(f, method=2)
        if not _simplex_set(dms) <= _simplex_set(full):
            mismatches += 1
        if _nz(dms) != _nz(full):
            mismatches += 1
        fz = [t for t in _nz(full) if t[0] != 1]
        if _nz(krus) != fz:
            mismatches += 1
    assert mismatches == 0


# -------------------------------------------------------- random small grids


@pytest.mark.parametrize("dims,seed", [((3, 3, 3), 0), ((4, 3, 5), 1), ((5, 5, 5), 2),
                                      ((7, 4, 3), 3), ((6, 6, 6), 4), ((8, 8, 8), 5),
                                      ((2, 9, 5), 6), ((10, 7, 6), 7)])
def test_dms_equals_full_reduction(orc, dims, seed):
    rng = np.random.default_rng(seed)
    f = rng.random(dims[::-1]).astype(np.float32)
    full = orc.pairs(f, method=1)
    dms = orc.pairs(f, method=0)
    assert _nz(dms) == _nz(full)
    # simplex level: critical pairs are pairs of the full reduction
    assert _simplex_set(dms) <= _simplex_set(full)
    # The gradient pairs themselves need not be pairs of the full reduction
    # (zero-persistence representatives are not unique), but every critical
    # cell is unpaired by the gradient and paired by the full reduction.
    vup, eup, tup = orc.gradient(f)
    crit = orc.critical(f)
    paired_full = {(int(p["dim"]), int(p["birth_cell"])) for p in full} | \
        {(int(p["dim"]) + 1, int(p["death_cell"])) for p in full if not p["essential"]}
    for d in range(4):
        for c in crit[d]:
            assert (d, int(c)) in paired_full
    # union-find variants
    krus = orc.pairs(f, method=2)
    assert _nz(krus) == [t for t in _nz(full) if t[0] != 1]


def test_dms_equals_kruskal_16(orc):
    rng = np.random.default_rng(11)
    f = rng.random((16, 14, 12)).astype(np.float32)
    assert _nz(orc.pairs(f, 0)) and \
        [t for t in _nz(orc.pairs(f, 0)) if t[0] != 1] == _nz(orc.pairs(f, 2))


def test_full_reduction_16(orc):
    rng = np.random.default_rng(12)
    f = rng.random((12, 10, 11)).astype(np.float32)
    assert _nz(orc.pairs(f, 0)) == _nz(orc.pairs(f, 1))


# ------------------------------------------------------------ invariants


def _crit_counts(orc, f):
    return [len(c) for c in orc.critical(f)]


@pytest.mark.parametrize("seed", range(3))
def test_euler_and_essential(orc, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(9, 11, 10)).astype(np.float32)
    c = _crit_counts(orc, f)
    assert c[0] - c[1] + c[2] - c[3] == 1
    P = orc.pairs(f, 0)
    # every critical cell is in exactly one pair except the global minimum
    crit_total = sum(c)
    assert 2 * (len(P) - 1) + 1 == crit_total
    ess = [p for p in P if p["essential"]]
    assert len(ess) == 1 and ess[0]["dim"] == 0


def test_gradient_is_valid_acyclic_matching(orc):
    dims = (7, 6, 5)
    rng = np.random.default_rng(3)
    f = rng.random(dims[::-1]).astype(np.float32)
    vup, eup, tup = orc.gradient(f)
    flat = f.ravel()
    order = sorted(range(flat.size), key=lambda v: (float(flat[v]), v))
    rank = {v: i for i, v in enumerate(order)}
    used = {1: set(), 2: set(), 3: set()}
    for d, arr in ((0, vup), (1, eup), (2, tup)):
        for c in np.nonzero(arr >= 0)[0]:
            lo = kuhn.cell_vertices(dims, d, c)
            hi = kuhn.cell_vertices(dims, d + 1, arr[c])
            assert set(lo) < set(hi)  # facet-cofacet
            assert max(lo, key=rank.get) == max(hi, key=rank.get)  # same lower star
            assert int(arr[c]) not in used[d + 1]
            used[d + 1].add(int(arr[c]))
    # a cell is paired at most once overall
    for d, arr in ((1, eup), (2, tup)):
        up = {int(c) for c in np.nonzero(arr >= 0)[0]}
        assert not (up & used[d])
    # acyclicity of the dim-1 V-paths: edge -> paired triangle -> other edges
    succ = {}
    for e in np.nonzero(eup >= 0)[0]:
        tri = kuhn.cell_vertices(dims, 2, eup[e])
        ev = set(kuhn.cell_vertices(dims, 1, e))
        succ[frozenset(ev)] = [frozenset(x) for x in itertools.combinations(tri, 2)
                               if set(x) != ev]
    state = {}

    def dfs(u):
        stack = [(u, iter(succ.get(u, [])))]
        state[u] = 1
        while stack:
            node, it = stack[-1]
            nxt = next(it, None)
            if nxt is None:
                state[node] = 2
                stack.pop()
                continue
            s = state.get(nxt, 0)
            assert s != 1, "cycle in V-paths"
            if s == 0:
                state[nxt] = 1
                stack.append((nxt, iter(succ.get(nxt, []))))

    for u in list(succ):
        if state.get(u, 0) == 0:
            dfs(u)


def test_interior_star_sizes(orc):
    # a strict local maximum in the interior has the whole star (14 edges, 36
    # triangles, 24 tetrahedra) as its lower star: 75 cells, one critical tet
    dims = (5, 5, 5)
    rank = np.arange(125, dtype=np.int32)
    v = kuhn.vid(dims, 2, 2, 2)
    rank[v], rank[124] = 124, rank[v]
    pairs, crit = orc.gradient_at(rank, dims, v)
    dims_of = [p[0] for p in pairs]
    assert 2 * len(pairs) + len(crit) == 75
    assert crit == [(3, crit[0][1])]
    assert dims_of.count(0) == 1


# -------------------------------------------------------------- hand-built


def _grid(dims):
    lx, ly, lz = dims
    z, y, x = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def test_linear_ramp_has_only_essential(orc):
    dims = (9, 7, 6)
    f = np.arange(int(np.prod(dims)), dtype=np.float32).reshape(dims[::-1])
    D = orc.diagram(f)
    assert len(D) == 1 and D[0]["essential"] == 1
    assert D[0]["v_birth"] == 0 and D[0]["v_death"] == f.size - 1
    c = _crit_counts(orc, f)
    assert c == [1, 0, 0, 0]


def _minimax_death(f, a, b, dims):
    """Brute force: lowest level t at which vertices a and b are connected in
    the sublevel graph of the triangulation's edges (14-neighbourhood)."""
    flat = f.ravel()
    levels = np.unique(flat)
    offs = []
    for m in range(1, 8):
        o = kuhn.corner(m)
        offs += [o, tuple(-c for c in o)]

    def connected(t):
        seen = {a}
        todo = [a]
        while todo:
            v = todo.pop()
            x, y, z = kuhn.xyz(dims, v)
            for ox, oy, oz in offs:
                X, Y, Z = x + ox, y + oy, z + oz
                if 0 <= X < dims[0] and 0 <= Y < dims[1] and 0 <= Z < dims[2]:
                    w = kuhn.vid(dims, X, Y, Z)
                    if w not in seen and flat[w] <= t:
                        seen.add(w)
                        todo.append(w)
        return b in seen

    lo, hi = 0, len(levels) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if connected(levels[mid]):
            hi = mid
        else:
            lo = mid + 1
    return levels[lo]


def test_two_wells(orc):
    dims = (15, 9, 8)
    x, y, z = _grid(dims)
    w1 = (x - 3) ** 2 + (y - 4) ** 2 + (z - 3.5) ** 2
    w2 = 0.5 + (x - 11) ** 2 + (y - 4) ** 2 + (z - 3.5) ** 2
    f = (np.minimum(w1, w2) + 1e-3 * (x + 0.37 * y + 0.11 * z)).astype(np.float32)
    D = orc.diagram(f)
    fin = [p for p in D if not p["essential"]]
    assert len(fin) == 1 and fin[0]["dim"] == 0
    p = fin[0]
    m2 = int(np.argmin(np.where(x.ravel() > 7, f.ravel(), np.inf)))
    m1 = int(np.argmin(f.ravel()))
    assert p["v_birth"] == m2
    assert p["death"] == _minimax_death(f, m1, m2, dims)


def test_spherical_shell_void(orc):
    dims = (15, 15, 15)
    x, y, z = _grid(dims)
    r = np.sqrt((x - 7.1) ** 2 + (y - 6.9) ** 2 + (z - 7.05) ** 2)
    f = np.abs(r - 5.0).astype(np.float32)
    D = orc.diagram(f)
    big = [p for p in D if not p["essential"] and p["death"] - p["birth"] > 2.0]
    assert len(big) == 1 and big[0]["dim"] == 2
    center = int(np.argmax(np.where(r.ravel() < 5, f.ravel(), -np.inf)))
    assert big[0]["v_death"] == center


def test_solid_torus_loop(orc):
    # sublevel sets of the distance to a circle of radius R: a 1-cycle is born
    # near -r... here at ~0 (the core circle) and dies at the axis (value ~R)
    dims = (24, 24, 12)
    x, y, z = _grid(dims)
    cx, cy, cz = 11.6, 11.4, 5.5
    R = 7.0
    rho = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    f = (np.sqrt((rho - R) ** 2 + (z - cz) ** 2) - 2.0).astype(np.float32)
    D = orc.diagram(f)
    big = [p for p in D if not p["essential"] and p["death"] - p["birth"] > 3.0]
    assert len(big) == 1 and big[0]["dim"] == 1
    assert abs(big[0]["birth"] - (-2.0)) < 1.0
    assert abs(big[0]["death"] - (R - 2.0)) < 1.5


def test_negative_zero_is_zero(orc):
    f = np.array([0.0, -0.0, 1.0, -1.0, 0.5, -0.0, 2.0, 3.0], dtype=np.float32)
    o, r = orc.order(f)
    # -0.0 and +0.0 tie and are ordered by index
    assert list(o) == [3, 0, 1, 5, 4, 2, 6, 7]
    # closed form via numpy's lexsort on (id, value with -0 -> +0)
    fv = np.where(f == 0, np.float32(0), f)
    assert list(np.lexsort((np.arange(8), fv))) == list(o)


def test_order_matches_lexsort(orc):
    rng = np.random.default_rng(5)
    f = rng.integers(0, 50, size=4000).astype(np.float32)  # many ties
    o, r = orc.order(f)
    ref = np.lexsort((np.arange(f.size), f))
    assert np.array_equal(o, ref)
    assert np.array_equal(r[o], np.arange(f.size))


def test_nonfinite_rejected(orc):
    f = np.zeros((3, 3, 3), np.float32)
    f[1, 1, 1] = np.nan
    with pytest.raises(orc.OracleError):
        orc.diagram(f)
