"""Pins of the oracle's still-pair join, reduced assignment and canonical form
(Sec. 4.3), and of list-mode signal selection (Sec. 3).

The assignment step is checked on hand-built diagrams whose expected
assignment follows from the rules by hand:
  - a point whose (dim, v_birth, v_death) matches a point of the previous
    diagram is still and keeps that point's assignment, even where a fresh
    solve of the whole problem would give it another target;
  - the dimension is part of the key;
  - equal keys are matched as multisets, the k-th occurrence with the k-th;
  - points that are not still are assigned exactly (Eq. (1)) to the targets
    that no still point holds; the essential point takes the essential target;
  - interchangeable points and targets are put in the canonical form (point
    classes in diagram order take the target classes by lowest id, diagonal
    last; a target class hands out its ids in increasing order).

List mode is checked on fields whose diagrams are known in closed form: a
pair left out of the list is pulled to its diagonal projection in one
halfway step (Sec. 5), a listed pair is held, whatever the persistences.
"""
import numpy as np
import pytest

from paper_2407_12399_amd import fields


def _rec(dim, vb, vd, b, d, ess=0, bcell=0, dcell=0):
    import oracle
    r = np.zeros(1, oracle.PAIR_DTYPE)
    r["dim"], r["essential"], r["v_birth"], r["v_death"] = dim, ess, vb, vd
    r["birth"], r["death"] = b, d
    r["birth_cell"], r["death_cell"] = bcell, dcell
    return r


def _cat(*recs):
    return np.concatenate(recs)


ESS = dict(dim=0, vb=0, vd=99, b=0.0, d=10.0, ess=1)
# D_T: t0 essential, t1 and t2 of dim 0, t3 of dim 1
TARGETS = [ESS, dict(dim=0, vb=1, vd=2, b=1.0, d=5.0), dict(dim=0, vb=3, vd=4, b=2.0, d=6.0),
           dict(dim=1, vb=5, vd=6, b=3.0, d=7.0)]


def _targets(extra=()):
    return _cat(*[_rec(**t) for t in list(TARGETS) + list(extra)])


def test_still_point_keeps_its_target(orc):
    """P keeps its key (1, 2) and inherits t1 although it now sits on t2; Q
    has a new birth vertex, so it is not still and takes the only free
    dim-0 target, t2.  A fresh solve of everything would give P -> t2 and
    Q -> t1 (both at cost 0)."""
    prev = _cat(_rec(**ESS), _rec(0, 1, 2, 1.0, 5.0), _rec(0, 3, 4, 2.0, 6.0))
    cur = _cat(_rec(**ESS), _rec(0, 1, 2, 2.0, 6.0), _rec(0, 7, 4, 1.0, 5.0))
    phi, n_still, n_red = orc.assign_step(prev, [0, 1, 2], cur, _targets())
    assert list(phi) == [0, 1, 2]
    assert (n_still, n_red) == (2, 1)


def test_dimension_is_part_of_the_key(orc):
    """R has the vertices of the previous dim-0 point but is of dim 1: it is
    not still, and goes to the free dim-1 target t3, never to t1."""
    prev = _cat(_rec(**ESS), _rec(0, 1, 2, 1.0, 5.0))
    cur = _cat(_rec(**ESS), _rec(1, 1, 2, 3.0, 7.0))
    phi, n_still, n_red = orc.assign_step(prev, [0, 1], cur, _targets())
    assert list(phi) == [0, 3]
    assert (n_still, n_red) == (1, 1)


def test_equal_keys_matched_in_order(orc):
    """Two previous points with the same key, assigned (t3, diagonal): the
    first current occurrence inherits t3, the second the diagonal; both are
    still."""
    prev = _cat(_rec(**ESS), _rec(1, 5, 6, 3.0, 7.0), _rec(1, 5, 6, 3.0, 7.0))
    cur = _cat(_rec(**ESS), _rec(1, 5, 6, 3.0, 7.0), _rec(1, 5, 6, 3.0, 7.0))
    phi, n_still, n_red = orc.assign_step(prev, [0, 3, -1], cur, _targets())
    assert list(phi) == [0, 3, -1]
    assert (n_still, n_red) == (3, 0)
    phi, _, _ = orc.assign_step(prev, [0, -1, 3], cur, _targets())
    assert list(phi) == [0, -1, 3]
    # one previous occurrence only: the second current one is not still and
    # t3 is held, so it goes to the diagonal
    phi, n_still, n_red = orc.assign_step(prev[:2], [0, 3], cur, _targets())
    assert list(phi) == [0, 3, -1]
    assert (n_still, n_red) == (2, 1)


def test_essential_point_takes_the_essential_target(orc):
    """A new global minimum makes the essential point not still; it still
    takes t0, and is not counted in the reduced problem.  A non-still
    dim-0 point facing only held dim-0 targets goes to the diagonal."""
    prev = _cat(_rec(**ESS), _rec(0, 1, 2, 1.0, 5.0), _rec(0, 3, 4, 2.0, 6.0))
    cur = _cat(_rec(0, 8, 99, -1.0, 10.0, ess=1), _rec(0, 1, 2, 1.0, 5.0),
               _rec(0, 3, 4, 2.0, 6.0), _rec(0, 9, 11, 1.5, 5.5))
    phi, n_still, n_red = orc.assign_step(prev, [0, 1, 2], cur, _targets())
    assert list(phi) == [0, 1, 2, -1]
    assert (n_still, n_red) == (2, 1)


def test_reduced_problem_is_exact(orc):
    """Two new dim-0 points against the two free dim-0 targets t1 = (1, 5)
    and t2 = (2, 6): A = (1.4, 5.4) is nearer to t1 (0.32 against 0.72) and
    B = (1, 5) sits on t1, so the optimum of Eq. (1) crosses the nearest
    choice: A -> t2, B -> t1 (0.72) beats A -> t1, B -> t2 (0.32 + 2)."""
    prev = _cat(_rec(**ESS))
    cur = _cat(_rec(**ESS), _rec(0, 20, 21, 1.4, 5.4), _rec(0, 22, 23, 1.0, 5.0))
    phi, n_still, n_red = orc.assign_step(prev, [0], cur, _targets())
    assert list(phi) == [0, 2, 1]
    assert (n_still, n_red) == (1, 2)


def test_pair_at_diagonal_cost_goes_to_diagonal(orc):
    """t1 is held by the still point P, so the new point A = (1, 3) can only
    take t2 = (2, 6): c(A, t2) = 1 + 9 = 10 equals diag(A) + diag(t2) =
    2 + 8 (exact in floating point), and a tie goes to the diagonal.  At
    A = (1, 3.5), c = 7.25 < 3.125 + 8, and A takes t2."""
    prev = _cat(_rec(**ESS), _rec(0, 1, 2, 1.0, 5.0))
    cur = _cat(_rec(**ESS), _rec(0, 1, 2, 1.0, 5.0), _rec(0, 20, 21, 1.0, 3.0))
    phi, n_still, n_red = orc.assign_step(prev, [0, 1], cur, _targets())
    assert list(phi) == [0, 1, -1]
    assert (n_still, n_red) == (2, 1)
    cur["death"][2] = 3.5
    phi, _, _ = orc.assign_step(prev, [0, 1], cur, _targets())
    assert list(phi) == [0, 1, 2]


def test_canonical_form_of_interchangeable_items(orc):
    """Two new points with equal key and coordinates against two free
    targets with equal key and coordinates (t4 duplicates t1): the first
    point takes the lower id.  With one such target only, the first point
    takes it and the second the diagonal."""
    t4 = dict(dim=0, vb=1, vd=2, b=1.0, d=5.0)
    prev = _cat(_rec(**ESS), _rec(0, 3, 4, 2.0, 6.0))
    cur = _cat(_rec(**ESS), _rec(0, 3, 4, 2.0, 6.0), _rec(0, 30, 31, 1.0, 5.0),
               _rec(0, 30, 31, 1.0, 5.0))
    phi, n_still, n_red = orc.assign_step(prev, [0, 2], cur, _targets([t4]))
    assert list(phi) == [0, 2, 1, 4]
    assert (n_still, n_red) == (2, 2)
    phi, _, _ = orc.assign_step(prev, [0, 2], cur, _targets())
    assert list(phi) == [0, 2, 1, -1]


# ---------------------------------------------------------------- list mode

def _two_dips():
    """A ramp (f = vertex id) with two single-vertex dips far apart: each
    dip v sits 0.5 (resp. 2.0) below its lowest neighbour w = v - (1, 1, 1),
    which gives exactly two finite pairs (v, w) of dim 0."""
    Lx, Ly, Lz = 9, 6, 5
    f = np.arange(Lx * Ly * Lz, dtype=np.float32).reshape(Lz, Ly, Lx)
    off = 1 + Lx + Lx * Ly
    v1 = 2 + Lx * (2 + Ly * 2)
    v2 = 6 + Lx * (3 + Ly * 2)
    fr = f.ravel()
    fr[v1] = fr[v1 - off] - np.float32(0.5)
    fr[v2] = fr[v2 - off] - np.float32(2.0)
    return f, [(v1, v1 - off), (v2, v2 - off)]


def _mid(f, v, w):
    return np.float32((np.float32(f.ravel()[v]) + np.float32(f.ravel()[w])) * np.float32(0.5))


def test_two_dips_diagram(orc):
    f, dips = _two_dips()
    D = orc.diagram(f)
    fin = D[D["essential"] == 0]
    assert sorted((int(p["v_birth"]), int(p["v_death"])) for p in fin) == sorted(dips)


@pytest.mark.parametrize("keep", [(), (0,), (1,), (0, 1)])
def test_list_mode_holds_listed_pairs(orc, keep):
    """Listed pairs are signal and stay; unlisted ones move to their
    midpoint in one halfway step.  Keeping only the small dip and
    cancelling the large one is something no threshold can express."""
    f, dips = _two_dips()
    D = orc.diagram(f)
    fin = D[D["essential"] == 0]
    by_v = {int(p["v_birth"]): p for p in fin}
    lst = np.array([by_v[dips[k][0]] for k in keep], dtype=orc.PAIR_DTYPE)
    g, rep = orc.simplify(f, signal_pairs=lst)
    if len(keep) == 2:
        assert rep.iterations == 0 and np.array_equal(g, f)
        return
    assert rep.iterations == 1 and rep.cancelled == 1
    for k, (v, w) in enumerate(dips):
        if k in keep:
            assert g.ravel()[v] == f.ravel()[v] and g.ravel()[w] == f.ravel()[w]
        else:
            m = _mid(f, v, w)
            assert abs(g.ravel()[v] - m) <= np.spacing(m)
            assert abs(g.ravel()[w] - m) <= np.spacing(m)
    rest = np.ones(f.size, bool)
    rest[[x for d in dips for x in d]] = False
    assert np.array_equal(g.ravel()[rest], f.ravel()[rest])


def test_list_mode_matches_on_dim_and_cells(orc):
    """A list entry matches a pair only on (dim, birth_cell, death_cell):
    the same cells under another dim, or another birth cell, select
    nothing."""
    f, dips = _two_dips()
    D = orc.diagram(f)
    fin = D[D["essential"] == 0]
    big = fin[np.argmax(fin["death"] - fin["birth"])]
    g_ref, _ = orc.simplify(f, signal_pairs=np.array([big]))
    wrong_dim = np.array([big]).copy()
    wrong_dim["dim"] = 1
    wrong_cell = np.array([big]).copy()
    wrong_cell["birth_cell"] += 1
    g_none, _ = orc.simplify(f, signal_pairs=np.zeros(0, orc.PAIR_DTYPE))
    for lst in (wrong_dim, wrong_cell):
        g, _ = orc.simplify(f, signal_pairs=lst)
        assert np.array_equal(g, g_none)
    assert not np.array_equal(g_ref, g_none)


def test_list_equal_to_threshold_set_gives_same_solve(orc):
    """The list of the pairs that the threshold rule keeps (persistence
    above 0.1 range; Sec. 3) gives the identical solve."""
    f = fields.gaussian_mixture((12, 11, 10), 8, 0.05, 0)
    D = orc.diagram(f)
    rng = float(f.max()) - float(f.min())
    thr = float(np.float32(0.1)) * rng
    pers = D["death"].astype(np.float64) - D["birth"].astype(np.float64)
    lst = D[(D["essential"] == 0) & (pers > thr)]
    assert 0 < len(lst) < len(D) - 1
    g1, r1 = orc.simplify(f, threshold=0.1, j_max=30)
    g2, r2 = orc.simplify(f, signal_pairs=lst, j_max=30)
    assert (r1.iterations, r1.n_targets) == (r2.iterations, r2.n_targets)
    assert np.array_equal(g1, g2)
