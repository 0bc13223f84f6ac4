"""Pins of the oracle's loss, assignment, update and solver loop.

Assignment: brute force over all partial matchings (Eq. 1 with q = 2 on the
augmented diagrams, Sec. 2.3).  Update: the closed form of the halfway step
(alpha_b = alpha_d = 1/2 moves an isolated pair's two vertices to its
diagonal projection, Sec. 5).  Solver: the stability bound of persistence
diagrams, the stop rules of Alg. 1 / Sec. 5.4, and signal preservation
(Sec. 3).
"""
import itertools

import numpy as np
import pytest

from paper_2407_12399_amd import fields


def _brute_assign(P, Q):
    """Minimum of sum c(p,q) over matched + diag over unmatched, over all
    injective partial maps points -> targets."""
    def c(p, q):
        return (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2

    def dg(p):
        return (p[1] - p[0]) ** 2 / 2

    best = np.inf
    m, k = len(P), len(Q)
    choices = list(range(k)) + [None]
    for combo in itertools.product(choices, repeat=m):
        used = [t for t in combo if t is not None]
        if len(set(used)) != len(used):
            continue
        cost = sum(c(P[i], Q[t]) if t is not None else dg(P[i]) for i, t in enumerate(combo))
        cost += sum(dg(Q[j]) for j in range(k) if j not in used)
        best = min(best, cost)
    return best


@pytest.mark.parametrize("seed", range(25))
def test_assignment_is_optimal(orc, seed):
    rng = np.random.default_rng(seed)
    m, k = rng.integers(0, 6), rng.integers(0, 6)
    pb = rng.random(m)
    pd = pb + rng.random(m) * 0.5
    qb = rng.random(k)
    qd = qb + rng.random(k) * 0.5
    match, cost = orc.assign(pb, pd, qb, qd)
    ref = _brute_assign(list(zip(pb, pd)), list(zip(qb, qd)))
    assert cost == pytest.approx(ref, rel=1e-12, abs=1e-15)
    # the returned matching realises the returned cost
    used = [t for t in match if t >= 0]
    assert len(set(used)) == len(used)
    real = sum((pb[i] - qb[t]) ** 2 + (pd[i] - qd[t]) ** 2 if t >= 0
               else (pd[i] - pb[i]) ** 2 / 2 for i, t in enumerate(match))
    real += sum((qd[j] - qb[j]) ** 2 / 2 for j in range(k) if j not in used)
    assert real == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_assignment_prefers_close_target(orc):
    # a point next to a target is matched to it, a point far from all is sent
    # to the diagonal, an unmatched target costs its diagonal distance
    match, cost = orc.assign([0.0, 0.5], [1.0, 0.52], [0.01, 5.0], [1.0, 9.0])
    assert list(match) == [0, -1]
    assert cost == pytest.approx(0.01 ** 2 + 0.02 ** 2 / 2 + 4.0 ** 2 / 2)


def test_halfway_step_closed_form(orc):
    """A single-vertex dip on a ramp gives one min-saddle pair (v, w) with w
    the lowest neighbour of v; with alpha = 1/2 both vertices move to the
    diagonal projection m = (f(v) + f(w)) / 2 in one step (Sec. 5), and the
    pair disappears."""
    dims = (6, 5, 4)
    f = np.arange(120, dtype=np.float32).reshape(4, 5, 6) * np.float32(1.0)
    v = 2 + 6 * (2 + 5 * 2)           # interior vertex (2,2,2)
    w = v - (1 + 6 + 30)              # its lowest neighbour, offset (-1,-1,-1)
    f.ravel()[v] = f.ravel()[w] - np.float32(0.5)
    D = orc.diagram(f)
    fin = [p for p in D if not p["essential"]]
    assert len(fin) == 1 and fin[0]["v_birth"] == v and fin[0]["v_death"] == w
    g, rep = orc.simplify(f, threshold=0.5, nonsignal_dims=(0,))
    m = np.float32((np.float32(f.ravel()[v]) + np.float32(f.ravel()[w])) * np.float32(0.5))
    assert rep.iterations == 1 and rep.cancelled == 1
    ulp = np.spacing(m)
    assert abs(g.ravel()[v] - m) <= ulp and abs(g.ravel()[w] - m) <= ulp
    other = np.ones(f.size, bool)
    other[[v, w]] = False
    assert np.array_equal(g.ravel()[other], f.ravel()[other])
    assert rep.loss0 == pytest.approx(0.5 ** 2 / 2)


@pytest.mark.parametrize("alpha_b,alpha_d", [(0.0, 0.5), (0.5, 0.0)])
def test_one_sided_steps_closed_form(orc, alpha_b, alpha_d):
    """Cut / fill variants (Sec. 5.3: only the death or only the birth
    vertex moves).  On the single-dip field the moving vertex goes to the
    current midpoint at every step, so the persistence halves per iteration
    while the other vertex keeps its value; the solver stops at the first
    iteration whose persistence is below 1e-6 of the range."""
    dims = (6, 5, 4)
    f = np.arange(120, dtype=np.float32).reshape(4, 5, 6) * np.float32(1.0)
    v = 2 + 6 * (2 + 5 * 2)
    w = v - (1 + 6 + 30)
    f.ravel()[v] = f.ravel()[w] - np.float32(0.5)
    g, rep = orc.simplify(f, threshold=0.5, nonsignal_dims=(0,), alpha_b=alpha_b,
                          alpha_d=alpha_d)
    b, d = np.float32(f.ravel()[v]), np.float32(f.ravel()[w])
    tol = 1e-6 * rep.range
    steps = 0
    while float(d) - float(b) >= tol:
        mid = np.float32((b + d) * np.float32(0.5))
        if alpha_b == 0.0:
            d = mid
        else:
            b = mid
        steps += 1
    assert rep.cancelled == 1 and rep.iterations == steps
    assert g.ravel()[v] == b and g.ravel()[w] == d
    other = np.ones(f.size, bool)
    other[[v, w]] = False
    assert np.array_equal(g.ravel()[other], f.ravel()[other])


def test_stability_of_diagrams(orc):
    """bottleneck(D(f), D(g)) <= ||f - g||_inf (stability theorem)."""
    rng = np.random.default_rng(0)
    for trial in range(4):
        f = rng.random((6, 7, 5)).astype(np.float32)
        eps = 0.02 * (trial + 1)
        g = (f + rng.uniform(-eps, eps, size=f.shape)).astype(np.float32)
        b = orc.bottleneck(orc.diagram(f), orc.diagram(g))
        assert b <= float(np.abs(f.astype(np.float64) - g).max()) + 1e-7


def test_bottleneck_trivial_cases(orc):
    D = orc.diagram(np.random.default_rng(1).random((5, 5, 5)).astype(np.float32))
    assert orc.bottleneck(D, D) == 0.0
    fin = D[D["essential"] == 0]
    # removing one finite point costs at most its half persistence (L_inf
    # distance to the diagonal), and exactly that when it is the only point
    k = int(np.argmax(fin["death"] - fin["birth"]))
    E = np.concatenate([D[D["essential"] == 1], np.delete(fin, k)])
    half = (float(fin[k]["death"]) - float(fin[k]["birth"])) / 2
    assert 0.0 < orc.bottleneck(D, E) <= half + 1e-12
    one = np.concatenate([D[D["essential"] == 1], fin[k:k + 1]])
    assert orc.bottleneck(one, D[D["essential"] == 1]) == pytest.approx(half, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_solver_cancels_and_preserves_signal(orc, seed):
    f = fields.gaussian_mixture((12, 12, 12), 8, 0.05, seed)
    g, rep = orc.simplify(f, threshold=0.1)
    assert rep.cancelled == 1 and rep.iterations < 1000
    assert rep.max_nonsignal_pers < 1e-6 * rep.range
    assert rep.loss < rep.loss0
    D0 = orc.diagram(f)
    Dg = orc.diagram(g)
    thr = 0.1 * rep.range
    sig0 = D0[(D0["death"].astype(np.float64) - D0["birth"]) > thr]
    # every signal point of D(f) is still present at its coordinates in D(g)
    # up to the signal displacement of the final assignment
    assert rep.max_signal_disp <= 1e-5
    big_g = Dg[(Dg["death"].astype(np.float64) - Dg["birth"]) > thr]
    assert len(big_g) == len(sig0)
    # every other point of D(g) has (numerically) zero persistence
    small = Dg[(Dg["death"].astype(np.float64) - Dg["birth"]) <= thr]
    assert (small["death"].astype(np.float64) - small["birth"]).max(initial=0) < 1e-6 * rep.range
    # stability: the diagram moved by no more than the field
    assert orc.bottleneck(D0, Dg) <= rep.linf + 1e-7


def test_loss_ratio_stop_rule(orc):
    # Alg. 1's stop rule L <= s L0 with the paper's s = 0.01
    f = fields.gaussian_mixture((12, 12, 12), 8, 0.05, 3)
    g, rep = orc.simplify(f, threshold=0.1, stop_mode=1)
    assert rep.cancelled == 1
    assert rep.loss <= 0.01 * rep.loss0
    assert rep.trace[-2] > 0.01 * rep.loss0 or rep.iterations == 1


def test_j_max_reports_not_cancelled(orc):
    f = fields.gaussian_mixture((12, 12, 12), 8, 0.05, 0)
    g, rep = orc.simplify(f, threshold=0.1, j_max=1)
    assert rep.iterations == 1 and rep.cancelled == 0 and rep.status == 1


def test_nothing_to_cancel_returns_input(orc):
    f = np.arange(64, dtype=np.float32).reshape(4, 4, 4)
    g, rep = orc.simplify(f, threshold=0.1)
    assert rep.iterations == 0 and rep.cancelled == 1
    assert np.array_equal(g, f)
