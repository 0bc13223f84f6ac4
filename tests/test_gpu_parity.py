"""GPU path vs the CPU oracle, stage by stage, through the C ABI.

Bit-exact: vertex order, gradient pairing, critical cells, persistence pairs
and the diagram (integer and ordering results; the diagram's coordinates are
gathered field values).  The solver's final field must match within
1e-6 * range (it is computed with the same FP32 operations in the same
order on both sides, so in practice it is bit-identical).
"""
import itertools

import numpy as np
import pytest

from paper_2407_12399_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_12399_amd as ts
    ts.lib()
    return ts


def _t(f):
    import torch
    return torch.from_numpy(np.ascontiguousarray(f)).cuda()


def _same_pairs(a, b):
    assert len(a) == len(b), (len(a), len(b))
    for k in ("dim", "essential", "birth_cell", "death_cell", "v_birth", "v_death"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["birth"].view(np.uint32), b["birth"].view(np.uint32))
    assert np.array_equal(a["death"].view(np.uint32), b["death"].view(np.uint32))


CASES = [((2, 2, 2), 0), ((3, 3, 3), 1), ((5, 4, 3), 2), ((8, 7, 6), 3), ((2, 9, 5), 4),
         ((16, 16, 16), 5), ((23, 19, 17), 6), ((33, 2, 9), 7)]


def _rand(dims, seed, kind="uniform"):
    rng = np.random.default_rng(seed)
    shp = dims[::-1]
    if kind == "uniform":
        return rng.random(shp).astype(np.float32)
    if kind == "ties":
        return rng.integers(0, 7, size=shp).astype(np.float32)
    return rng.normal(size=shp).astype(np.float32)


@pytest.mark.parametrize("n,seed", [(8, 0), (1000, 1), (100_003, 2), (1 << 20, 3)])
def test_order_bit_exact(gpu, orc, n, seed):
    rng = np.random.default_rng(seed)
    f = rng.integers(-20, 20, size=n).astype(np.float32) * np.float32(0.5)
    f[rng.random(n) < 0.05] = -0.0
    f = f.reshape(1, 1, n)
    o, r = gpu.order(_t(f))
    oo, ro = orc.order(f)
    assert np.array_equal(o.cpu().numpy(), oo)
    assert np.array_equal(r.cpu().numpy(), ro)


@pytest.mark.parametrize("dims,seed", CASES)
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_gradient_bit_exact(gpu, orc, dims, seed, kind):
    f = _rand(dims, seed, kind)
    for a, b in zip(gpu.gradient(_t(f)), orc.gradient(f)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", range(7))
def test_gradient_every_tile_shape(gpu, orc, monkeypatch, shape):
    """Every candidate launch shape of the lower-star kernel (3D tiles and
    runs of consecutive ids) gives the oracle's gradient, alone and in a
    batch of uneven fields whose edges cut the tiles."""
    monkeypatch.setenv("TS_K3_TILE", str(shape))
    for dims, seed in [((23, 19, 17), 6), ((33, 2, 9), 7), ((70, 9, 13), 8)]:
        f = _rand(dims, seed, "ties")
        for a, b in zip(gpu.gradient(_t(f)), orc.gradient(f)):
            assert np.array_equal(a, b)
    fs = _uneven_batch(5, 2, 21, shape)
    for d, f in zip(gpu.diagram_batch([_t(f) for f in fs]), fs):
        _same_pairs(d, orc.diagram(f))


def test_gradient_2x2x2_orders(gpu, orc):
    rng = np.random.default_rng(0)
    perms = list(itertools.permutations(range(8)))
    for k in rng.choice(len(perms), size=300, replace=False):
        f = np.asarray(perms[k], dtype=np.float32).reshape(2, 2, 2)
        for a, b in zip(gpu.gradient(_t(f)), orc.gradient(f)):
            assert np.array_equal(a, b)
        _same_pairs(gpu.pairs(_t(f)), orc.pairs(f, 0))


@pytest.mark.parametrize("dims,seed", CASES)
def test_critical_and_pairs_bit_exact(gpu, orc, dims, seed):
    f = _rand(dims, seed, "normal")
    for a, b in zip(gpu.critical(_t(f)), orc.critical(f)):
        assert np.array_equal(a, b)
    _same_pairs(gpu.pairs(_t(f)), orc.pairs(f, 0))
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_diagram_gaussian_32(gpu, orc, seed):
    f = fields.workload("gauss8_32", seed)
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def test_diagram_gaussian_64_noisy(gpu, orc):
    # the 128^3 generator (64 Gaussians, noise 0.1) at 64^3
    f = fields.gaussian_mixture((64, 64, 64), 64, 0.1, 0)
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def test_diagram_filament_48(gpu, orc):
    f = fields.filament_field((48, 40, 44), 0)
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def test_diagram_gaussian_128(gpu, orc):
    """The 128^3 workload (64 Gaussians, U[-0.1, 0.1] noise) at full size:
    the whole diagram, bit-exact."""
    f = fields.workload("gauss64_128", 0)
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def test_filament_256_full_size(gpu, orc):
    """The benchmark's 256^3 workload in the benchmark's launch
    configuration, where the oracle cannot run the whole map: the vertex
    order in full, the lower-star gradient on sampled vertices (the oracle
    processes one lower star at a time), and invariants of the critical cells
    and pairs that hold at any size."""
    dims = (256, 256, 256)
    f = fields.workload("filament_256", 0)
    order_o, rank_o = orc.order(f)
    ft = _t(f)
    order_g, rank_g = gpu.order(ft)
    assert np.array_equal(order_g.cpu().numpy(), order_o)
    assert np.array_equal(rank_g.cpu().numpy(), rank_o)
    del order_g, rank_g
    vup, eup, tup = gpu.gradient(ft)
    rng = np.random.default_rng(1)
    n = f.size
    for v in rng.integers(0, n, 3000):
        pairs, crit = orc.gradient_at(rank_o, dims, int(v))
        for fd, face, cof in pairs:
            arr = (vup, eup, tup)[fd]
            assert arr[face] == cof, (v, fd, face, cof)
        for cd, cid in crit:
            if cd < 3:
                assert (vup, eup, tup)[cd][cid] == -1, (v, cd, cid)
    crit = gpu.critical(ft)
    c = [len(a) for a in crit]
    assert c[0] - c[1] + c[2] - c[3] == 1
    P = gpu.pairs(ft)
    ess = P["essential"] == 1
    assert ess.sum() == 1
    # every critical d-cell is in exactly one pair: the birth of a d-pair or
    # the death of a (d-1)-pair (the global minimum in the essential one)
    for d in range(4):
        cells = []
        if d < 3:
            cells.append(P["birth_cell"][P["dim"] == d])
        if d > 0:
            cells.append(P["death_cell"][(P["dim"] == d - 1) & ~ess])
        assert np.array_equal(np.sort(np.concatenate(cells)), np.sort(crit[d])), d
    # birth before death in the filtration
    assert np.all(rank_o[P["v_birth"][~ess]] <= rank_o[P["v_death"][~ess]])
    D = gpu.diagram(ft)
    assert len(D) == int((P["v_birth"] != P["v_death"]).sum())
    assert np.all(D["death"] >= D["birth"])


def test_column_pool_growth(gpu, orc, monkeypatch):
    """The saddle-saddle column pool starts tiny, so that the boundary pass
    and the reduction both run out of it and grow it (the reduction compacts
    the live columns on the device): the diagram is unchanged."""
    f = fields.gaussian_mixture((40, 36, 33), 64, 0.1, 4)
    ref = orc.diagram(f)
    for words in ("256", "6000", "7500", "9000", "20000"):
        monkeypatch.setenv("TS_D1_POOL_WORDS", words)
        _same_pairs(gpu.diagram(_t(f)), ref)
    monkeypatch.delenv("TS_D1_POOL_WORDS")
    _same_pairs(gpu.diagram(_t(f)), ref)


@pytest.mark.parametrize("steps,cap,cap2", [(16, 256, 1024), (16, 4, 1024), (16, 4, 4)])
def test_boundary_fallback_kinds(gpu, orc, monkeypatch, steps, cap, cap2):
    """Saddle-saddle boundaries: with a first pass cut at 16 pops, the columns
    go on to the wave-queue kernel (256 entries); with that queue cut to 4
    edges, on to the 1024-entry wave queue; with that cut to 4 edges too, on
    to the LDS-heap kernel; every route gives the oracle's diagram."""
    monkeypatch.setenv("TS_D1_STEPS", str(steps))
    monkeypatch.setenv("TS_D1_WAVE_CAP", str(cap))
    monkeypatch.setenv("TS_D1_WAVE2_CAP", str(cap2))
    f = fields.workload("filament_256", seed=3, dims=(48, 40, 36))
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def test_critical_list_retry(gpu, orc, monkeypatch):
    """Critical-cell lists that start too small are sized from the counts
    and the gradient kernel is run again: same critical cells."""
    f = _rand((23, 19, 17), 6, "normal")
    monkeypatch.setenv("TS_CRIT_CAP", "8")
    for a, b in zip(gpu.critical(_t(f)), orc.critical(f)):
        assert np.array_equal(a, b)
    _same_pairs(gpu.diagram(_t(f)), orc.diagram(f))


def _uneven_batch(nf, lo, hi, seed):
    """Gaussian-mixture fields (8 Gaussians, uniform noise 0.05) whose three
    axes are drawn independently from lo..hi."""
    rng = np.random.default_rng(seed)
    return [fields.gaussian_mixture(tuple(int(a) for a in rng.integers(lo, hi + 1, 3)), 8, 0.05,
                                    seed * 1000 + i) for i in range(nf)]


def test_diagram_batch_small(gpu, orc):
    """A batch of small and degenerate grids, ties and negative zeros: each
    field's diagram equals the oracle's diagram of that field alone."""
    fs = [_rand(d, s, k) for (d, s), k in zip(CASES, ["uniform", "ties", "normal", "ties",
                                                      "uniform", "normal", "ties", "uniform"])]
    fs[3] = fs[3] - 3.0
    fs[3][fs[3] == 0] = -0.0
    fs += _uneven_batch(6, 2, 30, 7)
    out = gpu.diagram_batch([_t(f) for f in fs])
    assert len(out) == len(fs)
    for d, f in zip(out, fs):
        _same_pairs(d, orc.diagram(f))
    # host pointers give the same result
    out_h = gpu.diagram_batch([np.ascontiguousarray(f) for f in fs])
    for a, b in zip(out, out_h):
        _same_pairs(a, b)


def test_diagram_batch_uneven_64(gpu):
    """64 fields with axes drawn from 24..96 (13.8 M vertices in all): each
    field's diagram from the batch equals its own single-field diagram."""
    fs = _uneven_batch(64, 24, 96, 1)
    out = gpu.diagram_batch([_t(f) for f in fs])
    for d, f in zip(out, fs):
        _same_pairs(d, gpu.diagram(_t(f)))


@pytest.mark.parametrize("kw", [dict(j_max=1000), dict(stop_mode=1, j_max=1000),
                                dict(j_max=25, nonsignal_dims=(1,), ties_signal=1,
                                     full_gradient=True)])
def test_simplify_batch_matches_single(gpu, kw):
    """Fields solved as a batch: every field's g, iterations, stop and loss
    are those of solving it alone (fields stop at different iterations)."""
    fs = _uneven_batch(7, 6, 22, 3) + [_rand((9, 8, 7), 5, "ties")]
    gs, reps = gpu.simplify_batch([_t(f) for f in fs], threshold=0.1, **kw)
    its = set()
    for f, g, r in zip(fs, gs, reps):
        g1, r1 = gpu.simplify(_t(f), threshold=0.1, **kw)
        assert (r.iterations, r.cancelled) == (r1.iterations, r1.cancelled)
        assert np.array_equal(g.cpu().numpy(), g1.cpu().numpy())
        assert r.loss == r1.loss and r.loss0 == r1.loss0
        assert r.n_pairs == r1.n_pairs and r.n_targets == r1.n_targets
        its.add(r.iterations)
    if kw.get("j_max") == 1000:
        assert len(its) > 1  # the fields really stop at different iterations


def test_simplify_batch_oracle(gpu, orc):
    """A small batch against the oracle, field by field."""
    fs = [fields.gaussian_mixture(d, 8, 0.05, 40 + i)
          for i, d in enumerate([(12, 9, 7), (5, 11, 8), (10, 10, 10)])]
    gs, reps = gpu.simplify_batch([np.ascontiguousarray(f) for f in fs], threshold=0.1, j_max=200)
    for f, g, r in zip(fs, gs, reps):
        go, ro = orc.simplify(f, threshold=0.1, j_max=200)
        assert r.iterations == ro.iterations and r.cancelled == ro.cancelled
        assert np.array_equal(g, go)


def test_host_pointer_path(gpu, orc):
    f = _rand((9, 8, 7), 11, "normal")
    _same_pairs(gpu.diagram(f), orc.diagram(f))


@pytest.mark.parametrize("dims,seed,j_max", [((12, 12, 12), 0, 1000), ((12, 12, 12), 1, 1000),
                                            ((16, 14, 13), 2, 1000), ((32, 32, 32), 3, 25)])
def test_simplify_parity(gpu, orc, dims, seed, j_max):
    f = fields.gaussian_mixture(dims, 8, 0.05, seed)
    g, rep = gpu.simplify(_t(f), threshold=0.1, j_max=j_max)
    go, ro = orc.simplify(f, threshold=0.1, j_max=j_max)
    assert rep.iterations == ro.iterations
    assert rep.cancelled == ro.cancelled
    g = g.cpu().numpy()
    assert np.abs(g.astype(np.float64) - go).max() <= 1e-6 * ro.range
    assert np.array_equal(g, go)
    assert rep.loss == pytest.approx(ro.loss, rel=1e-9, abs=1e-15)
    assert rep.n_targets == ro.n_targets
    if rep.cancelled:
        assert rep.max_nonsignal_pers < 1e-6 * rep.range


def test_simplify_loss_ratio_and_dim_mask(gpu, orc):
    f = fields.gaussian_mixture((14, 13, 12), 8, 0.05, 7)
    for kw in (dict(stop_mode=1), dict(nonsignal_dims=(1,), ties_signal=1, j_max=40)):
        g, rep = gpu.simplify(_t(f), threshold=0.1, **kw)
        go, ro = orc.simplify(f, threshold=0.1, **kw)
        assert rep.iterations == ro.iterations
        assert np.array_equal(g.cpu().numpy(), go)


def _torus_sdf(n, seed, noise=0.02):
    """Signed distance to a torus (major radius 0.3, minor 0.1) in the unit
    cube, plus uniform noise: one dominant saddle-saddle loop among noise."""
    rng = np.random.default_rng(seed)
    t = np.arange(n) / (n - 1) - 0.5
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    d = np.sqrt((np.sqrt(x * x + y * y) - 0.3) ** 2 + z * z) - 0.1
    return (d + rng.uniform(-noise, noise, d.shape)).astype(np.float32)


@pytest.mark.parametrize("alpha_b,alpha_d", [(0.0, 0.5), (0.5, 0.0)])
def test_cut_and_fill_parity(gpu, orc, alpha_b, alpha_d):
    """One-sided steps (only deaths or only births move, Sec. 5.3) on a
    noisy torus distance field: same iterations and bit-identical g."""
    f = _torus_sdf(18, 3)
    kw = dict(threshold=0.1, alpha_b=alpha_b, alpha_d=alpha_d, j_max=30)
    g, rep = gpu.simplify(_t(f), **kw)
    go, ro = orc.simplify(f, **kw)
    assert rep.iterations == ro.iterations and rep.cancelled == ro.cancelled
    assert np.array_equal(g.cpu().numpy(), go)
    # the torus loop is signal: it survives
    D = gpu.diagram(g)
    pers = D["death"] - D["birth"]
    assert ((D["dim"] == 1) & (pers > 0.1 * ro.range)).sum() >= 1


@pytest.mark.parametrize("case", ["gauss32", "ties", "filament64", "gauss128"])
def test_fast_update_same_as_full(gpu, case):
    """The fast gradient update between iterations (Sec. 4.2) gives the solver
    the same maps as recomputing the whole gradient: the same iterations and a
    bit-identical g, with fewer lower stars processed."""
    if case == "gauss32":
        f, kw = fields.gaussian_mixture((32, 32, 32), 8, 0.05, 11), dict(threshold=0.1, j_max=80)
    elif case == "ties":
        # values on a coarse grid: many equal neighbours, ordered by index
        f = np.round(fields.gaussian_mixture((21, 18, 15), 8, 0.05, 12) * 16).astype(np.float32)
        kw = dict(threshold=0.1, j_max=40)
    elif case == "filament64":
        f = fields.workload("filament_256", seed=3, dims=(64, 64, 64))
        kw = dict(threshold=0.1, nonsignal_dims=(1,), ties_signal=1, j_max=4)
    else:
        f = fields.workload("gauss64_128", seed=4)
        kw = dict(threshold=0.1, j_max=3)
    n = f.size
    ga, ra = gpu.simplify(_t(f), full_gradient=True, **kw)
    gb, rb = gpu.simplify(_t(f), **kw)
    assert ra.iterations == rb.iterations and ra.iterations > 0
    assert ra.cancelled == rb.cancelled
    assert np.array_equal(ga.cpu().numpy(), gb.cpu().numpy())
    assert ra.loss == rb.loss
    assert ra.n_regradient == n * ra.iterations
    assert 0 < rb.n_regradient <= n * rb.iterations
    if case in ("gauss32", "ties"):  # long runs: late updates touch few vertices
        assert rb.n_regradient < n * rb.iterations


def test_paper_auction_precision(gpu, orc):
    """The paper's setting (auction at relative precision 0.01 with the
    loss-ratio stop L <= 0.01 L0, Sec. 5) is an option: on a 24^3 noisy field
    it reaches the stop and keeps the signal pairs, though its trajectory may
    differ from the exact oracle's."""
    f = fields.gaussian_mixture((24, 24, 24), 8, 0.05, 2)
    kw = dict(threshold=0.1, stop_mode=1, loss_ratio_s=0.01)
    g, rep = gpu.simplify(_t(f), assign_precision=0.01, **kw)
    go, ro = orc.simplify(f, **kw)
    assert rep.cancelled == 1 and ro.cancelled == 1
    assert rep.loss <= 0.01 * rep.loss0
    assert rep.n_targets == ro.n_targets
    D = gpu.diagram(g)
    Do = orc.diagram(go)
    thr = 0.1 * ro.range
    big = lambda X: sorted(zip(X["dim"][(X["death"] - X["birth"]) > thr].tolist()))
    assert big(D) == big(Do)
    with pytest.raises(gpu.TopsimpError):
        gpu.simplify(_t(f), assign_precision=-1.0)


def test_errors(gpu):
    import torch
    f = np.zeros((3, 3, 3), np.float32)
    f[1, 1, 1] = np.inf
    with pytest.raises(gpu.TopsimpError) as e:
        gpu.diagram(_t(f))
    assert e.value.code == -2
    with pytest.raises(gpu.TopsimpError) as e:
        gpu.diagram(_t(np.zeros((1, 3, 3), np.float32)))
    assert e.value.code == -1
    # the context still works after an error
    assert len(gpu.diagram(_t(np.arange(27, dtype=np.float32).reshape(3, 3, 3)))) == 1
    del torch


def test_batch_edges(gpu, orc):
    """A batch of one field is the field's own diagram; host arrays give the
    same solves as device tensors; a batch rejects a non-finite field, a
    grid below 2 and mixed memory kinds, and the context keeps working."""
    f = fields.gaussian_mixture((13, 11, 9), 8, 0.05, 21)
    (d,) = gpu.diagram_batch([_t(f)])
    _same_pairs(d, orc.diagram(f))
    fs = _uneven_batch(3, 5, 12, 9)
    gh, rh = gpu.simplify_batch([np.ascontiguousarray(x) for x in fs], threshold=0.1, j_max=50)
    gd, rd = gpu.simplify_batch([_t(x) for x in fs], threshold=0.1, j_max=50)
    for a, b, ra, rb in zip(gh, gd, rh, rd):
        assert np.array_equal(a, b.cpu().numpy()) and ra.iterations == rb.iterations
    bad = f.copy()
    bad[2, 3, 4] = np.nan
    with pytest.raises(gpu.TopsimpError) as e:
        gpu.diagram_batch([_t(f), _t(bad)])
    assert e.value.code == -2
    with pytest.raises(gpu.TopsimpError) as e:
        gpu.diagram_batch([_t(f), _t(np.zeros((1, 4, 4), np.float32))])
    assert e.value.code == -1
    with pytest.raises(ValueError):
        gpu.diagram_batch([_t(f), np.ascontiguousarray(f)])
    (d,) = gpu.diagram_batch([_t(f)])
    _same_pairs(d, orc.diagram(f))


def test_autotuned_launches_same_result(gpu, orc):
    """The first maps of a size class try each K3 tile shape and D1 block size
    in turn, later ones use the fastest: every map gives the oracle's diagram."""
    f = fields.gaussian_mixture((50, 47, 45), 64, 0.1, 13)
    want = orc.diagram(f)
    k3_key = "k3.tiles.%d" % f.size.bit_length()
    for _ in range(len(gpu.K3_TILE_SHAPES)):
        _same_pairs(gpu.diagram(_t(f)), want)
    # every K3 candidate tried once: the choice is made by now
    ch = gpu.launch_choices()
    assert 0 <= ch[k3_key] < len(gpu.K3_TILE_SHAPES)
    assert all(-1 <= v < len(gpu.K3_TILE_SHAPES) for v in ch.values())


def test_deterministic(gpu):
    f = fields.gaussian_mixture((40, 36, 33), 64, 0.1, 5)
    a = gpu.pairs(_t(f))
    b = gpu.pairs(_t(f))
    _same_pairs(a, b)


def _two_dips():
    from tests.test_oracle_still import _two_dips as make
    return make()


@pytest.mark.parametrize("keep", [(), (0,), (1,), (0, 1)])
def test_list_mode_parity(gpu, orc, keep):
    """Explicit signal lists (Sec. 3): the listed pairs are held, the others
    cancelled; same iterations and bit-identical g as the oracle."""
    f, dips = _two_dips()
    D = orc.diagram(f)
    fin = D[D["essential"] == 0]
    by_v = {int(p["v_birth"]): p for p in fin}
    lst = np.array([by_v[dips[k][0]] for k in keep], dtype=orc.PAIR_DTYPE)
    g, rep = gpu.simplify(_t(f), signal_pairs=lst)
    go, ro = orc.simplify(f, signal_pairs=lst)
    assert (rep.iterations, rep.n_targets) == (ro.iterations, ro.n_targets)
    assert np.array_equal(g.cpu().numpy(), go)


def test_list_equal_to_threshold_set(gpu, orc):
    """The list of the threshold rule's signal pairs gives the threshold
    solve, on the GPU as in the oracle; dropping the most persistent listed
    pair from the list changes the solve exactly as in the oracle."""
    f = fields.gaussian_mixture((12, 11, 10), 8, 0.05, 0)
    D = orc.diagram(f)
    rng = float(f.max()) - float(f.min())
    thr = float(np.float32(0.1)) * rng
    pers = D["death"].astype(np.float64) - D["birth"].astype(np.float64)
    lst = D[(D["essential"] == 0) & (pers > thr)]
    g1, r1 = gpu.simplify(_t(f), threshold=0.1, j_max=30)
    g2, r2 = gpu.simplify(_t(f), signal_pairs=lst, j_max=30)
    assert r1.iterations == r2.iterations
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())
    short = np.delete(lst, int(np.argmax(lst["death"] - lst["birth"])))
    g3, r3 = gpu.simplify(_t(f), signal_pairs=short, j_max=30)
    go, ro = orc.simplify(f, signal_pairs=short, j_max=30)
    assert r3.iterations == ro.iterations and r3.n_targets == len(short) + 1
    assert np.array_equal(g3.cpu().numpy(), go)


@pytest.mark.parametrize("kw", [dict(threshold=0.1), dict(threshold=0.1, nonsignal_dims=(1,),
                                                           ties_signal=1)])
def test_signal_mask(gpu, orc, kw):
    """The signal-vertex mask marks exactly the birth and death vertices of
    the pairs of D(f) that the threshold rule keeps (Sec. 3)."""
    f = fields.gaussian_mixture((20, 18, 16), 8, 0.05, 4)
    m, cnt = gpu.signal_mask(_t(f), **kw)
    D = orc.diagram(f)
    rng = float(f.max()) - float(f.min())
    thr = float(np.float32(kw["threshold"])) * rng
    pers = D["death"].astype(np.float64) - D["birth"].astype(np.float64)
    below = (pers < thr) | ((pers == thr) & (kw.get("ties_signal", 0) == 0))
    masked = np.isin(D["dim"], list(kw.get("nonsignal_dims", (0, 1, 2))))
    keep = (D["essential"] == 1) | ~(masked & below)
    want = np.zeros(f.size, np.float32)
    want[D["v_birth"][keep]] = 1.0
    want[D["v_death"][keep]] = 1.0
    assert cnt == int(keep.sum())
    assert np.array_equal(m.cpu().numpy().ravel(), want)
    # list mode: the mask of the list's own pairs
    lst = D[keep & (D["essential"] == 0)][:3]
    ml, cl = gpu.signal_mask(f, signal_pairs=lst)
    want = np.zeros(f.size, np.float32)
    for p in list(lst) + list(D[D["essential"] == 1]):
        want[p["v_birth"]] = want[p["v_death"]] = 1.0
    assert cl == 4 and np.array_equal(ml.ravel(), want)


def test_overlapping_buffers_rejected(gpu):
    import torch
    f = _t(fields.gaussian_mixture((8, 8, 8), 8, 0.05, 0))
    buf = torch.empty(2 * f.numel(), dtype=torch.float32, device=f.device)
    buf[: f.numel()] = f.ravel()
    src = buf[: f.numel()].view(f.shape)
    dst = buf[f.numel() // 2: f.numel() // 2 + f.numel()].view(f.shape)
    with pytest.raises(gpu.TopsimpError) as e:
        gpu.simplify(src, out=dst)
    assert e.value.code == -1
    g, _ = gpu.simplify(src, out=buf[f.numel():].view(f.shape), j_max=2)
    assert g.data_ptr() == buf[f.numel():].data_ptr()


def test_trace_matches_oracle(gpu, orc):
    """The per-iteration trace of a solve: the losses are the oracle's
    (Alg. 1, iteration by iteration), the last entry's largest non-signal
    persistence is the report's, and the times do not decrease."""
    f = fields.gaussian_mixture((16, 14, 13), 8, 0.05, 2)
    g, rep = gpu.simplify(_t(f), threshold=0.1, j_max=1000, trace=True)
    go, ro = orc.simplify(f, threshold=0.1, j_max=1000)
    assert rep.trace.shape == (rep.iterations + 1, 4)
    assert rep.iterations == ro.iterations
    np.testing.assert_allclose(rep.trace[:, 1], ro.trace, rtol=1e-9, atol=1e-15)
    assert rep.trace[-1, 2] == rep.max_nonsignal_pers
    assert np.all(np.diff(rep.trace[:, 0]) >= 0) and np.all(np.diff(rep.trace[:, 3]) >= 0)
