"""Python access to the CPU oracle (oracle/tso.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  The product path never
imports this module.

Fields are numpy float32 arrays of shape (Lz, Ly, Lx); dims are (Lx, Ly, Lz).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "tso.cpp")

PAIR_DTYPE = np.dtype([
    ("dim", "<i4"), ("essential", "<i4"),
    ("birth_cell", "<i8"), ("death_cell", "<i8"),
    ("v_birth", "<i8"), ("v_death", "<i8"),
    ("birth", "<f4"), ("death", "<f4"),
])
assert PAIR_DTYPE.itemsize == 48


OMP_LIB_PATH = os.path.join(HERE, "liboracle_omp.so")


def _compile(path, extra, force):
    if force or not os.path.exists(path) or os.path.getmtime(path) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "tso.h"))):
        tmp = path + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC",
                               "-shared"] + extra + [SRC, "-o", tmp])
        os.replace(tmp, path)
    return path


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain FP32, no contraction), and its
    multi-core timing build (-fopenmp; same source, same results)."""
    _compile(OMP_LIB_PATH, ["-fopenmp"], force)
    return _compile(LIB_PATH, [], force)


class _Signal(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threshold_rel", ctypes.c_float),
                ("nonsignal_dim_mask", ctypes.c_uint32), ("ties_signal", ctypes.c_int32),
                ("signal", ctypes.c_void_p), ("n_signal", ctypes.c_int64)]


class _Options(ctypes.Structure):
    _fields_ = [("alpha_b", ctypes.c_float), ("alpha_d", ctypes.c_float),
                ("j_max", ctypes.c_int32), ("stop_mode", ctypes.c_int32),
                ("cancel_tol_rel", ctypes.c_float), ("loss_ratio_s", ctypes.c_float)]


class _Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cancelled", ctypes.c_int32),
                ("loss0", ctypes.c_double), ("loss", ctypes.c_double),
                ("energy", ctypes.c_double), ("linf", ctypes.c_double),
                ("l2", ctypes.c_double), ("max_nonsignal_pers", ctypes.c_double),
                ("max_signal_disp", ctypes.c_double), ("range", ctypes.c_double),
                ("n_pairs", ctypes.c_int64 * 3), ("n_still", ctypes.c_int64),
                ("n_reduced", ctypes.c_int64), ("n_targets", ctypes.c_int64),
                ("total_s", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.tso_order.argtypes = [P, i64, P, P]
        L.tso_gradient.argtypes = [P, P, P, P, P]
        L.tso_gradient_at.argtypes = [P, P, i64, P, P, P, P, P, P, P]
        L.tso_critical.argtypes = [P, P, P, P, i64, P]
        L.tso_pairs.argtypes = [P, P, i32, P, i64, P]
        L.tso_diagram.argtypes = [P, P, P, i64, P]
        L.tso_assign.argtypes = [i64, P, P, i64, P, P, P, P]
        L.tso_bottleneck.argtypes = [P, i64, P, i64, P]
        L.tso_simplify.argtypes = [P, P, P, P, P, P, P, i64]
        L.tso_assign_step.argtypes = [P, i64, P, P, i64, P, i64, P, P, P]
        L.tso_threads.argtypes = []
        for fn in ("tso_order", "tso_gradient", "tso_gradient_at", "tso_critical",
                   "tso_pairs", "tso_diagram", "tso_assign", "tso_bottleneck",
                   "tso_simplify", "tso_assign_step", "tso_threads"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise OracleError(f"{what} failed with code {rc}")
    return rc


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _field(f):
    f = np.ascontiguousarray(f, dtype=np.float32)
    if f.ndim != 3:
        raise ValueError("field must have shape (Lz, Ly, Lx)")
    dims = np.array([f.shape[2], f.shape[1], f.shape[0]], dtype=np.int64)
    return f, dims


def order(f):
    f = np.ascontiguousarray(f, dtype=np.float32).ravel()
    o = np.empty(f.size, np.int32)
    r = np.empty(f.size, np.int32)
    _check(lib().tso_order(_ptr(f), f.size, _ptr(o), _ptr(r)), "tso_order")
    return o, r


def gradient(f):
    """Dense partner arrays (vup[n], eup[7n], tup[12n])."""
    f, dims = _field(f)
    n = f.size
    vup = np.empty(n, np.int32)
    eup = np.empty(7 * n, np.int32)
    tup = np.empty(12 * n, np.int32)
    _check(lib().tso_gradient(_ptr(f), _ptr(dims), _ptr(vup), _ptr(eup), _ptr(tup)),
           "tso_gradient")
    return vup, eup, tup


def gradient_at(rank, dims, v):
    """(pairs [(face_dim, face_id, coface_id)], critical [(dim, id)]) of L(v)."""
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    d = np.asarray(dims, dtype=np.int64)
    pd_ = np.empty(80, np.int32)
    pf = np.empty(80, np.int64)
    pc = np.empty(80, np.int64)
    npairs = np.zeros(1, np.int32)
    cd = np.empty(80, np.int32)
    ci = np.empty(80, np.int64)
    ncrit = np.zeros(1, np.int32)
    _check(lib().tso_gradient_at(_ptr(rank), _ptr(d), int(v), _ptr(pd_), _ptr(pf), _ptr(pc),
                                 _ptr(npairs), _ptr(cd), _ptr(ci), _ptr(ncrit)),
           "tso_gradient_at")
    k, c = int(npairs[0]), int(ncrit[0])
    return ([(int(pd_[i]), int(pf[i]), int(pc[i])) for i in range(k)],
            [(int(cd[i]), int(ci[i])) for i in range(c)])


def critical(f):
    """List of 4 int64 arrays: critical cell ids per dim, sorted by lex key."""
    f, dims = _field(f)
    cnt = np.zeros(1, np.int64)
    rc = lib().tso_critical(_ptr(f), _ptr(dims), None, None, 0, _ptr(cnt))
    if rc not in (0, -5, -1):
        _check(rc, "tso_critical")
    m = int(cnt[0])
    od = np.empty(max(m, 1), np.int32)
    oi = np.empty(max(m, 1), np.int64)
    _check(lib().tso_critical(_ptr(f), _ptr(dims), _ptr(od), _ptr(oi), m, _ptr(cnt)),
           "tso_critical")
    od, oi = od[:m], oi[:m]
    return [oi[od == d] for d in range(4)]


def _pairs_call(fn, f, *extra):
    f, dims = _field(f)
    cap = 1024
    while True:
        out = np.empty(cap, PAIR_DTYPE)
        cnt = np.zeros(1, np.int64)
        rc = fn(_ptr(f), _ptr(dims), *extra, _ptr(out), cap, _ptr(cnt))
        if rc == -5:
            cap = int(cnt[0]) + 1
            continue
        _check(rc, fn.__name__)
        return out[: int(cnt[0])].copy()


def pairs(f, method=0):
    """All persistence pairs incl. zero-persistence ones (method 0 DMS-style,
    1 full reduction, 2 Kruskal for dims 0 and 2)."""
    return _pairs_call(lib().tso_pairs, f, ctypes.c_int32(method))


def diagram(f):
    return _pairs_call(lib().tso_diagram, f)


_omp = None


def omp_lib():
    """The OpenMP timing build (gradient and vertex-order loops on all
    threads of OMP_NUM_THREADS); for the benchmark's CPU baseline only."""
    global _omp
    if _omp is None:
        build()
        L = ctypes.CDLL(OMP_LIB_PATH)
        P, i64 = ctypes.c_void_p, ctypes.c_int64
        L.tso_diagram.argtypes = [P, P, P, i64, P]
        L.tso_diagram.restype = ctypes.c_int
        L.tso_threads.argtypes = []
        L.tso_threads.restype = ctypes.c_int
        _omp = L
    return _omp


def diagram_omp(f):
    """diagram(f) by the OpenMP build; returns (records, threads used)."""
    L = omp_lib()
    return _pairs_call(L.tso_diagram, f), int(L.tso_threads())


def assign(pb, pd, qb, qd):
    pb, pd, qb, qd = (np.ascontiguousarray(a, dtype=np.float64) for a in (pb, pd, qb, qd))
    match = np.empty(max(len(pb), 1), np.int32)
    cost = np.zeros(1, np.float64)
    _check(lib().tso_assign(len(pb), _ptr(pb), _ptr(pd), len(qb), _ptr(qb), _ptr(qd),
                            _ptr(match), _ptr(cost)), "tso_assign")
    return match[: len(pb)].copy(), float(cost[0])


def assign_step(prev, phi_prev, cur, targets):
    """One iteration's assignment (Sec. 4.3): still join of `cur` against
    `prev` (records in diagram order), inheritance of `phi_prev`, exact
    reduced problem against the targets no still point holds, canonical
    form.  Returns (phi, n_still, n_reduced)."""
    prev = np.ascontiguousarray(prev, dtype=PAIR_DTYPE)
    cur = np.ascontiguousarray(cur, dtype=PAIR_DTYPE)
    targets = np.ascontiguousarray(targets, dtype=PAIR_DTYPE)
    phi_prev = np.ascontiguousarray(phi_prev, dtype=np.int32)
    assert len(phi_prev) == len(prev)
    phi = np.empty(max(len(cur), 1), np.int32)
    ns = np.zeros(1, np.int64)
    nr = np.zeros(1, np.int64)
    _check(lib().tso_assign_step(_ptr(prev), len(prev), _ptr(phi_prev), _ptr(cur), len(cur),
                                 _ptr(targets), len(targets), _ptr(phi), _ptr(ns), _ptr(nr)),
           "tso_assign_step")
    return phi[: len(cur)].copy(), int(ns[0]), int(nr[0])


def bottleneck(a, b):
    a = np.ascontiguousarray(a, dtype=PAIR_DTYPE)
    b = np.ascontiguousarray(b, dtype=PAIR_DTYPE)
    out = np.zeros(1, np.float64)
    _check(lib().tso_bottleneck(_ptr(a), len(a), _ptr(b), len(b), _ptr(out)),
           "tso_bottleneck")
    return float(out[0])


@dataclass
class Report:
    iterations: int
    cancelled: int
    loss0: float
    loss: float
    energy: float
    linf: float
    l2: float
    max_nonsignal_pers: float
    max_signal_disp: float
    range: float
    n_pairs: tuple
    n_still: int
    n_reduced: int
    n_targets: int
    total_s: float
    status: int
    trace: np.ndarray


def simplify(f, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0, alpha_b=0.5,
             alpha_d=0.5, j_max=1000, stop_mode=0, cancel_tol_rel=1e-6, loss_ratio_s=0.01,
             signal_pairs=None):
    f, dims = _field(f)
    sig = _Signal()
    if signal_pairs is not None:
        sp = np.ascontiguousarray(signal_pairs, dtype=PAIR_DTYPE)
        sig.mode, sig.signal, sig.n_signal = 1, sp.ctypes.data, len(sp)
    else:
        sig.mode = 0
        sig.threshold_rel = threshold
        sig.nonsignal_dim_mask = sum(1 << d for d in nonsignal_dims)
        sig.ties_signal = ties_signal
    opt = _Options(alpha_b, alpha_d, j_max, stop_mode, cancel_tol_rel, loss_ratio_s)
    rep = _Report()
    g = np.empty_like(f)
    trace = np.zeros(j_max + 1, np.float64)
    rc = lib().tso_simplify(_ptr(f), _ptr(dims), ctypes.byref(sig), ctypes.byref(opt),
                            _ptr(g), ctypes.byref(rep), _ptr(trace), len(trace))
    _check(rc, "tso_simplify")
    r = Report(rep.iterations, rep.cancelled, rep.loss0, rep.loss, rep.energy, rep.linf,
               rep.l2, rep.max_nonsignal_pers, rep.max_signal_disp, rep.range,
               tuple(rep.n_pairs), rep.n_still, rep.n_reduced, rep.n_targets, rep.total_s,
               rc, trace[: rep.iterations + 1].copy())
    return g, r
