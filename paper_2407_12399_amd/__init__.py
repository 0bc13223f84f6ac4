"""Python binding of the topsimp C ABI (include/topsimp.h).

Argument marshalling only: every step runs in libtopsimp.so (HIP kernels
for gfx950 plus the host-side exact assignment).  PyTorch is used for device
memory and the current HIP stream.  Importing this package does not load the
library; the first call does, and raises if it is missing.

Fields are float32 arrays of shape (Lz, Ly, Lx) (x fastest): a torch CUDA
tensor (used in place on its device and current stream) or anything numpy
accepts (copied through host memory).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtopsimp.so")

PAIR_DTYPE = np.dtype([
    ("dim", "<i4"), ("essential", "<i4"),
    ("birth_cell", "<i8"), ("death_cell", "<i8"),
    ("v_birth", "<i8"), ("v_death", "<i8"),
    ("birth", "<f4"), ("death", "<f4"),
])

TS_OK, TS_WARN_NOT_CANCELLED = 0, 1
ERRORS = {-1: "TS_ERR_ARG", -2: "TS_ERR_NONFINITE", -3: "TS_ERR_OOM", -4: "TS_ERR_HIP",
          -5: "TS_ERR_CAPACITY", -6: "TS_ERR_INTERNAL"}


class TopsimpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Signal(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threshold_rel", ctypes.c_float),
                ("nonsignal_dim_mask", ctypes.c_uint32), ("ties_signal", ctypes.c_int32),
                ("signal", ctypes.c_void_p), ("n_signal", ctypes.c_int64)]


class _Options(ctypes.Structure):
    _fields_ = [("alpha_b", ctypes.c_float), ("alpha_d", ctypes.c_float),
                ("j_max", ctypes.c_int32), ("stop_mode", ctypes.c_int32),
                ("cancel_tol_rel", ctypes.c_float), ("loss_ratio_s", ctypes.c_float),
                ("inputs_on_device", ctypes.c_int32), ("assign_precision", ctypes.c_float),
                ("full_gradient", ctypes.c_int32), ("init", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int64)]


class _Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cancelled", ctypes.c_int32),
                ("loss0", ctypes.c_double), ("loss", ctypes.c_double),
                ("energy", ctypes.c_double), ("linf", ctypes.c_double),
                ("l2", ctypes.c_double), ("max_nonsignal_pers", ctypes.c_double),
                ("max_signal_disp", ctypes.c_double), ("range", ctypes.c_double),
                ("n_pairs", ctypes.c_int64 * 3), ("n_still", ctypes.c_int64),
                ("n_reduced", ctypes.c_int64), ("n_targets", ctypes.c_int64),
                ("total_s", ctypes.c_double), ("persistence_s", ctypes.c_double),
                ("assign_s", ctypes.c_double), ("update_s", ctypes.c_double),
                ("n_regradient", ctypes.c_int64), ("init_used", ctypes.c_int32)]


_lib = None
_ctx = {}

EXPORTS = ["ts_create", "ts_destroy", "ts_last_error", "ts_diagram", "ts_diagram_batch",
           "ts_simplify", "ts_simplify_batch", "ts_unet_param_count", "ts_unet_forward",
           "ts_unet_backward", "ts_unet_adam",
           "ts_order", "ts_gradient", "ts_critical", "ts_pairs", "ts_assign", "ts_assign_auction",
           "ts_stage_times", "ts_signal_mask", "ts_order_noalloc", "ts_launch_choices"]


def lib():
    """Load libtopsimp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.ts_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
        L.ts_destroy.argtypes = [P]
        L.ts_last_error.argtypes = [P]
        L.ts_last_error.restype = ctypes.c_char_p
        L.ts_diagram.argtypes = [P, P, P, i32, P, i64, P]
        L.ts_diagram_batch.argtypes = [P, i32, P, P, i32, P, i64, P]
        L.ts_simplify.argtypes = [P, P, P, P, P, P, P]
        L.ts_simplify_batch.argtypes = [P, i32, P, P, P, P, P, P]
        L.ts_signal_mask.argtypes = [P, P, P, P, i32, P, P]
        L.ts_order_noalloc.argtypes = [P, i64, P, P, P]
        L.ts_unet_param_count.argtypes = [P]
        L.ts_unet_forward.argtypes = [P, P, P, P, P]
        L.ts_unet_backward.argtypes = [P, P, P, P, P, P, P]
        f32 = ctypes.c_float
        L.ts_unet_adam.argtypes = [P, P, P, P, P, i64, i64, f32, f32, f32, f32]
        L.ts_order.argtypes = [P, P, i64, i32, P, P]
        L.ts_gradient.argtypes = [P, P, P, i32, P, P, P]
        L.ts_critical.argtypes = [P, P, P, i32, P, P, i64, P]
        L.ts_pairs.argtypes = [P, P, P, i32, P, i64, P]
        L.ts_assign.argtypes = [i64, P, P, i64, P, P, P, P]
        L.ts_assign_auction.argtypes = [i64, P, P, i64, P, P, ctypes.c_double, P, P]
        L.ts_stage_times.argtypes = [P, ctypes.POINTER(ctypes.POINTER(ctypes.c_char_p)),
                                     ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
        L.ts_launch_choices.argtypes = [P, ctypes.POINTER(ctypes.POINTER(ctypes.c_char_p)),
                                        ctypes.POINTER(ctypes.POINTER(ctypes.c_int))]
        for fn in EXPORTS:
            if fn != "ts_last_error":
                getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def context(device=None):
    """Context bound to (device, current torch stream)."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("topsimp needs a ROCm GPU (torch.cuda.is_available() is False)")
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    if key not in _ctx:
        h = ctypes.c_void_p()
        rc = lib().ts_create(ctypes.byref(h), dev, ctypes.c_void_p(stream))
        if rc != 0:
            raise TopsimpError(rc, "ts_create failed")
        _ctx[key] = h
    return _ctx[key]


def _check(ctx, rc, allow=(0,)):
    if rc not in allow:
        msg = lib().ts_last_error(ctx)
        raise TopsimpError(rc, msg.decode() if msg else "")
    return rc


def _as_field(field):
    """(pointer, dims, on_device, keepalive)"""
    torch = _torch()
    if isinstance(field, torch.Tensor):
        if field.dtype != torch.float32 or field.dim() != 3:
            raise ValueError("field must be a 3D float32 tensor (Lz, Ly, Lx)")
        t = field.contiguous()
        dims = np.array([t.shape[2], t.shape[1], t.shape[0]], np.int64)
        if t.is_cuda:
            return ctypes.c_void_p(t.data_ptr()), dims, 1, t
        a = t.numpy()
    else:
        a = np.ascontiguousarray(field, dtype=np.float32)
        if a.ndim != 3:
            raise ValueError("field must have shape (Lz, Ly, Lx)")
        dims = np.array([a.shape[2], a.shape[1], a.shape[0]], np.int64)
    return a.ctypes.data_as(ctypes.c_void_p), dims, 0, a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


_cap_hint = {}


def _pairs_call(fn, field):
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    nv = int(np.prod(dims))
    # a capacity that usually fits, so that the map is not computed twice
    cap = max(4096, _cap_hint.get((fn.__name__, nv), nv // 4 + 16))
    torch = _torch()
    while True:
        # the records land in pinned host memory (a full-speed copy); the
        # returned array is a view that keeps that memory alive
        buf = torch.empty(cap * PAIR_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
        out = buf.numpy().view(PAIR_DTYPE)
        n = np.zeros(1, np.int64)
        rc = fn(ctx, fp, _ptr(dims), on_dev, _ptr(out), cap, _ptr(n))
        if rc == -5:
            cap = int(n[0]) + 1
            continue
        _check(ctx, rc)
        _cap_hint[(fn.__name__, int(np.prod(dims)))] = int(n[0]) + int(n[0]) // 8 + 16
        return out[: int(n[0])]


def diagram(field) -> np.ndarray:
    """Persistence diagram D(f) in diagram order (structured array)."""
    return _pairs_call(lib().ts_diagram, field)


def _batch_args(fields):
    """(pointer array, dims array, on_device, keepalive) of a list of fields,
    all device tensors or all host arrays."""
    if len(fields) == 0:
        raise ValueError("empty batch")
    parts = [_as_field(f) for f in fields]
    on_dev = {p[2] for p in parts}
    if len(on_dev) != 1:
        raise ValueError("a batch holds only device fields or only host fields")
    ptrs = (ctypes.c_void_p * len(parts))(*[p[0] for p in parts])
    dims = np.concatenate([p[1] for p in parts]).astype(np.int64)
    return ptrs, dims, on_dev.pop(), parts


def diagram_batch(fields) -> list:
    """Diagrams of a list of fields of any sizes, computed together (every
    stage runs once over the batch); one structured array per field."""
    ctx = context()
    ptrs, dims, on_dev, keep = _batch_args(fields)
    nf = len(fields)
    counts = np.zeros(nf, np.int64)
    nv = int(np.prod(dims.reshape(-1, 3), axis=1).sum())
    cap = max(4096, _cap_hint.get(("batch", nv), nv // 4 + 16))
    torch = _torch()
    while True:
        # pinned host memory: the records arrive in one full-speed copy
        buf = torch.empty(cap * PAIR_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
        out = buf.numpy().view(PAIR_DTYPE)
        rc = lib().ts_diagram_batch(ctx, nf, ptrs, _ptr(dims), on_dev, _ptr(out), cap, _ptr(counts))
        if rc == -5:
            cap = int(counts.sum()) + 1
            continue
        _check(ctx, rc)
        _cap_hint[("batch", nv)] = int(counts.sum()) * 9 // 8 + 16
        ends = np.cumsum(counts)
        return [out[e - c: e] for c, e in zip(counts, ends)]


def pairs(field) -> np.ndarray:
    """All pairs of critical cells incl. zero-persistence ones, plus the
    essential class, sorted by (dim, birth_cell, death_cell)."""
    return _pairs_call(lib().ts_pairs, field)


def order(field):
    """(order, rank) int32 arrays of the vertex order."""
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    n = int(np.prod(dims))
    torch = _torch()
    if on_dev:
        o = torch.empty(n, dtype=torch.int32, device=keep.device)
        r = torch.empty(n, dtype=torch.int32, device=keep.device)
        _check(ctx, lib().ts_order(ctx, fp, n, 1, ctypes.c_void_p(o.data_ptr()),
                                   ctypes.c_void_p(r.data_ptr())))
        return o, r
    o = np.empty(n, np.int32)
    r = np.empty(n, np.int32)
    _check(ctx, lib().ts_order(ctx, fp, n, 0, _ptr(o), _ptr(r)))
    return o, r


def gradient(field):
    """Dense partner arrays (vup[n], eup[7n], tup[12n]) of the gradient."""
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    n = int(np.prod(dims))
    vup = np.empty(n, np.int32)
    eup = np.empty(7 * n, np.int32)
    tup = np.empty(12 * n, np.int32)
    _check(ctx, lib().ts_gradient(ctx, fp, _ptr(dims), on_dev, _ptr(vup), _ptr(eup), _ptr(tup)))
    return vup, eup, tup


def critical(field):
    """Critical cell ids per dimension (4 int64 arrays), sorted by lex key."""
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    counts = np.zeros(4, np.int64)
    cap = 4096
    while True:
        od = np.empty(cap, np.int32)
        oi = np.empty(cap, np.int64)
        rc = lib().ts_critical(ctx, fp, _ptr(dims), on_dev, _ptr(od), _ptr(oi), cap, _ptr(counts))
        if rc == -5:
            cap = int(counts.sum()) + 1
            continue
        _check(ctx, rc)
        m = int(counts.sum())
        od, oi = od[:m], oi[:m]
        return [oi[od == d].copy() for d in range(4)]


def assign(pb, pd, qb, qd):
    """Exact one-dimension assignment (host only): (match, cost)."""
    pb, pd, qb, qd = (np.ascontiguousarray(a, dtype=np.float64) for a in (pb, pd, qb, qd))
    match = np.empty(max(len(pb), 1), np.int32)
    cost = np.zeros(1, np.float64)
    rc = lib().ts_assign(len(pb), _ptr(pb), _ptr(pd), len(qb), _ptr(qb), _ptr(qd), _ptr(match),
                         _ptr(cost))
    if rc != 0:
        raise TopsimpError(rc, "ts_assign failed")
    return match[: len(pb)].copy(), float(cost[0])


def assign_auction(pb, pd, qb, qd, rel_precision=0.0):
    """The auction alone (host only), stopped at the given relative precision
    (0: final epsilon): (match, cost)."""
    pb, pd, qb, qd = (np.ascontiguousarray(a, dtype=np.float64) for a in (pb, pd, qb, qd))
    match = np.empty(max(len(pb), 1), np.int32)
    cost = np.zeros(1, np.float64)
    rc = lib().ts_assign_auction(len(pb), _ptr(pb), _ptr(pd), len(qb), _ptr(qb), _ptr(qd),
                                 ctypes.c_double(rel_precision), _ptr(match), _ptr(cost))
    if rc != 0:
        raise TopsimpError(rc, "ts_assign_auction failed")
    return match[: len(pb)].copy(), float(cost[0])


def stage_times():
    """{stage name: device ms} of the last call on the current context."""
    ctx = context()
    names = ctypes.POINTER(ctypes.c_char_p)()
    ms = ctypes.POINTER(ctypes.c_double)()
    k = lib().ts_stage_times(ctx, ctypes.byref(names), ctypes.byref(ms))
    return {names[i].decode(): ms[i] for i in range(max(k, 0))}


# candidates of the tuned launches, in the library's index order ("runs":
# runs of 256 consecutive vertex ids instead of 3D tiles)
K3_TILE_SHAPES = ((256, 1, 1), (64, 4, 1), (32, 8, 1), (32, 4, 2), (16, 4, 4), (8, 8, 4), "runs")
D1_BLOCK_BITS = (16, 17, 18, 20, 24)


def launch_choices():
    """{launch key: candidate index in use, -1 while still trying} of the
    current context's launch tuner (keys "k3.tiles.<c>", "d1.block.<c>", ...)."""
    ctx = context()
    keys = ctypes.POINTER(ctypes.c_char_p)()
    ch = ctypes.POINTER(ctypes.c_int)()
    k = lib().ts_launch_choices(ctx, ctypes.byref(keys), ctypes.byref(ch))
    if k < 0:
        raise TopsimpError(k, "ts_launch_choices failed")
    return {keys[i].decode(): ch[i] for i in range(k)}


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
    persistence_s: float
    assign_s: float
    update_s: float
    n_regradient: int
    init_used: int
    status: int
    trace: object = None  # (iterations + 1, 4): wall s, loss, max non-signal persistence, assign s


def _signal(threshold, nonsignal_dims, ties_signal, signal_pairs):
    """ts_signal of the threshold rule, or of an explicit list; returns
    (struct, list array kept alive)."""
    sig = _Signal()
    sp = None
    if signal_pairs is not None:
        sp = np.ascontiguousarray(signal_pairs, dtype=PAIR_DTYPE)
        sig.mode, sig.signal, sig.n_signal = 1, sp.ctypes.data, len(sp)
    else:
        sig.mode = 0
        sig.threshold_rel = threshold
        sig.nonsignal_dim_mask = sum(1 << d for d in nonsignal_dims)
        sig.ties_signal = ties_signal
    return sig, sp


def signal_mask(field, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0,
                signal_pairs=None):
    """Signal-vertex mask of D(field) under the solver's signal rule (Sec. 3):
    1.0 at the birth and death vertices of the signal pairs, 0.0 elsewhere;
    same kind and shape as the field.  Returns (mask, number of signal pairs)."""
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    sig, _sp = _signal(threshold, nonsignal_dims, ties_signal, signal_pairs)
    if on_dev:
        m = _torch().empty_like(keep)
        mp = ctypes.c_void_p(m.data_ptr())
    else:
        m = np.empty_like(keep)
        mp = _ptr(m)
    cnt = ctypes.c_int64(0)
    _check(ctx, lib().ts_signal_mask(ctx, fp, _ptr(dims), ctypes.byref(sig), on_dev, mp,
                                     ctypes.byref(cnt)))
    return m, int(cnt.value)


def simplify(field, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0, alpha_b=0.5,
             alpha_d=0.5, j_max=1000, stop_mode=0, cancel_tol_rel=1e-6, loss_ratio_s=0.01,
             signal_pairs=None, out=None, assign_precision=0.0, full_gradient=False, init=None,
             trace=False):
    """Topological simplification; returns (g, Report).  g has the kind of
    the input (torch CUDA tensor in, torch CUDA tensor out).  init: optional
    start field of the same kind and shape (used unless its loss is higher)."""
    ctx = context()
    fp, dims, on_dev, keep = _as_field(field)
    sig, _sp = _signal(threshold, nonsignal_dims, ties_signal, signal_pairs)
    opt = _Options(alpha_b, alpha_d, j_max, stop_mode, cancel_tol_rel, loss_ratio_s, on_dev,
                   assign_precision, int(bool(full_gradient)))
    init_keep = None
    if init is not None:
        ip, idims, ion, init_keep = _as_field(init)
        if ion != on_dev or not np.array_equal(idims, dims):
            raise ValueError("init must match the field's kind and shape")
        opt.init = ip
    tr = None
    if trace:
        tr = np.zeros((j_max + 1, 4), np.float64)
        opt.trace, opt.trace_cap = tr.ctypes.data, j_max + 1
    rep = _Report()
    torch = _torch()
    if on_dev:
        g = out if out is not None else torch.empty_like(keep)
        gp = ctypes.c_void_p(g.data_ptr())
    else:
        g = np.empty_like(keep)
        gp = _ptr(g)
    rc = lib().ts_simplify(ctx, fp, _ptr(dims), ctypes.byref(sig), ctypes.byref(opt), gp,
                           ctypes.byref(rep))
    _check(ctx, rc, allow=(0, 1))
    r = _report(rep, rc)
    if tr is not None:
        r.trace = tr[: rep.iterations + 1].copy()
    return g, r


def _report(rep, rc):
    return Report(rep.iterations, rep.cancelled, rep.loss0, rep.loss, rep.energy, rep.linf,
                  rep.l2, rep.max_nonsignal_pers, rep.max_signal_disp, rep.range,
                  tuple(rep.n_pairs), rep.n_still, rep.n_reduced, rep.n_targets, rep.total_s,
                  rep.persistence_s, rep.assign_s, rep.update_s, rep.n_regradient,
                  rep.init_used, rc)


def simplify_batch(fields, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0, alpha_b=0.5,
                   alpha_d=0.5, j_max=1000, stop_mode=0, cancel_tol_rel=1e-6, loss_ratio_s=0.01,
                   assign_precision=0.0, full_gradient=False):
    """simplify() on a list of fields of any sizes, solved together (the
    persistence maps of all fields run as one batch); returns (list of g,
    list of Report).  Each field's result is that of simplify() on it alone;
    report times are those of the whole batch."""
    ctx = context()
    ptrs, dims, on_dev, parts = _batch_args(fields)
    nf = len(fields)
    sig = _Signal()
    sig.mode = 0
    sig.threshold_rel = threshold
    sig.nonsignal_dim_mask = sum(1 << d for d in nonsignal_dims)
    sig.ties_signal = ties_signal
    opt = _Options(alpha_b, alpha_d, j_max, stop_mode, cancel_tol_rel, loss_ratio_s, on_dev,
                   assign_precision, int(bool(full_gradient)))
    reps = (_Report * nf)()
    torch = _torch()
    gs = [torch.empty_like(p[3]) if on_dev else np.empty_like(p[3]) for p in parts]
    gptrs = (ctypes.c_void_p * nf)(*[ctypes.c_void_p(g.data_ptr()) if on_dev else _ptr(g)
                                     for g in gs])
    rc = lib().ts_simplify_batch(ctx, nf, ptrs, _ptr(dims), ctypes.byref(sig), ctypes.byref(opt),
                                 gptrs, reps)
    _check(ctx, rc, allow=(0, 1))
    return gs, [_report(r, 1 - r.cancelled) for r in reps]


# ---- the warm-start network (device tensors only) ----

def _dev(t, shape=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def unet_param_count() -> int:
    n = np.zeros(1, np.int64)
    _check(None, lib().ts_unet_param_count(_ptr(n)))
    return int(n[0])


def _unet_dims(inp):
    if inp.dim() != 4 or inp.shape[3] != 2:
        raise ValueError("input must be (Lz, Ly, Lx, 2)")
    return np.array([inp.shape[2], inp.shape[1], inp.shape[0]], np.int64)


def unet_forward(params, inp):
    """Network output (Lz, Ly, Lx) for input (Lz, Ly, Lx, 2)."""
    torch = _torch()
    dims = _unet_dims(inp)
    out = torch.empty(inp.shape[:3], dtype=torch.float32, device=inp.device)
    ctx = context()
    _check(ctx, lib().ts_unet_forward(ctx, _dev(params), _dev(inp), _ptr(dims), _dev(out)))
    return out


def unet_grad(params, inp, target):
    """(mean squared error, gradient w.r.t. params) of the network on one volume."""
    torch = _torch()
    dims = _unet_dims(inp)
    grad = torch.empty_like(params)
    loss = ctypes.c_double(0.0)
    ctx = context()
    _check(ctx, lib().ts_unet_backward(ctx, _dev(params), _dev(inp), _dev(target), _ptr(dims),
                                       _dev(grad), ctypes.byref(loss)))
    return loss.value, grad


def unet_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    ctx = context()
    _check(ctx, lib().ts_unet_adam(ctx, _dev(params), _dev(grad), _dev(m), _dev(v), params.numel(),
                                   step, lr, beta1, beta2, eps))
