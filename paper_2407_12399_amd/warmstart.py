"""The learned warm start: examples from the plain solver, training of the
3D U-Net with the library's own kernels (BF16 MFMA forward and backward,
Adam), and the warm-started solve.

The network sees (f normalised to [0, 1] by its range, signal-vertex mask)
and proposes (g - f) / range, where g is what the plain solver returns for f.
The exact solver then starts from g0 = f + range * proposal with the targets
of D(f); it falls back to f when g0's loss is higher, so the network changes
the iteration count, never what the solver accepts as a result.

Everything here runs on the GPU through the C ABI (device tensors).
"""
from __future__ import annotations

import time

import numpy as np

from . import (_torch, simplify, simplify_batch, unet_adam, unet_forward, unet_grad,
               unet_param_count)
from . import signal_mask as _signal_mask
from . import fields

# (input channels as stored, output channels) of the ten convolutions
LAYERS = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
          (48, 16), (16, 16)]
REAL_INPUTS = 2  # the first layer's channels 2..7 are zero padding


def init_params(seed: int = 0):
    """He-normal weights, zero biases; the head starts at zero (g0 = f)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    parts = []
    for i, (ci, co) in enumerate(LAYERS):
        fan = 27 * (REAL_INPUTS if i == 0 else ci)
        w = rng.normal(0.0, np.sqrt(2.0 / fan), (27, co, ci))
        if i == 0:
            w[:, :, REAL_INPUTS:] = 0.0
        parts += [w.ravel(), np.zeros(co)]
    parts += [np.zeros(17)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == unet_param_count()
    return torch.from_numpy(p).cuda()


def signal_mask(f, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0):
    """1 at the birth and death vertices of the signal pairs of D(f) (the
    solver's own signal rule, applied by the library), 0 elsewhere; same
    shape as f (device)."""
    m, _ = _signal_mask(f, threshold, nonsignal_dims, ties_signal)
    return m


def net_input(f, mask):
    """(input (Lz, Ly, Lx, 2), f.min(), range)."""
    torch = _torch()
    lo, hi = f.min(), f.max()
    rng = (hi - lo).clamp_min(1e-30)
    return torch.stack([(f - lo) / rng, mask], dim=-1).contiguous(), lo, rng


def proposal(params, f, mask):
    """g0 = f + range * network(f, mask)."""
    inp, _, rng = net_input(f, mask)
    return (f + rng * unet_forward(params, inp)).contiguous()


def make_examples(n, dims=(64, 64, 64), seed0=0, batch=64, log=None, **solver_kw):
    """n (input, target) pairs from the plain solver on config-1-style fields
    (8 Gaussians + U[-0.05, 0.05] noise) of the given dims, seeds seed0.. ;
    solved in batches.  Returns device tensors (n, Lz, Ly, Lx, 2), (n, Lz, Ly, Lx)."""
    torch = _torch()
    kw = dict(threshold=0.1)
    kw.update(solver_kw)
    ins, outs = [], []
    for b0 in range(0, n, batch):
        fs = [torch.from_numpy(fields.gaussian_mixture(dims, 8, 0.05, seed0 + i)).cuda()
              for i in range(b0, min(n, b0 + batch))]
        t0 = time.perf_counter()
        gs, reps = simplify_batch(fs, **kw)
        if log:
            log(f"examples {b0}..{b0 + len(fs)}: {time.perf_counter() - t0:.1f} s, "
                f"iterations {min(r.iterations for r in reps)}..{max(r.iterations for r in reps)}")
        for f, g in zip(fs, gs):
            m = signal_mask(f, kw["threshold"], kw.get("nonsignal_dims", (0, 1, 2)),
                            kw.get("ties_signal", 0))
            inp, _, rng = net_input(f, m)
            ins.append(inp)
            outs.append((g - f) / rng)
    return torch.stack(ins), torch.stack(outs)


def train(inputs, targets, steps, lr=1e-3, seed=0, params=None, log=None, log_every=100):
    """Adam on the mean squared error, one example per step in a seeded
    shuffled order.  Returns (params, list of (step, mean loss))."""
    torch = _torch()
    p = init_params(seed) if params is None else params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    order = np.random.default_rng(seed).permutation
    n = inputs.shape[0]
    perm = order(n)
    hist, acc = [], []
    for step in range(1, steps + 1):
        k = int(perm[(step - 1) % n])
        if (step - 1) % n == n - 1:
            perm = order(n)
        loss, g = unet_grad(p, inputs[k], targets[k])
        unet_adam(p, g, m, v, step, lr=lr)
        acc.append(loss)
        if step % log_every == 0 or step == steps:
            hist.append((step, float(np.mean(acc))))
            if log:
                log(f"step {step}: loss {hist[-1][1]:.3e}")
            acc = []
    return p, hist


def warm_solve(params, f, threshold=0.1, nonsignal_dims=(0, 1, 2), ties_signal=0, **solver_kw):
    """The exact solver started from the network's proposal (falls back to
    f when the proposal's loss is higher).  Returns (g, Report, seconds spent
    on the proposal)."""
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = signal_mask(f, threshold, nonsignal_dims, ties_signal)
    g0 = proposal(params, f, m)
    torch.cuda.synchronize()
    t_prop = time.perf_counter() - t0
    g, rep = simplify(f, threshold=threshold, nonsignal_dims=nonsignal_dims,
                      ties_signal=ties_signal, init=g0, **solver_kw)
    return g, rep, t_prop
