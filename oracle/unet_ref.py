"""CPU reference of the warm-start network (plain PyTorch on the CPU, FP64).

TEST INFRASTRUCTURE ONLY: the test suite is its only user; the product path
never imports it.  The network is not part of the paper (it proposes a start
point g0 for the exact solver); this module is written from its definition:

- input (Lz, Ly, Lx, 2): normalised field and signal-vertex mask, padded with
  zero channels to 8;
- ten 3x3x3 convolutions (zero padding) with ReLU:
  8->16, 16->16 | pool | 16->32, 32->32 | pool | 32->64, 64->64 | up, concat
  with the 32-channel skip | 96->32, 32->32 | up, concat with the 16-channel
  skip | 48->16, 16->16; pooling is the 2x2x2 mean, upsampling is nearest;
- a 1x1x1 head 16->1.

Parameters are one flat vector: per convolution weights [27][Cout][Cin] (tap
t = (dz+1)*9 + (dy+1)*3 + (dx+1)) then Cout biases; then 16 head weights and
its bias.

With bf16=True, the values the device path stores in BF16 are rounded to
BF16 at the same places (the convolution weights, the packed input, every
activation after its ReLU and every pooled tensor); the rounding passes
gradients straight through.  Everything else is FP64.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

LAYERS = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
          (48, 16), (16, 16)]


def param_count() -> int:
    return sum(27 * ci * co + co for ci, co in LAYERS) + 17


def _round(x, on):
    if not on:
        return x
    return x + (x.to(torch.bfloat16).to(x.dtype) - x).detach()


def _unpack(p):
    """[(W (Cout, Cin, 3, 3, 3), b)] * 10, head weights (16,), head bias."""
    out, o = [], 0
    for ci, co in LAYERS:
        w = p[o:o + 27 * co * ci].reshape(27, co, ci).permute(1, 2, 0).reshape(co, ci, 3, 3, 3)
        o += 27 * co * ci
        out.append((w, p[o:o + co]))
        o += co
    return out, p[o:o + 16], p[o + 16]


def forward(params, inp, bf16=True):
    """Network output (Lz, Ly, Lx).  params: flat tensor (FP64, may require
    grad); inp: (Lz, Ly, Lx, 2) tensor."""
    convs, hw, hb = _unpack(params)
    x = inp.permute(3, 0, 1, 2).unsqueeze(0)  # (1, 2, D, H, W)
    x = torch.cat([x, torch.zeros((1, 6) + x.shape[2:], dtype=x.dtype)], dim=1)
    x = _round(x, bf16)

    def conv(i, t):
        w, b = convs[i]
        return _round(F.relu(F.conv3d(t, _round(w, bf16), b, padding=1)), bf16)

    def pool(t):
        return _round(F.avg_pool3d(t, 2), bf16)

    def up(t):
        return t.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3).repeat_interleave(2, dim=4)

    a1 = conv(1, conv(0, x))
    a3 = conv(3, conv(2, pool(a1)))
    a5 = conv(5, conv(4, pool(a3)))
    a7 = conv(7, conv(6, torch.cat([up(a5), a3], dim=1)))
    a9 = conv(9, conv(8, torch.cat([up(a7), a1], dim=1)))
    return (a9[0] * hw.reshape(16, 1, 1, 1)).sum(dim=0) + hb


def loss_and_grad(params, inp, target, bf16=True):
    """(mean squared error, its gradient with respect to params), FP64."""
    p = torch.as_tensor(np.asarray(params), dtype=torch.float64).clone().requires_grad_(True)
    x = torch.as_tensor(np.asarray(inp), dtype=torch.float64)
    t = torch.as_tensor(np.asarray(target), dtype=torch.float64)
    loss = ((forward(p, x, bf16) - t) ** 2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy()
