"""Pins of the warm-start network's CPU reference (oracle/unet_ref.py)."""
import numpy as np
import torch

from oracle import unet_ref


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in unet_ref.LAYERS:
        parts.append(rng.normal(0, scale * np.sqrt(2.0 / (27 * ci)), 27 * co * ci))
        parts.append(rng.normal(0, 0.05, co))
    parts.append(rng.normal(0, 0.25, 16))
    parts.append(rng.normal(0, 0.05, 1))
    return np.concatenate(parts)


def test_param_count():
    assert unet_ref.param_count() == _params(0).size == 356305


def test_conv_layout_brute_force():
    """The first convolution through the reference's unpacking equals the
    definition Y[v][co] = b[co] + sum_t sum_ci X[v + off_t][ci] W[t][co][ci]
    with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), written out as loops."""
    rng = np.random.default_rng(1)
    D, H, W = 3, 4, 5
    p = _params(2)
    convs, _, _ = unet_ref._unpack(torch.as_tensor(p))
    w, b = convs[0]
    X = rng.normal(size=(D, H, W, 8))
    Y = torch.nn.functional.conv3d(torch.as_tensor(X).permute(3, 0, 1, 2)[None], w, b,
                                   padding=1)[0].permute(1, 2, 3, 0).numpy()
    Wf = p[:27 * 16 * 8].reshape(27, 16, 8)
    bias = p[27 * 16 * 8:27 * 16 * 8 + 16]
    for z, y, x in [(0, 0, 0), (1, 2, 3), (2, 3, 4), (1, 0, 4)]:
        want = bias.copy()
        for t in range(27):
            dx, dy, dz = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
            if 0 <= x + dx < W and 0 <= y + dy < H and 0 <= z + dz < D:
                want += Wf[t] @ X[z + dz, y + dy, x + dx]
        assert np.allclose(Y[z, y, x], want, rtol=1e-12, atol=1e-12)


def test_gradients_against_finite_differences():
    """FP64 reference without rounding: the input gradient by gradcheck and
    the parameter gradient along random directions by central differences."""
    torch.manual_seed(0)
    p = torch.as_tensor(_params(3), dtype=torch.float64)
    x = torch.rand(4, 4, 4, 2, dtype=torch.float64, requires_grad=True)
    t = torch.rand(4, 4, 4, dtype=torch.float64)
    assert torch.autograd.gradcheck(
        lambda xx: ((unet_ref.forward(p, xx, bf16=False) - t) ** 2).mean(), (x,), eps=1e-6,
        atol=1e-7)
    loss, g = unet_ref.loss_and_grad(p.numpy(), x.detach().numpy(), t.numpy(), bf16=False)
    rng = np.random.default_rng(4)
    for _ in range(3):
        d = rng.normal(size=p.numel())
        d /= np.linalg.norm(d)
        h = 1e-6

        def f(q):
            return float(((unet_ref.forward(torch.as_tensor(q), x.detach(), bf16=False) - t) ** 2)
                         .mean())
        fd = (f(p.numpy() + h * d) - f(p.numpy() - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(1e-3, abs(fd))


def test_pool_and_up_shapes():
    """A constant input gives a constant pooled value; output has the input's
    spatial shape."""
    p = torch.as_tensor(_params(5), dtype=torch.float64)
    x = torch.full((8, 4, 12, 2), 0.5, dtype=torch.float64)
    out = unet_ref.forward(p, x)
    assert out.shape == (8, 4, 12)
    assert torch.isfinite(out).all()
