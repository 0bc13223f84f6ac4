"""The warm-start network on the GPU (BF16 MFMA convolutions, FP32
accumulation) against its CPU reference (FP64 with the same BF16 roundings)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_12399_amd as ts
    ts.lib()
    return ts


def _params(seed):
    from oracle import unet_ref
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in unet_ref.LAYERS:
        parts.append(rng.normal(0, np.sqrt(2.0 / (27 * ci)), 27 * co * ci))
        parts.append(rng.normal(0, 0.05, co))
    parts.append(rng.normal(0, 0.25, 16))
    parts.append(rng.normal(0, 0.05, 1))
    return np.concatenate(parts).astype(np.float32)


def _case(seed, dims):
    rng = np.random.default_rng(seed)
    D, H, W = dims
    inp = np.stack([rng.random((D, H, W)), (rng.random((D, H, W)) < 0.1)], -1).astype(np.float32)
    target = rng.normal(0, 0.1, (D, H, W)).astype(np.float32)
    return inp, target


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def _close(a, ref, rtol, atol_frac, what):
    """Element by element: |a - ref| <= rtol * |ref| + atol_frac * max |ref|.
    The device stores weights and activations in BF16 (8-bit significand,
    relative rounding 2^-9) at the same places as the reference; where an
    FP32 sum (device) and an FP64 sum (reference) fall on different sides of
    a BF16 rounding boundary, one value differs by a BF16 ulp (2^-8
    relative), and that difference travels through the later layers, so
    the bound has a relative part and a part scaled to the tensor."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    err = np.abs(a - ref)
    bound = rtol * np.abs(ref) + atol_frac * scale
    worst = int(np.argmax(err - bound)) if ref.size else 0
    assert np.all(err <= bound), (what, "worst", worst, float(a.ravel()[worst]),
                                  float(ref.ravel()[worst]), "max err / scale",
                                  float(err.max() / max(scale, 1e-300)))


@pytest.mark.parametrize("dims", [(8, 12, 16), (4, 4, 4), (12, 8, 20), (32, 32, 32), (64, 64, 64)])
def test_unet_forward_and_gradient(gpu, dims):
    """Forward output and every parameter gradient, element by element, against
    the FP64 reference with the same BF16 roundings; the first layer's
    weights are compared on its two real input channels (f, mask)."""
    import torch
    from oracle import unet_ref
    p = _params(7)
    inp, target = _case(8, dims)
    pt = torch.from_numpy(p).cuda()
    it = torch.from_numpy(inp).cuda()
    tt = torch.from_numpy(target).cuda()
    out = gpu.unet_forward(pt, it).cpu().numpy()
    ref = unet_ref.forward(torch.as_tensor(p, dtype=torch.float64),
                           torch.as_tensor(inp, dtype=torch.float64)).detach().numpy()
    assert out.shape == ref.shape
    assert _rel(out, ref) < 1e-2
    _close(out, ref, 2e-2, 1e-2, "output")
    loss, grad = gpu.unet_grad(pt, it, tt)
    lref, gref = unet_ref.loss_and_grad(p.astype(np.float64), inp, target)
    assert abs(loss - lref) <= 1e-2 * lref
    grad = grad.cpu().numpy()
    o = 0
    for i, (ci, co) in enumerate(unet_ref.LAYERS):
        n = 27 * ci * co
        w, wr = grad[o:o + n].reshape(27, co, ci), gref[o:o + n].reshape(27, co, ci)
        if i == 0:  # channels 2..7 of the first layer are zero padding
            w, wr = w[:, :, :2], wr[:, :, :2]
        assert _rel(w, wr) < 5e-2, ("weights", i)
        _close(w, wr, 1e-1, 3e-2, ("weights", i))
        b, br = grad[o + n:o + n + co], gref[o + n:o + n + co]
        assert _rel(b, br) < 5e-2, ("bias", i)
        _close(b, br, 1e-1, 3e-2, ("bias", i))
        o += n + co
    assert _rel(grad[o:], gref[o:]) < 2e-2
    _close(grad[o:], gref[o:], 5e-2, 1e-2, "head")


def test_unet_adam_step(gpu):
    import torch
    rng = np.random.default_rng(3)
    n = 1000
    p, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = rng.normal(size=n).astype(np.float32) * 0.1, rng.random(n).astype(np.float32) * 0.1
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    gpu.unet_adam(tp, tg, tm, tv, step=3, lr=1e-2)
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    want = p - 1e-2 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    assert np.allclose(tp.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
    assert np.allclose(tm.cpu().numpy(), m2, rtol=1e-6, atol=1e-7)


def test_simplify_start_field(gpu):
    """A start field with a higher loss is rejected and the solve is the cold
    one, bit for bit; the solver's own result as the start field is used and
    stops at once; either way the exact solver judges the result."""
    import torch
    from paper_2407_12399_amd import fields
    f = torch.from_numpy(fields.gaussian_mixture((20, 16, 12), 8, 0.05, 5)).cuda()
    kw = dict(threshold=0.1, stop_mode=1, loss_ratio_s=1e-3, j_max=300)
    gc, rc = gpu.simplify(f, **kw)
    noisy = (f + torch.randn(f.shape, generator=torch.Generator().manual_seed(0)).cuda()).contiguous()
    gn, rn = gpu.simplify(f, init=noisy, **kw)
    assert rn.init_used == 0 and rc.init_used == 0
    assert rn.iterations == rc.iterations and torch.equal(gn, gc)
    gi, ri = gpu.simplify(f, init=gc.contiguous(), **kw)
    assert ri.init_used == 1 and ri.cancelled == 1
    assert ri.iterations <= 2 < rc.iterations
    assert ri.loss0 == rc.loss0  # the loss stays relative to the targets of D(f)


def test_warm_start_pipeline(gpu):
    """Examples from the batched solver, a few Adam steps with the library's
    kernels (the training loss falls), and a warm-started solve that meets
    the stop rule."""
    import torch
    from paper_2407_12399_amd import fields, warmstart
    X, Y = warmstart.make_examples(8, dims=(16, 16, 16), seed0=100, stop_mode=1,
                                   loss_ratio_s=1e-3, j_max=200)
    assert X.shape == (8, 16, 16, 16, 2) and Y.shape == (8, 16, 16, 16)
    p, hist = warmstart.train(X, Y, 80, lr=2e-3, log_every=40)
    assert hist[-1][1] < hist[0][1]
    f = torch.from_numpy(fields.gaussian_mixture((16, 16, 16), 8, 0.05, 999)).cuda()
    g, r, _ = warmstart.warm_solve(p, f, stop_mode=1, loss_ratio_s=1e-3, j_max=300)
    assert r.cancelled == 1 and r.init_used in (0, 1)
