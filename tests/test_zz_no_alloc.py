"""The allocation-free vertex order (ts_order_noalloc) against ts_order.

ts_order_noalloc keeps its temporaries in a static device array instead of
allocating; it must give ts_order's order and rank bit for bit, call after
call (the second call smaller than the first, so that stale contents of the
shared array would show), reject sizes beyond its array and non-finite
input, and keep working after an error."""
import ctypes

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


def _noalloc(ts, f):
    import torch
    n = f.numel()
    order = torch.empty(n, dtype=torch.int32, device=f.device)
    rank = torch.empty(n, dtype=torch.int32, device=f.device)
    stream = torch.cuda.current_stream().cuda_stream
    rc = ts.lib().ts_order_noalloc(ctypes.c_void_p(f.data_ptr()), n,
                                   ctypes.c_void_p(order.data_ptr()),
                                   ctypes.c_void_p(rank.data_ptr()), ctypes.c_void_p(stream))
    return rc, order, rank


def _field(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    f = rng.integers(-50, 50, size=n).astype(np.float32) * np.float32(0.25)
    f[rng.random(n) < 0.05] = -0.0  # ties and signed zeros
    return torch.from_numpy(f.reshape(1, 1, n)).cuda()


def test_noalloc_order_matches_ts_order(gpu):
    import torch
    for n, seed in [(1 << 21, 0), (100_003, 1), (1, 2), (4097, 3)]:
        f = _field(n, seed)
        rc, order, rank = _noalloc(gpu, f)
        torch.cuda.synchronize()
        assert rc == 0, (n, rc)
        o, r = gpu.order(f)
        assert torch.equal(order, o.ravel()), n
        assert torch.equal(rank, r.ravel()), n


def test_noalloc_order_errors(gpu):
    import torch
    rc, _, _ = _noalloc(gpu, torch.zeros((1, 1, (1 << 21) + 1), device="cuda"))
    assert rc == -1
    bad = _field(5000, 4)
    bad[0, 0, 17] = float("nan")
    rc, _, _ = _noalloc(gpu, bad)
    assert rc == -2
    # the flag is cleared by the next call
    f = _field(3000, 5)
    rc, order, rank = _noalloc(gpu, f)
    torch.cuda.synchronize()
    o, r = gpu.order(f)
    assert rc == 0 and torch.equal(order, o.ravel()) and torch.equal(rank, r.ravel())
