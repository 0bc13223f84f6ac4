"""Seeded synthetic scalar fields on 3D regular grids.

These generators stand in for the paper's 256^3 public volumes (vessels,
axons, cosmic-web filaments; Sec. 5), which are not available here.  They
hold none of the simplification method's arithmetic: they only draw random
numbers and evaluate closed-form bumps, in float64, and cast the result to
float32 once.  Both the GPU path and the CPU oracle receive the very same
array.

Conventions: an array has shape (Lz, Ly, Lx) (x fastest); the grid
coordinate of vertex (i, j, k) is (i/(Lx-1), j/(Ly-1), k/(Lz-1)); dims are
given as (Lx, Ly, Lz).  Draw order: geometry parameters first, then the
noise in linear-index order.
"""
from __future__ import annotations

import numpy as np

__all__ = ["gaussian_mixture", "filament_field", "workload", "WORKLOADS"]


def _axes(dims):
    lx, ly, lz = (int(d) for d in dims)
    return (np.arange(lx) / (lx - 1), np.arange(ly) / (ly - 1), np.arange(lz) / (lz - 1))


def gaussian_mixture(dims, n_gauss: int, noise_amp: float, seed: int) -> np.ndarray:
    """Sum of `n_gauss` isotropic Gaussians a*exp(-|p-c|^2/(2 s^2)) with
    c ~ U[0,1]^3, s ~ U[0.05, 0.15], a ~ U[0.5, 1], plus i.i.d. uniform noise
    in [-noise_amp, noise_amp].  Each Gaussian is evaluated as the product of
    its three 1D factors."""
    rng = np.random.default_rng(seed)
    lx, ly, lz = (int(d) for d in dims)
    centers = rng.uniform(0.0, 1.0, size=(n_gauss, 3))
    sigmas = rng.uniform(0.05, 0.15, size=n_gauss)
    amps = rng.uniform(0.5, 1.0, size=n_gauss)
    noise = rng.uniform(-noise_amp, noise_amp, size=lx * ly * lz)
    x, y, z = _axes(dims)
    f = np.zeros((lz, ly, lx), dtype=np.float64)
    for c, s, a in zip(centers, sigmas, amps):
        gx = np.exp(-((x - c[0]) ** 2) / (2 * s * s))
        gy = np.exp(-((y - c[1]) ** 2) / (2 * s * s))
        gz = np.exp(-((z - c[2]) ** 2) / (2 * s * s))
        f += a * (gz[:, None, None] * gy[None, :, None]) * gx[None, None, :]
    f += noise.reshape(lz, ly, lx)
    return f.astype(np.float32)


def filament_field(dims, seed: int, n_tubes: int = 32, n_points: int = 6,
                   noise_sigma: float = 0.02, s_range=(0.01, 0.03),
                   cutoff: float = 8.0) -> np.ndarray:
    """Sum of `n_tubes` random tubes plus Gaussian noise N(0, noise_sigma^2).
    A tube is a polyline through `n_points` points ~ U[0,1]^3 with value
    exp(-d^2/(2 s^2)), d the distance to the polyline and s ~ U[s_range];
    the bump is taken as exactly 0 beyond d > cutoff*s (exp(-32) ~ 1e-14)."""
    rng = np.random.default_rng(seed)
    lx, ly, lz = (int(d) for d in dims)
    pts = rng.uniform(0.0, 1.0, size=(n_tubes, n_points, 3))
    svals = rng.uniform(s_range[0], s_range[1], size=n_tubes)
    noise = rng.normal(0.0, noise_sigma, size=lx * ly * lz)
    x, y, z = _axes(dims)
    axes = (x, y, z)
    f = np.zeros((lz, ly, lx), dtype=np.float64)
    for t in range(n_tubes):
        s = float(svals[t])
        rad = cutoff * s
        lo = np.clip(pts[t].min(axis=0) - rad, 0.0, 1.0)
        hi = np.clip(pts[t].max(axis=0) + rad, 0.0, 1.0)
        sl = []
        for a in range(3):
            n_a = len(axes[a])
            i0 = int(np.floor(lo[a] * (n_a - 1)))
            i1 = int(np.ceil(hi[a] * (n_a - 1))) + 1
            sl.append(slice(max(i0, 0), min(i1, n_a)))
        bx, by, bz = x[sl[0]], y[sl[1]], z[sl[2]]
        d2 = np.full((len(bz), len(by), len(bx)), np.inf)
        for k in range(n_points - 1):
            p0, p1 = pts[t, k], pts[t, k + 1]
            seg = p1 - p0
            L2 = float(seg @ seg)
            # sub-box of this segment, in the tube box coordinates
            slo = np.minimum(p0, p1) - rad
            shi = np.maximum(p0, p1) + rad
            mx = (bx >= slo[0]) & (bx <= shi[0])
            my = (by >= slo[1]) & (by <= shi[1])
            mz = (bz >= slo[2]) & (bz <= shi[2])
            if not (mx.any() and my.any() and mz.any()):
                continue
            ix, iy, iz = np.nonzero(mx)[0], np.nonzero(my)[0], np.nonzero(mz)[0]
            sx = slice(ix[0], ix[-1] + 1)
            sy = slice(iy[0], iy[-1] + 1)
            sz = slice(iz[0], iz[-1] + 1)
            qx = bx[sx][None, None, :] - p0[0]
            qy = by[sy][None, :, None] - p0[1]
            qz = bz[sz][:, None, None] - p0[2]
            tt = (qx * seg[0] + qy * seg[1] + qz * seg[2]) / L2 if L2 > 0 else 0.0 * qx
            tt = np.clip(tt, 0.0, 1.0)
            dx = qx - tt * seg[0]
            dy = qy - tt * seg[1]
            dz = qz - tt * seg[2]
            dd = dx * dx + dy * dy + dz * dz
            np.minimum(d2[sz, sy, sx], dd, out=d2[sz, sy, sx])
        bump = np.where(d2 <= rad * rad, np.exp(-d2 / (2 * s * s)), 0.0)
        f[sl[2], sl[1], sl[0]] += bump
    f += noise.reshape(lz, ly, lx)
    return f.astype(np.float32)


# Named workloads: (generator, kwargs) with signal rules.  The signal rule is
# (threshold_rel, nonsignal_dim_mask, ties_signal).
WORKLOADS = {
    # 8 Gaussians + U[-0.05,0.05] noise; signal iff persistence > 0.1 range
    "gauss8_32": dict(kind="gauss", dims=(32, 32, 32), n_gauss=8, noise=0.05,
                      signal=(0.1, 0b111, 0)),
    # 64 Gaussians + U[-0.1,0.1] noise at 128^3
    "gauss64_128": dict(kind="gauss", dims=(128, 128, 128), n_gauss=64, noise=0.1,
                        signal=(0.1, 0b111, 0)),
    # 32 random tubes + N(0, 0.02^2) noise at 256^3; only saddle-saddle pairs
    # below 0.1 range are non-signal
    "filament_256": dict(kind="tube", dims=(256, 256, 256), signal=(0.1, 0b010, 1)),
}


def workload(name: str, seed: int = 0, dims=None) -> np.ndarray:
    """Field of a named workload (optionally at other dims)."""
    w = WORKLOADS[name]
    d = tuple(dims) if dims is not None else w["dims"]
    if w["kind"] == "gauss":
        return gaussian_mixture(d, w["n_gauss"], w["noise"], seed)
    return filament_field(d, seed)


def uneven_batch(n_fields: int = 64, lo: int = 24, hi: int = 96, seed: int = 0) -> list:
    """Batch of Gaussian-mixture fields (8 Gaussians, U[-0.05,0.05] noise) whose
    three axes are drawn independently and uniformly from lo..hi; field i has
    generator seed 1000 + i.  Signal rule as gauss8_32 (0.1 range, all dims)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        d = tuple(int(a) for a in rng.integers(lo, hi + 1, 3))
        out.append(gaussian_mixture(d, 8, 0.05, 1000 + i))
    return out
