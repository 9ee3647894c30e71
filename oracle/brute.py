"""Brute-force numpy versions of the oracle steps, for tiny cubes only.

TEST INFRASTRUCTURE ONLY.  Pure loops over voxels written straight from the
definitions, so the C oracle can be checked against something that shares
none of its code:
  - Eq. 2 (§2.1): the triple sum over the 3-D filter support, zero outside;
  - §3.3: per-voxel mean and population standard deviation over a clipped
    box window, in two passes (mean first, then squared deviations).
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_taps(sigma: float, truncate: float = 3.0) -> np.ndarray:
    r = int(math.ceil(truncate * sigma))
    g = np.array([math.exp(-(o * o) / (2.0 * sigma * sigma)) for o in range(-r, r + 1)])
    return g / g.sum()


def conv3d(d: np.ndarray, sigma_xy: float, sigma_z: float, truncate: float = 3.0) -> np.ndarray:
    """Eq. 2 with f = gxy (x) gxy (x) gz, built as an explicit 3-D array."""
    d = np.asarray(d, dtype=np.float64)
    gxy = gaussian_taps(sigma_xy, truncate)
    gz = gaussian_taps(sigma_z, truncate)
    rxy, rz = len(gxy) // 2, len(gz) // 2
    f = gxy[:, None, None] * gxy[None, :, None] * gz[None, None, :]
    nx, ny, nz = d.shape
    pad = np.zeros((nx + 2 * rxy, ny + 2 * rxy, nz + 2 * rz))
    pad[rxy:rxy + nx, rxy:rxy + ny, rz:rz + nz] = d
    out = np.empty(d.shape)
    for x in range(nx):
        for y in range(ny):
            for z in range(nz):
                blk = pad[x:x + 2 * rxy + 1, y:y + 2 * rxy + 1, z:z + 2 * rz + 1]
                out[x, y, z] = float(np.sum(blk * f))
    return out


def conv3d_weighted(d: np.ndarray, w: np.ndarray, sigma_xy: float, sigma_z: float,
                    truncate: float = 3.0) -> np.ndarray:
    """Eq. 1 read as sum(d w f) / sum(w f) over the explicit 3-D support, 0
    where the denominator is 0."""
    d = np.asarray(d, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    gxy = gaussian_taps(sigma_xy, truncate)
    gz = gaussian_taps(sigma_z, truncate)
    rxy, rz = len(gxy) // 2, len(gz) // 2
    f = gxy[:, None, None] * gxy[None, :, None] * gz[None, None, :]
    nx, ny, nz = d.shape
    out = np.zeros(d.shape)
    for x in range(nx):
        for y in range(ny):
            for z in range(nz):
                num = den = 0.0
                for ox in range(-rxy, rxy + 1):
                    for oy in range(-rxy, rxy + 1):
                        for oz in range(-rz, rz + 1):
                            ix, iy, iz = x + ox, y + oy, z + oz
                            if 0 <= ix < nx and 0 <= iy < ny and 0 <= iz < nz:
                                fw = f[ox + rxy, oy + rxy, oz + rz] * w[ix, iy, iz]
                                num += d[ix, iy, iz] * fw
                                den += fw
                out[x, y, z] = num / den if den != 0.0 else 0.0
    return out


def window_bounds(i: int, n: int, B: int) -> tuple[int, int]:
    lo = i - B // 2
    return max(lo, 0), min(lo + B, n)


def local_stats(F: np.ndarray, box) -> tuple[np.ndarray, np.ndarray]:
    """Two-pass windowed mean / population std at every voxel."""
    F = np.asarray(F, dtype=np.float64)
    bx, by, bz = box
    nx, ny, nz = F.shape
    mean = np.empty(F.shape)
    std = np.empty(F.shape)
    for x in range(nx):
        x0, x1 = window_bounds(x, nx, bx)
        for y in range(ny):
            y0, y1 = window_bounds(y, ny, by)
            for z in range(nz):
                z0, z1 = window_bounds(z, nz, bz)
                w = F[x0:x1, y0:y1, z0:z1]
                mu = float(w.sum()) / w.size
                mean[x, y, z] = mu
                std[x, y, z] = math.sqrt(float(((w - mu) ** 2).sum()) / w.size)
    return mean, std
