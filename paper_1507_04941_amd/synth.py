"""Seeded synthetic spectral cubes: N(0,1) noise plus 3-D Gaussian sources.

Stands in for the simulated survey cube the paper measures on (§4), which is
not available here.  This module only makes inputs: it contains none of the
source finder's arithmetic (no filter taps, window sums or thresholds), so
both the GPU path and the CPU oracle can be fed from it.

Recipe (numpy ``Generator(PCG64(seed))``, all in FP64, cast once to FP32 with
round-to-nearest):
  1. noise: ``standard_normal((nx, ny, nz))``, sigma 1;
  2. for each source, in order, draw x0, y0, z0 ~ U[0, n) (continuous),
     amplitude A ~ U[2, 6] (peak in noise sigma), s_xy ~ U[1, 3] pixels,
     s_z ~ U[2, 8] channels, and add
     A * exp(-((x-x0)^2 + (y-y0)^2) / (2 s_xy^2) - (z-z0)^2 / (2 s_z^2))
     to the voxels within +-ceil(4 s) of floor(centre) on each axis,
     clipped at the cube faces.
Layout: (nx, ny, nz) C-order, x slowest, z (spectral) contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One input configuration: cube shape, sources, filter bank, box, k."""
    name: str
    shape: tuple[int, int, int]
    n_sources: int
    seed: int
    filters: tuple[tuple[float, float], ...]
    box: tuple[int, int, int]
    k: float = 4.0
    truncate: float = 3.0
    meta: dict = field(default_factory=dict)

    @property
    def voxels(self) -> int:
        return int(self.shape[0]) * int(self.shape[1]) * int(self.shape[2])


# The 64x64x128 parity cube: 20 sources, filters (1,1), (2,2), (2,4),
# 32^3 statistics boxes, threshold mean + 4 std.
SMALL = Workload(
    name="cube64x64x128_f3_box32",
    shape=(64, 64, 128),
    n_sources=20,
    seed=1,
    filters=((1.0, 1.0), (2.0, 2.0), (2.0, 4.0)),
    box=(32, 32, 32),
)

# The 512x512x1024 (1 GiB FP32) cube: 2000 sources, sigma_xy in {1,2,4} x
# sigma_z in {2,8}, 64^3 statistics boxes, threshold mean + 4 std.
LARGE = Workload(
    name="cube512x512x1024_f6_box64",
    shape=(512, 512, 1024),
    n_sources=2000,
    seed=2,
    filters=((1.0, 2.0), (1.0, 8.0), (2.0, 2.0), (2.0, 8.0), (4.0, 2.0), (4.0, 8.0)),
    box=(64, 64, 64),
)

WORKLOADS = {w.name: w for w in (SMALL, LARGE)}


def _add_source(cube: np.ndarray, x0: float, y0: float, z0: float, amp: float,
                s_xy: float, s_z: float) -> None:
    nx, ny, nz = cube.shape
    hxy = int(math.ceil(4.0 * s_xy))
    hz = int(math.ceil(4.0 * s_z))
    cx, cy, cz = int(math.floor(x0)), int(math.floor(y0)), int(math.floor(z0))
    xs = np.arange(max(cx - hxy, 0), min(cx + hxy + 1, nx))
    ys = np.arange(max(cy - hxy, 0), min(cy + hxy + 1, ny))
    zs = np.arange(max(cz - hz, 0), min(cz + hz + 1, nz))
    if xs.size == 0 or ys.size == 0 or zs.size == 0:
        return
    ex = np.exp(-((xs - x0) ** 2) / (2.0 * s_xy * s_xy))
    ey = np.exp(-((ys - y0) ** 2) / (2.0 * s_xy * s_xy))
    ez = np.exp(-((zs - z0) ** 2) / (2.0 * s_z * s_z))
    blob = amp * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
    cube[xs[0]:xs[-1] + 1, ys[0]:ys[-1] + 1, zs[0]:zs[-1] + 1] += blob


def make_cube(shape, n_sources: int, seed: int, return_sources: bool = False):
    """Noise-plus-sources cube, FP32, (nx, ny, nz), following the recipe above."""
    nx, ny, nz = (int(s) for s in shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    cube = rng.standard_normal((nx, ny, nz))
    sources = []
    for _ in range(int(n_sources)):
        x0 = rng.uniform(0.0, nx)
        y0 = rng.uniform(0.0, ny)
        z0 = rng.uniform(0.0, nz)
        amp = rng.uniform(2.0, 6.0)
        s_xy = rng.uniform(1.0, 3.0)
        s_z = rng.uniform(2.0, 8.0)
        _add_source(cube, x0, y0, z0, amp, s_xy, s_z)
        sources.append((x0, y0, z0, amp, s_xy, s_z))
    out = cube.astype(np.float32)
    del cube
    if return_sources:
        return out, sources
    return out


def make_noise(shape, seed: int, scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """Plain N(offset, scale^2) FP32 cube (used for odd-shape and statistics cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (offset + scale * rng.standard_normal(tuple(int(s) for s in shape))).astype(np.float32)


def workload_cube(w: Workload) -> np.ndarray:
    return make_cube(w.shape, w.n_sources, w.seed)
