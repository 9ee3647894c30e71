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


@dataclass(frozen=True)
class BatchWorkload:
    """A batch of uneven sub-cubes, each a core plus an input-only halo.

    Core sizes: nx, ny ~ U{lo_xy..hi_xy}, nz ~ U{lo_z..hi_z} drawn in cube
    order from PCG64(size_seed); cube i is make_cube(core + 2*halo,
    round(V_core / 2^17) sources, seed cube_seed + i).  The halo (per side)
    is 3 x the largest sigma of the bank along each axis."""
    name: str
    n_cubes: int
    core_xy: tuple[int, int]
    core_z: tuple[int, int]
    halo: tuple[int, int, int]
    size_seed: int
    cube_seed: int
    filters: tuple[tuple[float, float], ...]
    box: tuple[int, int, int]
    k: float = 4.0


BATCH = BatchWorkload(
    name="batch96_core48-256x48-256x64-1024_halo12-12-24_f6_box64",
    n_cubes=96,
    core_xy=(48, 256),
    core_z=(64, 1024),
    halo=(12, 12, 24),
    size_seed=999,
    cube_seed=1000,
    filters=LARGE.filters,
    box=LARGE.box,
)


def batch_cores(b: BatchWorkload) -> list[tuple[int, int, int]]:
    rng = np.random.Generator(np.random.PCG64(b.size_seed))
    cores = []
    for _ in range(b.n_cubes):
        nx = int(rng.integers(b.core_xy[0], b.core_xy[1] + 1))
        ny = int(rng.integers(b.core_xy[0], b.core_xy[1] + 1))
        nz = int(rng.integers(b.core_z[0], b.core_z[1] + 1))
        cores.append((nx, ny, nz))
    return cores


def batch_cube(b: BatchWorkload, i: int) -> np.ndarray:
    """Sub-cube i of the batch: the full array (core plus halo), FP32."""
    core = batch_cores(b)[i]
    shape = tuple(c + 2 * h for c, h in zip(core, b.halo))
    n_src = int(round(core[0] * core[1] * core[2] / 2.0 ** 17))
    return make_cube(shape, n_src, b.cube_seed + i)


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
