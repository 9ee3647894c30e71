"""FP64 CPU oracle for the Gaussian source-finder hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product library never imports, links or calls
anything here, and this package imports nothing from the product.

The arithmetic lives in ``oracle_gsf.c`` (plain C, FP64, OpenMP over outer
loops); this module loads it with ctypes.  ``brute`` holds numpy triple-loop
versions for tiny cubes.  Each function cites the passage of the paper it
follows (Westerlund & Harris, Eq. 2 of §2.1 for the filter, §3.3 for the
local statistics, §1/§3.3 for the thresholds).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_gsf.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_gsf.so")
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_ptr = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (no GPU code involved)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_radius.restype = ctypes.c_int
    lib.oracle_radius.argtypes = [_dbl, _dbl]
    lib.oracle_taps.restype = ctypes.c_int
    lib.oracle_taps.argtypes = [_dbl, _dbl, _ptr, ctypes.c_int]
    for name in ("oracle_filter3d", "oracle_filter3d_direct"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [_ptr, _i64, _i64, _i64, _dbl, _dbl, _dbl, _ptr]
    lib.oracle_filter3d_weighted.restype = ctypes.c_int
    lib.oracle_filter3d_weighted.argtypes = [_ptr, _ptr, _i64, _i64, _i64, _dbl, _dbl, _dbl, _ptr]
    lib.oracle_filter3d_direct_at.restype = ctypes.c_int
    lib.oracle_filter3d_direct_at.argtypes = [_ptr, _i64, _i64, _i64, _dbl, _dbl, _dbl,
                                              _ptr, _i64, _ptr]
    lib.oracle_cube_mean.restype = _dbl
    lib.oracle_cube_mean.argtypes = [_ptr, _i64, _i64, _i64]
    lib.oracle_local_stats.restype = ctypes.c_int
    lib.oracle_local_stats.argtypes = [_ptr, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _ptr, _ptr]
    lib.oracle_local_stats_at.restype = ctypes.c_int
    lib.oracle_local_stats_at.argtypes = [_ptr, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, _ptr, _i64, _ptr, _ptr]
    lib.oracle_threshold.restype = None
    lib.oracle_threshold.argtypes = [_ptr, _ptr, _ptr, _i64, _dbl, _ptr]
    lib.oracle_threshold_f32.restype = None
    lib.oracle_threshold_f32.argtypes = [_ptr, _ptr, _ptr, _i64, _dbl, _ptr]
    lib.oracle_find.restype = ctypes.c_int
    lib.oracle_find.argtypes = [_ptr, _i64, _i64, _i64, _ptr, _ptr, _ptr, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, _dbl,
                                _ptr, _ptr, _ptr, _ptr]
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_get_threads.argtypes = []
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float32)
    if d.ndim != 3:
        raise ValueError("cube must be 3-D (nx, ny, nz)")
    return d


def _f64(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("cube must be 3-D (nx, ny, nz)")
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def radius(sigma: float, truncate: float = 3.0) -> int:
    """r = ceil(truncate * sigma) (truncation of the Gaussian filters, §2.1)."""
    return int(_load().oracle_radius(float(sigma), float(truncate)))


def taps(sigma: float, truncate: float = 3.0) -> np.ndarray:
    """Sampled unit-sum Gaussian taps for offsets -r..r (filter bank, §1/§2.1)."""
    g = np.zeros(1025, dtype=np.float64)
    r = _load().oracle_taps(float(sigma), float(truncate), _p(g), 1025)
    if r < 0:
        raise ValueError("invalid sigma/truncate")
    return g[: 2 * r + 1].copy()


def filter3d(d, sigma_xy: float, sigma_z: float, truncate: float = 3.0) -> np.ndarray:
    """Eq. 2 (§2.1) as z, y and x passes in FP64, zero outside the cube."""
    d = _f32(d)
    F = np.empty(d.shape, dtype=np.float64)
    rc = _load().oracle_filter3d(_p(d), *d.shape, float(sigma_xy), float(sigma_z),
                                 float(truncate), _p(F))
    if rc:
        raise RuntimeError(f"oracle_filter3d failed ({rc})")
    return F


def filter3d_weighted(d, w, sigma_xy: float, sigma_z: float, truncate: float = 3.0) -> np.ndarray:
    """Eq. 1 (§2.1), the weighted convolution, read as sum(d w f) / sum(w f)
    over the support (zero outside the cube); 0 where the denominator is 0."""
    d = _f32(d)
    w = _f32(w)
    if w.shape != d.shape:
        raise ValueError("weights must have the cube's shape")
    F = np.empty(d.shape, dtype=np.float64)
    if _load().oracle_filter3d_weighted(_p(d), _p(w), *d.shape, float(sigma_xy), float(sigma_z),
                                        float(truncate), _p(F)):
        raise RuntimeError("oracle_filter3d_weighted failed")
    return F


def filter3d_direct(d, sigma_xy: float, sigma_z: float, truncate: float = 3.0) -> np.ndarray:
    """Eq. 2 (§2.1) as the direct triple sum at every voxel (small cubes)."""
    d = _f32(d)
    F = np.empty(d.shape, dtype=np.float64)
    rc = _load().oracle_filter3d_direct(_p(d), *d.shape, float(sigma_xy), float(sigma_z),
                                        float(truncate), _p(F))
    if rc:
        raise RuntimeError(f"oracle_filter3d_direct failed ({rc})")
    return F


def filter3d_direct_at(d, sigma_xy: float, sigma_z: float, idx, truncate: float = 3.0) -> np.ndarray:
    """Eq. 2 (§2.1) as the direct triple sum at the given linear voxel indices."""
    d = _f32(d)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.shape, dtype=np.float64)
    rc = _load().oracle_filter3d_direct_at(_p(d), *d.shape, float(sigma_xy), float(sigma_z),
                                           float(truncate), _p(idx), idx.size, _p(out))
    if rc:
        raise RuntimeError(f"oracle_filter3d_direct_at failed ({rc})")
    return out


def cube_mean(F) -> float:
    F = _f64(F)
    return float(_load().oracle_cube_mean(_p(F), *F.shape))


def local_stats(F, box) -> tuple[np.ndarray, np.ndarray]:
    """Local mean and population std over the clipped box window (§3.3),
    as three directional sums.  box = (bx, by, bz) window lengths."""
    F = _f64(F)
    bx, by, bz = (int(b) for b in box)
    mean = np.empty(F.shape, dtype=np.float64)
    std = np.empty(F.shape, dtype=np.float64)
    rc = _load().oracle_local_stats(_p(F), *F.shape, bx, by, bz, _p(mean), _p(std))
    if rc:
        raise RuntimeError(f"oracle_local_stats failed ({rc})")
    return mean, std


def local_stats_at(F, box, idx) -> tuple[np.ndarray, np.ndarray]:
    """The plain two-pass window mean/std (§3.3) at the given linear indices."""
    F = _f64(F)
    bx, by, bz = (int(b) for b in box)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    mean = np.empty(idx.shape, dtype=np.float64)
    std = np.empty(idx.shape, dtype=np.float64)
    rc = _load().oracle_local_stats_at(_p(F), *F.shape, bx, by, bz, _p(idx), idx.size,
                                       _p(mean), _p(std))
    if rc:
        raise RuntimeError(f"oracle_local_stats_at failed ({rc})")
    return mean, std


def threshold(F, mean, std, k: float) -> np.ndarray:
    """Selection F > mean + k*std in FP64 (§1, §3.3).  Returns uint8 0/1."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    mean = np.ascontiguousarray(mean, dtype=np.float64)
    std = np.ascontiguousarray(std, dtype=np.float64)
    if not (F.shape == mean.shape == std.shape):
        raise ValueError("shape mismatch")
    out = np.empty(F.shape, dtype=np.uint8)
    _load().oracle_threshold(_p(F), _p(mean), _p(std), F.size, float(k), _p(out))
    return out


def threshold_f32(F, mean, std, k: float) -> np.ndarray:
    """Selection on FP32 inputs promoted exactly to FP64 (same expression)."""
    F = np.ascontiguousarray(F, dtype=np.float32)
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    std = np.ascontiguousarray(std, dtype=np.float32)
    if not (F.shape == mean.shape == std.shape):
        raise ValueError("shape mismatch")
    out = np.empty(F.shape, dtype=np.uint8)
    _load().oracle_threshold_f32(_p(F), _p(mean), _p(std), F.size, float(k), _p(out))
    return out


def find(d, filters, box, k: float, want_F: bool = False, want_stats: bool = False):
    """The whole path for one cube: for each (sigma_xy, sigma_z[, truncate])
    filter, Eq. 2, then local mean/std (§3.3), then F > mean + k*std.

    Returns dict with 'mask' (nfilt, nx, ny, nz) uint8 and optionally
    'F', 'mean', 'std' (nfilt, nx, ny, nz) float64."""
    d = _f32(d)
    nf = len(filters)
    sxy = np.array([float(f[0]) for f in filters], dtype=np.float64)
    sz = np.array([float(f[1]) for f in filters], dtype=np.float64)
    tr = np.array([float(f[2]) if len(f) > 2 else 3.0 for f in filters], dtype=np.float64)
    bx, by, bz = (int(b) for b in box)
    shape = (nf,) + d.shape
    masks = np.empty(shape, dtype=np.uint8)
    F = np.empty(shape, dtype=np.float64) if want_F else None
    mu = np.empty(shape, dtype=np.float64) if want_stats else None
    sd = np.empty(shape, dtype=np.float64) if want_stats else None
    null = ctypes.c_void_p(0)
    rc = _load().oracle_find(_p(d), *d.shape, _p(sxy), _p(sz), _p(tr), nf, bx, by, bz,
                             float(k), _p(masks), _p(F) if F is not None else null,
                             _p(mu) if mu is not None else null,
                             _p(sd) if sd is not None else null)
    if rc:
        raise RuntimeError(f"oracle_find failed ({rc})")
    out = {"mask": masks}
    if want_F:
        out["F"] = F
    if want_stats:
        out["mean"] = mu
        out["std"] = sd
    return out


def find_halo(d, halo, filters, box, k: float):
    """The whole path for a cube with an input-only border (the halo, per
    side along x, y, z): Eq. 2 over the whole array (zero outside it), the
    filtered core cut out, then local mean/std (§3.3) and the selection on
    that core as if it were the whole cube.  A plain composition of
    filter3d, local_stats and threshold.

    Returns dict with 'F', 'mean', 'std' (nfilt, core) float64 and 'mask'
    (nfilt, core) uint8."""
    d = _f32(d)
    hx, hy, hz = (int(h) for h in halo)
    core = (slice(hx, d.shape[0] - hx), slice(hy, d.shape[1] - hy), slice(hz, d.shape[2] - hz))
    out = {"F": [], "mean": [], "std": [], "mask": []}
    for f in filters:
        t = float(f[2]) if len(f) > 2 else 3.0
        F = np.ascontiguousarray(filter3d(d, float(f[0]), float(f[1]), t)[core])
        mu, sd = local_stats(F, box)
        out["F"].append(F)
        out["mean"].append(mu)
        out["std"].append(sd)
        out["mask"].append(threshold(F, mu, sd, k))
    return {key: np.stack(v) for key, v in out.items()}

