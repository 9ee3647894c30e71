"""Tolerances and comparison helpers shared by the GPU parity tests.

Readings (stated once here, used by every test):
  - filtered values: |F_gpu - F_oracle| <= 1e-5 * max(|F_oracle|, sigma_f * scale),
    sigma_f = sqrt(sum f^2) the filtered-noise sigma for unit input noise and
    `scale` the RMS of the input cube (a pure relative bound fails at zero
    crossings of F);
  - local mean / std: |err| <= 1e-5 * max(std_oracle, sigma_f * scale), plus
    half an FP32 ulp of the mean for the mean (it is stored in FP32);
  - masks: bit-exact wherever |F_o - thr_o| exceeds the margin those
    tolerances could move a voxel across (eps_F + eps_mean + k * eps_std);
    voxels inside that band are counted and reported, not failed;
  - the selection of identical FP32 inputs: bit-exact, no band.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle

REL = 1e-5
FP32_HALF_ULP = 2.0 ** -24


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def sigma_f(filt) -> float:
    gxy = oracle.taps(filt[0], filt[2] if len(filt) > 2 else 3.0)
    gz = oracle.taps(filt[1], filt[2] if len(filt) > 2 else 3.0)
    return float(np.sqrt(np.sum(gxy ** 2) ** 2 * np.sum(gz ** 2)))


def cube_scale(d: np.ndarray) -> float:
    s = float(np.sqrt(np.mean(np.square(d, dtype=np.float64))))
    return s if s > 0 else 1.0


def check_filtered(Fg: np.ndarray, Fo: np.ndarray, filt, scale: float, what: str = "F") -> float:
    """Assert the filtered-value bound; return the worst error in units of the bound."""
    Fg = np.asarray(Fg, dtype=np.float64)
    bound = REL * np.maximum(np.abs(Fo), sigma_f(filt) * scale)
    ratio = np.abs(Fg - Fo) / bound
    worst = float(ratio.max()) if ratio.size else 0.0
    if worst > 1.0:
        i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        raise AssertionError(f"{what}: worst error {worst:.3g} x bound at {i}: gpu={Fg[i]!r} "
                             f"oracle={Fo[i]!r}")
    return worst


def check_stats(mg, sg, mo, so, floor: float, what: str = "stats") -> tuple[float, float]:
    mg = np.asarray(mg, dtype=np.float64)
    sg = np.asarray(sg, dtype=np.float64)
    bound = REL * np.maximum(so, floor)
    # the mean is stored in FP32: allow its half-ulp representation error too
    rm = np.abs(mg - mo) / (bound + FP32_HALF_ULP * np.abs(mo))
    rs = np.abs(sg - so) / bound
    wm = float(rm.max()) if rm.size else 0.0
    ws = float(rs.max()) if rs.size else 0.0
    if wm > 1.0:
        i = np.unravel_index(int(np.argmax(rm)), rm.shape)
        raise AssertionError(f"{what} mean: worst {wm:.3g} x bound at {i}: gpu={mg[i]!r} oracle={mo[i]!r}")
    if ws > 1.0:
        i = np.unravel_index(int(np.argmax(rs)), rs.shape)
        raise AssertionError(f"{what} std: worst {ws:.3g} x bound at {i}: gpu={sg[i]!r} oracle={so[i]!r}")
    return wm, ws


def check_mask(mask_g: np.ndarray, Fo, mo, so, k: float, filt, scale: float,
               what: str = "mask") -> int:
    """Masks equal outside the near-threshold band; returns the band count."""
    thr = mo + k * so
    eps_f = REL * np.maximum(np.abs(Fo), sigma_f(filt) * scale)
    eps_s = REL * np.maximum(so, sigma_f(filt) * scale)
    eps_m = eps_s + FP32_HALF_ULP * np.abs(mo)
    band = np.abs(Fo - thr) <= (eps_f + eps_m + k * eps_s)
    mask_o = Fo > thr
    bad = (mask_g != mask_o) & ~band
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {int(bad.sum())} voxels differ outside the band, first at "
                             f"{tuple(i)}")
    return int(band.sum())
