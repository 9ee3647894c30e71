"""Pins for the oracle's local statistics (§3.3): per-voxel mean and population
standard deviation of the filtered cube over a box window around the voxel,
clipped at the faces.  Checked against closed forms (constant, linear ramps
including the clipped borders), numpy two-pass brute force, scipy's uniform
filter, and the oracle's own plain per-voxel two-pass evaluation.
"""
import numpy as np
import pytest
from scipy import ndimage as ndi

import oracle
from oracle import brute
from paper_1507_04941_amd import synth


def test_constant_gives_exact_mean_and_zero_std():
    F = np.full((9, 10, 40), -2.75)
    m, s = oracle.local_stats(F, (4, 5, 16))
    assert np.all(m == -2.75)
    assert np.all(s == 0.0)


def _ramp_expect(i, n, B, a, b):
    lo = max(i - B // 2, 0)
    hi = min(i - B // 2 + B, n)          # exclusive
    L = hi - lo
    mean = a * (lo + hi - 1) / 2.0 + b
    var = a * a * (L * L - 1) / 12.0
    return mean, var


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("B", [4, 5, 8])
def test_linear_ramp_closed_form(axis, B):
    shape = [7, 8, 9]
    shape[axis] = 23
    a, b = 0.37, -1.25
    idx = np.indices(shape)[axis].astype(np.float64)
    F = a * idx + b
    box = [3, 3, 3]
    box[axis] = B
    m, s = oracle.local_stats(F, tuple(box))
    n = shape[axis]
    for i in range(n):
        em, ev = _ramp_expect(i, n, B, a, b)
        sl = [slice(None)] * 3
        sl[axis] = i
        np.testing.assert_allclose(m[tuple(sl)], em, rtol=0, atol=1e-13)
        np.testing.assert_allclose(s[tuple(sl)] ** 2, ev, rtol=0, atol=1e-12)
    # interior: mean sits half a voxel below the centre for even B ([-B/2, B/2-1])
    if B % 2 == 0:
        i = n // 2
        sl = [0, 0, 0]
        sl[axis] = i
        assert abs(m[tuple(sl)] - (a * (i - 0.5) + b)) < 1e-12
        assert abs(s[tuple(sl)] ** 2 - a * a * (B * B - 1) / 12.0) < 1e-12


@pytest.mark.parametrize("shape,box", [
    ((6, 7, 11), (4, 5, 6)),
    ((3, 9, 5), (6, 4, 4)),          # box longer than the axis
    ((8, 8, 16), (8, 8, 8)),
    ((1, 1, 7), (2, 2, 3)),
])
def test_matches_bruteforce_two_pass(shape, box):
    F = synth.make_noise(shape, seed=21).astype(np.float64) * 0.3 + 1.7
    m, s = oracle.local_stats(F, box)
    bm, bs = brute.local_stats(F, box)
    np.testing.assert_allclose(m, bm, rtol=0, atol=1e-13)
    np.testing.assert_allclose(s, bs, rtol=0, atol=1e-12)


def test_matches_scipy_uniform_filter():
    F = synth.make_noise((24, 20, 48), seed=4).astype(np.float64)
    box = (8, 6, 16)
    B3 = float(np.prod(box))
    S1 = ndi.uniform_filter(F, size=box, mode="constant", cval=0.0) * B3
    S2 = ndi.uniform_filter(F * F, size=box, mode="constant", cval=0.0) * B3
    n = ndi.uniform_filter(np.ones_like(F), size=box, mode="constant", cval=0.0) * B3
    mu = S1 / n
    var = S2 / n - mu * mu
    m, s = oracle.local_stats(F, box)
    np.testing.assert_allclose(m, mu, rtol=0, atol=1e-11)
    np.testing.assert_allclose(s * s, var, rtol=0, atol=1e-10)


def test_directional_sums_match_plain_per_voxel():
    F = synth.make_noise((40, 36, 80), seed=8).astype(np.float64)
    box = (16, 16, 32)
    m, s = oracle.local_stats(F, box)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, F.size, size=300)
    idx = np.concatenate([idx, [0, F.size - 1, 35 * 80 + 79]])
    pm, ps = oracle.local_stats_at(F, box, idx)
    np.testing.assert_allclose(m.reshape(-1)[idx], pm, rtol=0, atol=1e-13)
    np.testing.assert_allclose(s.reshape(-1)[idx], ps, rtol=0, atol=1e-12)


def test_offset_cube_no_cancellation():
    # A large common offset must not cost precision (shifted sums).
    base = synth.make_noise((16, 16, 32), seed=12).astype(np.float64)
    m0, s0 = oracle.local_stats(base, (8, 8, 8))
    m1, s1 = oracle.local_stats(base + 1.0e4, (8, 8, 8))
    np.testing.assert_allclose(m1 - 1.0e4, m0, rtol=0, atol=1e-10)
    np.testing.assert_allclose(s1, s0, rtol=0, atol=1e-10)
