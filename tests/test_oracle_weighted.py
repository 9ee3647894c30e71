"""Pins for the oracle's weighted convolution (Eq. 1, read as the normalised
form sum(d w f) / sum(w f)): closed forms, invariances and brute force."""
import numpy as np

import oracle
from oracle import brute
from paper_1507_04941_amd import synth


def _weights(shape, seed, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 2.0, size=shape).astype(np.float32)
    if zero_frac:
        w[rng.random(shape) < zero_frac] = 0.0
    return w


def test_constant_cube_is_returned_for_any_positive_weights():
    d = np.full((11, 9, 30), 2.75, dtype=np.float32)
    F = oracle.filter3d_weighted(d, _weights(d.shape, 1), 2.0, 3.0)
    np.testing.assert_allclose(F, 2.75, rtol=1e-13, atol=0)


def test_unit_weights_renormalise_the_plain_filter_at_the_faces():
    d = synth.make_noise((14, 12, 40), seed=2)
    sxy, sz = 1.0, 2.0
    F = oracle.filter3d_weighted(d, np.ones_like(d), sxy, sz)
    gxy, gz = oracle.taps(sxy), oracle.taps(sz)

    def partial(g, n):          # in-range tap sum at each position
        r = len(g) // 2
        return np.array([sum(g[o + r] for o in range(-r, r + 1) if 0 <= i + o < n)
                         for i in range(n)])

    P = (partial(gxy, d.shape[0])[:, None, None] * partial(gxy, d.shape[1])[None, :, None]
         * partial(gz, d.shape[2])[None, None, :])
    np.testing.assert_allclose(F, oracle.filter3d(d, sxy, sz) / P, rtol=1e-12, atol=1e-14)


def test_scaling_the_weights_changes_nothing():
    d = synth.make_noise((10, 10, 24), seed=3)
    w = _weights(d.shape, 4, zero_frac=0.2)
    a = oracle.filter3d_weighted(d, w, 1.0, 1.0)
    b = oracle.filter3d_weighted(d, (w * 8.0).astype(np.float32), 1.0, 1.0)   # exact scaling
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_brute_force_with_zero_weights():
    d = synth.make_noise((7, 6, 12), seed=5)
    w = _weights(d.shape, 6, zero_frac=0.3)
    F = oracle.filter3d_weighted(d, w, 1.0, 1.0)
    np.testing.assert_allclose(F, brute.conv3d_weighted(d, w, 1.0, 1.0), rtol=1e-12, atol=1e-14)


def test_voxels_without_weighted_support_are_zero():
    d = synth.make_noise((12, 12, 40), seed=7) + 5.0
    w = np.ones_like(d)
    w[:, :, :20] = 0.0                  # channels 0..19 flagged
    F = oracle.filter3d_weighted(d, w, 1.0, 2.0)     # r_z = 6
    assert np.all(F[:, :, :14] == 0.0)              # support z..z+6 stays below 20
    assert np.all(F[:, :, 14:] != 0.0)
