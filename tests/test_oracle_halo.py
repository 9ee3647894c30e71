"""Pins for the oracle's sub-cube form (find_halo): a cube with an input-only
border.  Checked against the plain path, against the same voxels of a larger
cube, and against the brute-force triple sum over the array."""
import numpy as np

import oracle
from oracle import brute
from paper_1507_04941_amd import synth

FILTERS = [(1.0, 2.0), (2.0, 1.0)]


def test_zero_halo_is_the_plain_path():
    d = synth.make_cube((18, 15, 40), n_sources=2, seed=11)
    a = oracle.find_halo(d, (0, 0, 0), FILTERS, (8, 6, 10), 4.0)
    b = oracle.find(d, FILTERS, (8, 6, 10), 4.0, want_F=True, want_stats=True)
    for key in ("F", "mean", "std"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["mask"], b["mask"])


def test_wide_halo_reproduces_the_larger_cube():
    # a sub-cube whose halo covers the filter radius sees exactly the data the
    # larger cube's filter reads at those voxels: F agrees bit for bit
    big = synth.make_cube((40, 36, 80), n_sources=4, seed=12)
    halo = (6, 6, 12)                      # >= r_xy = 6, r_z = 6 for (2, 2)
    x0, y0, z0 = 9, 7, 20
    core = (14, 12, 30)
    sub = big[x0 - halo[0]:x0 + core[0] + halo[0], y0 - halo[1]:y0 + core[1] + halo[1],
              z0 - halo[2]:z0 + core[2] + halo[2]]
    f = (2.0, 2.0)
    got = oracle.find_halo(sub, halo, [f], (4, 4, 4), 4.0)["F"][0]
    ref = oracle.filter3d(big, *f)[x0:x0 + core[0], y0:y0 + core[1], z0:z0 + core[2]]
    np.testing.assert_array_equal(got, ref)


def test_thin_halo_matches_brute_force_over_the_array():
    d = synth.make_noise((10, 9, 14), seed=13)
    halo = (1, 2, 3)                       # thinner than the radius: zeros beyond the array
    f = (1.0, 1.0)
    got = oracle.find_halo(d, halo, [f], (3, 3, 3), 4.0)["F"][0]
    ref = brute.conv3d(d, *f)[1:-1, 2:-2, 3:-3]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_statistics_cover_the_core_only():
    # the window is clipped to the core: values in the halo never enter it
    d = synth.make_noise((12, 12, 16), seed=14)
    halo = (2, 2, 2)
    a = oracle.find_halo(d, halo, [(1.0, 1.0)], (5, 5, 5), 4.0)
    d2 = d.copy()
    d2[:2] += 100.0                        # change only the x halo planes ...
    b = oracle.find_halo(d2, halo, [(1.0, 1.0)], (5, 5, 5), 4.0)
    # ... so F changes only on core planes within the radius (r = 3) of them,
    # core planes 0..2 (array planes 2..4); the rest keep F exactly
    assert not np.array_equal(a["F"][0][:1], b["F"][0][:1])
    np.testing.assert_array_equal(a["F"][0][3:], b["F"][0][3:])
    mu, sd = brute.local_stats(a["F"][0], (5, 5, 5))
    np.testing.assert_allclose(a["mean"][0], mu, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a["std"][0], sd, rtol=0, atol=1e-12)
