"""The seeded synthetic inputs: sizes, truncation rules, non-overlap with the
stated gap, determinism, and the structure of the example geometries."""
import math

import numpy as np

import synth


def _min_gap(centers, radii):
    d = np.hypot(centers[:, None, 0] - centers[None, :, 0], centers[:, None, 1] - centers[None, :, 1])
    g = d - radii[:, None] - radii[None, :]
    np.fill_diagonal(g, np.inf)
    return g.min()


def test_one_rhs_recipe():
    c = synth.one_rhs()
    assert c.M == 400 and c.n_tot == 10000 and c.k == 2 * math.pi
    assert np.all(c.radii == 0.5) and np.all(c.n_modes == 12)
    assert c.centers.min() >= 0.0 and c.centers.max() <= 60.0
    assert _min_gap(c.centers, c.radii) >= 0.2
    c2 = synth.one_rhs()
    assert np.array_equal(c.centers, c2.centers)


def test_multi_rhs_recipe():
    c = synth.multi_rhs()
    assert c.M == 1000 and c.k == 10.0 and len(c.betas) == 256
    assert c.radii.min() >= 0.3 and c.radii.max() <= 1.0
    assert np.array_equal(c.n_modes, np.ceil(10.0 * c.radii).astype(np.int32) + 10)
    assert _min_gap(c.centers, c.radii) >= 0.1


def test_penetrable_example_geometry():
    c = synth.penetrable_example()
    assert c.M == 400 and c.n_tot == 400 * 17 and c.k == 1.0
    assert np.all(c.radii == 1.0)
    # the row and the column through the origin are removed, the rest is the lattice
    assert np.all(c.centers[:, 0] != 0.0) and np.all(c.centers[:, 1] != 0.0)
    assert set(np.unique(c.centers[:, 0])) == set(3.0 * np.r_[-10:0, 1:11])
    assert _min_gap(c.centers, c.radii) >= 1.0 - 1e-12
    # the point source at the origin lies outside every disk
    assert np.min(np.hypot(c.centers[:, 0], c.centers[:, 1])) > 1.0


def test_time_reversal_example_geometry():
    c = synth.dort_example(64)
    assert np.array_equal(c.centers, [[0.0, 20.0], [10.0, -10.0], [-10.0, -20.0]])
    assert np.array_equal(c.radii, [0.02, 0.01, 0.005])
    assert np.all(c.n_modes == 4) and len(c.betas) == 64
    assert np.allclose(c.thetas, c.betas + np.pi)


def test_small_random_is_seeded_and_separated():
    a = synth.small_random(7, 12, 0.3, 0.9, 8.0, 0.25, 3.0, 5)
    b = synth.small_random(7, 12, 0.3, 0.9, 8.0, 0.25, 3.0, 5)
    assert np.array_equal(a.centers, b.centers) and np.array_equal(a.radii, b.radii)
    assert _min_gap(a.centers, a.radii) >= 0.25
    assert np.array_equal(a.n_modes, np.ceil(3.0 * a.radii).astype(np.int32) + 5)
