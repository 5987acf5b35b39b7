"""The seeded input generators: deterministic, binary where they should be,
and at the requested volume fractions."""

import numpy as np

from paper_2103_05968_amd import microstructures as M


def test_c1_spheres_deterministic_and_fraction():
    a = M.config_c1()
    b = M.config_c1()
    assert a.shape == (32, 32, 32) and np.array_equal(a, b)
    assert set(np.unique(a)) == {0.3, 1.0}
    assert 0.15 <= np.mean(a == 0.3) < 0.25


def test_rsa_discs_non_overlapping_and_extruded():
    kap, centres = M.rsa_discs_extruded(96, 8, 5.0, 0.20, 10.0, 1.0, seed=2)
    assert kap.shape == (96, 96, 8)
    assert np.all(kap == kap[:, :, :1])
    assert 0.20 <= np.mean(kap == 10.0) < 0.23
    box = np.array([96.0, 96.0])
    for i in range(len(centres)):
        d = np.abs(centres[i + 1:] - centres[i])
        d = np.minimum(d, box - d)
        assert np.all(np.sqrt((d ** 2).sum(1)) >= 10.0)


def test_polydisperse_and_lognormal_and_cylinders():
    s = M.rsa_polydisperse_spheres(48, 3.0, 8.0, 0.25, 0.2, 1.0, seed=1000)
    assert 0.25 <= np.mean(s == 0.2) < 0.32
    g = M.gaussian_lognormal(32, 8.0, 0.5, seed=4)
    lg = np.log(g) / 0.5
    assert abs(lg.mean()) < 1e-12 and abs(lg.std() - 1.0) < 1e-12
    c = M.boolean_cylinders(64, 2.0, 20.0, 0.15, 5.0, 1.0, seed=5)
    assert 0.15 <= np.mean(c == 5.0) < 0.17
    assert np.array_equal(c, M.boolean_cylinders(64, 2.0, 20.0, 0.15, 5.0, 1.0, seed=5))


def test_single_sphere_and_laminate():
    s = M.single_sphere(16, 8.0, 10.0, 1.0)
    assert s[8, 8, 8] == 10.0 and s[0, 0, 0] == 1.0
    assert np.all(s[0] == 1.0)
    lam = M.laminate([1.0, 2.0, 3.0], (3, 2, 4), axis=0)
    assert lam.shape == (3, 2, 4) and np.all(lam[1] == 2.0)
