"""Seeded input generators (statistical checks) and the stored oracle fixture."""
import math
import os

import numpy as np

from paper_2511_02655_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_generators_are_seeded():
    a = inputs.plummer(1000, 5)
    b = inputs.plummer(1000, 5)
    np.testing.assert_array_equal(a.pos, b.pos)
    np.testing.assert_array_equal(a.vel, b.vel)
    c = inputs.plummer(1000, 6)
    assert not np.array_equal(a.pos, c.pos)


def test_uniform_cube():
    s = inputs.uniform_cube(4096, 1)
    assert s.pos.shape == (3, 4096) and s.pos.min() >= 0 and s.pos.max() < 1
    assert np.all(s.vel == 0)
    assert s.mass.min() >= 0.5 / 4096 and s.mass.max() < 1.5 / 4096
    assert abs(s.mass.sum() - 1.0) < 0.02


def test_plummer_mass_profile_and_centre():
    """Cumulative mass fraction inside r follows r^3/(1+r^2)^{3/2} (renormalised to the
    truncation radius 10); the centre of mass is at rest at the origin."""
    n = 65536
    s = inputs.plummer(n, 2)
    r = np.sqrt((s.pos ** 2).sum(axis=0))
    assert r.max() <= 10.0 + 1e-9
    cum = lambda x: x ** 3 / (1 + x * x) ** 1.5
    for x in [0.3, 0.7, 1.0, 2.0, 4.0]:
        expect = cum(x) / cum(10.0)
        got = np.mean(r < x)
        sigma = math.sqrt(expect * (1 - expect) / n)
        # recentring moves radii slightly; allow 5 sigma plus a small absolute slack
        assert abs(got - expect) < 5 * sigma + 2e-3, (x, got, expect)
    np.testing.assert_allclose((s.pos * s.mass).sum(axis=1), 0, atol=1e-15)
    np.testing.assert_allclose((s.vel * s.mass).sum(axis=1), 0, atol=1e-15)
    # every particle is bound: speed below the local escape speed of the untruncated profile
    v = np.sqrt((s.vel ** 2).sum(axis=0))
    assert np.all(v < math.sqrt(2.0) * (1 + r * r) ** -0.25 + 0.05)


def test_two_spheres_and_targets():
    s = inputs.two_spheres(8192, 4)
    assert s.n == 16384
    np.testing.assert_allclose(s.mass.sum(), 1.0)
    np.testing.assert_allclose(s.pos[0, :8192].mean(), -2.0, atol=1e-12)
    np.testing.assert_allclose(s.pos[0, 8192:].mean(), 2.0, atol=1e-12)
    np.testing.assert_allclose(s.vel[1, :8192].mean(), 0.3, atol=1e-12)
    np.testing.assert_allclose(s.vel[1, 8192:].mean(), -0.3, atol=1e-12)
    y = inputs.gaussian_targets(16384, 5)
    assert y.shape == (3, 16384) and abs(y.std() - 1) < 0.02


def test_batched_mix():
    b = inputs.batched_mix(512, 6)
    sizes = np.diff(b.offsets)
    assert len(sizes) == 512 and sizes.min() >= 64 and sizes.max() <= 8192
    assert b.offsets[0] == 0 and b.offsets[-1] == b.mass.shape[0]
    assert set(b.kinds) == {"cube", "plummer"}
    # log-uniform sizes: median near sqrt(64 * 8192) = 724
    assert 500 < np.median(sizes) < 1050


def test_kepler_pair_energy():
    """Pericentre state of a Kepler orbit has specific energy -G M / (2 a)."""
    s = inputs.kepler_pair(0.6, 0.4, 1.3, 0.5)
    rel_x = s.pos[:, 1] - s.pos[:, 0]
    rel_v = s.vel[:, 1] - s.vel[:, 0]
    eps_spec = 0.5 * rel_v @ rel_v - 1.0 / np.linalg.norm(rel_x)
    assert abs(eps_spec + 1.0 / (2 * 1.3)) < 1e-14


def test_golden_fixture_regression(oracle):
    """The oracle still reproduces the stored fixture it wrote."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    stored = mg.read(os.path.join(HERE, "golden", "cube1k_oracle.txt"))
    idx, acc, pot, x, v, energy = mg.cube1k()
    p = stored["particles"]
    np.testing.assert_array_equal(p[:, 0].astype(int), idx)
    np.testing.assert_allclose(p[:, 1:4].T, acc, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(p[:, 4], pot, rtol=1e-14)
    np.testing.assert_allclose(p[:, 5:8].T, x, rtol=1e-14)
    np.testing.assert_allclose(p[:, 8:11].T, v, rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(stored["energy"][:, 1:], energy, rtol=1e-13, atol=1e-18)
