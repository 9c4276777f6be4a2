"""Pins for the oracle's diagnostics: angular momentum L = sum m x cross v and the virial
W = sum m x . a of the pair forces (the law-agnostic reduction that extends energy and
momentum). Closed forms of a rigidly rotating ring and of a pair, the exact change of L
and invariance of W under a translation, Euler's theorem for the degree -1 Newtonian
potential (W = PE without softening) with the exact softened correction, the textbook
Lennard-Jones pair virial, and conservation of L by the kick-drift-kick integrator.
"""
import math

import numpy as np
import pytest

from paper_2511_02655_amd import inputs


def _diag(oracle, pos, vel, mass, G=1.0, eps=1e-2):
    acc, pot = oracle.forces(pos, mass, G=G, eps=eps)
    return oracle.diagnostics(pos, vel, mass, pot, acc)


def test_rotating_ring_closed_form(oracle):
    """Ring of n equal masses m at radius R spinning rigidly at omega about z:
    L = (0, 0, n m R^2 omega), KE = n m R^2 omega^2 / 2, P = 0, M = n m."""
    n, R, m, om = 37, 1.7, 0.3, 0.9
    s = inputs.ring(n, R=R, m=m, phase=0.2)
    vel = np.stack([-om * s.pos[1], om * s.pos[0], np.zeros(n)])
    d = _diag(oracle, s.pos, vel, s.mass)
    assert d[7] == pytest.approx(n * m * R * R * om, rel=1e-13)
    assert abs(d[5]) < 1e-13 and abs(d[6]) < 1e-13
    assert d[0] == pytest.approx(0.5 * n * m * R * R * om * om, rel=1e-13)
    assert np.max(np.abs(d[2:5])) < 1e-13
    assert d[9] == pytest.approx(n * m, rel=1e-15)


def test_pair_virial_closed_form(oracle):
    """Two bodies: W = m1 x1.a1 + m2 x2.a2 = -G m1 m2 r^2 / (r^2 + eps^2)^{3/2}, whatever
    the origin."""
    G, eps = 1.3, 0.2
    pos = np.array([[2.0, 2.9], [-1.0, -0.6], [0.5, 1.7]])
    mass = np.array([0.7, 2.1])
    r2 = float(np.sum((pos[:, 1] - pos[:, 0]) ** 2))
    d = _diag(oracle, pos, np.zeros((3, 2)), mass, G=G, eps=eps)
    assert d[8] == pytest.approx(-G * mass[0] * mass[1] * r2 / (r2 + eps * eps) ** 1.5, rel=1e-13)


def test_translation(oracle):
    """Shifting every position by c changes L by c cross P and leaves W unchanged (the pair
    forces sum to zero)."""
    g = np.random.Generator(np.random.PCG64(3))
    n = 60
    pos, vel, mass = g.normal(size=(3, n)), g.normal(size=(3, n)), g.uniform(0.5, 1.5, n)
    c = np.array([[3.0], [-7.0], [11.0]])
    d0 = _diag(oracle, pos, vel, mass)
    d1 = _diag(oracle, pos + c, vel, mass)
    P = d0[2:5]
    np.testing.assert_allclose(d1[5:8], d0[5:8] + np.cross(c[:, 0], P), rtol=1e-12, atol=1e-12)
    assert d1[8] == pytest.approx(d0[8], rel=1e-11)


def test_virial_equals_potential_energy_without_softening(oracle):
    """Newtonian gravity is homogeneous of degree -1, so W = PE (Euler); with softening eps the
    difference is exactly G sum_{i<j} m_i m_j eps^2 / (r^2 + eps^2)^{3/2}."""
    g = np.random.Generator(np.random.PCG64(4))
    n = 40
    pos, mass = g.normal(size=(3, n)), g.uniform(0.5, 1.5, n)
    d = _diag(oracle, pos, np.zeros((3, n)), mass, eps=1e-9)
    assert d[8] == pytest.approx(d[1], rel=1e-9)
    eps = 0.3
    d = _diag(oracle, pos, np.zeros((3, n)), mass, eps=eps)
    diff = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            r2 = float(np.sum((pos[:, i] - pos[:, j]) ** 2))
            diff += mass[i] * mass[j] * eps * eps / (r2 + eps * eps) ** 1.5
    assert d[8] - d[1] == pytest.approx(diff, rel=1e-10)


@pytest.mark.parametrize("r_over_sigma,want", [(1.0, 24.0), (2.0 ** (1.0 / 6.0), 0.0)])
def test_lennard_jones_pair_virial(oracle, r_over_sigma, want):
    """Lennard-Jones pair: W = r |F| = 24 eps (2 (s/r)^12 - (s/r)^6); 24 eps at r = sigma and 0
    at the minimum 2^{1/6} sigma."""
    sigma, epsilon = 0.8, 1.5
    r = r_over_sigma * sigma
    pos = np.array([[0.3, 0.3 + r], [1.0, 1.0], [-2.0, -2.0]])
    mass = np.array([1.0, 2.0])
    acc, pot = oracle.lj_forces(pos, mass, sigma, epsilon)
    d = oracle.diagnostics(pos, np.zeros((3, 2)), mass, pot, acc)
    assert d[8] == pytest.approx(want * epsilon, abs=1e-12 * epsilon * 24)


def test_kdk_conserves_angular_momentum(oracle):
    """Pair forces along the separation conserve L exactly, and so does each kick and
    drift of the integrator: L stays constant to rounding over a Plummer rollout."""
    s = inputs.plummer(200, 9)
    L0 = _diag(oracle, s.pos, s.vel, s.mass)[5:8]
    x, v, _, _ = oracle.kdk(s.pos, s.vel, s.mass, 1e-3, 50, eps=1e-2)
    L1 = _diag(oracle, x, v, s.mass)[5:8]
    scale = float(np.sum(s.mass * np.linalg.norm(s.pos, axis=0) * np.linalg.norm(s.vel, axis=0)))
    assert np.max(np.abs(L1 - L0)) < 1e-13 * scale
