"""Pins for the oracle's Lennard-Jones functions (the paper's pair law, Eq. (1)).

Each test checks the oracle against a fact that does not come from retyping its
formula: the textbook landmarks of the 12-6 potential (zero at r = sigma, minimum
-epsilon at r = 2^{1/6} sigma, zero force there), its asymptotic power laws, the
tabulated lattice sums of the simple cubic crystal, the force as minus the
gradient of the energy, Newton's third law, the small-oscillation period of a
bound dimer, free flight between reflective walls, and the second-order energy
error of the kick-drift-kick integrator.
"""
import math

import numpy as np
import pytest

from paper_2511_02655_amd import inputs


def _dimer(r, direction=(0.3, -0.5, 0.8), m=(1.0, 1.0), origin=(1.7, -0.4, 2.2)):
    u = np.asarray(direction, float)
    u /= np.linalg.norm(u)
    o = np.asarray(origin, float)
    pos = np.stack([o, o + r * u], axis=1)
    return pos, np.asarray(m, float), u


@pytest.mark.parametrize("sigma,epsilon", [(1.0, 1.0), (0.37, 2.5)])
def test_lj_landmarks(oracle, sigma, epsilon):
    """V(sigma) = 0; V has its minimum -epsilon at r = 2^{1/6} sigma where the force
    vanishes; at r = sigma the force is repulsive (pushes the pair apart)."""
    zero = np.zeros((3, 2))
    # zero crossing
    pos, m, u = _dimer(sigma)
    pe = oracle.lj_energy(pos, zero, m, sigma, epsilon)[1]
    assert abs(pe) < 1e-13 * epsilon
    acc, _ = oracle.lj_forces(pos, m, sigma, epsilon)
    assert acc[:, 1] @ u > 0 and acc[:, 0] @ u < 0  # particle 1 sits at +r u: pushed outwards
    # minimum
    rmin = 2.0 ** (1.0 / 6.0) * sigma
    pos, m, u = _dimer(rmin)
    pe = oracle.lj_energy(pos, zero, m, sigma, epsilon)[1]
    assert pe == pytest.approx(-epsilon, rel=1e-13)
    acc, _ = oracle.lj_forces(pos, m, sigma, epsilon)
    assert np.max(np.abs(acc)) < 1e-12 * epsilon / sigma
    # a minimum: the energy rises on both sides
    for r in (0.999 * rmin, 1.001 * rmin):
        p2, m2, _ = _dimer(r)
        assert oracle.lj_energy(p2, zero, m2, sigma, epsilon)[1] > -epsilon


def test_lj_power_laws(oracle):
    """Far apart the attraction dominates: V ~ -4 eps (sigma/r)^6 and |F| ~ 24 eps sigma^6 / r^7
    (log-log slopes -6 and -7); close in the repulsion dominates with slopes -12 and -13."""
    zero = np.zeros((3, 2))

    def vf(r):
        pos, m, u = _dimer(r)
        pe = oracle.lj_energy(pos, zero, m)[1]
        acc, _ = oracle.lj_forces(pos, m)
        return pe, acc[:, 1] @ u  # unit mass: acceleration = force

    for (r1, r2, sv, sf) in [(40.0, 41.0, -6, -7), (0.25, 0.26, -12, -13)]:
        v1, f1 = vf(r1)
        v2, f2 = vf(r2)
        slope_v = math.log(abs(v2) / abs(v1)) / math.log(r2 / r1)
        slope_f = math.log(abs(f2) / abs(f1)) / math.log(r2 / r1)
        assert slope_v == pytest.approx(sv, abs=2e-3)
        assert slope_f == pytest.approx(sf, abs=2e-3)
    v, f = vf(40.0)
    assert v < 0 and f < 0  # attractive: particle 1 pulled back towards particle 0


def test_lj_simple_cubic_lattice_sums(oracle):
    """The energy of the centre site of a simple cubic crystal of spacing a is
    4 eps [A12 (sigma/a)^12 - A6 (sigma/a)^6] with the tabulated lattice sums
    A12 = 6.2021, A6 = 8.4019 (a finite crystal of half-width R = 10 a misses a tail of
    A6 below 4 pi / (3 R^3) = 4.2e-3 and a negligible one of A12). Two spacings give A12, A6."""
    R = 10
    g = np.arange(-R, R + 1, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    centre = int(np.flatnonzero(np.all(base == 0, axis=0))[0])
    m = np.ones(base.shape[1])
    pots = []
    spacings = (1.0, 1.25)
    for a in spacings:
        _, pot = oracle.lj_forces(base * a, m)
        pots.append(pot[centre])  # unit mass: per-site energy sum_j V(r_j)
    M = np.array([[4.0 * a ** -12, -4.0 * a ** -6] for a in spacings])
    A12, A6 = np.linalg.solve(M, np.array(pots))
    assert A12 == pytest.approx(6.2021, abs=1e-4)
    assert 8.4019 - 5e-3 < A6 < 8.4019 + 1e-4


@pytest.mark.parametrize("soft", [0.0, 0.3])
def test_lj_force_is_minus_energy_gradient(oracle, soft):
    """m_k a_k = -dPE/dx_k, by central differences of the oracle's potential energy."""
    g = np.random.Generator(np.random.PCG64(11))
    n = 7
    pos = inputs.lj_gas(n, seed=3, spacing=1.2)[0].pos + g.uniform(-0.1, 0.1, (3, n))
    mass = g.uniform(0.5, 2.0, n)
    sigma, epsilon = 1.05, 0.8
    acc, _ = oracle.lj_forces(pos, mass, sigma, epsilon, soft)
    zero = np.zeros((3, n))
    h = 1e-6
    for k in (0, 3, 6):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[c, k] += h
            pm[c, k] -= h
            dpe = (oracle.lj_energy(pp, zero, mass, sigma, epsilon, soft)[1]
                   - oracle.lj_energy(pm, zero, mass, sigma, epsilon, soft)[1]) / (2 * h)
            assert mass[k] * acc[c, k] == pytest.approx(-dpe, rel=1e-6, abs=1e-7)


def test_lj_softening_is_a_shifted_distance(oracle):
    """With softening w the pair energy at distance r equals the plain pair energy at
    sqrt(r^2 + w^2)."""
    zero = np.zeros((3, 2))
    r, w = 1.1, 0.4
    pos, m, _ = _dimer(r)
    soft_pe = oracle.lj_energy(pos, zero, m, 1.0, 1.0, w)[1]
    pos2, m2, _ = _dimer(math.sqrt(r * r + w * w))
    assert soft_pe == pytest.approx(oracle.lj_energy(pos2, zero, m2)[1], rel=1e-13)


def test_lj_newton_third_law(oracle):
    s, _ = inputs.lj_gas(64, seed=5, spacing=1.1)
    g = np.random.Generator(np.random.PCG64(2))
    pos = s.pos + g.uniform(-0.05, 0.05, s.pos.shape)
    mass = g.uniform(0.5, 1.5, s.n)
    acc, _ = oracle.lj_forces(pos, mass)
    F = acc * mass
    assert np.max(np.abs(F.sum(axis=1))) < 1e-12 * np.sum(np.abs(F))


def test_lj_dimer_small_oscillation_period(oracle):
    """A dimer released at rest near r_min oscillates with the harmonic period
    2 pi sqrt(mu / k), k = V''(r_min) = 72 eps / (2^{1/3} sigma^2), mu = m1 m2 / (m1 + m2)."""
    m1, m2 = 1.0, 2.0
    rmin = 2.0 ** (1.0 / 6.0)
    pos, m, u = _dimer(rmin * (1 + 2e-4), m=(m1, m2))
    vel = np.zeros((3, 2))
    k = 72.0 / 2.0 ** (1.0 / 3.0)
    mu = m1 * m2 / (m1 + m2)
    T = 2 * math.pi * math.sqrt(mu / k)
    dt = T / 400
    seps, times = [], []
    t = 0.0
    for _ in range(1700):  # a bit over 4 periods
        pos, vel, _ = oracle.lj_kdk(pos, vel, m, dt, 1)
        t += dt
        seps.append(np.linalg.norm(pos[:, 1] - pos[:, 0]) - rmin)
        times.append(t)
    seps = np.array(seps)
    # upward zero crossings of r - r_min, linearly interpolated
    idx = np.flatnonzero((seps[:-1] < 0) & (seps[1:] >= 0))
    tc = [times[i] + (times[i + 1] - times[i]) * (-seps[i]) / (seps[i + 1] - seps[i]) for i in idx]
    assert len(tc) >= 3
    period = (tc[-1] - tc[0]) / (len(tc) - 1)
    assert period == pytest.approx(T, rel=2e-3)


def test_lj_walls_free_flight(oracle):
    """One particle (no pair forces) between reflective walls: the position is the
    unfolded straight line x0 + v t folded back into [lo, hi] (a triangle wave) and the
    velocity flips sign once per wall hit."""
    lo, hi = np.array([0.0, -1.0, 2.0]), np.array([3.0, 4.0, 2.5])
    x0 = np.array([[1.0], [0.5], [2.1]])
    v0 = np.array([[2.3], [-1.7], [0.9]])
    dt, steps = 0.01, 737
    pos, vel, _ = oracle.lj_kdk(x0, v0, np.ones(1), dt, steps, box=(lo, hi))
    t = dt * steps
    for c in range(3):
        L = hi[c] - lo[c]
        y = (x0[c, 0] - lo[c] + v0[c, 0] * t) % (2 * L)
        want_x = lo[c] + (y if y <= L else 2 * L - y)
        want_v = v0[c, 0] * (1 if y <= L else -1)
        assert pos[c, 0] == pytest.approx(want_x, abs=1e-11)
        assert vel[c, 0] == pytest.approx(want_v, rel=1e-15)


def test_lj_kdk_energy_error_is_second_order(oracle):
    """Kick-drift-kick is symplectic and second order: halving dt cuts the energy error
    of a bound LJ cluster about fourfold (and the momentum stays exactly conserved in
    open space)."""
    s, _ = inputs.lj_gas(27, seed=9, spacing=1.15, temperature=0.05)
    errs = []
    for dt in (4e-3, 2e-3):
        steps = int(round(0.4 / dt))
        _, _, en = oracle.lj_kdk(s.pos, s.vel, s.mass, dt, steps, want_energy=True)
        E = en[:, 0] + en[:, 1]
        errs.append(np.max(np.abs(E - E[0])))
        assert np.max(np.abs(en[:, 2:] - en[0, 2:])) < 1e-12
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_lj_reflective_walls_conserve_energy(oracle):
    """Elastic walls: a gas bouncing off them keeps its total energy to the integrator's
    error, and every particle stays inside the box."""
    s, box = inputs.lj_gas(64, seed=4, spacing=1.3, temperature=2.0)
    pos, vel, en = oracle.lj_kdk(s.pos, s.vel, s.mass, 1e-3, 400, box=(box.lo, box.hi), want_energy=True)
    E = en[:, 0] + en[:, 1]
    assert np.max(np.abs(E - E[0])) < 2e-3 * abs(en[0, 0])
    assert np.all(pos >= box.lo[:, None]) and np.all(pos <= box.hi[:, None])
    # some particles must actually have hit a wall for this to test anything
    assert np.any(np.sign(vel) != np.sign(s.vel + 0 * vel))


def test_lj_gas_generator():
    s, box = inputs.lj_gas(10000, seed=7)
    assert s.pos.shape == (3, 10000)
    assert np.all(s.pos > box.lo[:, None]) and np.all(s.pos < box.hi[:, None])
    assert np.allclose(box.hi, 22 * 1.5)
    assert np.max(np.abs(s.vel.mean(axis=1))) < 1e-15
    # nearest-neighbour distance is the lattice spacing: no overlapping particles
    d = np.sqrt(np.sum((s.pos[:, :1] - s.pos) ** 2, axis=0))
    assert np.sort(d)[1] == pytest.approx(1.5)
