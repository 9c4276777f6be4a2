"""Seeded synthetic inputs for the N-body workloads.

This module only draws initial conditions; it holds none of the force,
integrator, energy or adjoint arithmetic. Both the GPU path and the CPU oracle
receive the *same* arrays from here, so no cross-language random-number parity
is needed. Random numbers come from numpy's PCG64 generator.

All arrays are float64. Positions and velocities are SoA planes of shape (3, n).

The paper never specifies its initial state (its Lennard-Jones box, lattice and
time step are silent), so the workloads are the standard gravitational ones:
  * uniform cube: x ~ U[0,1)^3, v = 0, m ~ U[0.5,1.5)/n;
  * Plummer sphere (Aarseth, Henon & Wielen 1974 sampling), G = M = a = 1 by
    default, truncated at r <= 10 a, centre of mass moved to rest at the origin;
  * two Plummer spheres on a collision course (mass 1/2 each, offsets +-2 in x,
    bulk velocities +-0.3 in y) and a Gaussian target cloud;
  * a regular N-gon ring and a Kepler pair (closed-form test cases);
  * a batch of systems with log-uniform sizes, each a cube or a Plummer sphere;
  * a Lennard-Jones gas for the paper's own pair law: a simple cubic lattice in a
    box with reflective walls, Maxwell-Boltzmann velocities (reduced units).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class System:
    pos: np.ndarray   # (3, n)
    vel: np.ndarray   # (3, n)
    mass: np.ndarray  # (n,)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def uniform_cube(n: int, seed: int) -> System:
    """x ~ U[0,1)^3, v = 0, m ~ U[0.5, 1.5)/n. No recentring (total momentum is exactly 0)."""
    g = rng(seed)
    pos = g.random((3, n))
    mass = g.uniform(0.5, 1.5, n) / max(n, 1)
    return System(np.ascontiguousarray(pos), np.zeros((3, n)), np.ascontiguousarray(mass))


def _isotropic(g: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Vectors of length r with isotropic directions, shape (3, len(r))."""
    cos_t = g.uniform(-1.0, 1.0, r.shape[0])
    phi = g.uniform(0.0, 2.0 * math.pi, r.shape[0])
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return np.stack([r * sin_t * np.cos(phi), r * sin_t * np.sin(phi), r * cos_t])


def plummer(n: int, seed: int, M: float = 1.0, a: float = 1.0, G: float = 1.0,
            rmax: float = 10.0, recentre: bool = True) -> System:
    """Plummer sphere of total mass M and scale radius a (equal masses M/n).

    Radius from the inverse cumulative mass profile r = a (X^{-2/3} - 1)^{-1/2},
    rejecting r > rmax*a. Speed v = q v_esc(r), v_esc = sqrt(2GM/a) (1 + r^2/a^2)^{-1/4},
    with q drawn from g(q) = q^2 (1 - q^2)^{7/2} by rejection under the constant
    envelope 0.1 (max g is about 0.092). Directions are isotropic.
    """
    g = rng(seed)
    radii = np.empty(0)
    while radii.shape[0] < n:
        X = g.random(2 * (n - radii.shape[0]) + 16)
        X = X[X > 0.0]
        r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        radii = np.concatenate([radii, r[r <= rmax * a]])
    radii = radii[:n]
    pos = _isotropic(g, radii)

    q = np.empty(0)
    while q.shape[0] < n:
        m = 2 * (n - q.shape[0]) + 64
        x = g.random(m)
        y = g.uniform(0.0, 0.1, m)
        keep = y < x * x * (1.0 - x * x) ** 3.5
        q = np.concatenate([q, x[keep]])
    q = q[:n]
    vesc = math.sqrt(2.0 * G * M / a) * (1.0 + (radii / a) ** 2) ** -0.25
    vel = _isotropic(g, q * vesc)
    mass = np.full(n, M / max(n, 1))
    if recentre and n > 0:
        pos -= (pos * mass).sum(axis=1, keepdims=True) / mass.sum()
        vel -= (vel * mass).sum(axis=1, keepdims=True) / mass.sum()
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), np.ascontiguousarray(mass))


def two_spheres(n_each: int, seed: int, offset: float = 2.0, bulk_v: float = 0.3) -> System:
    """Two Plummer spheres (M = 0.5, a = 1 each), at x = -+offset moving at v_y = +-bulk_v."""
    s1 = plummer(n_each, seed, M=0.5)
    s2 = plummer(n_each, seed + 100003, M=0.5)
    s1.pos[0] -= offset
    s2.pos[0] += offset
    s1.vel[1] += bulk_v
    s2.vel[1] -= bulk_v
    return System(np.ascontiguousarray(np.concatenate([s1.pos, s2.pos], axis=1)),
                  np.ascontiguousarray(np.concatenate([s1.vel, s2.vel], axis=1)),
                  np.ascontiguousarray(np.concatenate([s1.mass, s2.mass])))


def gaussian_targets(n: int, seed: int) -> np.ndarray:
    """Target positions y_i ~ N(0, I_3), shape (3, n)."""
    return np.ascontiguousarray(rng(seed).standard_normal((3, n)))


def ring(n: int, R: float = 1.0, m: float = 1.0, phase: float = 0.0) -> System:
    """Regular n-gon of radius R in the z = 0 plane, equal masses m, at rest."""
    th = phase + 2.0 * math.pi * np.arange(n) / n
    pos = np.stack([R * np.cos(th), R * np.sin(th), np.zeros(n)])
    return System(np.ascontiguousarray(pos), np.zeros((3, n)), np.full(n, float(m)))


def kepler_pair(m1: float, m2: float, semi_major: float, ecc: float, G: float = 1.0) -> System:
    """Two bodies at pericentre of a Kepler orbit with the given semi-major axis and
    eccentricity, centre of mass at rest at the origin, orbit in the x-y plane."""
    M = m1 + m2
    rp = semi_major * (1.0 - ecc)
    vp = math.sqrt(G * M * (1.0 + ecc) / (semi_major * (1.0 - ecc)))
    rel_x = np.array([rp, 0.0, 0.0])
    rel_v = np.array([0.0, vp, 0.0])
    x1, x2 = -m2 / M * rel_x, m1 / M * rel_x
    v1, v2 = -m2 / M * rel_v, m1 / M * rel_v
    return System(np.ascontiguousarray(np.stack([x1, x2], axis=1)),
                  np.ascontiguousarray(np.stack([v1, v2], axis=1)),
                  np.array([m1, m2], dtype=np.float64))


@dataclass
class Batch:
    offsets: np.ndarray  # (S+1,) int64
    pos: np.ndarray      # (3, sum n)
    vel: np.ndarray
    mass: np.ndarray
    kinds: list


def batched_mix(n_systems: int, seed: int, nmin: int = 64, nmax: int = 8192) -> Batch:
    """n_systems independent systems; N_s = clamp(round(exp(U(ln nmin, ln nmax)))),
    a uniform cube if U < 0.5 else a Plummer sphere (M = 1), each from seed 1000*seed + s."""
    g = rng(seed)
    sizes = np.clip(np.rint(np.exp(g.uniform(math.log(nmin), math.log(nmax), n_systems))),
                    nmin, nmax).astype(np.int64)
    kinds_u = g.random(n_systems)
    offsets = np.zeros(n_systems + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    parts, kinds = [], []
    for s in range(n_systems):
        sub_seed = 1000 * seed + s
        if kinds_u[s] < 0.5:
            parts.append(uniform_cube(int(sizes[s]), sub_seed))
            kinds.append("cube")
        else:
            parts.append(plummer(int(sizes[s]), sub_seed))
            kinds.append("plummer")
    pos = np.concatenate([p.pos for p in parts], axis=1) if parts else np.zeros((3, 0))
    vel = np.concatenate([p.vel for p in parts], axis=1) if parts else np.zeros((3, 0))
    mass = np.concatenate([p.mass for p in parts]) if parts else np.zeros(0)
    return Batch(offsets, np.ascontiguousarray(pos), np.ascontiguousarray(vel),
                 np.ascontiguousarray(mass), kinds)


@dataclass
class Box:
    lo: np.ndarray  # (3,)
    hi: np.ndarray  # (3,)


def lj_gas(n: int, seed: int, spacing: float = 1.5, temperature: float = 1.0, m: float = 1.0,
           sigma: float = 1.0) -> tuple:
    """Lennard-Jones gas on a simple cubic lattice, returned as (System, Box).

    k = ceil(n^(1/3)) sites per edge at ((i + 1/2) a, (j + 1/2) a, (l + 1/2) a) with
    a = spacing * sigma; the first n sites in x-fastest order are occupied (the top
    layer is partly filled when n is not a cube). Box [0, k a]^3. Velocities are
    Maxwell-Boltzmann at temperature kT = temperature (each component ~ N(0, kT/m)),
    with the net momentum removed. Equal masses m."""
    k = max(1, int(math.ceil(round(n ** (1.0 / 3.0), 9))))
    while k ** 3 < n:
        k += 1
    a = spacing * sigma
    idx = np.arange(n)
    ix, iy, iz = idx % k, (idx // k) % k, idx // (k * k)
    pos = (np.stack([ix, iy, iz]).astype(np.float64) + 0.5) * a
    g = rng(seed)
    vel = g.normal(0.0, math.sqrt(temperature / m), (3, n))
    if n > 0:
        vel -= vel.mean(axis=1, keepdims=True)
    mass = np.full(n, float(m))
    box = Box(np.zeros(3), np.full(3, k * a))
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass), box


# ---- the five reference workloads (sizes, softening, step, seeds) ----

WORKLOADS = {
    "cube1k": dict(kind="cube", n=1024, eps=1e-2, dt=1e-3, steps=10, seed=1),
    "plummer64k": dict(kind="plummer", n=65536, eps=1e-2, dt=1e-3, steps=100, seed=2),
    "plummer1m": dict(kind="plummer", n=1048576, eps=1e-3, dt=5e-4, steps=10, seed=3),
    "merger2x8k": dict(kind="two_spheres", n=16384, eps=1e-2, dt=1e-3, steps=200, ckpt=20,
                       seed=4, target_seed=5),
    "batch512": dict(kind="batch", n_systems=512, eps=1e-2, dt=1e-3, steps=50, seed=6),
    # the paper's own experiment size: a Lennard-Jones gas of 10 000 particles, 2500 steps
    # (sigma = epsilon = m = 1, lattice spacing 1.5 sigma, kT = 1, dt = 0.002 in reduced units)
    "lj10k": dict(kind="lj", n=10000, sigma=1.0, epsilon=1.0, spacing=1.5, temperature=1.0, dt=2e-3,
                  steps=2500, seed=7),
}


def make(name: str, n: int | None = None):
    """Initial state of a named workload (optionally at a different n)."""
    w = WORKLOADS[name]
    if w["kind"] == "cube":
        return uniform_cube(n or w["n"], w["seed"])
    if w["kind"] == "plummer":
        return plummer(n or w["n"], w["seed"])
    if w["kind"] == "two_spheres":
        return two_spheres((n or w["n"]) // 2, w["seed"])
    if w["kind"] == "batch":
        return batched_mix(n or w["n_systems"], w["seed"])
    if w["kind"] == "lj":
        return lj_gas(n or w["n"], w["seed"], spacing=w["spacing"], temperature=w["temperature"],
                      sigma=w["sigma"])
    raise KeyError(name)
