"""FP64 CPU oracle for the all-pairs softened-gravity N-body hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. The GPU product path neither imports
nor calls anything here, and this package imports nothing from it.

The arithmetic lives in ``oracle.c`` (plain C, double precision, OpenMP over
particles, ascending-j sums with the self pair skipped); this module only
builds that file with gcc and marshals numpy arrays through ctypes.

Definitions (softened gravity in place of the paper's Lennard-Jones Eq. (1);
all-pairs structure of Sec. V-B; energy reduction of Sec. VI; the Verlet
half-step scheme of Sec. II-A read as kick-drift-kick):
    a_i   =  G sum_{j!=i} m_j d_ij s_ij^{-3/2},   d_ij = x_j - x_i, s_ij = |d_ij|^2 + eps^2
    phi_i = -G sum_{j!=i} m_j s_ij^{-1/2}
    KE = 1/2 sum m|v|^2, PE = 1/2 sum m phi, P = sum m v

The paper's own pair law, the Lennard-Jones gas of Eq. (1), with an optional
softening w (r^2 -> r^2 + w^2; w = 0 is the plain law) and the reflective-wall
boundary check applied after every drift:
    V(r) = 4 e [(s/r)^12 - (s/r)^6],  a_i = (1/m_i) sum_j 24 e [2 s^12/r^13 - s^6/r^7] r_hat_ji
    pot_i = (1/m_i) sum_{j!=i} V(r_ij)   (so PE = 1/2 sum m pot as for gravity)

Arrays are numpy float64, SoA planes of shape (3, n).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc: -O3 for the x86-64-v3 level (AVX2; the
    library is built on one host and run on others, so not -march=native), IEEE arithmetic kept
    exact (no fast-math, no contraction into fused multiply-adds: the FP64 results do not depend
    on the flags)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    lib.oracle_forces.argtypes = [I64, P, P, D, D, P, P]
    lib.oracle_forces.restype = None
    lib.oracle_forces_sample.argtypes = [I64, P, P, D, D, I64, P, P, P]
    lib.oracle_forces_sample.restype = None
    lib.oracle_energy_momentum.argtypes = [I64, P, P, P, D, D, P]
    lib.oracle_energy_momentum.restype = None
    lib.oracle_kdk.argtypes = [I64, D, D, D, I64, P, P, P, P, P]
    lib.oracle_kdk.restype = None
    lib.oracle_force_vjp.argtypes = [I64, P, P, D, D, P, P, P]
    lib.oracle_force_vjp.restype = None
    lib.oracle_force_vjp_sample.argtypes = [I64, P, P, D, D, P, I64, P, P, P]
    lib.oracle_force_vjp_sample.restype = None
    lib.oracle_rollout_adjoint.argtypes = [I64, D, D, D, I64, P, P, P, P, P, P, P, P]
    lib.oracle_rollout_adjoint.restype = None
    lib.oracle_loss_msd.argtypes = [I64, P, P, P]
    lib.oracle_loss_msd.restype = D
    lib.oracle_lj_forces.argtypes = [I64, P, P, D, D, D, P, P]
    lib.oracle_lj_forces.restype = None
    lib.oracle_lj_energy.argtypes = [I64, P, P, P, D, D, D, P]
    lib.oracle_lj_energy.restype = None
    lib.oracle_lj_kdk.argtypes = [I64, D, D, D, D, I64, P, P, P, P, P, P]
    lib.oracle_lj_kdk.restype = None
    lib.oracle_diagnostics.argtypes = [I64, P, P, P, P, P, P]
    lib.oracle_diagnostics.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def forces(pos, mass, G=1.0, eps=1e-2, want_pot=True):
    """Accelerations (3, n) and potentials (n,) (or None) of one system."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    acc = np.empty((3, n))
    pot = np.empty(n) if want_pot else None
    _load().oracle_forces(n, _p(pos), _p(mass), G, eps, _p(acc), _p(pot))
    return acc, pot


def forces_sample(pos, mass, idx, G=1.0, eps=1e-2):
    """Accelerations (3, k) and potentials (k,) of particles idx against all j."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("sample index out of range")
    k = idx.shape[0]
    acc = np.empty((3, k))
    pot = np.empty(k)
    _load().oracle_forces_sample(n, _p(pos), _p(mass), G, eps, k, _p(idx), _p(acc), _p(pot))
    return acc, pot


def energy_momentum(pos, vel, mass, G=1.0, eps=1e-2):
    """(KE, PE, Px, Py, Pz) of one system as a float64 array of 5."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    vel = _f64(vel, (3, n))
    out = np.empty(5)
    _load().oracle_energy_momentum(n, _p(pos), _p(vel), _p(mass), G, eps, _p(out))
    return out


def kdk(pos, vel, mass, dt, steps, G=1.0, eps=1e-2, want_traj=False, want_energy=False):
    """Run `steps` KDK steps. Returns (pos, vel, traj or None, energy or None)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n)).copy()
    vel = _f64(vel, (3, n)).copy()
    traj = np.empty((steps + 1, 3, n)) if want_traj else None
    energy = np.empty((steps + 1, 5)) if want_energy else None
    _load().oracle_kdk(n, G, eps, dt, steps, _p(pos), _p(vel), _p(mass), _p(traj), _p(energy))
    return pos, vel, traj, energy


def force_vjp(pos, mass, lam, G=1.0, eps=1e-2):
    """Gradient of sum_i lam_i . a_i w.r.t. positions (3, n) and masses (n,)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    lam = _f64(lam, (3, n))
    gx = np.zeros((3, n))
    gm = np.zeros(n)
    _load().oracle_force_vjp(n, _p(pos), _p(mass), G, eps, _p(lam), _p(gx), _p(gm))
    return gx, gm


def force_vjp_sample(pos, mass, lam, idx, G=1.0, eps=1e-2):
    """Rows idx of the force VJP: gx (3, k) and gm (k,) of particles idx (the full VJP's
    per-particle sums, evaluated for the sample only)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    lam = _f64(lam, (3, n))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("sample index out of range")
    k = idx.shape[0]
    gx = np.empty((3, k))
    gm = np.empty(k)
    _load().oracle_force_vjp_sample(n, _p(pos), _p(mass), G, eps, _p(lam), k, _p(idx), _p(gx), _p(gm))
    return gx, gm


def rollout_adjoint(pos0, vel0, mass, dt, steps, gpos_K, gvel_K, G=1.0, eps=1e-2):
    """Discrete-adjoint gradients (gpos0, gvel0, gmass) of a K-step KDK rollout."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos0 = _f64(pos0, (3, n))
    vel0 = _f64(vel0, (3, n))
    gpos_K = _f64(gpos_K, (3, n))
    gvel_K = _f64(gvel_K, (3, n))
    gx = np.empty((3, n))
    gv = np.empty((3, n))
    gm = np.empty(n)
    _load().oracle_rollout_adjoint(n, G, eps, dt, steps, _p(pos0), _p(vel0), _p(mass),
                                   _p(gpos_K), _p(gvel_K), _p(gx), _p(gv), _p(gm))
    return gx, gv, gm


def loss_msd(pos, target):
    """L = (1/n) sum_i |x_i - y_i|^2 and dL/dx (3, n)."""
    pos = _f64(pos)
    n = pos.shape[1]
    target = _f64(target, (3, n))
    grad = np.empty((3, n))
    val = _load().oracle_loss_msd(n, _p(pos), _p(target), _p(grad))
    return float(val), grad


def num_threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_num_threads())


def set_threads(t: int) -> None:
    """Run later oracle calls on t OpenMP threads (results do not depend on it)."""
    _load().oracle_set_threads(int(t))


# ---- batched systems: each system is an independent call (no cross-system pairs) ----

def forces_batched(pos, mass, offsets, G=1.0, eps=1e-2, want_pot=True):
    """Forces of concatenated systems; offsets[s]..offsets[s+1] delimit system s."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    acc = np.empty((3, n))
    pot = np.empty(n) if want_pot else None
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        ai, pi = forces(pos[:, a:b], mass[a:b], G, eps, want_pot)
        acc[:, a:b] = ai
        if want_pot:
            pot[a:b] = pi
    return acc, pot


# ---- Lennard-Jones gas (the paper's pair law, Eq. (1)) ----

def lj_forces(pos, mass, sigma=1.0, epsilon=1.0, soft=0.0, want_pot=True):
    """Accelerations F_i / m_i (3, n) and potential per unit mass (1/m_i) sum_j V(r_ij)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    acc = np.empty((3, n))
    pot = np.empty(n) if want_pot else None
    _load().oracle_lj_forces(n, _p(pos), _p(mass), sigma, epsilon, soft, _p(acc), _p(pot))
    return acc, pot


def lj_energy(pos, vel, mass, sigma=1.0, epsilon=1.0, soft=0.0):
    """(KE, PE, Px, Py, Pz) of a Lennard-Jones system."""
    mass = _f64(mass)
    n = mass.shape[0]
    out = np.empty(5)
    _load().oracle_lj_energy(n, _p(_f64(pos, (3, n))), _p(_f64(vel, (3, n))), _p(mass), sigma, epsilon, soft,
                             _p(out))
    return out


def lj_kdk(pos, vel, mass, dt, steps, sigma=1.0, epsilon=1.0, soft=0.0, box=None, want_energy=False):
    """KDK steps with reflective walls of box = (lo[3], hi[3]) (None: open space)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n)).copy()
    vel = _f64(vel, (3, n)).copy()
    lo = hi = None
    if box is not None:
        lo = _f64(box[0], (3,))
        hi = _f64(box[1], (3,))
    energy = np.empty((steps + 1, 5)) if want_energy else None
    _load().oracle_lj_kdk(n, sigma, epsilon, soft, dt, steps, _p(pos), _p(vel), _p(mass), _p(lo), _p(hi),
                          _p(energy))
    return pos, vel, energy


def diagnostics(pos, vel, mass, pot, acc):
    """(KE, PE, Px, Py, Pz, Lx, Ly, Lz, W, M) of one system from its state, the potential
    per unit mass and the acceleration (L = sum m x cross v, W = sum m x . a)."""
    mass = _f64(mass)
    n = mass.shape[0]
    out = np.empty(10)
    _load().oracle_diagnostics(n, _p(_f64(pos, (3, n))), _p(_f64(vel, (3, n))), _p(mass), _p(_f64(pot, (n,))),
                               _p(_f64(acc, (3, n))), _p(out))
    return out
