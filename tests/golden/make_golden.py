"""Write the stored oracle fixtures under tests/golden/.

Calls only the CPU oracle (and the seeded input generators). Each fixture is a
regression anchor for the oracle and a stored expectation for the GPU tests:

  cube1k_oracle.txt   uniform cube, n = 1024, seed 1, G = 1, eps = 1e-2,
                      10 kick-drift-kick steps of dt = 1e-3 (the all-pairs force of
                      Sec. V-B with the Verlet half-step scheme of Sec. II-A and the
                      energy reduction of Sec. VI, softened gravity as the pair law).
                      Rows for every 16th particle: initial a and phi, final x and v;
                      then the energy/momentum trace (KE, PE, Px, Py, Pz) per step.

Usage: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2511_02655_amd import inputs  # noqa: E402

STRIDE = 16


def cube1k():
    s = inputs.uniform_cube(1024, 1)
    acc, pot = oracle.forces(s.pos, s.mass, G=1.0, eps=1e-2)
    x, v, _, energy = oracle.kdk(s.pos, s.vel, s.mass, 1e-3, 10, G=1.0, eps=1e-2, want_energy=True)
    idx = np.arange(0, 1024, STRIDE)
    return idx, acc[:, idx], pot[idx], x[:, idx], v[:, idx], energy


def write(path):
    idx, acc, pot, x, v, energy = cube1k()
    with open(path, "w") as f:
        f.write("# oracle fixture: uniform cube n=1024 seed=1 G=1 eps=1e-2 dt=1e-3 steps=10\n")
        f.write("# written by tests/golden/make_golden.py (CPU oracle only)\n")
        f.write("# section particles: i ax ay az phi x y z vx vy vz  (a, phi at t=0; x, v after 10 steps)\n")
        f.write("particles %d\n" % len(idx))
        for k, i in enumerate(idx):
            vals = [acc[0, k], acc[1, k], acc[2, k], pot[k], x[0, k], x[1, k], x[2, k], v[0, k], v[1, k], v[2, k]]
            f.write("%d %s\n" % (i, " ".join("%.17e" % t for t in vals)))
        f.write("# section energy: step KE PE Px Py Pz\n")
        f.write("energy %d\n" % energy.shape[0])
        for s in range(energy.shape[0]):
            f.write("%d %s\n" % (s, " ".join("%.17e" % t for t in energy[s])))


def read(path):
    parts = {}
    with open(path) as f:
        lines = [l for l in f if not l.startswith("#")]
    k = 0
    while k < len(lines):
        name, cnt = lines[k].split()
        cnt = int(cnt)
        rows = np.array([[float(t) for t in lines[k + 1 + r].split()] for r in range(cnt)])
        parts[name] = rows
        k += 1 + cnt
    return parts


if __name__ == "__main__":
    write(os.path.join(HERE, "cube1k_oracle.txt"))
    print("wrote", os.path.join(HERE, "cube1k_oracle.txt"))
