"""GPU parity of the adaptive-separation FP32 mode ("fp32a", NBODY_FP32_ADAPT).

A single system on symmetric tiles is sorted along a Morton curve at every force pass, and
only sub-block pairs whose boxes lie within T = X_max / 256 take double-float separations.
Checked here: every symmetric variant forced through the tile table on sizes around the tile
and sort edges against the oracle (per-particle bound B_i of oracle/bounds.py, adaptive form);
outputs in the caller's order and bitwise deterministic; rollouts (step = rollout, checkpoint
interval invariance, energy trace on/off) bitwise consistent; degenerate inputs; the
Lennard-Jones law; and the paths that run as the double-float mode (batches, one-sided).
The N = 1M accuracy (max e_i <= 1e-5 on every particle) is checked in test_gpu_parity.py.
"""
import math

import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_02655_amd as nb
    nb.lib()
    return nb


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _sym_variants(nb):
    return [k for k, d in enumerate(nb.tile_variants("force", "fp32a")) if "sym=" in d]


def _bound(pos, mass, eps, G=1.0):
    from oracle import bounds
    return bounds.fp32_force_bound(pos, mass, eps, G, adaptive=True)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 1023, 2047, 2048, 2049, 5000])
def test_adaptive_every_symmetric_variant(nb, oracle, n):
    """Every symmetric variant in the adaptive mode, with and without the potential, against
    the oracle within the per-particle bound (uniform cube; sizes below, at and across the
    tile edges and the 2048-key edge of the sort)."""
    s = inputs.uniform_cube(n, 900 + n)
    acc_ref, pot_ref = oracle.forces(s.pos, s.mass, eps=1e-2)
    B = _bound(s.pos, s.mass, 1e-2)
    try:
        for v in _sym_variants(nb):
            nb.set_tile_table([dict(kernel="force", precision="fp32a", n_min=0, n_max=1 << 40, variant=v, j_split=1)])
            for want_pot in (True, False):
                acc, pot = nb.forces(dev(s.pos), dev(s.mass), eps=1e-2, precision="fp32a", want_pot=want_pot)
                a = host(acc)
                if n == 1:
                    assert np.all(a == 0)
                    continue
                d = np.sqrt(np.sum((a - acc_ref) ** 2, axis=0))
                assert np.max(d / B) <= 1.0, (v, want_pot, np.max(d / B))
                if want_pot:
                    assert np.max(np.abs(host(pot) - pot_ref) / np.abs(pot_ref)) <= 1e-6, v
    finally:
        nb.restore_tile_table()


def test_adaptive_plummer_and_determinism(nb, oracle):
    """A Plummer sphere at eps = 1e-3 on the tuned tile: every particle within the bound of the
    adaptive mode (checked against the oracle on a sample that includes the worst particles
    against the FP64 GPU path), below the compensated mode's error, and bitwise repeatable."""
    import torch
    n, eps = 40000, 1e-3
    s = inputs.plummer(n, 901)
    x, m = dev(s.pos), dev(s.mass)
    a64, _ = nb.forces(x, m, eps=eps, precision="fp64")
    mag = torch.sqrt((a64 ** 2).sum(0))
    floor = 1e-6 * float(torch.sqrt((mag ** 2).mean()))
    errs = {}
    for prec in ("fp32a", "fp32c"):
        a, _ = nb.forces(x, m, eps=eps, precision=prec)
        errs[prec] = host(torch.sqrt(((a - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor))
    a1, p1 = nb.forces(x, m, eps=eps, precision="fp32a", want_pot=True)
    a2, p2 = nb.forces(x, m, eps=eps, precision="fp32a", want_pot=True)
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    print("plummer 40k eps 1e-3: fp32a max e %.3e, fp32c max e %.3e" % (errs["fp32a"].max(), errs["fp32c"].max()))
    assert errs["fp32a"].max() <= 1e-5
    assert errs["fp32a"].max() < errs["fp32c"].max()
    g = np.random.Generator(np.random.PCG64(902))
    idx = np.unique(np.concatenate([np.argsort(errs["fp32a"])[-64:], g.choice(n, 64, replace=False), [0, n - 1]]))
    ref, _ = oracle.forces_sample(s.pos, s.mass, idx, eps=eps)
    from oracle import bounds
    B = bounds.fp32_force_bound(s.pos, s.mass, eps, adaptive=True, idx=idx)
    d = np.sqrt(np.sum((host(a1)[:, idx] - ref) ** 2, axis=0))
    assert np.max(d / B) <= 1.0, np.max(d / B)


def test_adaptive_degenerate_inputs(nb):
    """All particles at one point (zero-extent box: every Morton code equal, the order is the
    index order) give a = 0 exactly and phi_i = -G (M - m_i) / eps; particles on a line (two
    zero-extent axes) match the compensated mode within its own rounding."""
    n = 3000
    g = np.random.Generator(np.random.PCG64(903))
    mass = g.uniform(0.5, 1.5, n) / n
    pos = np.tile(np.array([[0.3], [-0.2], [0.7]]), (1, n))
    acc, pot = nb.forces(dev(pos), dev(mass), G=1.7, eps=0.05, precision="fp32a", want_pot=True)
    assert np.all(host(acc) == 0)
    np.testing.assert_allclose(host(pot), -1.7 * (mass.sum() - mass) / 0.05, rtol=1e-6)
    line = np.zeros((3, n))
    line[0] = g.uniform(-1, 1, n)
    a_a, _ = nb.forces(dev(line), dev(mass), eps=0.05, precision="fp32a")
    a_c, _ = nb.forces(dev(line), dev(mass), eps=0.05, precision="fp32c")
    assert np.all(host(a_a)[1:] == 0)
    np.testing.assert_allclose(host(a_a), host(a_c), rtol=1e-5, atol=1e-6 * np.abs(host(a_c)).max())


def test_adaptive_rollout_consistency(nb, oracle):
    """Rollouts in the adaptive mode (symmetric tile forced at n = 6000): five single steps equal
    a five-step rollout bitwise, the energy trace leaves the trajectory unchanged, the backward
    pass is bitwise independent of the checkpoint interval, and the state stays within rounding
    of the oracle."""
    n = 6000
    s = inputs.plummer(n, 904)
    v = _sym_variants(nb)[1]
    try:
        nb.set_tile_table([dict(kernel="force", precision="fp32a", n_min=0, n_max=1 << 40, variant=v, j_split=1)])
        p1, v1, m = dev(s.pos), dev(s.vel), dev(s.mass)
        a1, _ = nb.forces(p1, m, precision="fp32a")
        p2, v2, a2 = p1.clone(), v1.clone(), a1.clone()
        p3, v3, a3 = p1.clone(), v1.clone(), a1.clone()
        for _ in range(5):
            nb.step(p1, v1, m, a1, 1e-3, precision="fp32a")
        nb.rollout(p2, v2, m, a2, 1e-3, 5, precision="fp32a")
        _, tr = nb.rollout(p3, v3, m, a3, 1e-3, 5, energy_trace=True, precision="fp32a")
        assert np.array_equal(host(p1), host(p2)) and np.array_equal(host(v1), host(v2))
        assert np.array_equal(host(p1), host(p3)) and np.array_equal(host(v1), host(v3))
        xr, _, _, er = oracle.kdk(s.pos, s.vel, s.mass, 1e-3, 5, eps=1e-2, want_energy=True)
        assert np.max(np.abs(host(p1) - xr)) / math.sqrt(np.mean(s.pos ** 2)) <= 1e-6
        E, Er = host(tr)[:, 0, 0] + host(tr)[:, 0, 1], er[:, 0] + er[:, 1]
        assert np.max(np.abs(E - Er) / abs(Er[0])) <= 1e-6
        gxK = np.random.Generator(np.random.PCG64(905)).normal(size=(3, n))
        res = []
        for ck in (1, 2, 5):
            pos, vel = dev(s.pos), dev(s.vel)
            acc, _ = nb.forces(pos, m, precision="fp32a")
            ckpt, _ = nb.rollout(pos, vel, m, acc, 1e-3, 5, ckpt_every=ck, precision="fp32a")
            res.append([host(t) for t in nb.rollout_backward(m, ckpt, dev(gxK), dev(np.zeros((3, n))), 1e-3, 5, ck,
                                                             precision="fp32a")])
        for r in res[1:]:
            for a, b in zip(r, res[0]):
                assert np.array_equal(a, b)
    finally:
        nb.restore_tile_table()


def test_adaptive_lennard_jones(nb, oracle):
    """The Lennard-Jones gas in the adaptive mode (symmetric tile forced): forces against the
    oracle no worse than the compensated mode's, and a 20-step rollout with walls within
    rounding of the oracle."""
    g, box = inputs.lj_gas(4000, 906, spacing=1.2)
    v = _sym_variants(nb)[1]
    try:
        nb.set_tile_table([dict(kernel="lj_force", precision="fp32a", n_min=0, n_max=1 << 40, variant=v, j_split=1)])
        acc, pot = nb.lj_forces(dev(g.pos), dev(g.mass), precision="fp32a", want_pot=True)
        a_r, p_r = oracle.lj_forces(g.pos, g.mass)
        a_c, _ = nb.lj_forces(dev(g.pos), dev(g.mass), precision="fp32c")
        # the gas's forces cancel to near zero on lattice sites: compare with the scale of the terms
        scale = np.abs(a_r).max()
        assert np.max(np.abs(host(acc) - a_r)) <= 2 * np.max(np.abs(host(a_c) - a_r)) + 1e-7 * scale
        pos, vel, m = dev(g.pos), dev(g.vel), dev(g.mass)
        a0, _ = nb.lj_forces(pos, m, precision="fp32a")
        nb.lj_rollout(pos, vel, m, a0, 2e-3, 20, box=(box.lo, box.hi), precision="fp32a")
        pr, _, _ = oracle.lj_kdk(g.pos, g.vel, g.mass, 2e-3, 20, box=(box.lo, box.hi))
        assert np.max(np.abs(host(pos) - pr)) <= 1e-6
    finally:
        nb.restore_tile_table()


def test_adaptive_other_paths_run_double_float(nb):
    """Where the adaptive mode does not sort (batches, one-sided passes) it runs as the
    double-float mode: results bitwise equal to fp32ds."""
    b = inputs.batched_mix(6, 907, nmin=64, nmax=1500)
    a_a, p_a = nb.forces(dev(b.pos), dev(b.mass), precision="fp32a", want_pot=True, offsets=b.offsets)
    a_d, p_d = nb.forces(dev(b.pos), dev(b.mass), precision="fp32ds", want_pot=True, offsets=b.offsets)
    assert np.array_equal(host(a_a), host(a_d)) and np.array_equal(host(p_a), host(p_d))
    s = inputs.plummer(1500, 908)  # one-sided at this size with the tuned tiles
    vid, _ = nb.tile_lookup("force", "fp32a", 1500)
    assert "sym=" not in nb.tile_variants("force", "fp32a")[vid]
    a_a, _ = nb.forces(dev(s.pos), dev(s.mass), precision="fp32a")
    a_d, _ = nb.forces(dev(s.pos), dev(s.mass), precision="fp32ds")
    assert np.array_equal(host(a_a), host(a_d))
