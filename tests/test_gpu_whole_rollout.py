"""Whole batched rollout in one launch (NBODY_FLAG_WHOLE_ROLLOUT): systems advance
independently through a task queue with per-system waits, running the same tile and
per-particle code as one launch per pass, so the trajectory must be bitwise that of the
per-step path (which the other GPU tests pin to the oracle), and within FP32 rounding of
the oracle itself.
"""
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


def _sym_batched(nb, prec="fp32c"):
    return [k for k, d in enumerate(nb.tile_variants("force_batched", prec)) if "sym=" in d]


def _mixed_batch(seed):
    """Empty, single-particle, two-particle and ragged systems across tile edges."""
    g = np.random.Generator(np.random.PCG64(seed))
    sizes = [0, 1, 2, 700, 0, 1500, 64, 2049, 3, 1100, 5, 0]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    pos = g.normal(size=(3, n))
    vel = g.normal(size=(3, n)) * 0.1
    mass = g.uniform(0.5, 1.5, n) / 1000
    return off, pos, vel, mass


def _run(nb, off, pos, vel, mass, steps, flags, prec, **kw):
    p, v, m = dev(pos), dev(vel), dev(mass)
    a, _ = nb.forces(p, m, eps=1e-2, precision=prec, offsets=off)
    out = nb.rollout(p, v, m, a, 1e-3, steps, eps=1e-2, precision=prec, offsets=off, flags=flags, **kw)
    return host(p), host(v), host(a), out


@pytest.mark.parametrize("prec", ["fp32c", "fp32", "fp32ds"])
def test_whole_rollout_bitwise_equals_per_step(nb, prec):
    """Every symmetric batched variant, every FP32 mode: positions, velocities and final
    accelerations bitwise equal to one launch per pass, over 7 steps of a ragged batch."""
    off, pos, vel, mass = _mixed_batch(1)
    try:
        for v in _sym_batched(nb, prec):
            nb.set_tile_table([dict(kernel="force_batched", precision=prec, n_min=0, n_max=1 << 40, variant=v,
                                    j_split=1)])
            ref = _run(nb, off, pos, vel, mass, 7, nb.FLAG_PER_PASS, prec)
            got = _run(nb, off, pos, vel, mass, 7, nb.FLAG_WHOLE_ROLLOUT, prec)
            for a, b in zip(ref[:3], got[:3]):
                assert np.array_equal(a, b), (v, prec)
    finally:
        nb.restore_tile_table()


def test_whole_rollout_vs_oracle(nb, oracle):
    """Against the oracle per system (20 steps, FP32 compensated): the same FP32 bound as the
    per-step batched rollout."""
    off, pos, vel, mass = _mixed_batch(2)
    x, _, _, _ = _run(nb, off, pos, vel, mass, 20, nb.FLAG_WHOLE_ROLLOUT, "fp32c")
    for s in range(len(off) - 1):
        sl = slice(off[s], off[s + 1])
        if off[s + 1] == off[s]:
            continue
        xr, _, _, _ = oracle.kdk(pos[:, sl], vel[:, sl], mass[sl], 1e-3, 20, eps=1e-2)
        assert np.max(np.abs(x[:, sl] - xr)) <= 1e-6 * max(1.0, float(np.max(np.abs(xr))))


@pytest.mark.parametrize("steps", [0, 1, 2])
def test_whole_rollout_few_steps(nb, steps):
    off, pos, vel, mass = _mixed_batch(3)
    ref = _run(nb, off, pos, vel, mass, steps, nb.FLAG_PER_PASS, "fp32c")
    got = _run(nb, off, pos, vel, mass, steps, nb.FLAG_WHOLE_ROLLOUT, "fp32c")
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)


def test_whole_rollout_flag_ignored_where_it_does_not_apply(nb):
    """Energy trace, checkpoints, a single system, the FP64 path (one-sided batched units)
    and the per-system loop run as before with the flag set."""
    import torch
    off, pos, vel, mass = _mixed_batch(4)
    W = nb.FLAG_WHOLE_ROLLOUT
    ref = _run(nb, off, pos, vel, mass, 5, 0, "fp32c", energy_trace=True)
    got = _run(nb, off, pos, vel, mass, 5, W, "fp32c", energy_trace=True)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(host(ref[3][1]), host(got[3][1]))
    ref = _run(nb, off, pos, vel, mass, 6, 0, "fp32c", ckpt_every=3)
    got = _run(nb, off, pos, vel, mass, 6, W, "fp32c", ckpt_every=3)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(host(ref[3][0]), host(got[3][0]))
    for prec in ("fp64",):
        ref = _run(nb, off, pos, vel, mass, 4, 0, prec)
        got = _run(nb, off, pos, vel, mass, 4, W, prec)
        assert np.array_equal(ref[0], got[0])
    ref = _run(nb, off, pos, vel, mass, 4, nb.FLAG_LOOP_SYSTEMS, "fp32c")
    got = _run(nb, off, pos, vel, mass, 4, nb.FLAG_LOOP_SYSTEMS | W, "fp32c")
    assert np.array_equal(ref[0], got[0])
    s = inputs.plummer(3000, 5)
    outs = []
    for flags in (0, W):
        p, v, m = dev(s.pos), dev(s.vel), dev(s.mass)
        a, _ = nb.forces(p, m, precision="fp32c")
        nb.rollout(p, v, m, a, 1e-3, 4, precision="fp32c", flags=flags)
        outs.append(host(p))
    assert np.array_equal(outs[0], outs[1])
    del torch


def test_whole_rollout_lennard_jones_walls(nb):
    """Batched Lennard-Jones gases with reflective walls (the walls are per call): bitwise
    equal to the per-step path, and every particle stays in its box."""
    gases = [inputs.lj_gas(n, 40 + n, spacing=1.2, temperature=2.0) for n in (500, 1300, 90)]
    lo = np.min([b.lo for _, b in gases], axis=0)
    hi = np.max([b.hi for _, b in gases], axis=0)
    pos = np.concatenate([g.pos for g, _ in gases], axis=1)
    vel = np.concatenate([g.vel for g, _ in gases], axis=1)
    mass = np.concatenate([g.mass for g, _ in gases])
    off = np.zeros(len(gases) + 1, dtype=np.int64)
    off[1:] = np.cumsum([g.n for g, _ in gases])
    outs = []
    for flags in (nb.FLAG_PER_PASS, nb.FLAG_WHOLE_ROLLOUT):
        p, v, m = dev(pos), dev(vel), dev(mass)
        a, _ = nb.lj_forces(p, m, precision="fp32c", offsets=off)
        nb.lj_rollout(p, v, m, a, 2e-3, 30, box=(lo, hi), precision="fp32c", offsets=off, flags=flags)
        outs.append((host(p), host(v)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    x = outs[1][0]
    assert np.all(x >= lo[:, None]) and np.all(x <= hi[:, None])


@pytest.mark.parametrize("name,steps,reps", [("batch512", 50, 3), ("tiny", 50, 3)])
def test_whole_rollout_many_systems(nb, name, steps, reps):
    """The 512-system mix (N_s log-uniform in [64, 8192]) and 4096 systems of 16-300
    particles, 50 steps with the tuned tile, repeated: every repetition bitwise equal to one
    launch per pass (the cross-workgroup hand-offs must never expose stale data)."""
    b = inputs.make("batch512") if name == "batch512" else inputs.batched_mix(4096, 21, nmin=16, nmax=300)
    p, v, m = dev(b.pos), dev(b.vel), dev(b.mass)
    a, _ = nb.forces(p, m, eps=1e-2, precision="fp32c", offsets=b.offsets)
    nb.rollout(p, v, m, a, 1e-3, steps, eps=1e-2, precision="fp32c", offsets=b.offsets, flags=nb.FLAG_PER_PASS)
    ref = (host(p), host(v), host(a))
    for _ in range(reps):
        p, v, m = dev(b.pos), dev(b.vel), dev(b.mass)
        a, _ = nb.forces(p, m, eps=1e-2, precision="fp32c", offsets=b.offsets)
        nb.rollout(p, v, m, a, 1e-3, steps, eps=1e-2, precision="fp32c", offsets=b.offsets,
                   flags=nb.FLAG_WHOLE_ROLLOUT)
        for x, y in zip(ref, (host(p), host(v), host(a))):
            assert np.array_equal(x, y)


def test_single_tile_batches_take_one_launch_by_default(nb):
    """A batch whose systems all fit one tile runs every step in one launch without the flag
    (no waits, no read-back); the result is bitwise that of one launch per pass."""
    import torch
    b = inputs.batched_mix(2048, 31, nmin=8, nmax=200)
    outs = []
    for flags in (nb.FLAG_PER_PASS, 0):
        p, v, m = dev(b.pos), dev(b.vel), dev(b.mass)
        a, _ = nb.forces(p, m, eps=1e-2, precision="fp32c", offsets=b.offsets)
        nb.rollout(p, v, m, a, 1e-3, 30, eps=1e-2, precision="fp32c", offsets=b.offsets, flags=flags)
        torch.cuda.synchronize()
        outs.append((host(p), host(v), host(a)))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_whole_rollout_wait_limit_reports_error(nb):
    """Failure path, forced from the host: two large systems, so that a reduction task is
    taken while its system's tiles still run and must wait; with a one-probe wait limit it
    gives up, every workgroup leaves the launch, and the call returns the device error. With
    the default limit restored the same rollout completes and matches one launch per pass
    bitwise."""
    b = inputs.batched_mix(2, 41, nmin=6000, nmax=8192)

    def run(flags):
        p, v, m = dev(b.pos), dev(b.vel), dev(b.mass)
        a, _ = nb.forces(p, m, eps=1e-2, precision="fp32c", offsets=b.offsets)
        nb.rollout(p, v, m, a, 1e-3, 5, eps=1e-2, precision="fp32c", offsets=b.offsets, flags=flags)
        return host(p)

    sym = [k for k, d in enumerate(nb.tile_variants("force_batched", "fp32c")) if "sym=1024" in d][0]
    try:
        nb.set_tile_table([dict(kernel="force_batched", precision="fp32c", n_min=0, n_max=1 << 40, variant=sym,
                                j_split=1)])
        nb.set_wait_limit(1)
        with pytest.raises(nb.NBodyError) as ei:
            run(nb.FLAG_WHOLE_ROLLOUT)
        assert ei.value.code == 2 and "gave up" in str(ei.value)
        nb.set_wait_limit()
        assert np.array_equal(run(nb.FLAG_WHOLE_ROLLOUT), run(nb.FLAG_PER_PASS))
    finally:
        nb.set_wait_limit()
        nb.restore_tile_table()
