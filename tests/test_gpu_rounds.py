"""The round schedule of the symmetric force pass: tiles of 1024-particle blocks in rounds of
disjoint block pairs, each tile adding its sums to per-particle double accumulators (workspace
linear in n). Forced with NBODY_FLAG_SYM_ROUNDS at small sizes; taken by the library itself
where the slot schedule's partial sums would exceed its cap (checked at 1.6M particles).

Against the oracle every particle is held to its FP32 rounding bound (oracle/bounds.py, the
same bound as the slot schedule: the sums are the same float tile sums, added in double);
potentials within the per-mode relative tolerance of the parity tests."""
import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu

TOL_P = {"fp32c": 1e-6, "fp32": 1e-5, "fp32ds": 1e-6, "fp32a": 1e-6}


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2511_02655_amd as m
    m.lib()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _bound(pos, mass, eps, prec, idx=None):
    from oracle import bounds
    if prec == "fp32a":
        return bounds.fp32_force_bound(pos, mass, eps, adaptive=True, idx=idx)
    return bounds.fp32_force_bound(pos, mass, eps, accumulate_plain=(prec == "fp32"),
                                   exact_coords=(prec == "fp32ds"), idx=idx)


@pytest.mark.parametrize("n", [1, 2, 100, 1023, 1024, 1025, 2048, 2049, 5000])
def test_rounds_vs_oracle(nb, oracle, n):
    """Sizes below, at and across one and two blocks (odd and even block counts: the padding
    block of the circle method), every FP32 mode (the adaptive one sorted, on its adaptive
    tiles), with and without the potential."""
    s = inputs.uniform_cube(n, 1200 + n)
    a_r, p_r = oracle.forces(s.pos, s.mass, eps=1e-2)
    for prec in ("fp32c", "fp32", "fp32ds", "fp32a"):
        B = _bound(s.pos, s.mass, 1e-2, prec) if n > 1 else None
        for want_pot in (True, False):
            a, p = nb.forces(dev(s.pos), dev(s.mass), eps=1e-2, precision=prec, want_pot=want_pot,
                             flags=nb.FLAG_SYM_ROUNDS)
            a = host(a)
            if n == 1:
                assert np.all(a == 0)
                continue
            d = np.sqrt(np.sum((a - a_r) ** 2, axis=0))
            assert np.max(d / B) <= 1.0, (prec, want_pot, float(np.max(d / B)))
            if want_pot:
                assert np.max(np.abs(host(p) - p_r) / np.abs(p_r)) <= TOL_P[prec], prec


def test_rounds_lennard_jones_vs_oracle(nb, oracle):
    """The Lennard-Jones law on the round schedule, held to the Lennard-Jones parity checks."""
    from test_gpu_lj import _gas, check_lj
    for n in (100, 3000):
        pos, mass, _, _ = _gas(n, 1201 + n)
        a_r, p_r = oracle.lj_forces(pos, mass, 1.1, 0.7)
        for prec in ("fp32c", "fp32", "fp32ds", "fp32a"):
            a, p = nb.lj_forces(dev(pos), dev(mass), sigma=1.1, epsilon=0.7, precision=prec, want_pot=True,
                                flags=nb.FLAG_SYM_ROUNDS)
            # the adaptive mode's separations are never worse than the compensated mode's float
            # ones (exact on near sub-block pairs), so the compensated bound holds for it
            check_lj(host(a), host(p), a_r, p_r, pos, mass, "fp32c" if prec == "fp32a" else prec, sigma=1.1,
                     epsilon=0.7)


def test_rounds_deterministic_and_consistent(nb):
    """Repeated calls are bitwise equal; a step's accelerations and potential are bitwise those of
    a force pass at the new positions; trajectories do not depend on the energy trace; in the
    adaptive mode five single steps equal a five-step rollout, with and without the trace."""
    import torch
    n = 7000
    s = inputs.plummer(n, 1202)
    x, m = dev(s.pos), dev(s.mass)
    F = nb.FLAG_SYM_ROUNDS
    a1, p1 = nb.forces(x, m, precision="fp32c", want_pot=True, flags=F)
    a2, p2 = nb.forces(x, m, precision="fp32c", want_pot=True, flags=F)
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    pos, vel = dev(s.pos), dev(s.vel)
    acc = a1.clone()
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    nb.step(pos, vel, m, acc, 1e-3, precision="fp32c", out_pot=pot, flags=F)
    a3, p3 = nb.forces(pos, m, precision="fp32c", want_pot=True, flags=F)
    assert torch.equal(acc, a3) and torch.equal(pot, p3)
    outs = []
    for trace in (False, True):
        p_, v_ = dev(s.pos), dev(s.vel)
        nb.rollout(p_, v_, m, a1.clone(), 1e-3, 5, energy_trace=trace, precision="fp32c", flags=F)
        outs.append((host(p_), host(v_)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    b1, q1 = nb.forces(x, m, precision="fp32a", want_pot=True, flags=F)
    b2, q2 = nb.forces(x, m, precision="fp32a", want_pot=True, flags=F)
    assert torch.equal(b1, b2) and torch.equal(q1, q2)
    p1, v1 = dev(s.pos), dev(s.vel)
    a_s = b1.clone()
    for _ in range(5):
        nb.step(p1, v1, m, a_s, 1e-3, precision="fp32a", flags=F)
    for trace in (False, True):
        p_, v_ = dev(s.pos), dev(s.vel)
        nb.rollout(p_, v_, m, b1.clone(), 1e-3, 5, energy_trace=trace, precision="fp32a", flags=F)
        assert torch.equal(p_, p1) and torch.equal(v_, v1), trace


def test_rounds_match_slots(nb):
    """At N = 40 000 the round schedule and the slot schedule agree within FP32 rounding of
    the separate sums (both against the FP64 GPU path)."""
    import torch
    s = inputs.plummer(40000, 1203)
    x, m = dev(s.pos), dev(s.mass)
    a64, _ = nb.forces(x, m, precision="fp64")
    mag = torch.sqrt((a64 ** 2).sum(0))
    floor = 1e-6 * float(torch.sqrt((mag ** 2).mean()))
    for prec in ("fp32c", "fp32ds", "fp32a"):
        ar, _ = nb.forces(x, m, precision=prec, flags=nb.FLAG_SYM_ROUNDS)
        asl, _ = nb.forces(x, m, precision=prec)
        er = float(torch.max(torch.sqrt(((ar - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor)))
        es = float(torch.max(torch.sqrt(((asl - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor)))
        assert er <= 1e-5 and es <= 1e-5, (prec, er, es)


def test_rounds_taken_beyond_the_slot_cap(nb, oracle):
    """N = 1.6M: the tuned tile's partial sums would exceed the library's 16 GiB cap, so the pass
    runs on the round schedule by itself (bitwise equal to forcing it); sampled particles,
    including the worst against the FP64 GPU path, against the oracle within their bounds."""
    import torch
    n = 1600000
    s = inputs.plummer(n, 1204)
    x, m = dev(s.pos), dev(s.mass)
    a, _ = nb.forces(x, m, eps=1e-2, precision="fp32c")
    af, _ = nb.forces(x, m, eps=1e-2, precision="fp32c", flags=nb.FLAG_SYM_ROUNDS)
    assert torch.equal(a, af)
    a64, _ = nb.forces(x, m, eps=1e-2, precision="fp64")
    d = host(torch.sqrt(((a - a64) ** 2).sum(0)))
    g = np.random.Generator(np.random.PCG64(1205))
    idx = np.unique(np.concatenate([np.argsort(d)[-32:], g.choice(n, 32, replace=False)]))
    ref, _ = oracle.forces_sample(s.pos, s.mass, idx, eps=1e-2)
    B = _bound(s.pos, s.mass, 1e-2, "fp32c", idx=idx)
    dd = np.sqrt(np.sum((host(a)[:, idx] - ref) ** 2, axis=0))
    assert np.max(dd / B) <= 1.0, float(np.max(dd / B))


def test_adaptive_rounds_beyond_the_slot_cap(nb, oracle):
    """N = 1.6M at eps = 1e-3 in the adaptive mode, which the library runs on the round schedule
    (sorted, adaptive tiles): every particle within 1e-5 of the FP64 GPU path, and sampled
    particles, including the worst, against the oracle within the adaptive mode's bound."""
    import torch
    n, eps = 1600000, 1e-3
    s = inputs.plummer(n, 1208)
    x, m = dev(s.pos), dev(s.mass)
    a, _ = nb.forces(x, m, eps=eps, precision="fp32a")
    af, _ = nb.forces(x, m, eps=eps, precision="fp32a", flags=nb.FLAG_SYM_ROUNDS)
    assert torch.equal(a, af)
    a64, _ = nb.forces(x, m, eps=eps, precision="fp64")
    mag = torch.sqrt((a64 ** 2).sum(0))
    floor = 1e-6 * float(torch.sqrt((mag ** 2).mean()))
    e = host(torch.sqrt(((a - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor))
    print("adaptive rounds 1.6M eps 1e-3: max e %.3e" % e.max())
    assert e.max() <= 1e-5
    g = np.random.Generator(np.random.PCG64(1209))
    idx = np.unique(np.concatenate([np.argsort(e)[-32:], g.choice(n, 32, replace=False)]))
    ref, _ = oracle.forces_sample(s.pos, s.mass, idx, eps=eps)
    B = _bound(s.pos, s.mass, eps, "fp32a", idx=idx)
    dd = np.sqrt(np.sum((host(a)[:, idx] - ref) ** 2, axis=0))
    assert np.max(dd / B) <= 1.0, float(np.max(dd / B))


def test_rounds_from_two_threads_on_two_streams(nb):
    """Round-schedule passes and steps issued at once from two host threads, each on its own
    stream (both share the library's two round streams, each call ordered by its own events):
    every result equals the same calls made alone, bitwise."""
    import threading

    import torch
    F = nb.FLAG_SYM_ROUNDS
    systems = [inputs.plummer(5000, 1206), inputs.plummer(20000, 1207)]
    data = [(dev(s.pos), dev(s.vel), dev(s.mass)) for s in systems]
    torch.cuda.synchronize()  # the inputs, made on the default stream, are read from others

    def work(k, stream, out):
        p0, v0, m = data[k]
        with torch.cuda.stream(stream):
            for _ in range(3):
                a, pot = nb.forces(p0, m, precision="fp32c", want_pot=True, flags=F, stream=stream)
                p, v = p0.clone(), v0.clone()
                nb.rollout(p, v, m, a.clone(), 1e-3, 3, precision="fp32c", flags=F, stream=stream)
                out.append((a, pot, p, v))
            stream.synchronize()

    alone = []
    for k in range(2):
        o = []
        work(k, torch.cuda.Stream(), o)
        alone.append(o[0])
    outs = [[], []]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    threads = [threading.Thread(target=work, args=(k, streams[k], outs[k])) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    for k in range(2):
        assert len(outs[k]) == 3
        for got in outs[k]:
            for x, y in zip(got, alone[k]):
                assert torch.equal(x, y), k


@pytest.mark.parametrize("n", [100, 1025, 3000])
def test_rounds_adjoint_vs_oracle(nb, oracle, n):
    """The adjoint pass on the round schedule (NBODY_FLAG_SYM_ROUNDS on the backward): a
    one-step backward (two adjoint passes) in every FP32 mode against the oracle's discrete
    adjoint, rel-L2 and per particle as the symmetric adjoint's parity test; bitwise repeatable;
    the checkpoint interval leaves a 6-step backward bitwise unchanged."""
    from test_gpu_parity import _grad_ok
    s = inputs.plummer(n, 1210 + n)
    g = np.random.Generator(np.random.PCG64(1211))
    gxK, gvK = g.normal(size=(3, n)), g.normal(size=(3, n))
    ref = oracle.rollout_adjoint(s.pos, s.vel, s.mass, 1e-3, 1, gxK, gvK, eps=1e-2)
    tol = {"fp32c": 1e-4, "fp32": 1e-3, "fp32ds": 1e-4}
    F = nb.FLAG_SYM_ROUNDS
    for prec in ("fp32c", "fp32", "fp32ds"):
        pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
        acc, _ = nb.forces(pos, mass, precision=prec, flags=F)
        ckpt, _ = nb.rollout(pos, vel, mass, acc, 1e-3, 1, ckpt_every=1, precision=prec, flags=F)
        out = [host(t) for t in nb.rollout_backward(mass, ckpt, dev(gxK), dev(gvK), 1e-3, 1, 1, precision=prec,
                                                     flags=F)]
        for a, b in zip(out, ref):
            _grad_ok(a, b, tol[prec], "rounds %s n=%d" % (prec, n))
        out2 = [host(t) for t in nb.rollout_backward(mass, ckpt, dev(gxK), dev(gvK), 1e-3, 1, 1, precision=prec,
                                                      flags=F)]
        for a, b in zip(out, out2):
            assert np.array_equal(a, b)
    res = []
    for ck in (1, 3, 6):
        pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
        acc, _ = nb.forces(pos, mass, precision="fp32c", flags=F)
        ckpt, _ = nb.rollout(pos, vel, mass, acc, 1e-3, 6, ckpt_every=ck, precision="fp32c", flags=F)
        res.append([host(t) for t in nb.rollout_backward(mass, ckpt, dev(gxK), dev(gvK), 1e-3, 6, ck,
                                                         precision="fp32c", flags=F)])
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            assert np.array_equal(a, b)


def test_adjoint_rounds_beyond_the_slot_cap(nb):
    """N = 1.1M: the tuned symmetric adjoint tile's slots would exceed the 16 GiB cap, so the
    adjoint pass runs on the round schedule by itself (bitwise equal to forcing it) and agrees
    with the FP64 backward within the FP32 gradient tolerance."""
    import torch
    n = 1100000
    s = inputs.plummer(n, 1212)
    g = np.random.Generator(np.random.PCG64(1213))
    gxK = dev(g.normal(size=(3, n)))
    gvK = torch.zeros_like(gxK)
    outs = {}
    for prec, fl in (("fp32c", 0), ("fp32c", nb.FLAG_SYM_ROUNDS), ("fp64", 0)):
        pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
        acc, _ = nb.forces(pos, mass, precision=prec, flags=fl)
        ckpt, _ = nb.rollout(pos, vel, mass, acc, 1e-3, 1, ckpt_every=1, precision=prec, flags=fl)
        outs[(prec, fl)] = nb.rollout_backward(mass, ckpt, gxK, gvK, 1e-3, 1, 1, precision=prec, flags=fl)
        del ckpt
        torch.cuda.empty_cache()
    for a, b in zip(outs[("fp32c", 0)], outs[("fp32c", nb.FLAG_SYM_ROUNDS)]):
        assert torch.equal(a, b)
    for a, b in zip(outs[("fp32c", 0)], outs[("fp64", 0)]):
        rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        assert rel <= 1e-4, rel


def test_rounds_per_system_loop(nb, oracle):
    """Batches whose systems are looped one by one (NBODY_FLAG_LOOP_SYSTEMS) run each system on
    the round schedule with the flag: forces of every system against the oracle within its
    bound, and a 3-step rollout plus its backward equal, system by system, the same calls on the
    systems alone, bitwise. Without the loop flag the batched kernels ignore it (bitwise equal)."""
    import torch
    b = inputs.batched_mix(4, 1214, nmin=300, nmax=3000)
    off = b.offsets
    F = nb.FLAG_SYM_ROUNDS
    L = nb.FLAG_LOOP_SYSTEMS
    x, v, m = dev(b.pos), dev(b.vel), dev(b.mass)
    a, _ = nb.forces(x, m, precision="fp32c", offsets=off, flags=F | L)
    a_b, _ = nb.forces(x, m, precision="fp32c", offsets=off, flags=F)
    a_n, _ = nb.forces(x, m, precision="fp32c", offsets=off)
    assert torch.equal(a_b, a_n)
    g = np.random.Generator(np.random.PCG64(1215))
    gxK = g.normal(size=b.pos.shape)
    for k in range(len(off) - 1):
        lo, hi = int(off[k]), int(off[k + 1])
        a_r, _ = oracle.forces(b.pos[:, lo:hi], b.mass[lo:hi], eps=1e-2)
        B = _bound(b.pos[:, lo:hi], b.mass[lo:hi], 1e-2, "fp32c")
        d = np.sqrt(np.sum((host(a)[:, lo:hi] - a_r) ** 2, axis=0))
        assert np.max(d / B) <= 1.0, (k, float(np.max(d / B)))
    p, vv = x.clone(), v.clone()
    ckpt, _ = nb.rollout(p, vv, m, a.clone(), 1e-3, 3, ckpt_every=1, precision="fp32c", offsets=off, flags=F | L)
    grads = nb.rollout_backward(m, ckpt, dev(gxK), torch.zeros_like(x), 1e-3, 3, 1, precision="fp32c", offsets=off,
                                flags=F | L)
    for k in range(len(off) - 1):
        lo, hi = int(off[k]), int(off[k + 1])
        xs, vs, ms = x[:, lo:hi].contiguous(), v[:, lo:hi].contiguous(), m[lo:hi].contiguous()
        a1, _ = nb.forces(xs, ms, precision="fp32c", flags=F)
        assert torch.equal(a1, a[:, lo:hi].contiguous()), k
        ps, vs2 = xs.clone(), vs.clone()
        ck1, _ = nb.rollout(ps, vs2, ms, a1.clone(), 1e-3, 3, ckpt_every=1, precision="fp32c", flags=F)
        assert torch.equal(ps, p[:, lo:hi].contiguous()) and torch.equal(vs2, vv[:, lo:hi].contiguous()), k
        g1 = nb.rollout_backward(ms, ck1, dev(gxK[:, lo:hi]), torch.zeros_like(xs), 1e-3, 3, 1, precision="fp32c",
                                 flags=F)
        for u, w in zip(g1, grads):
            ww = w[..., lo:hi].contiguous()
            assert torch.equal(u, ww), k
