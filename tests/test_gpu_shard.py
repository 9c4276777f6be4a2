"""One GPU's share of the paper's ring decomposition (nbody_forces_shard, Sec. V-B and Fig. 1):
block g of P against all n particles, one double partial per j-block added in block order.

Checked: the P shares together are bitwise the full one-sided call with P j-ranges (acc and
pot, every FP32 mode and FP64, ragged sizes, fewer blocks than P); each share against the oracle
within the per-particle FP32 bound (FP64: 1e-12); rows outside the share untouched; and the real
shape of one of 8 GPUs at N = 1,048,576 (131 072 x 1 048 576) on sampled rows against the oracle
and bitwise against the full call."""
import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_02655_amd as m
    m.lib()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _full(nb, x, m, prec, P, eps=1e-2):
    """nbody_forces on the one-sided tile variant 0 with P j-ranges."""
    try:
        nb.set_tile_table([dict(kernel="force", precision=prec, n_min=0, n_max=1 << 40, variant=0, j_split=P)])
        return nb.forces(x, m, eps=eps, precision=prec, want_pot=True)
    finally:
        nb.restore_tile_table()


@pytest.mark.parametrize("n", [1000, 5000, 70001])
def test_shares_assemble_the_full_call(nb, n):
    import torch
    s = inputs.plummer(n, 1300 + n)
    x, m = dev(s.pos), dev(s.mass)
    for prec in ("fp64", "fp32c", "fp32", "fp32ds"):
        for P in (1, 3, 8):
            a_f, p_f = _full(nb, x, m, prec, P)
            acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
            pot = torch.zeros(n, dtype=torch.float64, device="cuda")
            covered = 0
            for g in range(P):
                _, _, (i0, i1) = nb.forces_shard(x, m, P, g, precision=prec, want_pot=True, out_acc=acc, out_pot=pot)
                assert i0 == min(n, covered) and i1 >= i0
                covered = i1
            assert covered == n
            assert torch.equal(acc, a_f) and torch.equal(pot, p_f), (prec, P)


def test_share_vs_oracle(nb, oracle):
    """Each of 4 shares of a 3000-particle cube against the oracle: FP32 within the per-particle
    bound, FP64 within 1e-12 relative; the rows outside the share stay as they were."""
    from oracle import bounds
    import torch
    n, P = 3000, 4
    s = inputs.uniform_cube(n, 1301)
    a_r, p_r = oracle.forces(s.pos, s.mass, eps=1e-2)
    x, m = dev(s.pos), dev(s.mass)
    B = bounds.fp32_force_bound(s.pos, s.mass, 1e-2)
    mag = np.sqrt(np.sum(a_r ** 2, axis=0))
    for prec in ("fp32c", "fp64"):
        for g in range(P):
            acc = torch.full((3, n), 7.0, dtype=torch.float64, device="cuda")
            pot = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
            _, _, (i0, i1) = nb.forces_shard(x, m, P, g, precision=prec, want_pot=True, out_acc=acc, out_pot=pot)
            a, p = host(acc), host(pot)
            out = np.ones(n, dtype=bool)
            out[i0:i1] = False
            assert np.all(a[:, out] == 7.0) and np.all(p[out] == 7.0)
            d = np.sqrt(np.sum((a[:, i0:i1] - a_r[:, i0:i1]) ** 2, axis=0))
            if prec == "fp64":
                assert np.max(d / mag[i0:i1]) <= 1e-12
                assert np.max(np.abs(p[i0:i1] - p_r[i0:i1]) / np.abs(p_r[i0:i1])) <= 1e-12
            else:
                assert np.max(d / B[i0:i1]) <= 1.0, (g, float(np.max(d / B[i0:i1])))
                assert np.max(np.abs(p[i0:i1] - p_r[i0:i1]) / np.abs(p_r[i0:i1])) <= 1e-6


def test_share_at_the_real_shape(nb, oracle):
    """Share 3 of 8 at N = 1,048,576 (the share of one of 8 GPUs: 131 072 particles against all):
    rows [393 216, 524 288) only, sampled rows against the oracle within the FP32 bound, and
    bitwise the full one-sided call's rows."""
    from oracle import bounds
    import torch
    n, P, g = 1 << 20, 8, 3
    s = inputs.plummer(n, 1302)
    x, m = dev(s.pos), dev(s.mass)
    acc, _, (i0, i1) = nb.forces_shard(x, m, P, g, eps=1e-3, precision="fp32c")
    assert (i0, i1) == (393216, 524288)
    a = host(acc)
    assert np.all(a[:, :i0] == 0) and np.all(a[:, i1:] == 0)
    a_f, _ = _full(nb, x, m, "fp32c", P, eps=1e-3)
    assert torch.equal(acc[:, i0:i1], a_f[:, i0:i1])
    rng = np.random.Generator(np.random.PCG64(1303))
    idx = np.sort(rng.choice(np.arange(i0, i1), 48, replace=False))
    ref, _ = oracle.forces_sample(s.pos, s.mass, idx, eps=1e-3)
    B = bounds.fp32_force_bound(s.pos, s.mass, 1e-3, idx=idx)
    d = np.sqrt(np.sum((a[:, idx] - ref) ** 2, axis=0))
    assert np.max(d / B) <= 1.0, float(np.max(d / B))
