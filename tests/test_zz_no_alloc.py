"""nbody_step_noalloc (the allocation-free step: its workspace is the library's static device
scratch array) through the C ABI against nbody_step with a caller workspace, on calls in a row
(the second with a smaller system), bitwise.

The allocation-free step takes the first of: the tile nbody_step takes, the tile table's tile for
the largest systems, the round schedule, whose whole workspace fits the scratch; nbody_step is run
on that same tile (the tile table set to it) or schedule (NBODY_FLAG_SYM_ROUNDS). Each case checks
first, from nbody_workspace_size, that the choice it expects is the one the rule makes for its
size. The step is also captured into a HIP graph and replayed against eager steps."""
import ctypes

import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu

SCRATCH = 128 << 20     # NBODY_NOALLOC_SCRATCH_BYTES


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_02655_amd as nb
    nb.lib()
    return nb


def _fits(nb, n, prec, flags=0):
    """Whether one step's whole workspace (nbody_workspace_size) fits the scratch."""
    c = nb._Cfg(prec, flags=flags)
    b = ctypes.c_size_t()
    assert nb.lib().nbody_workspace_size(ctypes.byref(c.cfg), n, 1, 0, ctypes.byref(b)) == 0
    return b.value <= SCRATCH


def _expected_tile(nb, n, prec):
    """(variant, j_split, which) of the rule."""
    v, js = nb.tile_lookup("force", prec, n)
    if _fits(nb, n, prec):
        return v, js, "tuned"
    # the table's entry for the largest systems (its last bucket holds 1M particles)
    vb, jb = nb.tile_lookup("force", prec, 1 << 20)
    table_prec = "fp32c" if prec == "fp32a" else prec
    try:
        nb.set_tile_table([dict(kernel="force", precision=table_prec, n_min=0, n_max=1 << 40, variant=vb,
                                j_split=jb)])
        big = _fits(nb, n, prec)
    finally:
        nb.restore_tile_table()
    if big:
        return vb, jb, "largest block"
    assert _fits(nb, n, prec, nb.FLAG_SYM_ROUNDS)
    return None, None, "rounds"


def _two_steps(nb, step, n, prec, s, a0, **kw):
    import torch
    m = dev(s.mass)
    p, v, a = dev(s.pos), dev(s.vel), a0.clone()
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        step(p, v, m, a, 1e-3, precision=prec, out_pot=pot, **kw)
    torch.cuda.synchronize()
    return p, v, a, pot


def test_step_noalloc_matches_step(nb):
    cases = ((60000, "fp32c", "largest block"), (3000, "fp32c", "tuned"), (40000, "fp32a", "tuned"),
             (300000, "fp32c", "rounds"))
    for n, prec, which in cases:
        v, js, got = _expected_tile(nb, n, prec)
        assert got == which, (n, prec, got)
        print("step_noalloc n=%d %s: %s, variant %s" % (n, prec, which, v), flush=True)
        s = inputs.plummer(n, 950 + n)
        a0, _ = nb.forces(dev(s.pos), dev(s.mass), precision=prec)  # one starting acceleration for both
        table_prec = "fp32c" if prec == "fp32a" else prec
        try:
            if which == "largest block":
                nb.set_tile_table([dict(kernel="force", precision=table_prec, n_min=0, n_max=1 << 40, variant=v,
                                        j_split=js)])
            ref = _two_steps(nb, nb.step, n, prec, s, a0, flags=nb.FLAG_SYM_ROUNDS if which == "rounds" else 0)
        finally:
            nb.restore_tile_table()
        out = _two_steps(nb, nb.step_noalloc, n, prec, s, a0)
        import torch
        for r, o, name in zip(ref, out, ("pos", "vel", "acc", "pot")):
            assert torch.equal(r, o), (n, prec, name)


@pytest.mark.parametrize("n,prec", [(3000, "fp32c"), (40000, "fp32a"), (300000, "fp32c")])
def test_step_noalloc_graph_replays(nb, n, prec):
    """The step captured into a HIP graph (torch.cuda.graph on a side stream) and replayed: every
    replay equals the same step run eagerly, bitwise, with eager steps and synchronizations
    between the replays. Cases: the tuned one-sided tile, the adaptive mode's sort and symmetric
    tiles, the round schedule (whose launches go in order on the captured stream)."""
    import torch
    print("graph capture of step_noalloc n=%d %s" % (n, prec), flush=True)
    s = inputs.plummer(n, 970 + n)
    m = dev(s.mass)
    a0, _ = nb.forces(dev(s.pos), m, precision=prec)
    st = torch.cuda.Stream()
    p, v, a = dev(s.pos), dev(s.vel), a0.clone()
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    pe, ve, ae = p.clone(), v.clone(), a.clone()
    pote = torch.empty_like(pot)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):  # a first call on the device outside the capture
        nb.step_noalloc(p.clone(), v.clone(), m, a.clone(), 1e-3, precision=prec, out_pot=pot, stream=st)
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        nb.step_noalloc(p, v, m, a, 1e-3, precision=prec, out_pot=pot, stream=st)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        nb.step_noalloc(pe, ve, m, ae, 1e-3, precision=prec, out_pot=pote)
        torch.cuda.synchronize()
        for x, y, name in ((p, pe, "pos"), (v, ve, "vel"), (a, ae, "acc"), (pot, pote, "pot")):
            assert torch.equal(x, y), (n, prec, k, name)
