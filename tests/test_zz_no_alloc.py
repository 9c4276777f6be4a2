"""nbody_step_noalloc (the allocation-free step: its workspace is the library's static device
scratch array) through the C ABI against nbody_step with a caller workspace, on calls in a row
(the second with a smaller system), bitwise.

Where the tile nbody_step takes fits the scratch, both use it. Where its partial sums do not
fit, the allocation-free step takes the tile table's tile for the largest systems, or the
one-sided pass with one j-range when even that does not fit; nbody_step is then run with the
tile table set to that same tile. Each case checks first that the tile it expects is the one
the rule picks for its size."""
import math

import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu

SCRATCH = 128 << 20     # NBODY_NOALLOC_SCRATCH_BYTES
MARGIN = 512            # bytes per particle kept for the rest of the step's workspace


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


def _edge(desc):
    return int(desc.split("sym=")[1].split(",")[0]) if "sym=" in desc else 0


def _slot_bytes(desc, n):
    return math.ceil(n / _edge(desc)) * 16.0 * n


def _expected_tile(nb, n, prec):
    """(variant, j_split, which) of the rule for a symmetric tuned tile."""
    descs = nb.tile_variants("force", prec)
    cap = max(0.0, SCRATCH - MARGIN * n)
    v, js = nb.tile_lookup("force", prec, n)
    if "sym=" not in descs[v] or _slot_bytes(descs[v], n) <= cap:
        return v, js, "tuned"
    # the table's entry for the largest systems (its last bucket holds 1M particles; looked up at
    # 1M, whose partial sums stay under the library's default cap)
    vb, jb = nb.tile_lookup("force", prec, 1 << 20)
    if "sym=" in descs[vb] and _slot_bytes(descs[vb], n) <= cap:
        return vb, jb, "largest block"
    return 0, 1, "one-sided"


def _two_steps(nb, step, n, prec, s, a0):
    import torch
    m = dev(s.mass)
    p, v, a = dev(s.pos), dev(s.vel), a0.clone()
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        step(p, v, m, a, 1e-3, precision=prec, out_pot=pot)
    torch.cuda.synchronize()
    return p, v, a, pot


def test_step_noalloc_matches_step(nb):
    cases = ((60000, "fp32c", "largest block"), (3000, "fp32c", "tuned"), (40000, "fp32a", "tuned"),
             (300000, "fp32c", "one-sided"))
    for n, prec, which in cases:
        v, js, got = _expected_tile(nb, n, prec)
        assert got == which, (n, prec, got)
        print("step_noalloc n=%d %s: %s tile, variant %d" % (n, prec, which, v), flush=True)
        s = inputs.plummer(n, 950 + n)
        a0, _ = nb.forces(dev(s.pos), dev(s.mass), precision=prec)  # one starting acceleration for both
        table_prec = "fp32c" if prec == "fp32a" else prec
        try:
            if which != "tuned":
                nb.set_tile_table([dict(kernel="force", precision=table_prec, n_min=0, n_max=1 << 40, variant=v,
                                        j_split=js)])
            ref = _two_steps(nb, nb.step, n, prec, s, a0)
        finally:
            nb.restore_tile_table()
        out = _two_steps(nb, nb.step_noalloc, n, prec, s, a0)
        import torch
        for r, o, name in zip(ref, out, ("pos", "vel", "acc", "pot")):
            assert torch.equal(r, o), (n, prec, name)
