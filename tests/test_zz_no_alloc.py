"""nbody_step_noalloc (the allocation-free step: its workspace is the library's static device
scratch array) through the C ABI against nbody_step with a caller workspace: two calls in a row,
the second with a smaller system, then the adaptive mode; results bitwise equal."""
import numpy as np
import pytest

from paper_2511_02655_amd import inputs

pytestmark = pytest.mark.gpu


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


def test_step_noalloc_matches_step(nb):
    import torch
    for n, prec in ((60000, "fp32c"), (3000, "fp32c"), (40000, "fp32a")):
        print("step_noalloc n=%d %s" % (n, prec), flush=True)
        s = inputs.plummer(n, 950 + n)
        m = dev(s.mass)
        p1, v1 = dev(s.pos), dev(s.vel)
        a1, _ = nb.forces(p1, m, precision=prec)
        p2, v2, a2 = p1.clone(), v1.clone(), a1.clone()
        pot1 = torch.empty(n, dtype=torch.float64, device="cuda")
        pot2 = torch.empty(n, dtype=torch.float64, device="cuda")
        for _ in range(2):
            nb.step(p1, v1, m, a1, 1e-3, precision=prec, out_pot=pot1)
            nb.step_noalloc(p2, v2, m, a2, 1e-3, precision=prec, out_pot=pot2)
        torch.cuda.synchronize()
        assert torch.equal(p1, p2) and torch.equal(v1, v2) and torch.equal(a1, a2) and torch.equal(pot1, pot2)
