"""Integration parity at the size boundaries of the two layouts, rtol 1e-10
against the oracle: the wavefront path's padded sizes (N = 32 and 56 fill
their padding exactly, N = 57 moves to the next one) and its largest N (64),
the first size on the workgroup path (N = 65) and the workgroup path's
largest N (255, whose first panels exceed the register panel)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import make_mechanism, make_states  # noqa: E402

DEV = "cuda:0"
RTOL, ATOL = 1e-10, 1e-14
P = 1e6

# (species K, reactions, max atoms per species, cells, dt)
CASES = [
    (31, 120, None, 4, 1e-10),
    (55, 280, None, 4, 1e-10),
    (56, 280, None, 4, 1e-10),
    (63, 300, None, 4, 1e-10),
    (64, 300, None, 4, 1e-10),
    (254, 1600, 8, 2, 2e-11),
]


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


@pytest.mark.parametrize("K,R,max_atoms,nc,dt", CASES, ids=[f"N{c[0] + 1}" for c in CASES])
def test_integrate_parity_at_size_boundaries(chem, K, R, max_atoms, nc, dt):
    mech = make_mechanism(K, R, R // 10, R // 20, 7000 + K, max_atoms=max_atoms)
    st0 = make_states(mech, nc, 8000 + K, [(900.0, 2200.0)])
    m = chem.Mechanism(mech)
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = torch.zeros(nc, dtype=torch.int32, device=DEV)
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    chem.integrate(m, s, h, P, dt, RTOL, ATOL, steps=steps, status=status)
    torch.cuda.synchronize()
    got, st = s.cpu().numpy(), status.cpu().numpy()
    assert np.all(st == 0)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0, None, P, dt, RTOL, ATOL)
    assert np.all(rst == 0)
    dev_ = np.abs(got - ref)
    rel = dev_ / (np.abs(ref) + 100 * ATOL)
    print(f"[N={K + 1}] steps gpu {steps.cpu().numpy()} oracle {rs}; max rel dev {rel.max():.3e}")
    assert np.all(dev_ <= 1e-8 * np.abs(ref) + 100 * ATOL)
