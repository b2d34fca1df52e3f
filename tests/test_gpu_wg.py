"""Parity of the workgroup path (one cell per 256-thread workgroup, 64 < N)
with the oracle, through the C ABI.  Bounds as in test_gpu_parity.py."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, make_mechanism, make_states  # noqa: E402

TIGHT_RTOL, TIGHT_ATOL = 1e-10, 1e-14


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


DEV = "cuda:0"
_C5 = {}


def c5():
    if not _C5:
        w = WORKLOADS["c5_150sp"]
        _C5["w"], _C5["mech"] = w, w.mechanism()
    return _C5["w"], _C5["mech"]


def run(chem, mech, st0, p, dt, rtol, atol, **opt):
    m = chem.Mechanism(mech)
    s = torch.tensor(st0, device=DEV)
    nc = st0.shape[1]
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = torch.zeros(nc, dtype=torch.int32, device=DEV)
    rej = torch.zeros(nc, dtype=torch.int32, device=DEV)
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    chem.integrate(m, s, h, p, dt, rtol, atol, options=chem.Options(**opt) if opt else None, steps=steps,
                   rejects=rej, status=status)
    torch.cuda.synchronize()
    return s.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), rej.cpu().numpy(), status.cpu().numpy()


@pytest.mark.parametrize("n", [65, 100, 151, 160, 256])
def test_lu_solve_matches_lapack_large(chem, n):
    say(f"[lu wg] n={n}")
    rng = np.random.default_rng(n)
    nmat = 11
    A = rng.standard_normal((nmat, n, n)) + np.eye(n) * rng.uniform(-2, 2, (nmat, 1, 1))
    b = rng.standard_normal((nmat, n))
    x, info = chem.lu_solve(torch.tensor(A, device=DEV), torch.tensor(b, device=DEV))
    torch.cuda.synchronize()
    x, info = x.cpu().numpy(), info.cpu().numpy()
    assert np.all(info == 0)
    for i in range(nmat):
        ref = np.linalg.solve(A[i], b[i])
        res = np.abs(A[i] @ x[i] - b[i]).max() / (np.abs(A[i]).max() * np.abs(x[i]).max())
        assert res <= 20 * n * np.finfo(float).eps, (i, res)
        np.testing.assert_allclose(x[i], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("n", [100, 151, 256])
def test_lu_solve_pivot_ties_large(chem, n):
    """Entries from {+-1, +-(1 + 2^-40), +-2}: columns hold many pivot candidates
    of equal magnitude (exact ties) and of equal upper 32 bits that differ only
    in the lower bits, so the pivot search takes its tie-breaking path."""
    rng = np.random.default_rng(100 + n)
    nmat = 6
    vals = np.array([1.0, 1.0 + 2.0 ** -40, 2.0])
    A = rng.choice(vals, (nmat, n, n)) * rng.choice([-1.0, 1.0], (nmat, n, n))
    b = rng.standard_normal((nmat, n))
    x, info = chem.lu_solve(torch.tensor(A, device=DEV), torch.tensor(b, device=DEV))
    torch.cuda.synchronize()
    x, info = x.cpu().numpy(), info.cpu().numpy()
    assert np.all(info == 0)
    for i in range(nmat):
        ref = np.linalg.solve(A[i], b[i])
        res = np.abs(A[i] @ x[i] - b[i]).max() / (np.abs(A[i]).max() * np.abs(x[i]).max())
        assert res <= 20 * n * np.finfo(float).eps, (i, res)
        np.testing.assert_allclose(x[i], ref, rtol=1e-6, atol=1e-8 * np.abs(ref).max())


def test_lu_zero_pivot_large(chem):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((2, 100, 100))
    A[0, :, 37] = 0.0  # column 37 is zero: the factorisation meets a zero pivot at step 38
    b = rng.standard_normal((2, 100))
    x, info = chem.lu_solve(torch.tensor(A, device=DEV), torch.tensor(b, device=DEV))
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] == 38 and info[1] == 0
    np.testing.assert_allclose(x.cpu().numpy()[1], np.linalg.solve(A[1], b[1]), rtol=1e-9, atol=1e-11)


def test_rhs_and_jacobian_match_oracle_150sp(chem):
    w, mech = c5()
    st = w.states(mech, 9)
    m = chem.Mechanism(mech)
    f = chem.rhs(m, torch.tensor(st, device=DEV), w.p_pa).cpu().numpy()
    J, fj = chem.jacobian(m, torch.tensor(st, device=DEV), w.p_pa)
    J, fj = J.cpu().numpy(), fj.cpu().numpy()
    mm = oracle.Mech(mech)
    for c in range(st.shape[1]):
        ref = oracle.rhs(mm, w.p_pa, st[:, c])
        scale = np.abs(ref[1:]).max()
        for got in (f[:, c], fj[:, c]):
            assert abs(got[0] - ref[0]) <= 1e-10 * abs(ref[0]), (c, got[0], ref[0])
            assert np.all(np.abs(got[1:] - ref[1:]) <= 1e-10 * np.abs(ref[1:]) + 1e-12 * scale), c
        Jr = oracle.jac(mm, w.p_pa, st[:, c])
        dev_ = np.abs(J[c] - Jr) / np.abs(Jr).max(axis=1, keepdims=True)
        assert dev_.max() <= 1e-10, (c, dev_.max(), np.unravel_index(dev_.argmax(), dev_.shape))


def _tight(got, ref, tag):
    dev_ = np.abs(got - ref)
    rel = dev_ / (np.abs(ref) + 100 * TIGHT_ATOL)
    say(f"[{tag}] max rel dev {rel.max():.3e} median {np.median(rel):.3e}")
    assert np.all(dev_ <= 1e-8 * np.abs(ref) + 100 * TIGHT_ATOL), (tag, rel.max())


def test_integrate_parity_150sp_tight(chem):
    """150 species / 1000 reactions, rtol 1e-10 over 1e-10 s (500-2800 steps per cell)."""
    w, mech = c5()
    st0 = w.states(mech, 6)
    dt = 1e-10
    got, h, steps, rej, status = run(chem, mech, st0, w.p_pa, dt, TIGHT_RTOL, TIGHT_ATOL)
    assert np.all(status == 0)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0, None, w.p_pa, dt, TIGHT_RTOL, TIGHT_ATOL)
    say(f"[c5 tight] steps gpu {steps} oracle {rs}")
    _tight(got, ref, "c5 tight")


def test_integrate_parity_80sp_tight(chem):
    """A second size (N = 81, padded to 96), 8 cells at rtol 1e-10."""
    mech = make_mechanism(80, 300, 30, 15, 1080)
    st0 = make_states(mech, 8, 2080, [(900.0, 2200.0)])
    dt, p = 1e-9, 1e6
    got, h, steps, rej, status = run(chem, mech, st0, p, dt, TIGHT_RTOL, TIGHT_ATOL)
    assert np.all(status == 0)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0, None, p, dt, TIGHT_RTOL, TIGHT_ATOL)
    _tight(got, ref, "k80 tight")


def test_integrate_150sp_metric_and_bitwise(chem):
    """rtol 1e-6 over the CFD step on 24 cells; repeated, graph and cost-ordered
    launches give bitwise identical results."""
    w, mech = c5()
    st0 = w.states(mech, 24)
    a = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol)
    assert np.all(a[4] == 0)
    assert np.abs(a[0][1:].sum(axis=0) - 1).max() <= 1e-12
    idx = np.arange(0, 24, 4)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, w.dt, w.rtol, w.atol)
    bound = 100 * (w.rtol * np.abs(ref) + w.atol)
    say(f"[c5 metric] max dev / bound {np.max(np.abs(a[0][:, idx] - ref) / bound):.3e}; "
        f"steps gpu {a[2][idx]} oracle {rs}")
    assert np.all(np.abs(a[0][:, idx] - ref) <= bound)
    b = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    m = chem.Mechanism(mech)
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(24, dtype=torch.float64, device=DEV)
    steps = torch.tensor(a[2], device=DEV)
    opt = chem.Options(persistent=1, use_graph=1, cost_order=1)
    for rep in range(3):
        s.copy_(torch.tensor(st0, device=DEV))
        h.zero_()
        chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), a[0]), rep
        assert np.array_equal(steps.cpu().numpy(), a[2]), rep


def test_wg_adjoint_unsupported_and_failures(chem):
    w, mech = c5()
    m = chem.Mechanism(mech)
    s = torch.tensor(w.states(mech, 3), device=DEV)
    with pytest.raises(chem.ChemError):
        chem.integrate_adjoint(m, s, torch.zeros(3, dtype=torch.float64, device=DEV), w.p_pa, w.dt, w.rtol, w.atol,
                               torch.ones_like(s))
    st = w.states(mech, 4)
    st[0, 1] = np.nan
    st[0, 2] = -5.0
    got, h, steps, rej, status = run(chem, mech, st, w.p_pa, w.dt, w.rtol, w.atol, max_steps=3)
    assert status[1] == 4 and status[2] == 4
    assert status[0] == 1 and status[3] == 1  # 3 attempts cannot cover the CFD step
