"""Full-size workloads in the launch configurations bench.py times, checked on
sampled cells against the oracle and through properties that hold at any
size: the 262,144-cell batching workload (persistent, graph, cost-ordered
queue), the 150-species workload at the 16,384 cells its bench line covers,
and the adjoint over all 16,384 cells of its workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, objective_weights  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def say(*a):
    print(*a, flush=True)


def integrate(chem, m, st0, w, opt=None, steps_in=None):
    nc = st0.shape[1]
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = (torch.tensor(steps_in, device=DEV) if steps_in is not None
             else torch.zeros(nc, dtype=torch.int32, device=DEV))
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, status=status)
    torch.cuda.synchronize()
    return s.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()


def sampled_parity(mech, st0, got, w, idx, tag):
    ref, _, rs, _, rst = oracle.integrate(mech, np.ascontiguousarray(st0[:, idx]), None, w.p_pa, w.dt, w.rtol,
                                          w.atol)
    assert np.all(rst == 0)
    bound = 100 * (w.rtol * np.abs(ref) + w.atol)
    dev_ = np.abs(got[:, idx] - ref)
    say(f"[{tag}] sampled {len(idx)} cells: max dev / bound {np.max(dev_ / bound):.3e}")
    assert np.all(dev_ <= bound)


def test_batching_workload_full_size(chem):
    w = WORKLOADS["c3_batch"]
    mech = w.mechanism()
    st0 = w.states(mech)
    m = chem.Mechanism(mech)
    plain, steps, status = integrate(chem, m, st0, w, chem.Options(persistent=0))
    assert np.all(status == 0)
    # the bench configuration: persistent, hipGraph, queue ordered by the previous call's counts
    opt = chem.Options(persistent=1, use_graph=1, cost_order=1)
    for rep in range(2):
        got, s2, st2 = integrate(chem, m, st0, w, opt, steps_in=steps)
        assert np.array_equal(got, plain) and np.array_equal(s2, steps) and np.all(st2 == 0), rep
    assert np.abs(got[1:].sum(axis=0) - 1.0).max() <= 1e-12
    say(f"[c3 full] steps min {steps.min()} median {np.median(steps)} max {steps.max()}")
    idx = np.unique(np.concatenate([np.argsort(steps)[-8:], np.linspace(0, st0.shape[1] - 1, 24).astype(int)]))
    sampled_parity(mech, st0, got, w, idx, "c3 full")


def test_150sp_workload_bench_size(chem):
    w = WORKLOADS["c5_150sp"]
    mech = w.mechanism()
    st0 = np.ascontiguousarray(w.states(mech)[:, :16384])
    m = chem.Mechanism(mech)
    got, steps, status = integrate(chem, m, st0, w)
    assert np.all(status == 0)
    assert np.abs(got[1:].sum(axis=0) - 1.0).max() <= 1e-12
    idx = np.linspace(0, 16383, 6).astype(int)
    sampled_parity(mech, st0, got, w, idx, "c5 16k")


def test_adjoint_full_size(chem):
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    st0 = w.states(mech)
    nc = st0.shape[1]
    K, R = mech["n_species"], mech["n_reactions"]
    lam = np.zeros((K + 1, nc))
    lam[0] = 1.0
    lam[1:] = objective_weights(K)[:, None]
    m = chem.Mechanism(mech)

    def adjoint(cols):
        s0 = torch.tensor(np.ascontiguousarray(st0[:, cols]), device=DEV)
        h = torch.zeros(s0.shape[1], dtype=torch.float64, device=DEV)
        lt = torch.tensor(np.ascontiguousarray(lam[:, cols]), device=DEV)
        out, lam0, grad, steps, status = chem.integrate_adjoint(m, s0, h, w.p_pa, w.dt, w.rtol, w.atol, lt)
        torch.cuda.synchronize()
        return out.cpu().numpy(), lam0.cpu().numpy(), grad.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()

    out, lam0, grad, steps, status = adjoint(np.arange(nc))
    assert np.all(status == 0) and np.all(np.isfinite(grad)) and np.all(np.isfinite(lam0))
    # the forward half is chem_integrate, bit for bit
    fwd, fsteps, fstatus = integrate(chem, m, st0, w)
    assert np.array_equal(out, fwd) and np.array_equal(steps, fsteps)
    # the summed gradient is the sum of the gradients of four quarters of the cells
    parts = [adjoint(np.arange(q * nc // 4, (q + 1) * nc // 4))[2] for q in range(4)]
    gsum = sum(parts)
    rel = np.abs(gsum - grad) / (np.abs(grad) + 1e-12 * np.abs(grad).max())
    say(f"[c4 full] gradient vs sum of quarters: max rel {rel.max():.2e}")
    assert rel.max() <= 1e-9
    # lambda0 of sampled cells: lambda_final . dy(dt) = lambda0 . dy0 along random state directions
    om = oracle.Mech(mech)
    rng = np.random.default_rng(11)
    checked = 0
    for c in np.linspace(0, nc - 1, 12).astype(int):
        _, _, hs, st, _ = oracle.integrate_record(om, st0[:, c], None, w.p_pa, w.dt, w.rtol, w.atol)
        if st != 0 or len(hs) != steps[c]:
            continue  # another accepted-step sequence: the identity does not apply exactly
        dy0 = rng.standard_normal(K + 1) * np.abs(st0[:, c]) * 1e-3
        _, dyo = oracle.tlm(om, st0[:, c], hs, w.p_pa, dy0=dy0)
        lhs, rhs = lam[:, c] @ dyo, lam0[:, c] @ dy0
        scale = np.abs(lam[:, c]) @ np.abs(dyo)
        assert abs(lhs - rhs) <= 1e-7 * scale, (c, lhs, rhs)
        checked += 1
    say(f"[c4 full] lambda0 identity on {checked} sampled cells")
    assert checked >= 4
