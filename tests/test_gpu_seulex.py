"""Parity of the Seulex-family integrator (method 2) with the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def run(chem, mech, st0, p, dt, rtol, atol, **opt):
    m = chem.Mechanism(mech)
    nc = st0.shape[1]
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = torch.zeros(nc, dtype=torch.int32, device=DEV)
    rej = torch.zeros(nc, dtype=torch.int32, device=DEV)
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    chem.integrate(m, s, h, p, dt, rtol, atol, options=chem.Options(method=2, **opt), steps=steps, rejects=rej,
                   status=status)
    torch.cuda.synchronize()
    return s.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), rej.cpu().numpy(), status.cpu().numpy()


@pytest.mark.parametrize("name,nc,dt", [("c1_10sp", 128, None), ("c2_54sp", 24, 1e-7), ("c4_adj", 16, 1e-7)])
def test_seulex_tight_parity(chem, name, nc, dt):
    w = WORKLOADS[name]
    mech = w.mechanism()
    st0 = w.states(mech, nc)
    dt = dt or w.dt
    rtol, atol = 1e-10, 1e-14
    got, h, steps, rej, status = run(chem, mech, st0, w.p_pa, dt, rtol, atol)
    assert np.all(status == 0)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0, None, w.p_pa, dt, rtol, atol, method="seulex")
    assert np.all(rst == 0)
    dev_ = np.abs(got - ref)
    rel = dev_ / (np.abs(ref) + 100 * atol)
    same = (steps == rs) & (rej == rr)
    print(f"[seulex {name}] max rel dev {rel.max():.3e}; identical (steps, rejects) {same.mean():.2f}; "
          f"steps gpu {steps[:6]} oracle {rs[:6]}")
    assert np.all(dev_ <= 1e-8 * np.abs(ref) + 100 * atol)


def test_seulex_metric_and_launch_shapes(chem):
    w = WORKLOADS["c2_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 203)
    a = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol, persistent=0, waves_per_block=1)
    b = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol, persistent=1)
    assert np.all(a[4] == 0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    idx = np.arange(0, 203, 17)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, w.dt, w.rtol, w.atol,
                                              method="seulex")
    bound = 100 * (w.rtol * np.abs(ref) + w.atol)
    print(f"[seulex c2 metric] max dev / bound {np.max(np.abs(a[0][:, idx] - ref) / bound):.3e}; "
          f"mean steps {a[2].mean():.1f}")
    assert np.all(np.abs(a[0][:, idx] - ref) <= bound)


def test_seulex_unsupported_combinations(chem):
    w = WORKLOADS["c1_10sp"]
    mech = w.mechanism()
    m = chem.Mechanism(mech)
    s = torch.tensor(w.states(mech, 4), device=DEV)
    h = torch.zeros(4, dtype=torch.float64, device=DEV)
    with pytest.raises(chem.ChemError):
        chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=chem.Options(method=2, jac_mode=1))
    with pytest.raises(chem.ChemError):
        chem.integrate_adjoint(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, torch.ones_like(s),
                               options=chem.Options(method=2))
    with pytest.raises(chem.ChemError):
        chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=chem.Options(method=3))


def test_seulex_instrumented_counts(chem):
    """The instrumented kernel takes the same steps as the plain one and counts
    its factorisations (2..6 columns per attempt) and substeps (n_j = j)."""
    w = WORKLOADS["c2_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 64)
    a = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol)
    pc = torch.zeros((64, 8), dtype=torch.int64, device=DEV)
    b = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol, phase_cycles=pc)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    pcn = pc.cpu().numpy()
    att = a[2] + a[3]
    nlu, nsub = pcn[:, 6], pcn[:, 7]
    assert np.all(nlu >= 2 * att) and np.all(nlu <= 6 * att)
    # columns 1..k take 1..k substeps: k(k+1)/2 substeps for k factorisations
    assert np.all(nsub >= 1.5 * nlu) and np.all(nsub <= 3.5 * nlu)
    print(f"[seulex counts] LU per attempt {nlu.sum() / att.sum():.2f}, substeps per LU {nsub.sum() / nlu.sum():.2f}")


@pytest.mark.parametrize("case", ["c5_150sp", "N65"])
def test_seulex_workgroup_path_tight(chem, case):
    """Seulex on the workgroup path (N > 64): 150 species over 1e-10 s and the
    first workgroup size (N = 65) over 1e-9 s, rtol 1e-10, against the oracle."""
    from paper_2105_12070_amd.inputs import make_mechanism, make_states
    if case == "c5_150sp":
        w = WORKLOADS[case]
        mech = w.mechanism()
        st0 = w.states(mech, 4)
        p, dt = w.p_pa, 1e-10
    else:
        mech = make_mechanism(64, 300, 30, 15, 7064)
        st0 = make_states(mech, 4, 8064, [(900.0, 2200.0)])
        p, dt = 1e6, 1e-9
    rtol, atol = 1e-10, 1e-14
    got, h, steps, rej, status = run(chem, mech, st0, p, dt, rtol, atol)
    assert np.all(status == 0)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0, None, p, dt, rtol, atol, method="seulex")
    assert np.all(rst == 0)
    dev_ = np.abs(got - ref)
    rel = dev_ / (np.abs(ref) + 100 * atol)
    print(f"[seulex wg {case}] steps gpu {steps} oracle {rs}; max rel dev {rel.max():.3e}")
    assert np.all(dev_ <= 1e-8 * np.abs(ref) + 100 * atol)


def test_seulex_workgroup_path_metric_and_counts(chem):
    """150 species at the metric setting: repeated launches bitwise equal, the
    instrumented kernel takes the same steps and counts its work, sampled
    parity with the oracle."""
    w = WORKLOADS["c5_150sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 40)
    a = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol)
    assert np.all(a[4] == 0)
    pc = torch.zeros((40, 8), dtype=torch.int64, device=DEV)
    b = run(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol, phase_cycles=pc)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    pcn = pc.cpu().numpy()
    att = a[2] + a[3]
    assert np.all(pcn[:, 6] >= 2 * att) and np.all(pcn[:, 6] <= 6 * att)
    idx = np.arange(0, 40, 8)
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, w.dt, w.rtol, w.atol,
                                              method="seulex")
    bound = 100 * (w.rtol * np.abs(ref) + w.atol)
    print(f"[seulex wg metric] max dev / bound {np.max(np.abs(a[0][:, idx] - ref) / bound):.3e}; "
          f"mean steps {a[2].mean():.1f}")
    assert np.all(np.abs(a[0][:, idx] - ref) <= bound)
