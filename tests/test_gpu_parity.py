"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances:
  * integration at rtol 1e-10, atol 1e-16: |x_gpu - x_ref| <= 1e-8 |x_ref| +
    1e-14 per component (T and every Y).  Relative 1e-8 is the bar stated for
    this path; the absolute floor 1e-14 covers trace species, which atol =
    1e-16 resolves to ~1e-16 (measured on the oracle itself: one flipped
    accept/reject decision moves a run by at most 0.24 of this bound);
  * integration at the metric setting (rtol 1e-6, atol 1e-10): accept/reject
    decisions taken with err close to 1 may flip on rounding, after which two
    valid runs differ by their global error.  Measured on the same 18 cells,
    the oracle moves by 20.7 (rtol |x| + atol) when its own safety factor
    changes by 1e-7 relative, so the bound is 100 (rtol |x_ref| + atol).  Cells
    whose step and reject counts equal the oracle's are reported separately:
    there only rounding differs (pivot order, reciprocal, exp/log, summation
    order), but stiff iteration matrices have condition numbers near 1e10, so
    no fixed multiple of eps bounds them at this tolerance;
  * f and J: the GPU sums reactions in a different order, so each component is
    compared against the size of that row (cancellation in omega_k).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


_MECH = {}


def mech_of(name):
    if name not in _MECH:
        w = WORKLOADS[name]
        _MECH[name] = (w, w.mechanism())
    return _MECH[name]


def run_gpu(chem, m, st0, h0, p, dt, rtol, atol, dev, **opt):
    st = torch.tensor(st0, device=dev)
    h = torch.tensor(h0 if h0 is not None else np.zeros(st0.shape[1]), device=dev)
    nc = st0.shape[1]
    steps = torch.zeros(nc, dtype=torch.int32, device=dev)
    rej = torch.zeros(nc, dtype=torch.int32, device=dev)
    status = torch.full((nc,), -1, dtype=torch.int32, device=dev)
    o = chem.Options(**opt) if opt else None
    chem.integrate(m, st, h, p, dt, rtol, atol, options=o, steps=steps, rejects=rej, status=status)
    torch.cuda.synchronize()
    return (st.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), rej.cpu().numpy(), status.cpu().numpy())


# ------------------------------------------------------------------ LU
@pytest.mark.parametrize("n", [1, 3, 11, 16, 17, 33, 54, 55, 64])
def test_lu_solve_matches_lapack(chem, dev, n):
    say(f"[lu] n={n}")
    rng = np.random.default_rng(n)
    nmat = 37
    A = rng.standard_normal((nmat, n, n)) + np.eye(n) * rng.uniform(-2, 2, (nmat, 1, 1))
    b = rng.standard_normal((nmat, n))
    x, info = chem.lu_solve(torch.tensor(A, device=dev), torch.tensor(b, device=dev))
    torch.cuda.synchronize()
    x, info = x.cpu().numpy(), info.cpu().numpy()
    assert np.all(info == 0)
    for i in range(nmat):
        ref = np.linalg.solve(A[i], b[i])
        res = np.abs(A[i] @ x[i] - b[i]).max() / (np.abs(A[i]).max() * np.abs(x[i]).max())
        assert res <= 20 * n * np.finfo(float).eps, (i, res)
        np.testing.assert_allclose(x[i], ref, rtol=1e-8, atol=1e-10 * np.abs(ref).max())


def test_lu_reports_zero_pivot(chem, dev):
    A = np.array([[[1.0, 0.0, 3.0], [2.0, 0.0, 6.0], [1.0, 0.0, 1.0]], [[2.0, 1.0, 0.0], [1.0, 3.0, 1.0], [0.0, 1.0, 4.0]]])
    b = np.ones((2, 3))
    x, info = chem.lu_solve(torch.tensor(A, device=dev), torch.tensor(b, device=dev))
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] == 2 and info[1] == 0
    np.testing.assert_allclose(x.cpu().numpy()[1], np.linalg.solve(A[1], b[1]), rtol=1e-13)


# ------------------------------------------------------- f and J parity
@pytest.mark.parametrize("name", ["c1_10sp", "c2_54sp", "c4_adj"])
def test_rhs_matches_oracle(chem, dev, name):
    say(f"[rhs] {name}")
    w, mech = mech_of(name)
    st = w.states(mech, 37)
    m = chem.Mechanism(mech)
    f = chem.rhs(m, torch.tensor(st, device=dev), w.p_pa)
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    mm = oracle.Mech(mech)
    for c in range(st.shape[1]):
        ref = oracle.rhs(mm, w.p_pa, st[:, c])
        scale = np.abs(ref[1:]).max()
        assert abs(f[0, c] - ref[0]) <= 1e-10 * abs(ref[0]) + 1e-12 * abs(ref[0]), (c, f[0, c], ref[0])
        assert np.all(np.abs(f[1:, c] - ref[1:]) <= 1e-10 * np.abs(ref[1:]) + 1e-12 * scale), c


@pytest.mark.parametrize("name", ["c1_10sp", "c2_54sp", "c4_adj"])
def test_jacobian_matches_oracle(chem, dev, name):
    say(f"[jac] {name}")
    w, mech = mech_of(name)
    st = w.states(mech, 13)
    m = chem.Mechanism(mech)
    J, f = chem.jacobian(m, torch.tensor(st, device=dev), w.p_pa)
    torch.cuda.synchronize()
    J, f = J.cpu().numpy(), f.cpu().numpy()
    mm = oracle.Mech(mech)
    for c in range(st.shape[1]):
        ref = oracle.jac(mm, w.p_pa, st[:, c])
        scale = np.abs(ref).max(axis=1, keepdims=True)
        dev_ = np.abs(J[c] - ref) / scale
        assert dev_.max() <= 1e-10, (c, dev_.max(), np.unravel_index(dev_.argmax(), dev_.shape))
        fr = oracle.rhs(mm, w.p_pa, st[:, c])
        assert np.all(np.abs(f[:, c] - fr) <= 1e-10 * np.abs(fr) + 1e-12 * np.abs(fr[1:]).max())


# ------------------------------------------------------ integration parity
TIGHT_RTOL, TIGHT_ATOL = 1e-10, 1e-16
TIGHT_FLOOR = 1e-14


def _tight_check(got, ref, tag):
    dev_ = np.abs(got - ref)
    bound = 1e-8 * np.abs(ref) + TIGHT_FLOOR
    ok = dev_ <= bound
    rel = dev_ / bound
    say(f"[{tag}] max dev / bound {rel.max():.3e} median {np.median(rel):.3e}")
    assert np.all(ok), (tag, np.argwhere(~ok)[:5], rel.max())


def test_integrate_parity_c1_tight(chem, dev):
    """Config 1 (10 species / 27 reactions, 1,024 cells) at rtol 1e-10."""
    w, mech = mech_of("c1_10sp")
    st0 = w.states(mech)
    rtol, atol = TIGHT_RTOL, TIGHT_ATOL
    say("[c1 tight] gpu")
    got, h, steps, rej, status = run_gpu(chem, chem.Mechanism(mech), st0, None, w.p_pa, w.dt, rtol, atol, dev)
    assert np.all(status == 0)
    idx = np.arange(0, st0.shape[1], 8)  # 128 cells the oracle finishes in seconds
    say("[c1 tight] oracle")
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, w.dt, rtol, atol)
    assert np.all(rst == 0)
    _tight_check(got[:, idx], ref, "c1 tight")
    same = (steps[idx] == rs) & (rej[idx] == rr)
    say(f"[c1 tight] cells with identical (steps, rejects): {same.mean():.3f}")
    assert same.mean() >= 0.9


@pytest.mark.parametrize("name", ["c2_54sp", "c4_adj"])
def test_integrate_parity_large_mech_tight(chem, dev, name):
    """54- and 53-species mechanisms, 70 cells (ragged over 4-cell workgroups), rtol 1e-10, over a short
    dt (the full flow step of these configurations is tested in test_gpu_tight.py)."""
    w, mech = mech_of(name)
    st0 = w.states(mech, 70)
    dt, rtol, atol = 1e-8, TIGHT_RTOL, TIGHT_ATOL
    say(f"[{name} tight] gpu")
    got, h, steps, rej, status = run_gpu(chem, chem.Mechanism(mech), st0, None, w.p_pa, dt, rtol, atol, dev)
    assert np.all(status == 0)
    idx = np.arange(0, 70, 3)
    say(f"[{name} tight] oracle on {len(idx)} cells")
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, dt, rtol, atol)
    _tight_check(got[:, idx], ref, f"{name} tight")
    same = (steps[idx] == rs) & (rej[idx] == rr)
    say(f"[{name} tight] cells with identical (steps, rejects): {same.mean():.3f}")


def test_integrate_full_size_c2_metric(chem, dev):
    """Full 65,536-cell config 2 at rtol 1e-6 in the benchmark launch; sampled cells vs oracle."""
    w, mech = mech_of("c2_54sp")
    st0 = w.states(mech)
    say("[c2 full] gpu")
    got, h, steps, rej, status = run_gpu(chem, chem.Mechanism(mech), st0, None, w.p_pa, w.dt, w.rtol, w.atol, dev)
    assert np.all(status == 0)
    assert np.abs(got[1:].sum(axis=0) - 1).max() <= 1e-12
    assert np.all((h > 0) & (h <= w.dt))
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(st0.shape[1], 16, replace=False))
    idx = np.concatenate([idx, [0, st0.shape[1] - 1]])
    say("[c2 full] oracle on sampled cells")
    ref, href, rs, rr, rst = oracle.integrate(mech, st0[:, idx], None, w.p_pa, w.dt, w.rtol, w.atol)
    bound = 100 * (w.rtol * np.abs(ref) + w.atol)
    dev_ = np.abs(got[:, idx] - ref)
    same = (steps[idx] == rs) & (rej[idx] == rr)
    tight = 1e-7 * np.abs(ref[:, same]) + 10 * w.atol
    say(f"[c2 full] max dev / bound {np.max(dev_ / bound):.3e}; identical step counts in {same.sum()}/{len(idx)}; "
        f"their max dev / (1e-7|x| + 10 atol) {np.max(dev_[:, same] / tight) if same.any() else 0:.3e}")
    assert np.all(dev_ <= bound)


def test_persistent_equals_plain_bitwise(chem, dev):
    w, mech = mech_of("c2_54sp")
    st0 = w.states(mech, 203)
    m = chem.Mechanism(mech)
    a = run_gpu(chem, m, st0, None, w.p_pa, 1e-7, 1e-6, 1e-10, dev, persistent=1)
    b = run_gpu(chem, m, st0, None, w.p_pa, 1e-7, 1e-6, 1e-10, dev, persistent=0, waves_per_block=1)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_graph_replays_match_eager(chem, dev):
    """The cached hipGraph (reset kernel + persistent kernel) replayed several
    times, with eager work in between, gives the eager result every time."""
    w, mech = mech_of("c1_10sp")
    st0 = w.states(mech, 300)
    m = chem.Mechanism(mech)
    ref = run_gpu(chem, m, st0, None, w.p_pa, w.dt, w.rtol, w.atol, dev, persistent=1)
    st = torch.empty((st0.shape[0], st0.shape[1]), dtype=torch.float64, device=dev)
    h = torch.empty(st0.shape[1], dtype=torch.float64, device=dev)
    status = torch.empty(st0.shape[1], dtype=torch.int32, device=dev)
    src = torch.tensor(st0, device=dev)
    o = chem.Options(persistent=1, use_graph=1)
    for rep in range(4):
        st.copy_(src)
        h.zero_()
        chem.integrate(m, st, h, w.p_pa, w.dt, w.rtol, w.atol, options=o, status=status)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=dev).sum().item()  # eager work between replays
        np.testing.assert_array_equal(st.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(h.cpu().numpy(), ref[1])
        assert np.isfinite(junk)


def test_failure_statuses_per_cell(chem, dev):
    w, mech = mech_of("c1_10sp")
    st0 = w.states(mech, 6)
    m = chem.Mechanism(mech)
    clean = run_gpu(chem, m, st0, None, w.p_pa, w.dt, w.rtol, w.atol, dev)
    st = st0.copy()
    st[3, 1] = np.nan
    st[0, 2] = -5.0
    out = run_gpu(chem, m, st, None, w.p_pa, w.dt, w.rtol, w.atol, dev)
    assert list(out[4]) == [0, 4, 4, 0, 0, 0]
    for c in (0, 3, 4, 5):
        np.testing.assert_array_equal(out[0][:, c], clean[0][:, c])
    few = run_gpu(chem, m, st0[:, :2], None, w.p_pa, w.dt, w.rtol, w.atol, dev, max_steps=1)
    assert np.all(few[4] == 1)
    under = run_gpu(chem, m, st0[:, :2], None, w.p_pa, w.dt, 0.0, 0.0, dev)
    assert np.all(under[4] == 2)


def test_ld_padding_and_empty(chem, dev):
    w, mech = mech_of("c1_10sp")
    m = chem.Mechanism(mech)
    nc, ld = 50, 64
    st0 = w.states(mech, ld)
    st = torch.tensor(st0, device=dev)
    h = torch.zeros(ld, dtype=torch.float64, device=dev)
    chem.integrate(m, st, h, w.p_pa, w.dt, w.rtol, w.atol, ncells=nc)
    chem.integrate(m, st, h, w.p_pa, w.dt, w.rtol, w.atol, ncells=0)
    torch.cuda.synchronize()
    out = st.cpu().numpy()
    np.testing.assert_array_equal(out[:, nc:], st0[:, nc:])
    assert np.all(h.cpu().numpy()[nc:] == 0)
    ref = oracle.integrate(mech, st0[:, :nc], None, w.p_pa, w.dt, w.rtol, w.atol)[0]
    assert np.all(np.abs(out[:, :nc] - ref) <= 100 * (w.rtol * np.abs(ref) + w.atol))


def test_rodas3_parity(chem, dev):
    w, mech = mech_of("c1_10sp")
    st0 = w.states(mech, 40)
    rtol, atol = 1e-9, 1e-14
    got = run_gpu(chem, chem.Mechanism(mech), st0, None, w.p_pa, w.dt, rtol, atol, dev, method=1)
    ref = oracle.integrate(mech, st0, None, w.p_pa, w.dt, rtol, atol, method="rodas3")
    assert np.all(got[4] == 0)
    assert np.all(np.abs(got[0] - ref[0]) <= 1e-7 * np.abs(ref[0]) + 1e-13)


def test_warm_h_and_second_call(chem, dev):
    """h returned by one call seeds the next (the sub-step persisting between CFD steps)."""
    w, mech = mech_of("c1_10sp")
    st0 = w.states(mech, 64)
    m = chem.Mechanism(mech)
    a = run_gpu(chem, m, st0, None, w.p_pa, w.dt, w.rtol, w.atol, dev)
    b = run_gpu(chem, m, a[0], a[1], w.p_pa, w.dt, w.rtol, w.atol, dev)
    ra = oracle.integrate(mech, st0, None, w.p_pa, w.dt, w.rtol, w.atol)
    rb = oracle.integrate(mech, ra[0], ra[1], w.p_pa, w.dt, w.rtol, w.atol)
    assert np.all(np.abs(b[0] - rb[0]) <= 100 * (w.rtol * np.abs(rb[0]) + w.atol))
    np.testing.assert_allclose(a[1], ra[1], rtol=1e-3)


def test_cost_ordered_queue_bitwise(chem, dev):
    """Cost-ordered persistent queue (eager and through the graph) gives the
    same per-cell results as the unordered launch; the order comes from the
    step counts passed in."""
    w, mech = mech_of("c3_batch")
    st0 = w.states(mech, n_cells=4096)
    m = chem.Mechanism(mech)
    outs = []
    for cfg in (dict(persistent=1), dict(persistent=1, cost_order=1), dict(persistent=1, cost_order=1, use_graph=1)):
        s = torch.tensor(st0, device=dev)
        h = torch.zeros(st0.shape[1], dtype=torch.float64, device=dev)
        steps = torch.tensor(np.arange(st0.shape[1], dtype=np.int32) % 700, device=dev)
        status = torch.zeros(st0.shape[1], dtype=torch.int32, device=dev)
        for rep in range(2 if cfg.get("use_graph") else 1):
            s.copy_(torch.tensor(st0, device=dev))
            h.zero_()
            chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=chem.Options(**cfg), steps=steps,
                           status=status)
            torch.cuda.synchronize()
        outs.append((s.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()))
    say("c3 sample steps percentiles", np.percentile(outs[0][2], [0, 50, 90, 99, 100]))
    assert np.all(outs[0][3] == 0)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
