"""Parity of the discrete adjoint on the workgroup path (N > 64: one cell per
256-thread workgroup, transposed solves with the blocked LU's factors) with
the oracle's tangent-linear model, through the C ABI.

Skipped: a sweep kernel for this layout returned non-finite results on its
first runs and then faulted the GPU with a memory aperture violation; no
access out of bounds was found in its code, so it was taken out and
chem_integrate_adjoint keeps rejecting N > 64.  These checks are what it has
to pass when it returns.

The checks mirror the wavefront-path adjoint tests: the dot-product identity
lambda_final . dy(dt) = lambda0 . dy0 + grad . dparams along random
directions on cells whose GPU step count equals the oracle's, single entries
of the gradient and of lambda0 along unit directions, central differences of
the oracle's replay, a closed form, and the replay's bitwise invariants.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the workgroup-path adjoint is switched off: its kernel faulted the GPU "
                                      "(memory aperture violation) with the cause not found")]

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, make_mechanism, make_states, objective_weights  # noqa: E402

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from mechs import isomer_mech  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def n65():
    """The first workgroup-path size: 64 species / 300 reactions."""
    mech = make_mechanism(64, 300, 30, 15, 7064)
    return mech, 1e6


def gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam, ck=8, max_tape=0, method=0):
    m = chem.Mechanism(mech)
    s0 = torch.tensor(st0, device=DEV)
    h = torch.zeros(st0.shape[1], dtype=torch.float64, device=DEV)
    lt = torch.tensor(lam, device=DEV)
    out, lam0, grad, steps, status = chem.integrate_adjoint(m, s0, h, p, dt, rtol, atol, lt,
                                                            options=chem.Options(method=method),
                                                            checkpoint_every=ck, max_tape=max_tape)
    torch.cuda.synchronize()
    return (out.cpu().numpy(), lam0.cpu().numpy(), grad.cpu().numpy(), steps.cpu().numpy(),
            status.cpu().numpy())


def gpu_integrate(chem, mech, st0, p, dt, rtol, atol):
    m = chem.Mechanism(mech)
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(st0.shape[1], dtype=torch.float64, device=DEV)
    steps = torch.zeros(st0.shape[1], dtype=torch.int32, device=DEV)
    chem.integrate(m, s, h, p, dt, rtol, atol, steps=steps)
    return s.cpu().numpy(), steps.cpu().numpy()


def objective_lambda(K, nc):
    lam = np.zeros((K + 1, nc))
    lam[0] = 1.0
    lam[1:] = objective_weights(K)[:, None]
    return lam


def dot_product(chem, mech, st0, p, dt, rtol, atol, ndir, tol, seed=11, max_tape=0):
    nc = st0.shape[1]
    K, R = mech["n_species"], mech["n_reactions"]
    om = oracle.Mech(mech)
    recs = [oracle.integrate_record(om, st0[:, c], None, p, dt, rtol, atol) for c in range(nc)]
    _, gs = gpu_integrate(chem, mech, st0, p, dt, rtol, atol)
    same = np.array([len(r[2]) == gs[c] for c, r in enumerate(recs)])
    say(f"N={K + 1}: {same.sum()}/{nc} cells with the oracle's step count; steps {gs.min()}..{gs.max()}")
    assert same.sum() >= max(2, nc // 2)
    lam = objective_lambda(K, nc) * same[None, :]
    _, lam0, grad, steps, status = gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam, max_tape=max_tape)
    assert np.all(status == 0) and np.array_equal(steps, gs)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for d in range(ndir):
        dy0 = rng.standard_normal(st0.shape) * np.abs(st0) * 1e-3
        dp = [rng.standard_normal(R), rng.standard_normal(R), rng.standard_normal(R) * 100.0]
        lhs, scale = 0.0, 0.0
        for c in np.nonzero(same)[0]:
            _, dyo = oracle.tlm(om, st0[:, c], recs[c][2], p, dy0=dy0[:, c], dlnA=dp[0], db=dp[1], dtheta=dp[2])
            lhs += lam[:, c] @ dyo
            scale += np.abs(lam[:, c]) @ np.abs(dyo)
        got = np.sum(lam0 * dy0) + sum(grad[i] @ dp[i] for i in range(3))
        err = abs(got - lhs) / scale
        assert np.isfinite(err), (lhs, got)
        worst = max(worst, err)
        say(f"  dir {d}: oracle {lhs:.12e}  gpu {got:.12e}  rel {err:.2e}")
    assert worst <= tol, worst


def test_adjoint_wg_dot_product_n65_tight(chem):
    mech, p = n65()
    st0 = make_states(mech, 8, 8064, [(900.0, 2200.0)])
    dot_product(chem, mech, st0, p, 1e-9, 1e-10, 1e-14, 3, 1e-9, max_tape=8192)


def test_adjoint_wg_dot_product_n65_metric(chem):
    mech, p = n65()
    st0 = make_states(mech, 8, 8065, [(900.0, 2200.0)])
    dot_product(chem, mech, st0, p, 1e-6, 1e-6, 1e-10, 3, 1e-7)


def test_adjoint_wg_dot_product_c5_metric(chem):
    """150 species / 1000 reactions at the workload's dt and tolerances."""
    w = WORKLOADS["c5_150sp"]
    mech = w.mechanism()
    st0 = np.ascontiguousarray(w.states(mech, 3))
    dot_product(chem, mech, st0, w.p_pa, w.dt, w.rtol, w.atol, 2, 1e-7)


def test_adjoint_wg_elements_n65(chem):
    """Single gradient and lambda0 entries of one cell along unit directions,
    and central differences (h = 1e-6) of the oracle's replay on ln A."""
    mech, p = n65()
    K, R = mech["n_species"], mech["n_reactions"]
    st0 = make_states(mech, 2, 8066, [(900.0, 2200.0)])
    dt, rtol, atol = 1e-6, 1e-6, 1e-10
    om = oracle.Mech(mech)
    rec = oracle.integrate_record(om, st0[:, 0], None, p, dt, rtol, atol)
    _, gs = gpu_integrate(chem, mech, st0, p, dt, rtol, atol)
    assert gs[0] == len(rec[2])
    lam = objective_lambda(K, 2)
    lam[:, 1] = 0.0
    _, lam0, grad, _, status = gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam)
    assert status[0] == 0 and np.all(lam0[:, 1] == 0.0)
    gmax = np.abs(grad).max(axis=1)
    names = ("dlnA", "db", "dtheta")
    picks = []
    for comp in range(3):
        picks += [(comp, int(r)) for r in np.argsort(-np.abs(grad[comp]))[:3]]
        picks += [(comp, int(r)) for r in np.random.default_rng(comp + 5).choice(R, 2, replace=False)]
    for comp, r in picks:
        e = np.zeros(R)
        e[r] = 1.0
        _, dyo = oracle.tlm(om, st0[:, 0], rec[2], p, **{names[comp]: e})
        ref = lam[:, 0] @ dyo
        say(f"  {names[comp]}[{r}]: oracle {ref:.10e} gpu {grad[comp, r]:.10e}")
        assert abs(grad[comp, r] - ref) <= 1e-7 * abs(ref) + 1e-9 * gmax[comp]
    for r in np.argsort(-np.abs(grad[0]))[:2]:
        vals = []
        for sgn in (1.0, -1.0):
            lnA = mech["lnA"].copy()
            lnA[r] += sgn * 1e-6
            vals.append(lam[:, 0] @ oracle.replay(oracle.Mech(mech, lnA=lnA), st0[:, 0], rec[2], p))
        fd = (vals[0] - vals[1]) / 2e-6
        say(f"  FD dlnA[{r}]: {fd:.8e} adjoint {grad[0, r]:.8e}")
        assert abs(fd - grad[0, r]) <= 1e-5 * abs(grad[0, r]) + 1e-7 * gmax[0]
    comps = [0] + [int(i) for i in np.argsort(-np.abs(lam0[1:, 0]))[:3] + 1]
    for i in comps:
        e = np.zeros(K + 1)
        e[i] = 1.0
        _, dyo = oracle.tlm(om, st0[:, 0], rec[2], p, dy0=e)
        ref = lam[:, 0] @ dyo
        say(f"  lambda0[{i}]: oracle {ref:.10e} gpu {lam0[i, 0]:.10e}")
        assert abs(lam0[i, 0] - ref) <= 1e-7 * abs(ref) + 1e-9 * np.abs(lam0[:, 0]).max()


@pytest.mark.parametrize("kind", ["elementary", "thirdbody"])
def test_adjoint_wg_isomer_closed_form(chem, kind):
    """A <=> B with identical thermo and 68 inert species (N = 71): T stays
    constant and Y_A - Y_B decays as exp(-2 k t), so Y_A(dt) and its
    derivatives are known in closed form."""
    n_inert = 68
    mech = isomer_mech(kind, n_inert=n_inert)
    p, T = 101325.0, 1200.0
    YA, YB = 0.6, 0.1
    st0 = np.zeros((3 + n_inert, 1))
    st0[:3, 0] = [T, YA, YB]
    st0[3:, 0] = 0.3 / n_inert
    lam = np.zeros_like(st0)
    lam[1, 0] = 1.0  # objective Y_A(dt)
    R_u = oracle.gas_constant()
    k = np.exp(mech["lnA"][0] + mech["b"][0] * np.log(T) - mech["theta"][0] / T)
    if kind == "thirdbody":
        k *= 10.0 * p / (R_u * T)
    dt = 0.75 / k
    _, lam0, grad, steps, status = gpu_adjoint(chem, mech, st0, p, dt, 1e-12, 1e-16, lam)
    assert status[0] == 0
    E = np.exp(-2.0 * k * dt)
    dYA_dlnk = 0.5 * (YA - YB) * E * (-2.0 * k * dt)
    dlnk_dT = mech["b"][0] / T + mech["theta"][0] / T ** 2 - (1.0 / T if kind == "thirdbody" else 0.0)
    ref_grad = np.array([dYA_dlnk, dYA_dlnk * np.log(T), -dYA_dlnk / T])
    ref_lam0 = np.zeros(3 + n_inert)
    ref_lam0[:3] = [dYA_dlnk * dlnk_dT, 0.5 * (1 + E), 0.5 * (1 - E)]
    say(f"{kind}: steps {steps[0]}, grad {grad[:, 0]} ref {ref_grad}; lam0[:3] {lam0[:3, 0]} ref {ref_lam0[:3]}")
    np.testing.assert_allclose(grad[:, 0], ref_grad, rtol=1e-7)
    np.testing.assert_allclose(lam0[:, 0], ref_lam0, rtol=1e-7, atol=1e-12)


def test_adjoint_wg_forward_and_replay_invariants(chem):
    """The forward half equals chem_integrate bit for bit; the result does not
    depend on the checkpoint interval and repeats bitwise; a cell whose tape
    overflows is reported and not swept."""
    mech, p = n65()
    nc = 40
    st0 = make_states(mech, nc, 8067, [(900.0, 2200.0)])
    dt, rtol, atol = 1e-6, 1e-6, 1e-10
    ref_out, ref_steps = gpu_integrate(chem, mech, st0, p, dt, rtol, atol)
    lam = objective_lambda(mech["n_species"], nc)
    a = gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam, ck=8)
    assert np.all(a[4] == 0)
    assert np.array_equal(a[0], ref_out) and np.array_equal(a[3], ref_steps)
    for ck, mt in ((8, 0), (1, 2048), (5, 4000)):
        b = gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam, ck=ck, max_tape=mt)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), ck
    cap = int(np.median(ref_steps))
    cap -= cap % 4
    _, lam0, grad, steps, status = gpu_adjoint(chem, mech, st0, p, dt, rtol, atol, lam, ck=4, max_tape=cap)
    full = steps > cap
    say(f"tape {cap}: {full.sum()}/{nc} cells over")
    assert full.any() and (~full).any()
    assert np.all(status[full] == 5) and np.all(status[~full] == 0)
    assert np.all(lam0[:, full] == lam[:, full])
    assert np.array_equal(lam0[:, ~full], a[1][:, ~full])
