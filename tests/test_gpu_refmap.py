"""Reference-cell mapping on the GPU against the oracle's (same seeded zonal
workload), through the C ABI: the classification is exact, mapped cells carry
the reference's increment bit for bit, integrated cells match the oracle
within the integration bound and the unmapped integration bitwise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, make_states  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def run(chem, m, st0, p, dt, rtol, atol, rm=None, ref_out=True, **opt):
    nc = st0.shape[1]
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = torch.zeros(nc, dtype=torch.int32, device=DEV)
    rej = torch.zeros(nc, dtype=torch.int32, device=DEV)
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    ref_of = torch.full((nc,), 7, dtype=torch.int32, device=DEV) if (rm and ref_out) else None
    refmap = None
    if rm is not None:
        refmap = chem.RefMap(torch.tensor(rm["weight"], device=DEV), rm["z0"], rm["z_max"], rm["dT"], ref_of)
    chem.integrate(m, s, h, p, dt, rtol, atol, options=chem.Options(refmap=refmap, **opt), steps=steps,
                   rejects=rej, status=status)
    torch.cuda.synchronize()
    out = [s.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), rej.cpu().numpy(), status.cpu().numpy()]
    out.append(ref_of.cpu().numpy() if ref_of is not None else None)
    return out


def classify(st, weight, z0, z_max, dT):
    z = z0 + weight @ st[1:]  # exact for one-hot indicators
    zone = z <= z_max
    if not zone.any():
        return np.full(st.shape[1], -1)
    r = int(np.argmax(zone))
    mapped = zone & (np.abs(st[0] - st[0, r]) <= dT)
    mapped[r] = False
    return np.where(mapped, r, -1)


def check_mapped(st0, out, ref_of):
    mapped = ref_of >= 0
    if not mapped.any():
        return
    r = int(ref_of[mapped][0])
    assert np.all(ref_of[mapped] == r)
    inc = out[0][:, r] - st0[:, r]
    assert np.array_equal(out[0][:, mapped], st0[:, mapped] + inc[:, None])
    assert np.all(out[1][mapped] == out[1][r]) and np.all(out[4][mapped] == out[4][r])
    assert np.all(out[2][mapped] == 0) and np.all(out[3][mapped] == 0)


def test_refmap_matches_oracle(chem):
    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 384)
    rm = w.refmap_params()
    m = chem.Mechanism(mech)
    g = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, rm)
    ref = oracle.integrate_refmap(mech, st0, None, w.p_pa, w.dt, w.rtol, w.atol, **rm)
    assert np.array_equal(g[5], ref[5])
    assert np.array_equal(g[5], classify(st0, **rm))
    mapped = g[5] >= 0
    print(f"[refmap] {mapped.sum()} of {len(mapped)} cells mapped")
    assert mapped.sum() > 100
    check_mapped(st0, g, g[5])
    assert np.all(g[4] == 0)
    bound = 100 * (w.rtol * np.abs(ref[0]) + w.atol)
    dev_ = np.abs(g[0] - ref[0])
    print(f"[refmap] max dev / bound {np.max(dev_ / bound):.3e}")
    assert np.all(dev_ <= bound)
    # the integrated cells are those of a run without mapping, bit for bit
    plain = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol)
    for x, y in zip(g[:5], plain[:5]):
        assert np.array_equal(x[..., ~mapped], y[..., ~mapped])


@pytest.mark.parametrize("method", [0, 2])
def test_refmap_launch_shapes_graph_and_order(chem, method):
    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 777)
    rm = w.refmap_params()
    m = chem.Mechanism(mech)
    base = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, rm, method=method, persistent=1)
    check_mapped(st0, base, base[5])
    variants = [dict(persistent=0, waves_per_block=1), dict(persistent=0), dict(persistent=1, grid_mult=2)]
    for v in variants:
        o = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, rm, method=method, **v)
        for x, y in zip(o, base):
            assert np.array_equal(x, y), v
    # library-owned flags (ref_of NULL) give the same results
    o = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, rm, ref_out=False, method=method)
    for x, y in zip(o[:5], base[:5]):
        assert np.array_equal(x, y)
    # cost order (steps of a previous call) and graph replays with eager work between
    nc = st0.shape[1]
    wt = torch.tensor(rm["weight"], device=DEV)
    ref_of = torch.zeros(nc, dtype=torch.int32, device=DEV)
    refmap = chem.RefMap(wt, rm["z0"], rm["z_max"], rm["dT"], ref_of)
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(nc, dtype=torch.float64, device=DEV)
    steps = torch.tensor(np.random.default_rng(5).integers(0, 900, nc).astype(np.int32), device=DEV)
    rej = torch.zeros(nc, dtype=torch.int32, device=DEV)
    status = torch.zeros(nc, dtype=torch.int32, device=DEV)
    opt = chem.Options(method=method, persistent=1, cost_order=1, use_graph=1, refmap=refmap)
    for rep in range(3):
        s.copy_(torch.tensor(st0, device=DEV))
        h.zero_()
        chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, rejects=rej, status=status)
        torch.cuda.synchronize()
        got = [s.cpu().numpy(), h.cpu().numpy(), steps.cpu().numpy(), rej.cpu().numpy(), status.cpu().numpy(),
               ref_of.cpu().numpy()]
        for x, y in zip(got, base):
            assert np.array_equal(x, y), rep
        _ = torch.randn(1000, device=DEV).sum().item()  # eager work between replays


def test_refmap_full_size(chem):
    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech)
    rm = w.refmap_params()
    m = chem.Mechanism(mech)
    g = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, rm)
    exp = classify(st0, **rm)
    assert np.array_equal(g[5], exp)
    check_mapped(st0, g, g[5])
    assert np.all(g[4] == 0)
    # sampled integrated cells (the reference among them) against the oracle
    integ = np.nonzero(g[5] < 0)[0]
    r = int(g[5][g[5] >= 0][0])
    idx = np.unique(np.concatenate([[r], integ[:: max(1, len(integ) // 40)]]))
    ref = oracle.integrate(mech, np.ascontiguousarray(st0[:, idx]), None, w.p_pa, w.dt, w.rtol, w.atol)
    bound = 100 * (w.rtol * np.abs(ref[0]) + w.atol)
    assert np.all(np.abs(g[0][:, idx] - ref[0]) <= bound)
    print(f"[refmap full] mapped {np.mean(g[5] >= 0):.3f}; steps mean {g[2].mean():.1f}")


def test_refmap_edge_cases(chem):
    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 200)
    rm = w.refmap_params()
    m = chem.Mechanism(mech)
    plain = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol)
    # empty zone: the plain integration
    g = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, dict(rm, z_max=-1.0))
    assert np.all(g[5] == -1)
    for x, y in zip(g[:5], plain[:5]):
        assert np.array_equal(x, y)
    # infinite window: the whole zone but the reference is mapped
    g = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, dict(rm, dT=float("inf")))
    assert np.array_equal(g[5], classify(st0, **dict(rm, dT=float("inf"))))
    check_mapped(st0, g, g[5])
    # every cell in the zone: all but cell 0 mapped
    g = run(chem, m, st0, w.p_pa, w.dt, w.rtol, w.atol, dict(rm, z_max=10.0, dT=float("inf")))
    assert g[5][0] == -1 and np.all(g[5][1:] == 0)
    check_mapped(st0, g, g[5])
    # empty input and invalid parameters
    e = torch.zeros((55, 0), dtype=torch.float64, device=DEV)
    he = torch.zeros(0, dtype=torch.float64, device=DEV)
    chem.integrate(m, e, he, w.p_pa, w.dt, w.rtol, w.atol,
                   options=chem.Options(refmap=chem.RefMap(torch.tensor(rm["weight"], device=DEV), 0.0, 1.0, 1.0)))
    s = torch.tensor(st0, device=DEV)
    h = torch.zeros(200, dtype=torch.float64, device=DEV)
    wt = torch.tensor(rm["weight"], device=DEV)
    for bad in (dict(z_max=float("nan")), dict(dT=-1.0), dict(z0=float("nan"))):
        kw = dict(dict(z0=0.0, z_max=1e-10, dT=2.0), **bad)
        with pytest.raises(chem.ChemError):
            chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol,
                           options=chem.Options(refmap=chem.RefMap(wt, kw["z0"], kw["z_max"], kw["dT"])))
    with pytest.raises(chem.ChemError):
        chem.integrate_adjoint(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, torch.ones_like(s),
                               options=chem.Options(refmap=chem.RefMap(wt, 0.0, 1e-10, 2.0)))


def test_refmap_workgroup_path(chem):
    """N > 64 (one cell per workgroup): identical cells are mapped onto the
    first; the others integrate as without mapping."""
    w = WORKLOADS["c5_150sp"]
    mech = w.mechanism()
    st0 = w.states(mech, 8)
    st0[:, 4:] = st0[:, 3:4]
    st0[1, 3:] = 0.0       # species 0 absent in the zone cells 3..7
    st0[1:, 3:] /= st0[1:, 3:].sum(axis=0)
    st0[1, :3] = np.maximum(st0[1, :3], 1e-3)
    st0[1:, :3] /= st0[1:, :3].sum(axis=0)
    wt = np.zeros(150)
    wt[0] = 1.0
    rm = dict(weight=wt, z0=0.0, z_max=0.0, dT=0.0)
    m = chem.Mechanism(mech)
    dt = 1e-7
    g = run(chem, m, st0, w.p_pa, dt, w.rtol, w.atol, rm)
    assert np.array_equal(g[5], [-1, -1, -1, -1, 3, 3, 3, 3])
    check_mapped(st0, g, g[5])
    plain = run(chem, m, st0, w.p_pa, dt, w.rtol, w.atol)
    for x, y in zip(g[:5], plain[:5]):
        assert np.array_equal(x[..., :4], y[..., :4])
    # identical cells: a + (b - a) is b up to two roundings of max(|a|, |b|)
    big = np.maximum(np.abs(st0[:, 4:]), np.abs(plain[0][:, 4:]))
    assert np.all(np.abs(g[0][:, 4:] - plain[0][:, 4:]) <= 4.5e-16 * big)
