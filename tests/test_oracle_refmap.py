"""Pins of the oracle's reference-cell mapping (section 2.2: the chemistry
solution of a reference cell is mapped onto low-reactivity cells instead of
integrating them; the criterion is the library's stated reading), CPU only.

The expected classification and increments are written out here in numpy from
the definition; the integrated cells are checked against plain integration."""
import numpy as np
import pytest

import oracle
from paper_2105_12070_amd.inputs import WORKLOADS


def classify(st, weight, z0, z_max, dT):
    """The mapping rule written out: zone, reference, mapped set."""
    z = z0 + weight @ st[1:]  # exact for the one-hot indicators used here
    zone = z <= z_max
    if not zone.any():
        return -1, np.full(st.shape[1], -1)
    r = int(np.argmax(zone))
    mapped = zone & (np.abs(st[0] - st[0, r]) <= dT)
    mapped[r] = False
    return r, np.where(mapped, r, -1)


@pytest.fixture(scope="module")
def zonal(oracle_lib):
    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st = w.states(mech, 48)
    return w, mech, st, w.refmap_params()


def test_no_zone_is_plain_integration(zonal):
    w, mech, st, rm = zonal
    a = oracle.integrate_refmap(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol, rm["weight"], 0.0, -1.0, 2.0)
    b = oracle.integrate(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol)
    assert np.all(a[5] == -1)
    for x, y in zip(a[:5], b):
        assert np.array_equal(x, y)


def test_mapped_cells_take_the_reference_increment(zonal):
    w, mech, st, rm = zonal
    out, h, steps, rej, status, ref_of = oracle.integrate_refmap(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol,
                                                                 **rm)
    r, exp = classify(st, rm["weight"], rm["z0"], rm["z_max"], rm["dT"])
    assert r >= 0 and np.array_equal(ref_of, exp)
    mapped = exp >= 0
    assert 10 < mapped.sum() < 48
    # every integrated cell (reference included) equals its plain integration
    plain = oracle.integrate(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol)
    for x, y in zip((out, h, steps, rej, status), plain):
        assert np.array_equal(x[..., ~mapped], y[..., ~mapped])
    # mapped: Phi_c(0) + (Phi_r(dt) - Phi_r(0)), the reference's h and status, no work
    inc = plain[0][:, r] - st[:, r]
    assert np.array_equal(out[:, mapped], st[:, mapped] + inc[:, None])
    assert np.all(h[mapped] == plain[1][r]) and np.all(status[mapped] == plain[4][r])
    assert np.all(steps[mapped] == 0) and np.all(rej[mapped] == 0)
    # mass fractions keep their sum (the reference's increments sum to zero)
    assert np.all(np.abs(out[1:, mapped].sum(axis=0) - st[1:, mapped].sum(axis=0)) < 1e-14)


def test_identical_cells_reproduce_their_own_integration(zonal):
    w, mech, st, rm = zonal
    r, _ = classify(st, rm["weight"], rm["z0"], rm["z_max"], rm["dT"])
    dup = np.repeat(st[:, r:r + 1], 5, axis=1)
    out, *_, ref_of = oracle.integrate_refmap(mech, dup, None, w.p_pa, w.dt, w.rtol, w.atol, **rm)
    assert np.array_equal(ref_of, [-1, 0, 0, 0, 0])
    # a + (b - a) is b up to two roundings of max(|a|, |b|)
    big = np.maximum(np.abs(dup[:, 1:]), np.abs(out[:, :1]))
    assert np.all(np.abs(out[:, 1:] - out[:, :1]) <= 4.5e-16 * big)


def test_temperature_window_is_inclusive(oracle_lib):
    w = WORKLOADS["c1_10sp"]
    mech = w.mechanism()
    st = w.states(mech, 6)
    st[1:, :] = st[1:, :1]  # one composition
    st[1, :] = 0.0          # species 0 absent: the zone indicator
    st[1:] /= st[1:].sum(axis=0)
    st[0] = [1000.0, 1002.0, np.nextafter(1002.0, 2000.0), 998.0, 1000.0, 997.5]
    wt = np.zeros(10)
    wt[0] = 1.0
    *_, ref_of = oracle.integrate_refmap(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol, wt, 0.0, 0.0, 2.0)
    assert np.array_equal(ref_of, [-1, 0, -1, 0, 0, -1])
    # a cell outside the zone is never mapped, even at the reference's temperature
    st2 = st.copy()
    st2[1, 4] = 1e-3
    st2[1:, 4] /= st2[1:, 4].sum()
    *_, ref2 = oracle.integrate_refmap(mech, st2, None, w.p_pa, w.dt, w.rtol, w.atol, wt, 0.0, 0.0, 2.0)
    assert np.array_equal(ref2, [-1, 0, -1, 0, -1, -1])
    # the reference is the zone cell of lowest index: with cell 0 out of the
    # zone it is cell 1 (1002 K), and the window moves with it
    st3 = st.copy()
    st3[1, 0] = 1e-3
    st3[1:, 0] /= st3[1:, 0].sum()
    *_, ref3 = oracle.integrate_refmap(mech, st3, None, w.p_pa, w.dt, w.rtol, w.atol, wt, 0.0, 0.0, 2.0)
    assert np.array_equal(ref3, [-1, -1, 1, -1, 1, -1])


def test_mapping_error_is_first_order_in_the_temperature_offset(zonal):
    """Mapping is an approximation: a mapped cell's own increment differs from
    the reference's by a term proportional to their temperature offset (the
    jittered ambient cells re-equilibrate).  Scaling every offset by 1/10
    scales the error by about 1/10; identical cells map exactly (above)."""
    w, mech, st, rm = zonal
    r, exp = classify(st, rm["weight"], rm["z0"], rm["z_max"], rm["dT"])
    mapped = exp >= 0
    errs = []
    for scale in (1.0, 0.1):
        s2 = st.copy()
        s2[0, mapped] = st[0, r] + scale * (st[0, mapped] - st[0, r])
        out, *_, ref_of = oracle.integrate_refmap(mech, s2, None, w.p_pa, w.dt, w.rtol, w.atol, **rm)
        assert np.array_equal(ref_of, exp)
        own = oracle.integrate(mech, s2, None, w.p_pa, w.dt, w.rtol, w.atol)[0]
        errs.append(np.abs(out[0, mapped] - own[0, mapped]).max())  # temperature, K
    print(f"mapping error in T: {errs[0]:.3e} K (offsets up to 2 K), {errs[1]:.3e} K (offsets / 10)")
    assert 0.04 < errs[1] / errs[0] < 0.25
