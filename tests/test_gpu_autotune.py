"""The autotuner (chem_autotune, chem_set_variant and the binding's JSON
cache): every launch variant computes the same bits, so the tuned default and
every explicitly selected variant must reproduce the default launch's results
exactly; the cache returns the stored variant without timing."""
import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2105_12070_amd.inputs import WORKLOADS  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def _run(chem, m, st0, w, opt=None, dt=None):
    st = torch.tensor(st0, device=DEV)
    h = torch.zeros(st0.shape[1], dtype=torch.float64, device=DEV)
    steps = torch.zeros(st0.shape[1], dtype=torch.int32, device=DEV)
    status = torch.zeros(st0.shape[1], dtype=torch.int32, device=DEV)
    chem.integrate(m, st, h, w.p_pa, dt or w.dt, w.rtol, w.atol, options=opt, steps=steps, status=status)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (st, h, steps, status)]


@pytest.mark.parametrize("name,n,dt", [("c2_54sp", 700, 2e-7), ("c4_adj", 300, 2e-7), ("c1_10sp", 500, None),
                                       ("c5_150sp", 40, 1e-8)])
def test_tuned_and_explicit_variants_bitwise(chem, tmp_path, name, n, dt):
    w = WORKLOADS[name]
    mech = w.mechanism()
    st0 = w.states(mech, n)
    m = chem.Mechanism(mech)
    ref = _run(chem, m, st0, w, dt=dt)
    assert np.all(ref[3] == 0)
    cache = str(tmp_path / "tune.json")
    h0 = torch.zeros(n, dtype=torch.float64, device=DEV)
    variant, ms = chem.autotune(m, torch.tensor(st0, device=DEV), h0, w.p_pa, dt or w.dt, w.rtol, w.atol,
                                cache=cache)
    say(f"[{name}] tuned {variant} ({ms:.2f} ms)")
    assert ms is not None
    got = _run(chem, m, st0, w, dt=dt)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    # the cache answers the second call, without timing, and installs the variant
    m2 = chem.Mechanism(mech)
    v2, ms2 = chem.autotune(m2, torch.tensor(st0, device=DEV), h0, w.p_pa, dt or w.dt, w.rtol, w.atol, cache=cache)
    assert ms2 is None and v2 == variant
    assert list(json.load(open(cache)).values()) == [variant]
    got2 = _run(chem, m2, st0, w, dt=dt)
    for a, b in zip(ref, got2):
        np.testing.assert_array_equal(a, b)
    # explicit variants: private blocks, shared slots, plain launches
    variants = [dict(persistent=0, waves_per_block=1, jac_slots=-1), dict(persistent=1, waves_per_block=2,
                                                                          jac_slots=-1, grid_mult=2)]
    if w.N > 16 and w.N <= 64:
        variants += [dict(persistent=1, waves_per_block=5, jac_slots=2), dict(persistent=1, waves_per_block=6,
                                                                              jac_slots=3),
                     dict(persistent=0, waves_per_block=7, jac_slots=2), dict(persistent=1, waves_per_block=8,
                                                                              jac_slots=2)]
    if w.N > 64:
        variants = [dict(grid_mult=1), dict(grid_mult=2)]
    for kv in variants:
        out = _run(chem, m, st0, w, chem.Options(**kv), dt=dt)
        for a, b in zip(ref, out):
            np.testing.assert_array_equal(a, b)


def test_set_variant_rejects_what_does_not_fit(chem):
    w = WORKLOADS["c2_54sp"]
    m = chem.Mechanism(w.mechanism())
    for bad in (dict(persistent=1, waves_per_block=8, grid_mult=1, jac_slots=8),  # 8 slots exceed the LDS
                dict(persistent=1, waves_per_block=9, grid_mult=1, jac_slots=2),
                dict(persistent=2, waves_per_block=1, grid_mult=1, jac_slots=-1),
                dict(persistent=1, waves_per_block=5, grid_mult=1, jac_slots=-1)):  # 5 private blocks do not fit
        with pytest.raises(chem.ChemError) as e:
            chem.set_variant(m, bad)
        assert e.value.code == -1
    chem.set_variant(m, dict(persistent=1, waves_per_block=7, grid_mult=1, jac_slots=3))
