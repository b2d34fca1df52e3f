"""Exercised under AddressSanitizer + UndefinedBehaviorSanitizer by
test_sanitizers.py (run in a child process with the sanitizer runtime
preloaded): every host-side entry point of the oracle, and the host-side
validation and packing of the C-ABI library (no GPU needed: the library
stops at its first device call)."""
import ctypes as C
import sys

import numpy as np

sys.path.insert(0, sys.argv[3])


def oracle_part(lib_path):
    import oracle.oracle as OO
    OO._lib = C.CDLL(lib_path)
    OO._lib.oracle_gas_constant.restype = C.c_double
    import oracle
    from paper_2105_12070_amd.inputs import WORKLOADS
    for name in ("c1_10sp", "c2_54sp"):
        w = WORKLOADS[name]
        mech = w.mechanism()
        st = w.states(mech, 3)
        for method in ("ros4", "rodas3", "seulex"):
            r = oracle.integrate(mech, st, None, w.p_pa, 1e-7, w.rtol, w.atol, method=method, nthreads=2)
            assert np.all(r[4] == 0), (name, method)
        oracle.integrate(mech, st, None, w.p_pa, 1e-8, w.rtol, w.atol, jac_mode=1, lu_pivot=1, nthreads=1)
        for mode in ("analytic", "ad", "fd"):
            assert np.all(np.isfinite(oracle.jac(mech, w.p_pa, st[:, 0], mode)))
        oracle.rates(mech, w.p_pa, st[:, 0])
        oracle.op_counts(mech, w.p_pa, st[:, 0])
        y, h, hs, status, _ = oracle.integrate_record(mech, st[:, 0], None, w.p_pa, 1e-8, w.rtol, w.atol)
        oracle.tlm(mech, st[:, 0], hs, w.p_pa, dy0=np.ones(w.N))
        rm = np.zeros(w.n_species)
        rm[0] = 1.0
        oracle.integrate_refmap(mech, st, None, w.p_pa, 1e-8, w.rtol, w.atol, rm, 0.0, 1.0, 5.0, nthreads=1)
    A = np.random.default_rng(0).standard_normal((7, 7))
    LU, piv, info = oracle.lu_factor(A)
    oracle.lu_solve(LU, piv, np.ones(7), trans=True)
    oracle.controller_test("ros4", [-3e4, -40.0], [1.0, 0.5], 2e-2, 1e-4, 1e-12)
    oracle.controller_test("seulex", [-400.0, -0.5], [1.0, 1.0], 0.3, 1e-7, 1e-12, h=1e-4)
    oracle.controller_test("rodas3", [190.0, -5.0], [1.0, 1.0], 1e-2, 1e-5, 1e-12, bound=10.0)
    oracle.ros_test("ros4", 0, 0.05, 4, [1.0, 1.0])
    oracle.sx_test(0, 0.1, 3, 4, [1.0, 1.0])


def library_part(lib_path):
    from paper_2105_12070_amd import chem
    from paper_2105_12070_amd.inputs import WORKLOADS
    chem.LIB_PATH = lib_path
    L = chem.lib()
    out = C.c_void_p()
    assert L.chem_load_mechanism(None, C.byref(out)) == -1
    for name in ("c1_10sp", "c2_54sp", "c5_150sp"):
        m = WORKLOADS[name].mechanism()
        cases = {"ok": dict(m)}
        cases["W"] = dict(m, W=m["W"].copy())
        cases["W"]["W"][1] = -1.0
        cases["reac"] = dict(m, reac=m["reac"].copy())
        cases["reac"]["reac"][0, 0] = 10_000
        cases["elem"] = dict(m, prod=m["prod"].copy())
        cases["elem"]["prod"][1][0] = (cases["elem"]["prod"][1][0] + 3) % m["n_species"]
        cases["noelem"] = dict(m, elem=None)
        for tag, desc in cases.items():
            try:
                chem.Mechanism(desc)
            except chem.ChemError as e:
                # without a GPU a valid mechanism stops at its first device call
                assert (e.code == -1) == (tag in ("W", "reac", "elem")), (name, tag, str(e))
    vp = None
    assert L.chem_integrate(vp, 4, 4, vp, vp, 1e5, 1e-6, 1e-6, 1e-10, vp, vp, vp, vp, vp) == -1
    assert L.chem_integrate_noalloc(vp, 4, 4, vp, vp, 1e5, 1e-6, 1e-6, 1e-10, vp, vp, vp, vp, vp) == -1
    assert L.chem_lu_solve(1, 0, vp, vp, vp, vp) == -1
    assert L.chem_lu_factor(1, 300, vp, vp, vp, vp, vp) == -1
    assert L.chem_failed_count(vp, vp, vp) == -1
    assert L.chem_set_adjoint_record_budget(C.c_uint64(1 << 20)) == 0
    assert L.chem_max_n() == 255


if __name__ == "__main__":
    {"oracle": oracle_part, "library": library_part}[sys.argv[1]](sys.argv[2])
    print("sanitized run ok", sys.argv[1], flush=True)
