"""Pins of the oracle's LU, Rosenbrock tables, step and controller (CPU only)."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2105_12070_amd.inputs import WORKLOADS


# ------------------------------------------------------------------ LU
@pytest.mark.parametrize("n", [1, 2, 7, 11, 55])
def test_lu_matches_lapack_getrf(n, oracle_lib):
    """Same factors and pivots as LAPACK getrf (scipy.linalg.lu_factor) on generic matrices."""
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n))
    LU, piv, info = oracle.lu_factor(A)
    assert info == 0
    LU_ref, piv_ref = scipy.linalg.lu_factor(A)
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(LU, LU_ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [3, 11, 55])
@pytest.mark.parametrize("trans", [False, True])
def test_lu_solve_backward_error(n, trans, oracle_lib):
    rng = np.random.default_rng(7 * n + trans)
    A = rng.standard_normal((n, n)) + np.diag(rng.uniform(-3, 3, n))
    b = rng.standard_normal(n)
    LU, piv, info = oracle.lu_factor(A)
    x = oracle.lu_solve(LU, piv, b, trans)
    Aop = A.T if trans else A
    res = np.abs(Aop @ x - b).max() / (np.abs(A).max() * np.abs(x).max())
    assert res <= 10 * n * np.finfo(float).eps
    np.testing.assert_allclose(x, np.linalg.solve(Aop, b), rtol=1e-9)


def test_lu_reports_singular(oracle_lib):
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    A[:, 1] = 0.0
    _, _, info = oracle.lu_factor(A)
    assert info == 2  # LAPACK convention: 1-based index of the zero pivot


# ------------------------------------------------------- Rosenbrock tables
def _global_error(method, nsteps):
    y, _ = oracle.ros_test(method, 0, 1.0 / nsteps, nsteps, np.array([1.0, 1.0]))
    return np.abs(y - np.array([0.5, 2.0])).max()


@pytest.mark.parametrize("method,order", [("ros4", 4), ("rodas3", 3)])
def test_table_global_order(method, order, oracle_lib):
    """y1' = -y1^2, y2' = y1 y2 from (1,1): exact (1/(1+t), 1+t); error ~ h^order."""
    e = [_global_error(method, n) for n in (20, 40, 80)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(rates - order) < 0.15), rates


@pytest.mark.parametrize("method,order", [("ros4", 4), ("rodas3", 3)])
def test_table_error_estimate_order(method, order, oracle_lib):
    """The embedded estimate of one step is O(h^order) (local error of the lower-order method)."""
    est = []
    for h in (0.1, 0.05, 0.025):
        _, err = oracle.ros_test(method, 0, h, 1, np.array([1.0, 1.0]))
        est.append(np.abs(err).max())
    rates = np.log2(np.array(est[:-1]) / np.array(est[1:]))
    assert np.all(np.abs(rates - order) < 0.2), rates


@pytest.mark.parametrize("method,bound", [("ros4", 2e-5), ("rodas3", 1e-10)])
def test_table_stiff_decay(method, bound, oracle_lib):
    """|R(z)| for z = -1e12 (L-stability in practice) and the estimate stays bounded."""
    y, err = oracle.ros_test(method, 1, 1.0, 1, np.array([1.0, -1e12]))
    assert abs(y[0]) < bound
    assert abs(err[0]) < 1.0


def test_stability_function_near_origin(oracle_lib):
    """R(z) = e^z + O(z^5) for the order-4 table on y' = lambda y."""
    for z in (-1e-2, -2e-2):
        y, _ = oracle.ros_test("ros4", 1, 1.0, 1, np.array([1.0, z]))
        assert abs(y[0] - np.exp(z)) < 5e-2 * abs(z) ** 5


def test_eq2_is_the_one_stage_special_case(oracle_lib):
    """Eq. 2: (I - h J)(y_new - y) = h f.  The 1-stage table must reproduce it exactly."""
    w = WORKLOADS["c1_10sp"]
    m = w.mechanism()
    y0 = w.states(m, 3)[:, 2]
    mm = oracle.Mech(m)
    for h in (1e-12, 1e-10):
        ynew = oracle.replay(mm, y0, np.array([h]), w.p_pa, method="euler")
        J = oracle.jac(mm, w.p_pa, y0)
        f = oracle.rhs(mm, w.p_pa, y0)
        dy = np.linalg.solve(np.eye(len(y0)) - h * J, h * f)
        np.testing.assert_allclose(ynew, y0 + dy, rtol=1e-12, atol=1e-14 * np.abs(y0).max())
