"""Pins of the oracle's ablation modes (CPU only): the one-sided
finite-difference Jacobian that section 2.3 contrasts with the analytical one,
and the LU without pivoting that it contrasts with LAPACK's."""
import numpy as np
import pytest

import oracle
from paper_2105_12070_amd.inputs import WORKLOADS


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["c1_10sp"]
    m = w.mechanism()
    return w, m, w.states(m, 8)


def test_fd_jacobian_matches_analytic_to_truncation(c1, oracle_lib):
    w, mech, st = c1
    om = oracle.Mech(mech)
    for c in range(st.shape[1]):
        y = st[:, c]
        Ja = oracle.jac(om, w.p_pa, y)
        Jf = oracle.jac(om, w.p_pa, y, mode="fd")
        scale = np.abs(Ja).max(axis=1, keepdims=True)
        # one-sided differences: error ~ sqrt(eps) relative to the row scale
        assert np.max(np.abs(Jf - Ja) / scale) < 1e-5
        # and it is a difference quotient, not the analytic matrix
        assert np.max(np.abs(Jf - Ja) / scale) > 1e-12


def test_fd_jacobian_column_is_a_forward_difference(c1, oracle_lib):
    """Column j equals (f(y + d e_j) - f(y)) / d with the documented step."""
    w, mech, st = c1
    om = oracle.Mech(mech)
    y = st[:, 3]
    Jf = oracle.jac(om, w.p_pa, y, mode="fd")
    f0 = oracle.rhs(om, w.p_pa, y)
    for j in (0, 1, 5):
        d = 1.4901161193847656e-08 * max(abs(y[j]), 1e-10)
        d = (y[j] + d) - y[j]
        yp = y.copy()
        yp[j] += d
        col = (oracle.rhs(om, w.p_pa, yp) - f0) / d
        np.testing.assert_array_equal(Jf[:, j], col)


def test_unpivoted_lu_equals_pivoted_without_interchanges_and_fails_on_zero_leading_pivot(oracle_lib):
    rng = np.random.default_rng(4)
    A = rng.standard_normal((9, 9)) + np.diag(np.full(9, 20.0))  # diagonally dominant: no interchanges
    L1, p1, i1 = oracle.lu_factor(A)
    L2, p2, i2 = oracle.lu_factor(A, pivot=False)
    assert i1 == i2 == 0 and np.array_equal(p1, np.arange(9)) and np.array_equal(L1, L2)
    B = np.array([[0.0, 1.0], [1.0, 0.0]])
    assert oracle.lu_factor(B)[2] == 0
    assert oracle.lu_factor(B, pivot=False)[2] == 1
    # generic matrix: no interchanges are made and L U reproduces A
    C = rng.standard_normal((7, 7))
    LU, piv, info = oracle.lu_factor(C, pivot=False)
    assert info == 0 and np.array_equal(piv, np.arange(7))
    Lm = np.tril(LU, -1) + np.eye(7)
    Um = np.triu(LU)
    np.testing.assert_allclose(Lm @ Um, C, atol=1e-9 * np.abs(C).max())


def test_integration_with_ablation_modes_stays_within_tolerance(c1, oracle_lib):
    w, mech, st = c1
    rtol, atol = 1e-8, 1e-12
    ref = oracle.integrate(mech, st, None, w.p_pa, w.dt, rtol, atol)[0]
    fd, _, sfd, rfd, stfd = oracle.integrate(mech, st, None, w.p_pa, w.dt, rtol, atol, jac_mode=1)
    npv, _, snp, rnp, stnp = oracle.integrate(mech, st, None, w.p_pa, w.dt, rtol, atol, lu_pivot=1)
    assert np.all(stfd == 0) and np.all(stnp == 0)
    bound = 100 * (rtol * np.abs(ref) + atol)
    assert np.all(np.abs(fd - ref) <= bound)
    assert np.all(np.abs(npv - ref) <= bound)
