"""Pins of the oracle's step-size controller and Seulex order selection (CPU only).

The paper leaves both to "theoretical relations and heuristics" (section 2.3),
so the rules are this library's reading: for the Rosenbrock methods,

  R1  h starts at min(h_in, dt), dt when h_in is not a positive finite number;
  R3  sc_i = atol + rtol max(|y_i|, |ynew_i|) over every component;
  R4  err = sqrt(sum_i (e_i / sc_i)^2 / N);
  R5  fac = min(fac_max, max(fac_min, fac_safe err^(-1/q))), q = 4 (ROS4), 3 (Rodas3);
  R6  accept iff err <= 1;
  R7  after a rejection the next accepted step does not grow h;
  R8  a non-finite err (or ynew) rejects with fac_min;
  R9  the last step is clipped to dt - t and t is then dt exactly;
  R10 h_out is the last unclipped proposal, capped at dt;
  R11 max_steps attempts give TOO_MANY_STEPS, h < h_min gives STEP_UNDERFLOW;
  R12 a zero pivot halves h, at most 5 times in one step, then SINGULAR;

and for the Seulex family (extrapolated linearly implicit Euler, n_j = j,
work A_j = sum_{i<=j} (n_i + 1), column proposals H_j = H min(fac_max,
max(fac_min, fac_safe err_j^(-1/j)))), after an accepted step of k columns:
k-1 if A_{k-1}/H_{k-1} < 0.8 A_k/H_k; else k+1 with H_k A_{k+1}/A_k if k < 6
and A_k/H_k < 0.9 A_{k-1}/H_{k-1}; else k; a rejection keeps k and takes H_k;
no order or step growth right after a rejection.

The test system is y' = diag(lam) y with J = diag(lam) exactly.  On it every
stage of a Rosenbrock step is a rational function of z = h lam_i, and every
entry of the extrapolation table a rational function of H lam_i, so the whole
trace of a run (each attempt's h, error norm and outcome, and the column
count for Seulex) follows in closed form.  `_ros_model` / `_sx_model` below
evaluate the stage recursions in exact rational arithmetic (fractions) from the
published coefficient tables and walk the rules above in plain Python; the
oracle must reproduce the trace.  Each rule has a switch in the model, and the
test cases are chosen so that flipping any one of them changes the trace: a
one-token change to a controller rule in the oracle turns a test red.
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle

# Published tables (Sandu et al. 1997, transformed form of Hairer & Wanner IV.7):
# M K_i = f(y + sum_j a_ij K_j) + sum_j (c_ij/h) K_j, M = I/(gamma h) - J.
ROS4 = dict(
    gamma=0.57282, q=4.0,
    a=[[], [2.0], [1.867943637803922, 0.2344449711399156], [1.867943637803922, 0.2344449711399156, 0.0]],
    c=[[], [-7.137615036412310], [2.580708087951457, 0.6515950076447975],
       [-2.137148994382534, -0.3214669691237626, -0.6949742501781779]],
    m=[2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163],
    e=[-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163])
RODAS3 = dict(
    gamma=0.5, q=3.0,
    a=[[], [0.0], [2.0, 0.0], [2.0, 0.0, 1.0]],
    c=[[], [4.0], [1.0, -1.0], [1.0, -1.0, -8.0 / 3.0]],
    m=[2.0, 0.0, 1.0, 1.0],
    e=[0.0, 0.0, 0.0, 1.0])
TABLES = {"ros4": ROS4, "rodas3": RODAS3}
DEF = dict(max_steps=100000, fac_safe=0.9, fac_min=0.2, fac_max=6.0, h_min=1e-20)
ACC, REJ, NONFIN, SING = 0, 1, 2, 3


# --------------------------------------------------------------- closed forms
def _stage_ratios(tab, z):
    """Exact K_i / y for y' = lam y at z = h lam: (1/gamma - z) k_i = z (1 + sum a_ij k_j) + sum c_ij k_j.
    Also returns the stage points Y_i / y = 1 + sum_j a_ij k_j."""
    g = F(tab["gamma"])
    ks, pts = [], []
    for i in range(4):
        pt = F(1) + sum((F(a) * k for a, k in zip(tab["a"][i], ks)), F(0))
        pts.append(pt)
        num = z * pt + sum((F(c) * k for c, k in zip(tab["c"][i], ks)), F(0))
        ks.append(num / (1 / g - z))
    return ks, pts


def _ros_candidate(tab, lam, y, h, bound):
    """(ynew, err_i, singular, nonfinite) of one attempt, exact then rounded."""
    ynew, err = [], []
    for li, yi in zip(lam, y):
        # the zero-pivot decision is taken on the matrix entry as the
        # integrator rounds it: 1/(gamma h) - lam in FP64
        if 1.0 / (tab["gamma"] * h) - li == 0.0:
            return None, None, True, False
        z = F(h) * F(li)
        ks, pts = _stage_ratios(tab, z)
        # stage i > 0 evaluates f at Y_i; f is NaN there if |Y_i| > bound
        if bound > 0 and any(abs(float(p * F(yi))) > bound for p in pts[1:]):
            return None, None, False, True
        R = 1 + sum(F(mc) * k for mc, k in zip(tab["m"], ks))
        E = sum(F(ec) * k for ec, k in zip(tab["e"], ks))
        ynew.append(float(R * F(yi)))
        err.append(float(E * F(yi)))
    return ynew, err, False, False


def _ros_model(method, lam, y0, dt, rtol, atol, h_in=None, bound=0.0, mut=(), **kw):
    """Trace [(h, err, outcome)], final y, h_out, status, steps, rejects under
    the rules R1..R12; `mut` names rules to flip (the model of a one-token bug)."""
    o = dict(DEF, **kw)
    tab = TABLES[method]
    q = tab["q"] + (1.0 if "exponent" in mut else 0.0)
    N = len(lam)
    valid = h_in is not None and math.isfinite(h_in) and h_in > 0
    hprop = (min(h_in, dt) if "start_min" not in mut else h_in) if valid else dt
    y = [float(v) for v in y0]
    t, rej_last, attempts, steps, rejects = 0.0, False, 0, 0, 0
    trace, status = [], 0
    while t < dt and status == 0:
        nsing = 0
        while True:
            if attempts >= o["max_steps"]:
                status = 1
                break
            if not hprop >= o["h_min"]:
                status = 2
                break
            h, clipped = hprop, False
            if h >= dt - t:
                h, clipped = dt - t, ("no_clip" not in mut)
                if "no_clip" in mut:
                    h = hprop
            attempts += 1
            ynew, err, sing, nonfin = _ros_candidate(tab, lam, y, h, bound)
            if sing:
                trace.append((h, math.nan, SING))
                rejects += 1
                nsing += 1
                if nsing > (5 if "sing_limit" not in mut else 6):
                    status = 3
                    break
                hprop = 0.5 * h if "sing_half" not in mut else 0.2 * h
                rej_last = True
                continue
            if nonfin:
                trace.append((h, math.nan, NONFIN))
                rejects += 1
                hprop = (o["fac_min"] if "nonfinite_fac" not in mut else 0.5) * h
                rej_last = True
                continue
            s2 = 0.0
            for i in range(N):
                big = max(abs(y[i]), abs(ynew[i])) if "sc_max" not in mut else abs(y[i])
                s2 += (err[i] / (atol + rtol * big)) ** 2
            en = math.sqrt(s2 / (N if "rms_mean" not in mut else 1))
            fac = min(o["fac_max"] if "fac_max" not in mut else 5.0,
                      max(o["fac_min"] if "fac_min" not in mut else 0.25,
                          o["fac_safe"] * (en ** (-1.0 / q) if en > 0 else math.inf)))
            if (en <= 1.0) if "accept" not in mut else (en < 0.99):
                trace.append((h, en, ACC))
                steps += 1
                t = dt if clipped else t + h
                y = ynew
                hn = h * fac
                if rej_last and "no_growth" not in mut:
                    hn = min(hn, h)
                if clipped and "h_out" not in mut:
                    hn = max(hn, hprop)
                hprop = hn
                rej_last = False
                break
            trace.append((h, en, REJ))
            rejects += 1
            hprop = h * fac
            rej_last = True
    return trace, y, min(hprop, dt), status, steps, rejects


def _sx_table(lam_i, y_i, H, kcols):
    """Exact extrapolation table entries T[j][l] / y (0-based j, l <= j) for y' = lam y."""
    n = list(range(1, kcols + 1))
    T = []
    for j in range(kcols):
        # n_j linearly implicit Euler substeps of h = H / n_j: y_{m+1} = y_m / (1 - h lam)
        row = [(1 / (1 - F(H) * F(lam_i) / n[j])) ** n[j]]
        for l in range(1, j + 1):
            row.append(row[l - 1] + (row[l - 1] - T[j - 1][l - 1]) / (F(n[j], n[j - l]) - 1))
        T.append(row)
    return T


def _sx_err(y, a, b, rtol, atol):
    s2 = sum(((ai - bi) / (atol + rtol * max(abs(yi), abs(ai)))) ** 2 for yi, ai, bi in zip(y, a, b))
    return math.sqrt(s2 / len(y))


def _sx_model(lam, y0, dt, rtol, atol, h_in=None, mut=(), rec=None, **kw):
    """Seulex-family trace [(h, err, outcome, k)] under the order rules in the module docstring."""
    o = dict(DEF, **kw)
    kmax = 6
    A = [0.0] * (kmax + 2)
    for j in range(1, kmax + 2):
        A[j] = A[j - 1] + (j + 1 if "work" not in mut else j)
    valid = h_in is not None and math.isfinite(h_in) and h_in > 0
    hprop = min(h_in, dt) if valid else dt
    y = [float(v) for v in y0]
    k = 3
    t, rej_last, attempts, steps, rejects = 0.0, False, 0, 0, 0
    trace, status = [], 0

    def hopt(H, e, j):
        return H * min(o["fac_max"], max(o["fac_min"], o["fac_safe"] * (e ** (-1.0 / j) if e > 0 else math.inf)))

    while t < dt and status == 0:
        while True:
            if attempts >= o["max_steps"]:
                status = 1
                break
            H, clipped = hprop, False
            if H >= dt - t:
                H, clipped = dt - t, True
            attempts += 1
            tabs = [_sx_table(li, yi, H, k) for li, yi in zip(lam, y)]
            col = lambda j, l: [float(tb[j][l] * F(yi)) for tb, yi in zip(tabs, y)]
            yk = col(k - 1, k - 1)
            ek = _sx_err(y, yk, col(k - 1, k - 2), rtol, atol)
            Hk = hopt(H, ek, k)
            Hk1 = 0.0
            if k >= 3:
                Hk1 = hopt(H, _sx_err(y, col(k - 2, k - 2), col(k - 2, k - 3), rtol, atol), k - 1)
            if ek <= 1.0:
                trace.append((H, ek, ACC, k))
                steps += 1
                t = dt if clipped else t + H
                y = yk
                lo, hi = (0.8, 0.9) if "thresholds" not in mut else (0.9, 0.8)
                if rec is not None and k >= 3 and Hk1 > 0:
                    rec += [(A[k - 1] / Hk1) / (A[k] / Hk) / lo, (A[k] / Hk) / (A[k - 1] / Hk1) / hi]
                knew, hnew = k, Hk
                if k >= 3 and Hk1 > 0 and A[k - 1] / Hk1 < lo * (A[k] / Hk):
                    knew, hnew = k - 1, Hk1
                elif k < kmax and (k == 2 or Hk1 <= 0 or A[k] / Hk < hi * (A[k - 1] / Hk1)):
                    knew, hnew = k + 1, (Hk * (A[k + 1] / A[k]) if "raise_step" not in mut else Hk)
                if rej_last and "no_growth" not in mut:
                    hnew, knew = min(hnew, H), min(knew, k)
                if clipped:
                    hnew = max(hnew, hprop)
                hprop, k, rej_last = hnew, knew, False
                break
            trace.append((H, ek, REJ, k))
            rejects += 1
            hprop = Hk
            if "reject_order" in mut:
                k = max(2, k - 1)
            rej_last = True
    return trace, y, min(hprop, dt), status, steps, rejects


# ------------------------------------------------------------------ helpers
def _run(method, lam, y0, dt, rtol, atol, h_in=None, bound=0.0, **kw):
    return oracle.controller_test(method, lam, y0, dt, rtol, atol, h=h_in, bound=bound, **kw)


def _same(model, got, seulex=False, hrel=1e-9):
    """Oracle run == model trace: outcomes (and k) exactly, step sizes, final y and h_out to hrel."""
    trace, y, hout, status, steps, rejects = model
    gy, gh, gst, gsteps, grej, gtr = got
    if (status, steps, rejects) != (gst, gsteps, grej) or len(trace) != len(gtr):
        return False
    for (row, g) in zip(trace, gtr):
        if int(g[2]) != row[2] or (seulex and int(g[3]) != row[3]):
            return False
        if abs(g[0] - row[0]) > hrel * abs(row[0]):
            return False
    if abs(gh - hout) > hrel * abs(hout):
        return False
    # components that decayed far below their start carry the relative rounding of many steps
    return np.allclose(gy, y, rtol=hrel, atol=1e-14 * max(1.0, float(np.abs(gy).max())))


def _order_margins_ok(tol=1e-5, **c):
    """No work-per-step comparison of the Seulex order rule is within tol of its threshold."""
    ratios = []
    _sx_model(**c, rec=ratios)
    return all(abs(r - 1.0) > tol for r in ratios)


def _margins_ok(trace, tol=1e-7):
    """No error norm is within tol of the accept threshold (rounding cannot flip a decision)."""
    return all(not (abs(r[1] - 1.0) < tol) for r in trace if math.isfinite(r[1]))


# -------------------------------------------------------------------- cases
# Each case lists the rules whose flip it must detect.
ROS_CASES = {
    # two stiff-ish decays from h_in = dt: rejections clamped by fac_min, growth
    # clamped by fac_max, no growth right after the rejections, a clipped last step
    "decay2": dict(lam=[-3.0e4, -40.0], y0=[1.0, 0.5], dt=2e-2, rtol=1e-4, atol=1e-12,
                   rules=["exponent", "fac_min", "rms_mean", "fac_max", "no_clip", "h_out"]),
    # a growing component decides the scale through max(|y|, |ynew|)
    "growth": dict(lam=[-3.0e3, 20.0], y0=[1.0, 0.5], dt=2e-2, rtol=1e-4, atol=1e-12,
                   rules=["sc_max", "exponent", "h_out"]),
    # h_in larger than dt starts at dt (the min with dt itself is not observable:
    # the clip to dt - t and the cap of h_out at dt cover it)
    "start": dict(lam=[-5.0], y0=[1.0], dt=1e-1, rtol=1e-6, atol=1e-12, h_in=0.5,
                  rules=["fac_min", "h_out", "no_clip"]),
    # f is NaN where |y| > 10: long steps of y' = 200 y overshoot inside a stage
    "nonfinite": dict(lam=[190.0, -5.0], y0=[1.0, 1.0], dt=1e-2, rtol=1e-5, atol=1e-12, bound=10.0,
                      rules=["nonfinite_fac", "no_growth", "exponent", "sc_max"]),
}


@pytest.mark.parametrize("method", ["ros4", "rodas3"])
@pytest.mark.parametrize("case", sorted(ROS_CASES))
def test_ros_controller_trace(method, case, oracle_lib):
    c = dict(ROS_CASES[case])
    rules = c.pop("rules")
    model = _ros_model(method, **c)
    assert _margins_ok(model[0])
    got = _run(method, **c)
    assert _same(model, got), (model[0][:6], got[5][:6], model[2], got[1])
    # the case exercises its rules: the model with any one of them flipped differs
    for r in rules:
        assert not _same(_ros_model(method, **c, mut=(r,)), got), f"case {case} does not pin rule {r}"


def test_ros_trace_properties(oracle_lib):
    """Hand-checkable consequences on the decay case: accepted steps sum to dt
    with the last one clipped, rejections multiply h by at least fac_min, an
    accepted step after a rejection is no larger than the rejected one, and
    steps never grow by more than fac_max."""
    c = dict(ROS_CASES["decay2"])
    c.pop("rules")
    y, hout, st, steps, rej, tr = _run("ros4", **c)
    assert st == 0 and rej >= 3 and steps > 10
    acc = tr[tr[:, 2] == ACC]
    assert math.fsum(acc[:, 0]) == pytest.approx(c["dt"], rel=1e-13)
    assert tr[0, 0] == c["dt"]  # no h_in: the first attempt is dt itself
    for a in range(1, len(tr)):
        ratio = tr[a, 0] / tr[a - 1, 0]
        if tr[a - 1, 2] == REJ:
            assert ratio >= 0.2 * (1 - 1e-15) and ratio < 1.0
        elif a + 1 < len(tr):  # (the last attempt may be clipped)
            assert ratio <= 6.0 * (1 + 1e-15)
        if tr[a - 1, 2] == REJ and tr[a, 2] == ACC and a + 1 < len(tr):
            assert tr[a + 1, 0] <= tr[a, 0] * (1 + 1e-15)
    # the first rejection of an enormous error is clamped at fac_min exactly
    assert tr[0, 2] == REJ and tr[1, 0] == pytest.approx(0.2 * tr[0, 0], rel=1e-15)


@pytest.mark.parametrize("h_in", [None, 0.0, -1.0, math.nan, math.inf, 2.0])
def test_invalid_or_large_h_in_starts_at_dt(h_in, oracle_lib):
    _, _, st, _, _, tr = _run("ros4", [-5.0], [1.0], 1e-3, 1e-6, 1e-12, h_in=h_in)
    assert st == 0 and tr[0, 0] == 1e-3


def test_h_out_is_the_unclipped_proposal(oracle_lib):
    """After a clipped last step the returned h is the proposal that the clip
    shortened, not the clipped step times its factor."""
    c = dict(ROS_CASES["decay2"])
    c.pop("rules")
    trace, _, hout, *_ = _ros_model("ros4", **c)
    y, gh, st, steps, rej, tr = _run("ros4", **c)
    assert tr[-1, 0] < tr[-2, 0]  # the clip shortened the last step
    assert gh == pytest.approx(hout, rel=1e-9)
    # the proposal before the clipped step, carried past it
    assert gh >= tr[-2, 0] and gh < c["dt"]


@pytest.mark.parametrize("method,lam", [("ros4", -66.38), ("rodas3", -29.36)])
def test_accept_threshold_and_clipped_first_step(method, lam, oracle_lib):
    """A first step of h = dt whose error norm is just below 1 (0.995) is
    accepted (accept iff err <= 1), it is clipped (h >= dt - t), so h_out is
    dt although the factor is below 1."""
    c = dict(lam=[lam], y0=[1.0], dt=1e-3, rtol=1e-6, atol=1e-12)
    got = _run(method, **c)
    y, h, st, steps, rej, tr = got
    assert st == 0 and steps == 1 and rej == 0 and 0.99 < tr[0, 1] < 1.0 and h == 1e-3
    assert _same(_ros_model(method, **c), got)
    for r in ("accept", "no_clip", "h_out"):
        assert not _same(_ros_model(method, **c, mut=(r,)), got), r


def test_too_many_steps_and_underflow(oracle_lib):
    y, h, st, steps, rej, tr = _run("ros4", [-3.0e4, -40.0], [1.0, 0.5], 2e-2, 1e-6, 1e-12, max_steps=7)
    assert st == 1 and len(tr) == 7 and steps + rej == 7
    # h_min above the step sizes the error control needs: underflow after the rejections
    y, h, st, steps, rej, tr = _run("ros4", [-3.0e4, -40.0], [1.0, 0.5], 2e-2, 1e-6, 1e-12, h_min=1e-3)
    assert st == 2 and steps == 0 and np.all(tr[:, 0] >= 1e-3) and np.all(tr[:, 2] == REJ)
    # the last rejection proposed a step below h_min (fac_min = 0.2 of 0.004)
    assert tr[-1, 0] == pytest.approx(4e-3, rel=1e-15) and h == pytest.approx(8e-4, rel=1e-15)


def _singular_lams(method, h0, count, n):
    """lam_i = 2^i / (gamma h0) for i < count: 1/(gamma h) - lam_i is exactly zero at h = h0 2^-i."""
    g = TABLES[method]["gamma"] if method != "seulex" else 1.0
    base = 1.0 / (g * h0)
    lam = [base * 2.0 ** i for i in range(count)]
    return lam + [-1.0] * (n - count)


@pytest.mark.parametrize("method", ["ros4", "rodas3", "seulex"])
def test_singular_matrix_halves_h_then_fails(method, oracle_lib):
    """Six singular iteration matrices in a row (h0, h0/2, ..., h0/32) end the
    cell with SINGULAR after six rejections; five are survived."""
    h0, dt = 1e-3, 1e-2
    lam = _singular_lams(method, h0, 6, 7)
    y, h, st, steps, rej, tr = _run(method, lam, [0.0] * 6 + [1.0], dt, 1e-6, 1e-12, h_in=h0)
    assert st == 3 and steps == 0 and rej == 6
    assert np.all(tr[:, 2] == SING) and np.allclose(tr[:, 0], h0 * 0.5 ** np.arange(6), rtol=0, atol=0)
    # five singular halvings, then a regular step at h0/32 and on to dt
    lam = _singular_lams(method, h0, 5, 6)
    c = (lam, [0.0] * 5 + [1.0], dt, 1e-6, 1e-12)
    got = _run(method, *c, h_in=h0)
    y, h, st, steps, rej, tr = got
    assert st == 0 and rej >= 5 and np.all(tr[:5, 2] == SING) and tr[5, 0] == h0 / 32 and tr[5, 2] == ACC
    if method != "seulex":
        assert _same(_ros_model(method, *c, h_in=h0), got)
        assert not _same(_ros_model(method, *c, h_in=h0, mut=("sing_half",)), got)
        # the accepted step after the halvings does not grow h (its error would allow it)
        assert tr[6, 0] == tr[5, 0]
        assert not _same(_ros_model(method, *c, h_in=h0, mut=("no_growth",)), got)


def test_singular_limit_is_five_halvings(oracle_lib):
    """The sixth singular matrix (not the seventh) ends the step."""
    h0 = 1e-3
    lam = _singular_lams("ros4", h0, 6, 7)
    c = (lam, [0.0] * 6 + [1.0], 1e-2, 1e-6, 1e-12)
    got = _run("ros4", *c, h_in=h0)
    assert _same(_ros_model("ros4", *c, h_in=h0), got)
    assert not _same(_ros_model("ros4", *c, h_in=h0, mut=("sing_limit",)), got)
    assert not _same(_ros_model("ros4", *c, h_in=h0, mut=("sing_half",)), got)


# --------------------------------------------------------------- Seulex order
SX_CASES = {
    # a stiff start from h_in = dt at a loose tolerance: rejections keep k, no
    # order growth right after them, the order climbs to 6 and falls back
    "stiff": dict(lam=[-2.0e3, -0.5], y0=[1.0, 1.0], dt=0.05, rtol=1e-3, atol=1e-8,
                  rules=["thresholds", "raise_step", "work", "reject_order", "no_growth"]),
    # a tight tolerance from a small h_in: the order climbs and settles
    "climb": dict(lam=[-400.0, -0.5], y0=[1.0, 1.0], dt=0.3, rtol=1e-7, atol=1e-12, h_in=1e-4,
                  rules=["thresholds", "raise_step", "work", "reject_order", "no_growth"]),
    # a smooth problem at a loose tolerance: low columns win on work per unit step, k falls to 2
    "loose": dict(lam=[-30.0, -7.0], y0=[1.0, 1.0], dt=0.3, rtol=1e-3, atol=1e-8, h_in=1e-4,
                  rules=["thresholds", "raise_step", "work"]),
}


@pytest.mark.parametrize("case", sorted(SX_CASES))
def test_seulex_order_and_step_trace(case, oracle_lib):
    c = dict(SX_CASES[case])
    rules = c.pop("rules")
    model = _sx_model(**c)
    # the extrapolated differences of high columns cancel: the oracle's FP64
    # table carries ~1e-9 relative error in err_k, hence the looser margins
    assert _margins_ok(model[0], tol=1e-5) and _order_margins_ok(**c)
    got = _run("seulex", **c)
    assert _same(model, got, seulex=True, hrel=1e-6), ([r[2:] for r in model[0][:10]], got[5][:10, 2:].tolist())
    ks = [r[3] for r in model[0]]
    assert len(set(ks)) >= 2  # the case moves the order
    for r in rules:
        assert not _same(_sx_model(**c, mut=(r,)), got, seulex=True, hrel=1e-6), f"case {case} does not pin rule {r}"


def test_seulex_order_moves_both_ways(oracle_lib):
    """Across the cases the column count both rises to 6 and falls."""
    ks_all = []
    for case in SX_CASES.values():
        c = dict(case)
        c.pop("rules")
        tr = _run("seulex", **c)[5]
        ks_all.append(tr[:, 3].astype(int))
    assert any(k.max() == 6 for k in ks_all)
    assert any(np.any(np.diff(k) < 0) for k in ks_all)
    assert any(k.min() == 2 for k in ks_all)
