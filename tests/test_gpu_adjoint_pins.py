"""The discrete adjoint against the oracle's forward sensitivities and against
finite differences, entry by entry (53 species / 325 reactions, 975
Arrhenius parameters).

* Full sensitivity matrix: every entry of d Phi(dt) / d (Phi0, lnA, b,
  theta)  (54 x 1029) from the oracle's tangent-linear replay of its own
  accepted steps, against the GPU adjoint called once per output component
  (lambda_final = e_i gives row i: lambda0 and the parameter gradient), on 2
  cells over 2e-10 s (a few hundred steps), |dS| <= 1e-10 max(|S|, 1e-6
  max_row |S|), and on 64 cells over 2e-11 s, |dS| <= 1e-12 max_row |S| and
  |dS| <= 1e-11 |S| where |S| >= 1e-3 max_row |S|.
* All 975 parameters on 32 cells: the gradient of Psi = sum_cells
  [T + w.Y](dt) against central differences with replayed step sizes
  (tests/golden/make_adjoint_fd.py, oracle only), |dg| <= 1e-5 max(|g|,
  1e-3 max|g|) per parameter.
* 20 random parameters on 1,024 cells: against the oracle's tangent-linear
  derivative of the same replays, |dg| <= 1e-9 max(|g|, 1e-6 max|g|) (summed
  over 1,024 cells, the central differences' rounding noise, ~1e-4 absolute,
  exceeds the difference bound for the smallest entries; their deviation is
  reported).  The same 20 parameters on all 16,384 cells of the workload
  against the oracle's tangent-linear derivatives (make_adjoint_fd.py
  all-cells), same bound.
Cells are compared only where the GPU takes the oracle's number of steps (the
adjoint differentiates the GPU's own step sequence).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, objective_weights  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    from paper_2105_12070_amd import chem as c
    assert torch.cuda.is_available()
    return c


def _adjoint(chem, m, st0, w, dt, lam):
    s0 = torch.tensor(np.ascontiguousarray(st0), device=DEV)
    h = torch.zeros(st0.shape[1], dtype=torch.float64, device=DEV)
    out, lam0, grad, steps, status = chem.integrate_adjoint(m, s0, h, w.p_pa, dt, w.rtol, w.atol,
                                                            torch.tensor(np.ascontiguousarray(lam), device=DEV),
                                                            max_tape=8192)
    torch.cuda.synchronize()
    return lam0.cpu().numpy(), grad.cpu().numpy().reshape(-1), steps.cpu().numpy(), status.cpu().numpy()


@pytest.mark.timeout(600)
def test_full_sensitivity_matrix(chem):
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    m = chem.Mechanism(mech)
    om = oracle.Mech(mech)
    dt = 2e-10
    N = w.N
    st = w.states(mech, 2)
    for c in range(st.shape[1]):
        y, h, hs, status, _ = oracle.integrate_record(om, st[:, c], None, w.p_pa, dt, w.rtol, w.atol)
        assert status == 0
        say(f"[cell {c}] oracle: {len(hs)} steps; tangent-linear matrix")
        S = oracle.tlm_matrix(om, st[:, c], hs, w.p_pa)
        G = np.zeros_like(S)
        for i in range(N):
            lam = np.zeros((N, 1))
            lam[i, 0] = 1.0
            lam0, grad, steps, stat = _adjoint(chem, m, st[:, c:c + 1], w, dt, lam)
            assert stat[0] == 0 and steps[0] == len(hs), (steps[0], len(hs))
            G[i, :N] = lam0[:, 0]
            G[i, N:] = grad
        scale = np.maximum(np.abs(S), 1e-6 * np.abs(S).max(axis=1, keepdims=True))
        ratio = np.abs(G - S) / scale
        say(f"[cell {c}] max |dS| / scale {ratio.max():.3e} (state block {ratio[:, :N].max():.3e}, "
            f"parameter block {ratio[:, N:].max():.3e}) over {S.size} entries")
        assert ratio.max() <= 1e-10, np.unravel_index(np.argmax(ratio), ratio.shape)


@pytest.mark.timeout(900)
def test_full_sensitivity_matrix_64_cells(chem):
    """The whole 54 x 1,029 matrix on 64 cells spread over the workload's 16,384, over dt = 2e-11 s (50 to 200 steps
    each, so that the oracle's 64 matrices take minutes): one single-cell adjoint call per output component and cell
    (lambda_final = e_i gives row i), every entry against the oracle's tangent-linear matrix.

    The adjoint and the tangent-linear replay sum the same chain-rule terms in opposite orders, so the rounding error
    of an entry follows the size of the terms of its row, not of the entry: an entry that is the small difference of
    large terms carries an absolute error of a few ulps of the row's largest entry.  Two bounds: |dS| <= 1e-12
    max_row |S| on every entry, and |dS| <= 1e-11 |S| on entries of at least 1e-3 max_row |S|."""
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    m = chem.Mechanism(mech)
    om = oracle.Mech(mech)
    dt = 2e-11
    N = w.N
    idx = np.linspace(0, w.n_cells - 1, 64).astype(np.int64)
    st = np.ascontiguousarray(w.states(mech, w.n_cells)[:, idx])
    worst_abs, worst_rel, compared = 0.0, 0.0, 0
    for c in range(st.shape[1]):
        y, h, hs, status, _ = oracle.integrate_record(om, st[:, c], None, w.p_pa, dt, w.rtol, w.atol)
        assert status == 0
        S = oracle.tlm_matrix(om, st[:, c], hs, w.p_pa)
        G = np.zeros_like(S)
        same = True
        for i in range(N):
            lam = np.zeros((N, 1))
            lam[i, 0] = 1.0
            lam0, grad, steps, stat = _adjoint(chem, m, st[:, c:c + 1], w, dt, lam)
            assert stat[0] == 0
            if steps[0] != len(hs):
                same = False
                break
            G[i, :N] = lam0[:, 0]
            G[i, N:] = grad
        if not same:
            say(f"[cell {idx[c]}] step count differs from the oracle's ({len(hs)}): not compared")
            continue
        rowmax = np.abs(S).max(axis=1, keepdims=True)
        d = np.abs(G - S)
        ab = (d / rowmax).max()
        big = np.abs(S) >= 1e-3 * rowmax
        rel = (d[big] / np.abs(S[big])).max()
        worst_abs, worst_rel = max(worst_abs, ab), max(worst_rel, rel)
        compared += 1
        if c % 8 == 0:
            say(f"[cell {idx[c]}] {len(hs)} steps, max |dS| / max_row |S| {ab:.3e}, relative on the large entries "
                f"{rel:.3e}")
    say(f"64 cells: {compared} compared ({compared * N * (N + 3 * w.n_reactions)} entries), max |dS| / max_row |S| "
        f"{worst_abs:.3e}, max |dS| / |S| where |S| >= 1e-3 max_row |S|: {worst_rel:.3e}")
    assert compared >= 56
    assert worst_abs <= 1e-12
    assert worst_rel <= 1e-11


@pytest.fixture(scope="module")
def fd():
    with np.load(os.path.join(HERE, "golden", "adjoint_fd.npz"), allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    with open(os.path.join(HERE, "golden", "adjoint_fd.json")) as f:
        meta = json.load(f)
    return g, meta


def _fd_case(chem, fd, ncells):
    g, meta = fd
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    st = w.states(mech, 1024)
    assert hashlib.sha256(st.tobytes()).hexdigest() == meta["input_sha256"], "input generator changed"
    st = np.ascontiguousarray(st[:, :ncells])
    weights = np.concatenate([[1.0], objective_weights(w.n_species)])
    m = chem.Mechanism(mech)
    # first pass: which cells take the oracle's number of steps
    lam = np.repeat(weights[:, None], ncells, axis=1)
    _, _, steps, status = _adjoint(chem, m, st, w, meta["dt"], lam)
    assert np.all(status == 0)
    same = steps == g["steps"][:ncells]
    say(f"{ncells} cells: {same.sum()} with the oracle's step count")
    assert same.sum() >= 0.9 * ncells
    lam[:, ~same] = 0.0
    _, grad, _, _ = _adjoint(chem, m, st, w, meta["dt"], lam)
    return grad, same


def _fd_check(got, ref, tag, rel=1e-5, floor=1e-3):
    bound = rel * np.maximum(np.abs(ref), floor * np.abs(ref).max())
    ratio = np.abs(got - ref) / bound
    say(f"[{tag}] max |dg| / bound {ratio.max():.3e}, median {np.median(ratio):.3e}")
    assert np.all(ratio <= 1.0), (np.argmax(ratio), got[np.argmax(ratio)], ref[np.argmax(ratio)])


def test_fd_all_parameters_32_cells(chem, fd):
    grad, same = _fd_case(chem, fd, 32)
    ref = fd[0]["all32"][same].sum(axis=0)
    _fd_check(grad, ref, "975 parameters, 32 cells")


def test_random_parameters_1024_cells(chem, fd):
    grad, same = _fd_case(chem, fd, 1024)
    pick = fd[0]["pick"]
    fdv = fd[0]["rand1k"][same].sum(axis=0)
    dev = np.abs(grad[pick] - fdv)
    say(f"[20 parameters, 1,024 cells] central differences: max |dg| {dev.max():.3e} "
        f"(max |g| {np.abs(fdv).max():.3e})")
    ref = fd[0]["tlm1k"][same].sum(axis=0)
    _fd_check(grad[pick], ref, "20 parameters, 1,024 cells, tangent-linear", rel=1e-9, floor=1e-6)


def test_random_parameters_all_cells(chem):
    with np.load(os.path.join(HERE, "golden", "adjoint_tlm_all.npz"), allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    with open(os.path.join(HERE, "golden", "adjoint_tlm_all.json")) as f:
        meta = json.load(f)
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    st = w.states(mech, w.n_cells)
    assert hashlib.sha256(st.tobytes()).hexdigest() == meta["input_sha256"], "input generator changed"
    n = st.shape[1]
    weights = np.concatenate([[1.0], objective_weights(w.n_species)])
    m = chem.Mechanism(mech)
    lam = np.repeat(weights[:, None], n, axis=1)
    _, _, steps, status = _adjoint(chem, m, st, w, meta["dt"], lam)
    assert np.all(status == 0)
    same = steps == g["steps"]
    say(f"{n} cells: {same.sum()} with the oracle's step count")
    assert same.sum() >= 0.9 * n
    lam[:, ~same] = 0.0
    _, grad, _, _ = _adjoint(chem, m, st, w, meta["dt"], lam)
    ref = g["tlm"][same].sum(axis=0)
    _fd_check(grad[g["pick"]], ref, f"20 parameters, {n} cells, tangent-linear", rel=1e-9, floor=1e-6)
