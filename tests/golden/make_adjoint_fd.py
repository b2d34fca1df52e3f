#!/usr/bin/env python3
"""Writes adjoint_fd.npz: central finite differences of the adjoint
workload's objective with respect to the Arrhenius parameters, replaying the
oracle's own accepted step sizes (with the controller re-run, the step
sequence would change under the perturbation and the differences would be
meaningless).

Workload: the 53-species / 325-reaction mechanism (c4_adj) at its pressure,
rtol 1e-6, atol 1e-10, over dt = 2e-10 s (a few hundred steps per cell: the
initial transients of the random states are that fast), objective
Psi = sum_cells [T + sum_k w_k Y_k](dt) with the seeded weights w.  Steps:
1e-6 for lnA and b, 1e-6 max(|theta|, 1) for theta.

  * all 975 parameters on the first 32 cells (per-cell differences stored);
  * 20 seeded random parameters on the first 1,024 cells (per cell), as
    central differences and as the oracle's tangent-linear derivative of the
    same replay.  Summed over 1,024 cells the differences carry the rounding
    noise of every cell's replay (about 1e-14 of Psi per cell over a few
    hundred steps, divided by the 1e-6 step): about 1e-4 absolute, above the
    bound for the smallest entries, so that check uses the tangent-linear
    values, which are exact derivatives of the replayed map.

The oracle's step counts per cell are stored so that the GPU test compares
only cells whose adjoint takes the same steps.  Only the oracle is called.
Run from the repository root:  python tests/golden/make_adjoint_fd.py

With the argument "all-cells" it writes adjoint_tlm_all.npz instead: the same
20 parameters' tangent-linear derivatives of each cell's objective on all
16,384 cells of the workload (the generator's 16,384-cell draw, which is not
an extension of its 1,024-cell one), with the oracle's step counts.
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, objective_weights  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "adjoint_fd.npz")
OUT_ALL = os.path.join(HERE, "adjoint_tlm_all.npz")
DT = 2e-10


def fd_column(mech, w, st, recs, weights, kind, r, cells):
    """Central difference of each cell's objective along parameter (kind, r)."""
    base = {k: np.array(mech[k], dtype=np.float64) for k in ("lnA", "b", "theta")}
    key = ("lnA", "b", "theta")[kind]
    step = 1e-6 if kind < 2 else 1e-6 * max(abs(base[key][r]), 1.0)
    vals = []
    for sgn in (1.0, -1.0):
        prm = {k: v.copy() for k, v in base.items()}
        prm[key][r] += sgn * step
        om = oracle.Mech(mech, **prm)
        vals.append(np.array([oracle.replay(om, st[:, c], recs[c][2], w.p_pa) @ weights for c in cells]))
    return (vals[0] - vals[1]) / (2.0 * step)


def tlm_column(mech, w, st, recs, weights, kind, r, cells):
    """Each cell's d Psi_c / d p along parameter (kind, r) by the tangent-linear replay."""
    R = mech["n_reactions"]
    d = [np.zeros(R), np.zeros(R), np.zeros(R)]
    d[kind][r] = 1.0
    om = oracle.Mech(mech)
    return np.array([oracle.tlm(om, st[:, c], recs[c][2], w.p_pa, dlnA=d[0], db=d[1], dtheta=d[2])[1] @ weights
                     for c in cells])


def pick_parameters(R):
    rng = np.random.default_rng(4005)
    return np.sort(rng.choice(3 * R, 20, replace=False))


def cell_tlm_row(mech, om, w, y0, weights, pick):
    """One cell: record its accepted steps, then d Psi_c / d p for each picked parameter."""
    R = mech["n_reactions"]
    rec = oracle.integrate_record(om, y0, None, w.p_pa, DT, w.rtol, w.atol)
    assert rec[3] == 0
    row = np.zeros(len(pick))
    for j, q in enumerate(pick):
        d = [np.zeros(R), np.zeros(R), np.zeros(R)]
        d[q // R][q % R] = 1.0
        row[j] = oracle.tlm(om, y0, rec[2], w.p_pa, dlnA=d[0], db=d[1], dtheta=d[2])[1] @ weights
    return len(rec[2]), row


def main_all_cells():
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    weights = np.concatenate([[1.0], objective_weights(w.n_species)])
    st = w.states(mech, w.n_cells)
    om = oracle.Mech(mech)
    pick = pick_parameters(mech["n_reactions"])
    t0 = time.time()
    out = [None] * w.n_cells

    def work(c):
        out[c] = cell_tlm_row(mech, om, w, st[:, c], weights, pick)
        if c % 1024 == 0:
            print(f"cell {c}: {time.time() - t0:.0f} s", flush=True)

    with ThreadPoolExecutor(os.cpu_count() or 8) as ex:
        list(ex.map(work, range(w.n_cells)))
    steps = np.array([o[0] for o in out], dtype=np.int32)
    tlm = np.stack([o[1] for o in out])  # [n_cells, 20]
    np.savez(OUT_ALL, steps=steps, pick=pick, tlm=tlm)
    meta = {"dt": DT, "rtol": w.rtol, "atol": w.atol, "n_cells": w.n_cells,
            "input_sha256": hashlib.sha256(st.tobytes()).hexdigest(),
            "steps_min_max": [int(steps.min()), int(steps.max())], "seconds": round(time.time() - t0, 1)}
    with open(OUT_ALL.replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


def main():
    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    R = mech["n_reactions"]
    weights = np.concatenate([[1.0], objective_weights(w.n_species)])
    st = w.states(mech, 1024)
    om = oracle.Mech(mech)
    t0 = time.time()
    recs = [oracle.integrate_record(om, st[:, c], None, w.p_pa, DT, w.rtol, w.atol) for c in range(1024)]
    assert all(r[3] == 0 for r in recs)
    steps = np.array([len(r[2]) for r in recs], dtype=np.int32)
    nthreads = os.cpu_count() or 8
    with ThreadPoolExecutor(nthreads) as ex:
        cells32 = list(range(32))
        cols = list(ex.map(lambda q: fd_column(mech, w, st, recs, weights, q // R, q % R, cells32), range(3 * R)))
        all32 = np.stack(cols, axis=1)  # [32 cells, 3R]
        pick = pick_parameters(R)
        cells1k = list(range(1024))
        cols = list(ex.map(lambda q: fd_column(mech, w, st, recs, weights, q // R, q % R, cells1k), pick))
        rand1k = np.stack(cols, axis=1)  # [1024 cells, 20]
        cols = list(ex.map(lambda q: tlm_column(mech, w, st, recs, weights, q // R, q % R, cells1k), pick))
        tlm1k = np.stack(cols, axis=1)  # [1024 cells, 20]
    np.savez(OUT, steps=steps, all32=all32, pick=pick, rand1k=rand1k, tlm1k=tlm1k)
    meta = {"dt": DT, "rtol": w.rtol, "atol": w.atol, "input_sha256": hashlib.sha256(st.tobytes()).hexdigest(),
            "steps_min_max": [int(steps.min()), int(steps.max())], "seconds": round(time.time() - t0, 1)}
    with open(OUT.replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "all-cells":
        main_all_cells()
    else:
        main()
