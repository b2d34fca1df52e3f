#!/usr/bin/env python3
"""Writes tight_parity.npz: oracle results for the tight-tolerance parity tests.

At rtol 1e-10 / atol 1e-16 a cell of the 54- to 150-species workloads takes
10^4 to 10^5 Rosenbrock steps over the full flow step (1e-6 s; 1e-5 s for the
batching workload), so the oracle needs minutes for the sampled cells.  This
script runs it once and stores its results; the GPU tests regenerate the same
input states from the seeded generator, check them against the SHA-256 stored
here, and compare the GPU's results with the stored ones.  Only the oracle is
called.

Samples (ROS4, max_steps 400,000 on both sides):
  c2_54sp   32 cells evenly spaced over the 65,536 (both temperature strata);
  c4_adj    32 cells evenly spaced over the 16,384;
  c3_batch  the 8 cells with the most oracle steps at the metric setting
            (rtol 1e-6, atol 1e-10) among the first 4,096 cells, dt 1e-5 s,
            one per distinct state (the cells are drawn from a pool with
            replacement, so the stiffest states recur);
  c5_150sp  8 cells evenly spaced over the 131,072.

Run from the repository root:  python tests/golden/make_tight_parity.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tight_parity.npz")
RTOL, ATOL, MAX_STEPS = 1e-10, 1e-16, 400000


def sample(name):
    """(cell indices, their initial states [N, n]) of a workload's tight-parity sample."""
    w = WORKLOADS[name]
    mech = w.mechanism()
    if name == "c3_batch":
        st = w.states(mech, 4096)
        _, _, steps, _, status = oracle.integrate(mech, st, None, w.p_pa, w.dt, w.rtol, w.atol)
        assert np.all(status == 0)
        idx, seen = [], set()
        for c in np.argsort(-steps, kind="stable"):
            key = st[:, c].tobytes()
            if key not in seen:
                seen.add(key)
                idx.append(int(c))
            if len(idx) == 8:
                break
        idx = np.sort(np.array(idx, dtype=np.int64))
        return idx, np.ascontiguousarray(st[:, idx])
    n = 8 if name == "c5_150sp" else 32
    idx = np.linspace(0, w.n_cells - 1, n).astype(np.int64)
    st = w.states(mech, w.n_cells)
    return idx, np.ascontiguousarray(st[:, idx])


def state_hash(st):
    return hashlib.sha256(np.ascontiguousarray(st, dtype=np.float64).tobytes()).hexdigest()


def main():
    out, meta = {}, {}
    for name in ("c2_54sp", "c4_adj", "c3_batch", "c5_150sp"):
        w = WORKLOADS[name]
        mech = w.mechanism()
        idx, st0 = sample(name)
        t0 = time.time()
        st, h, steps, rej, status = oracle.integrate(mech, st0, None, w.p_pa, w.dt, RTOL, ATOL,
                                                     max_steps=MAX_STEPS)
        el = time.time() - t0
        out[f"{name}_idx"] = idx
        out[f"{name}_state"] = st
        out[f"{name}_h"] = h
        out[f"{name}_steps"] = steps
        out[f"{name}_rejects"] = rej
        out[f"{name}_status"] = status
        meta[name] = {"input_sha256": state_hash(st0), "cells": idx.tolist(), "dt": w.dt,
                      "steps": steps.tolist(), "rejects": rej.tolist(), "status": status.tolist(),
                      "oracle_seconds": round(el, 1), "threads": oracle.num_threads()}
        print(name, json.dumps(meta[name]), flush=True)
    meta["_settings"] = {"rtol": RTOL, "atol": ATOL, "max_steps": MAX_STEPS, "method": "ros4"}
    np.savez(OUT, **out)
    with open(OUT.replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
