#!/usr/bin/env python3
"""Writes c3_relaxed_pool.npy: the state pool of the batching workload.

The batching workload needs cells of very uneven stiffness.  The pool holds
2,048 states of the 54-species mechanism at 60 bar, each obtained by
integrating a random state (T ~ U(700, 1600) K, Y ~ Dirichlet(1), state seed
2003) with the oracle over a relaxation time tau: 1,536 states with
tau = 1e-3 s (relaxed to near equilibrium: 1-10 steps per 1e-5 s afterwards)
and 512 states with tau log-uniform in [3e-7, 1e-5] s (sixteen buckets;
tens to hundreds of steps afterwards).  The workload samples its 262,144
cells from the pool with replacement.  Only the oracle is called here.

Run from the repository root:  python tests/golden/make_relaxed_pool.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2105_12070_amd.inputs import WORKLOADS, make_states  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_relaxed_pool.npy")


def main():
    w = WORKLOADS["c3_batch"]
    mech = w.mechanism()
    n_eq, n_part = 1536, 512
    base = make_states(mech, n_eq + n_part, 2003, [(700.0, 1600.0)])
    rng = np.random.default_rng(2103)
    taus = np.empty(n_eq + n_part)
    taus[:n_eq] = 1e-3
    buckets = np.exp(np.linspace(np.log(3e-7), np.log(1e-5), 16))
    taus[n_eq:] = buckets[rng.integers(0, 16, n_part)]
    pool = np.empty_like(base)
    for tau in np.unique(taus):
        idx = np.nonzero(taus == tau)[0]
        st, _, _, _, status = oracle.integrate(mech, np.ascontiguousarray(base[:, idx]), None, w.p_pa, tau,
                                               w.rtol, w.atol)
        assert np.all(status == 0)
        pool[:, idx] = st
    # shuffle so that any prefix mixes both kinds
    perm = rng.permutation(pool.shape[1])
    pool = np.ascontiguousarray(pool[:, perm])
    np.save(OUT, pool, allow_pickle=False)
    _, _, steps, _, status = oracle.integrate(mech, pool.copy(), None, w.p_pa, w.dt, w.rtol, w.atol)
    meta = {"sha256": hashlib.sha256(pool.tobytes()).hexdigest(), "shape": list(pool.shape),
            "steps_percentiles_0_10_25_50_75_90_99_100_at_dt_1e-5": np.percentile(
                steps, [0, 10, 25, 50, 75, 90, 99, 100]).tolist(),
            "steps_mean": float(steps.mean()), "status_ok": int(np.sum(status == 0))}
    with open(OUT.replace(".npy", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
