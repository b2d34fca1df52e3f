#!/usr/bin/env python3
"""Writes zonal_ambient_state.npy: the ambient state of the zonal workload.

The reference-mapping workload mixes reacting cells with cells of a quiescent
ambient zone (in the manner of the Spray A case of section 3, whose ambient
gas is far less reactive than the igniting region).  The ambient state is one
random state of the 54-species mechanism at 60 bar (T = 900 K, Y ~
Dirichlet(1), seed 2006) integrated by the oracle over 1e-3 s, which leaves it
near chemical equilibrium.  Only the oracle is called here.

Run from the repository root:  python tests/golden/make_ambient_state.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zonal_ambient_state.npy")


def main():
    w = WORKLOADS["c2_54sp"]
    mech = w.mechanism()
    base = make_states(mech, 1, 2006, [(900.0, 900.0)])
    st, _, steps, _, status = oracle.integrate(mech, base, None, w.p_pa, 1e-3, w.rtol, w.atol)
    assert status[0] == 0
    amb = np.ascontiguousarray(st[:, 0])
    np.save(OUT, amb, allow_pickle=False)
    # steps the ambient state takes over one flow time step afterwards
    _, _, s2, _, _ = oracle.integrate(mech, amb[:, None].copy(), None, w.p_pa, w.dt, w.rtol, w.atol)
    meta = {"sha256": hashlib.sha256(amb.tobytes()).hexdigest(), "shape": list(amb.shape),
            "T": float(amb[0]), "relax_steps": int(steps[0]), "steps_over_dt_1e-6": int(s2[0]),
            "min_Y": float(amb[1:].min()), "argmin_Y": int(np.argmin(amb[1:]))}
    with open(OUT.replace(".npy", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
