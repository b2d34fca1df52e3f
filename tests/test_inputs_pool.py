"""The stored state pool of the batching workload matches its recorded hash
and feeds the workload's cells (host-only checks)."""
import hashlib
import json
import os

import numpy as np

from paper_2105_12070_amd.inputs import POOL_DIR, WORKLOADS


def test_pool_hash_and_sampling():
    pool = np.load(os.path.join(POOL_DIR, "c3_relaxed_pool.npy"), allow_pickle=False)
    meta = json.load(open(os.path.join(POOL_DIR, "c3_relaxed_pool.json")))
    assert list(pool.shape) == meta["shape"] == [55, 2048]
    assert hashlib.sha256(np.ascontiguousarray(pool).tobytes()).hexdigest() == meta["sha256"]
    w = WORKLOADS["c3_batch"]
    st = w.states(n_cells=1000)
    assert st.shape == (55, 1000)
    cols = {c.tobytes() for c in pool.T}
    assert all(c.tobytes() in cols for c in st.T)
    assert np.all(np.abs(st[1:].sum(axis=0) - 1.0) < 1e-12)
