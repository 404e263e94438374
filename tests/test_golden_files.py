"""The stored oracle outputs under tests/golden/ were written by the oracle as it stands: the SHA-256 of
the oracle source recorded beside them must match (else rerun tests/golden/make_oracle_trajectories.py)."""
import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_trajectories_match_the_oracle_source():
    with open(os.path.join(HERE, "golden", "oracle_trajectories.json")) as f:
        meta = json.load(f)
    with open(os.path.join(ROOT, "oracle", "ipc_oracle.cpp"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    assert meta["oracle_sha256"] == sha, "oracle changed: rerun tests/golden/make_oracle_trajectories.py"
    data = np.load(os.path.join(HERE, "golden", "oracle_trajectories.npz"))
    for case, m in meta["cases"].items():
        for k in m["checkpoints"]:
            pos = data[f"{case}_pos_{k}"]
            assert pos.ndim == 2 and pos.shape[1] == 3 and np.isfinite(pos).all()
        assert len(data[f"{case}_status"]) == m["steps_run"]
