"""Regression check of the oracle against fixtures written by
tests/golden/make_golden.py (which calls only the oracle)."""
import glob
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads

FIXTURES = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*_tau*.json")))


@pytest.mark.parametrize("path", FIXTURES, ids=os.path.basename)
def test_oracle_matches_fixture(path):
    with open(path) as f:
        g = json.load(f)
    wl = workloads.WORKLOADS[g["workload"]]
    A = wl.matrix()
    r = oracle.spamm(A, A, g["leaf"], g["tau"], want_C=False)
    assert [int(v) for v in r.Kt] == g["Kt"]
    keys = np.ascontiguousarray(r.keys.astype("<u8"))
    assert hashlib.sha256(keys.tobytes()).hexdigest() == g["keys_sha256"]
