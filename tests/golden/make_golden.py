"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

Each fixture records the kept triple count per tier and a SHA-256 of the sorted
task keys ((linear_index(I,J) << 32) | K, little-endian uint64) for a named
synthetic workload.  Inputs come from the seeded generators in ``workloads``.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

CASES = [
    ("expdecay-n1024", 1e-6),
    ("expdecay-n1024", 0.0),
]


def main():
    for name, tau in CASES:
        wl = workloads.WORKLOADS[name]
        A = wl.matrix()
        r = oracle.spamm(A, A, wl.leaf, tau, want_C=False)
        keys = np.ascontiguousarray(r.keys.astype("<u8"))
        out = {
            "workload": name, "n": wl.n, "leaf": wl.leaf, "tau": tau,
            "Kt": [int(v) for v in r.Kt],
            "keys_sha256": hashlib.sha256(keys.tobytes()).hexdigest(),
            "written_by": "tests/golden/make_golden.py (oracle only)",
        }
        path = os.path.join(HERE, f"{name}_tau{tau:g}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(path, out["Kt"])


if __name__ == "__main__":
    main()
