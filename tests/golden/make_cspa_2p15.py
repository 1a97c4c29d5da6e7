"""Writes cspa_2p15.json: the CSPA-shaped program's result on the seeded
2^15-id literal-reading input (workloads.cspa(15)), computed by the oracle's
matrix-product naive evaluator: per-relation sizes, per-iteration delta
sizes, and a SHA-256 of each relation's sorted row-major uint32 rows.

Run from the repository root: python tests/golden/make_cspa_2p15.py
(several minutes on one CPU socket).  Calls only oracle/ and workloads/.
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import matrix_naive  # noqa: E402

IDB = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}


def main():
    prog = open(os.path.join(ROOT, "workloads", "programs", "cspa_shaped.dl")).read()
    wl = workloads.cspa(15)
    res = matrix_naive.evaluate(prog, wl["edb"], IDB)
    out = {"workload": "workloads.cspa(15): Zipf(1.2), 2^15 ids, literal reading",
           "program": "workloads/programs/cspa_shaped.dl",
           "evaluator": "oracle.matrix_naive", "iterations": res.iterations,
           "active_ids": res.active_ids, "relations": {}}
    for n in IDB:
        rows = np.ascontiguousarray(res.relations[n], dtype=np.uint32)
        out["relations"][n] = {"size": int(len(rows)), "deltas": res.deltas[n],
                               "sha256": hashlib.sha256(rows.tobytes()).hexdigest()}
    path = os.path.join(ROOT, "tests", "golden", "cspa_2p15.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
