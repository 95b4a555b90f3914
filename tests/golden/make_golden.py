"""Writes the stored expected values of the named workloads by running the
CPU oracle (and nothing else) on the seeded synthetic inputs.

    python tests/golden/make_golden.py small mid [seismic]

Each JSON file records the input's sha256, the max-flow value, the optimal
energy and the sha256 of the minimal-cut surface (int32 [nx][ny]).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_17026_amd import synth  # noqa: E402

MAKERS = {"small": synth.config_small, "mid": synth.config_mid, "seismic": synth.config_seismic}


def main(names):
    for name in names:
        cost, delta = MAKERS[name]()
        t = time.time()
        r = oracle.solve(cost, delta)
        assert r.conservation_ok and r.capacity_ok and r.flow == r.cut and r.smin_in_smax
        out = {
            "workload": name,
            "shape": list(cost.shape),
            "delta": delta,
            "cost_sha256": synth.sha256(cost),
            "flow": int(r.flow),
            "energy": int(r.energy),
            "surface_sha256": synth.sha256(r.hmin.astype(np.int32)),
            "surface_max_sha256": synth.sha256(r.hmax.astype(np.int32)),
            "oracle": "Dinic on the explicit graph (oracle/oracle.c)",
            "oracle_seconds": round(time.time() - t, 1),
        }
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["small", "mid"])
