"""Write the stored expected values used by the full-size parity tests.

Calls only the CPU oracle (and the seeded input generators).  Each fixture
records the generator call that rebuilds its inputs and the oracle's float64
R_i = (G^-1)_ii (paper Sec. II-B, Eq. 2 with the bumps merged into the
grounded supply) for a seeded sample of nodes.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import reff_oracle as ro  # noqa: E402
from paper_2607_05818_amd import gen  # noqa: E402

SAMPLE_SEED = 2002
N_GOLD = 128


def config2_sample():
    desc = gen.config2()
    nodes = gen.sample_free_nodes(desc, 16384, SAMPLE_SEED)[:N_GOLD]
    t0 = time.time()
    R = ro.diag(desc, nodes=nodes)
    dt = time.time() - t0
    return {
        "what": "R_i = (G^-1)_ii, float64 oracle (sparse LU), config 2 stack",
        "inputs": "gen.config2(seed=1002); nodes = gen.sample_free_nodes(desc, 16384, 2002)[:128]",
        "oracle_seconds": dt,
        "nodes": [int(v) for v in nodes],
        "R": [float(r) for r in R],
    }


N_PLANS3 = 8


def config3_sample():
    plans = gen.config3_plans()
    nodes = gen.config3_samples(plans)
    t0 = time.time()
    R = [ro.diag(plans[i], nodes=nodes[i]) for i in range(N_PLANS3)]
    dt = time.time() - t0
    return {
        "what": "R_i = (G^-1)_ii, float64 oracle (sparse LU), first batching plans",
        "inputs": ("plans = gen.config3_plans(seed=1003); nodes = gen.config3_samples(plans); "
                   "plans 0..7"),
        "oracle_seconds": dt,
        "nodes": [[int(v) for v in nodes[i]] for i in range(N_PLANS3)],
        "R": [[float(r) for r in R[i]] for i in range(N_PLANS3)],
    }


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2", "config3"]
    for name, fn in (("config2", config2_sample), ("config3", config3_sample)):
        if name not in which:
            continue
        out = fn()
        with open(os.path.join(HERE, name + "_sample.json"), "w") as f:
            json.dump(out, f, indent=0)
        print("wrote", name + "_sample.json", out["oracle_seconds"])
