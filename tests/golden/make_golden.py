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


if __name__ == "__main__":
    out = config2_sample()
    with open(os.path.join(HERE, "config2_sample.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote config2_sample.json", out["oracle_seconds"])
