"""The large workload at its full size (8 tiers of 2048 x 2048, 33,554,432
nodes, anisotropic edges, 16,384 clustered TSVs, 4096 pads).

No exact oracle solve of this stack fits one host (its sparse factor alone
would take hours; the quarter-size stack is checked against stored oracle
values in test_gpu_fullmap.py), so sixteen seeded nodes are checked against
two-sided bounds that hold at any size: Rayleigh window bounds, exact
float64 solves of the window around each node with the outside cut (upper)
or merged into the supply (lower), from oracle/bounds.py.  The mixed
path's values must lie inside them within its 1e-3 bar; where a window
holds no way down to a pad the upper bound is infinite and only the lower
one binds.
"""
import numpy as np
import pytest

from oracle import bounds as ob
from paper_2607_05818_amd import gen

pytestmark = pytest.mark.gpu

HALF = 64  # window half-width: 129 x 129 columns through the 8 tiers


def test_config5_full_size_within_rayleigh_bounds():
    from paper_2607_05818_amd import reff
    d = gen.config5()
    nodes = gen.sample_free_nodes(d, 16, 5005)
    print("[case] config5 full size, 16 nodes, mixed", flush=True)
    h = reff.reff_build_pdn(d)
    R, st = reff.reff_solve_diag(h, nodes, precision=reff.REFF_PREC_MIXED, rel_tol=1e-3)
    h.close()
    print("solve", st["iters_total"], "iterations,", round(st["seconds"], 1), "s", flush=True)
    finite = 0
    for v, r in zip(nodes, R):
        lo, hi = ob.window_bounds(d, v, HALF)
        print(f"node {v}: {lo:.6f} <= {r:.6f} <= {hi:.6f}", flush=True)
        assert lo * (1 - 1e-3) <= r
        assert r <= hi * (1 + 1e-3)
        finite += np.isfinite(hi)
    print("finite upper bounds", finite, "of", len(nodes), flush=True)
