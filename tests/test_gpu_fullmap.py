"""Full-size parity against the stored full map of the mixed-precision stack
(4 x 512 x 512, every node id; tests/golden/config2_fullmap_f32.npy, written
by tests/golden/make_golden.py from the oracle's selected inversion).

Node ids are drawn uniformly over the whole stack (pads included, which must
come out exactly 0), solved in the launch configuration the benchmark times
(mixed precision, rel_tol 1e-3, default preconditioner) and compared element
by element at 1e-3; a float64 subset at 1e-6 (float32 storage of the map
rounds at 6e-8 relative).  The whole map is run by `bench.py --full-map`.
"""
import os

import numpy as np
import pytest

from paper_2607_05818_amd import gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _max_rel(got, want):
    m = want > 0
    assert np.all(got[~m] == 0.0), "pads must be exactly 0"
    rel = np.abs(got[m] - want[m]) / want[m]
    i = int(np.argmax(rel))
    print(f"  worst: {np.flatnonzero(m)[i]} got {got[m][i]!r} want {want[m][i]!r}; "
          f"median {np.median(rel):.3e}", flush=True)
    return float(rel[i])


@pytest.fixture(scope="module")
def stack():
    from paper_2607_05818_amd import reff
    d = gen.config2()
    full = np.load(os.path.join(HERE, "golden", "config2_fullmap_f32.npy")).astype(np.float64)
    assert full.shape == (gen.n_nodes(d),)
    return reff, reff.reff_build_pdn(d), full


def test_config2_fullmap_uniform_sample_mixed(stack):
    reff, h, full = stack
    rng = np.random.default_rng(7101)
    ids = rng.choice(len(full), size=2048, replace=False).astype(np.int64)
    ids[:4] = gen.pad_ids(gen.config2())[:4]          # pads in the request
    print("[case] config2 full-map sample, 2048 ids, mixed rel_tol 1e-3", flush=True)
    got, st = reff.reff_solve_diag(h, ids, precision=reff.REFF_PREC_MIXED, rel_tol=1e-3)
    err = _max_rel(got, full[ids])
    print("mixed", err, st["iters_total"], flush=True)
    assert err <= 1e-3
    assert st["n_unconverged"] == 0


def test_config2_fullmap_sample_fp64(stack):
    reff, h, full = stack
    rng = np.random.default_rng(7102)
    ids = rng.choice(len(full), size=64, replace=False).astype(np.int64)
    print("[case] config2 full-map sample, 64 ids, fp64 rel_tol 1e-8", flush=True)
    got, st = reff.reff_solve_diag(h, ids, precision=reff.REFF_PREC_FP64, rel_tol=1e-8)
    err = _max_rel(got, full[ids])
    print("fp64", err, st["iters_total"], flush=True)
    assert err <= 1e-6


def test_large_recipe_quarter_area_against_oracle():
    """The large workload's recipe (8 tiers, anisotropic edges, clustered
    TSVs, pads at pitch 32) on a quarter of its area, 8 x 1024 x 1024
    (8,388,608 nodes): 64 seeded nodes against the stored oracle values
    (tests/golden/config5_quarter_sample.json), mixed precision at the 1e-3
    bar in the launch configuration of the large bench line."""
    import json
    from paper_2607_05818_amd import reff
    g = json.load(open(os.path.join(HERE, "golden", "config5_quarter_sample.json")))
    d = gen.config5(side=1024)
    nodes = np.array(g["nodes"], dtype=np.int64)
    assert np.array_equal(nodes, gen.sample_free_nodes(d, 64, 5005))
    want = np.array(g["R"])
    print("[case] large recipe 8 x 1024 x 1024, 64 nodes, mixed rel_tol 1e-3", flush=True)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_solve_diag(h, nodes, precision=reff.REFF_PREC_MIXED, rel_tol=1e-3)
    err = _max_rel(got, want)
    print("mixed", err, st["iters_total"], st["seconds"], flush=True)
    assert err <= 1e-3
