"""Sparse-direct full maps on the GPU (reff_selinv_diag) against the oracle.

The oracle is the definition: R_i = (G^-1)_ii from one unit-current solve
per node (oracle/reff_oracle.diag) on small stacks, and the oracle's own
selected inversion (oracle/selinv.py, pinned against dense inverses and
closed forms) on larger ones.  Both sides compute in float64 without a
tolerance, so the bar is rounding: 1e-10 relative (the fronts' Cholesky and
Takahashi products accumulate some 10^3..10^4 terms in a different order on
each side; the stacks are well conditioned at these sizes).  Pads must come
out exactly 0.
"""
import os

import numpy as np
import pytest

from oracle import reff_oracle as ro
from oracle import selinv as osel
from paper_2607_05818_amd import gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10


def _reff():
    from paper_2607_05818_amd import reff
    return reff


def _say(*a):
    print("[case]", *a, flush=True)


def _max_rel(got, want):
    m = want > 0
    assert np.all(got[~m] == 0.0), "pads must be exactly 0"
    if not np.any(m):
        return 0.0
    rel = np.abs(got[m] - want[m]) / want[m]
    return float(rel.max())


SMALL = [
    # seed, nt, nx, ny, n_tsv, n_pads: ragged and degenerate shapes
    (101, 1, 7, 5, 0, 1), (102, 3, 1, 9, 1, 1), (103, 2, 33, 3, 4, 2),
    (104, 4, 10, 10, 6, 3), (105, 1, 1, 1, 0, 1), (106, 2, 17, 19, 9, 5),
    (107, 5, 6, 4, 3, 1), (108, 2, 5, 40, 7, 2), (109, 8, 9, 7, 12, 3),
]


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL)
def test_small_stacks_match_unit_solves(seed, nt, nx, ny, ntsv, npad):
    reff = _reff()
    d = gen.small_random_desc(seed, nt, nx, ny, max(ntsv, 1 if nt > 1 else 0), npad)
    _say("selinv small", seed, nt, nx, ny, ntsv, npad)
    want = ro.diag(d)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_selinv_diag(h)
    err = _max_rel(got, want)
    print("max rel err", err, st, flush=True)
    assert err <= TOL
    h.close()


@pytest.mark.parametrize("nt,side,ntsv,npad", [(4, 100, 300, 40), (3, 150, 200, 12),
                                              (2, 97, 50, 7)])
def test_multi_panel_fronts_match_oracle_selected_inversion(nt, side, ntsv, npad):
    """Separators of 97..600 pivots: several 64-column panels per front, a
    ragged last panel, and update sets that span tiers."""
    reff = _reff()
    d = gen.small_random_desc(5000 + side, nt, side, side - 3, ntsv, npad)
    _say("selinv multi-panel", nt, side, side - 3, ntsv, npad)
    want = osel.diag_full(d)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_selinv_diag(h)
    err = _max_rel(got, want)
    print("max rel err", err, "max front", st["max_front"], flush=True)
    assert st["max_front"] > 128
    assert err <= TOL
    # a second call reuses the plan and gives the same bits
    got2, st2 = reff.reff_selinv_diag(h)
    assert np.array_equal(got, got2)
    assert st2["seconds_plan"] < st["seconds_plan"] + 1e-3
    h.close()


def test_node_subset_duplicates_pads_and_device_output():
    import torch
    reff = _reff()
    d = gen.config1()
    _say("selinv config1 subset, duplicates, pads, device output")
    want = ro.diag(d)
    rng = np.random.default_rng(31)
    nodes = rng.integers(0, len(want), size=300)
    nodes[:5] = ro.pad_nodes(d)[:5]
    nodes[5:9] = nodes[10]
    h = reff.reff_build_pdn(d)
    out = torch.full((len(nodes),), -1.0, dtype=torch.float64, device="cuda")
    reff.reff_selinv_diag(h, nodes, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(got[:5] == 0.0)
    assert _max_rel(got, want[nodes]) <= TOL
    host, _ = reff.reff_selinv_diag(h, nodes)
    assert np.array_equal(host, got)
    empty, _ = reff.reff_selinv_diag(h, np.zeros(0, dtype=np.int64))
    assert len(empty) == 0
    with pytest.raises(reff.ReffError):
        reff.reff_selinv_diag(h, [len(want)])
    h.close()


def test_config2_full_map():
    """The whole 4 x 512 x 512 stack (1,048,576 node ids) against the stored
    oracle map (float32 storage: 2^-24 relative rounding, bar 1.2e-7) and
    32 sampled nodes against float64 oracle solves."""
    reff = _reff()
    d = gen.config2()
    _say("selinv config2 full map")
    full = np.load(os.path.join(HERE, "golden", "config2_fullmap_f32.npy")).astype(np.float64)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_selinv_diag(h)
    print({k: v for k, v in st.items()}, flush=True)
    assert _max_rel(got, full) <= 1.2e-7
    ids = np.random.default_rng(7201).choice(len(full), size=32, replace=False)
    want = osel.solve_nodes(d, ids)
    assert _max_rel(got[ids], want) <= TOL
    h.close()
