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


def test_batch_of_ragged_plans_matches_unit_solves_and_single_calls():
    """reff_selinv_batch over plans of different shapes and depths (their
    dissection trees merged by depth): all nodes of some plans, subsets
    with duplicates and pads of others, host and device output; every value
    against the oracle's unit solves (1e-10) and against reff_selinv_diag of
    the plan alone (1e-12: the batch may split products differently)."""
    import torch
    reff = _reff()
    shapes = [(201, 2, 17, 19, 9, 5), (202, 1, 7, 5, 0, 1), (203, 4, 10, 10, 6, 3),
              (204, 3, 40, 33, 30, 6), (205, 1, 1, 1, 0, 1), (206, 8, 9, 7, 12, 3)]
    plans = [gen.small_random_desc(s, nt, nx, ny, max(k, 1 if nt > 1 else 0), p)
             for s, nt, nx, ny, k, p in shapes]
    rng = np.random.default_rng(77)
    nodes = []
    for i, d in enumerate(plans):
        if i % 2 == 0:
            nodes.append(None)
        else:
            ids = rng.integers(0, gen.n_nodes(d), size=50)
            ids[:2] = ro.pad_nodes(d)[:1].repeat(2)
            nodes.append(ids)
    _say("selinv batch of 6 ragged plans")
    outs, st = reff.reff_selinv_batch(plans, nodes)
    print(st, flush=True)
    dev = [torch.empty(gen.n_nodes(d) if nodes[i] is None else len(nodes[i]),
                       dtype=torch.float64, device="cuda") for i, d in enumerate(plans)]
    reff.reff_selinv_batch(plans, nodes, dev)
    torch.cuda.synchronize()
    for i, d in enumerate(plans):
        want = ro.diag(d, nodes[i])
        assert _max_rel(outs[i], want) <= TOL
        assert np.array_equal(dev[i].cpu().numpy(), outs[i])
        h = reff.reff_build_pdn(d)
        alone, _ = reff.reff_selinv_diag(h, nodes[i])
        h.close()
        m = alone > 0
        assert np.all(outs[i][~m] == 0.0)
        if m.any():  # a 1 x 1 x 1 stack is all pad
            assert np.max(np.abs(outs[i][m] - alone[m]) / alone[m]) <= 1e-12
    # the pooled device memory goes back to the device, and calls still work
    reff.reff_release_cached_memory(0)
    again, _ = reff.reff_selinv_batch(plans, nodes)
    for i in range(len(plans)):
        assert np.array_equal(again[i], outs[i])


def test_batch_all_256_recipe_plans_against_stored_oracle_values():
    """The batching workload (256 plans, 2-4 tiers, sides 64-256, 21.1M
    nodes) in one reff_selinv_batch call: the seeded 64-node block of every
    plan against the oracle's float64 values stored in
    tests/golden/config3_sample.json, at the float64 bar."""
    import json
    import os
    reff = _reff()
    plans = gen.config3_plans()
    nodes = gen.config3_samples(plans)
    gold = json.load(open(os.path.join(HERE, "golden", "config3_sample.json")))
    assert [list(x) for x in nodes] == gold["nodes"], "sample drifted from the fixture"
    _say("selinv batch, all 256 recipe plans")
    outs, st = reff.reff_selinv_batch(plans, nodes)
    print({k: v for k, v in st.items()}, flush=True)
    worst = max(_max_rel(outs[i], np.array(gold["R"][i])) for i in range(len(plans)))
    print("worst relative error over 16,384 nodes", worst, flush=True)
    assert worst <= TOL


@pytest.mark.parametrize("seed,nt,side,ntsv,npad,count", [(61, 4, 100, 300, 40, 5),
                                                          (62, 2, 97, 50, 7, 1),
                                                          (63, 3, 64, 80, 6, 200)])
def test_node_request_inverts_only_needed_fronts(seed, nt, side, ntsv, npad, count):
    """A node list makes the selected inversion visit only the fronts that
    hold the nodes and their ancestors; each front's arithmetic is the same,
    so the values equal those of the full map bit for bit, and the reported
    inversion flops drop with the request."""
    reff = _reff()
    d = gen.small_random_desc(seed, nt, side, side - 3, ntsv, npad)
    _say("selinv node request", seed, nt, side, count)
    h = reff.reff_build_pdn(d)
    full, st_full = reff.reff_selinv_diag(h)
    ids = np.random.default_rng(seed).integers(0, len(full), size=count)
    ids[0] = ro.pad_nodes(d)[0]
    got, st = reff.reff_selinv_diag(h, ids)
    print("inversion flops", st["flops_selinv"], "of", st_full["flops_selinv"], flush=True)
    assert np.array_equal(got, full[ids])
    assert got[0] == 0.0
    assert st["flops_selinv"] < st_full["flops_selinv"]
    assert st["flops_factor"] == st_full["flops_factor"]
    # the full map afterwards is unchanged by the partial call
    again, _ = reff.reff_selinv_diag(h)
    assert np.array_equal(again, full)
    h.close()


def test_batch_node_requests_equal_full_batch():
    """Batched requests take the same partial inversion over the merged
    forest: equal bit for bit to the all-node batch at the same ids."""
    reff = _reff()
    shapes = [(301, 2, 40, 33, 20, 4), (302, 3, 50, 21, 30, 2), (303, 1, 9, 70, 0, 3)]
    plans = [gen.small_random_desc(s, nt, nx, ny, k, p) for s, nt, nx, ny, k, p in shapes]
    _say("selinv batch node requests vs all-node batch")
    full, st_full = reff.reff_selinv_batch(plans, [None] * len(plans))
    rng = np.random.default_rng(303)
    nodes = [rng.integers(0, gen.n_nodes(d), size=7) for d in plans]
    nodes[1] = None  # one plan asks for every node
    got, st = reff.reff_selinv_batch(plans, nodes)
    for i in range(len(plans)):
        want = full[i] if nodes[i] is None else full[i][nodes[i]]
        assert np.array_equal(got[i], want)
    assert st["flops_selinv"] < st_full["flops_selinv"]


def test_batch_in_chunks_all_nodes_equal_single_calls():
    """A batch above 8M nodes runs as several chunks of plans (the host
    analysis of one under the device work of the previous): every node of
    every plan, written to device memory, against reff_selinv_diag of the
    plan alone (1e-12: the forests may split products differently)."""
    import torch
    reff = _reff()
    plans = gen.config3_plans()
    order = np.argsort([-gen.n_nodes(d) for d in plans], kind="stable")
    pick, tot = [], 0
    for i in order:
        pick.append(plans[int(i)])
        tot += gen.n_nodes(plans[int(i)])
        if tot > 9 << 20:
            break
    _say("selinv batch in chunks,", len(pick), "plans,", tot, "nodes")
    dev = [torch.full((gen.n_nodes(d),), -1.0, dtype=torch.float64, device="cuda") for d in pick]
    _, st = reff.reff_selinv_batch(pick, None, dev)
    torch.cuda.synchronize()
    print({k: v for k, v in st.items()}, flush=True)
    worst = 0.0
    for d, out in zip(pick, dev):
        h = reff.reff_build_pdn(d)
        alone, _ = reff.reff_selinv_diag(h)
        h.close()
        got = out.cpu().numpy()
        m = alone > 0
        assert np.all(got[~m] == 0.0)
        worst = max(worst, float(np.max(np.abs(got[m] - alone[m]) / alone[m])))
    print("worst relative difference to single calls", worst, flush=True)
    assert worst <= 1e-12
