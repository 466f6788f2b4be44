"""Iteration chunks replayed as HIP graphs give bitwise the results of plain
launches (same kernels in the same order; the solver's reductions are
deterministic).  Each solve replays a captured chunk of four iterations
many times with host-side convergence checks in between, and in a batch
whose blocks converge at different iterations the same chunk stays valid
while converged blocks leave the device-resident work lists.  Graph replay
is the default; the NULL stream path runs on a stream of its own."""
import numpy as np
import pytest

from paper_2607_05818_amd import gen

pytestmark = pytest.mark.gpu


def _reff():
    from paper_2607_05818_amd import reff
    return reff


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_solve_graph_replay_matches_plain_launches(prec):
    import torch
    reff = _reff()
    d = gen.config2(side=128, n_tsv=64, sigma=10.0)
    nodes = gen.sample_free_nodes(d, 100, 41)
    h = reff.reff_build_pdn(d)
    s = torch.cuda.Stream()
    _say("graphs solve prec", prec)
    with torch.cuda.stream(s):
        out_g = torch.empty(len(nodes), dtype=torch.float64, device="cuda")
        reff.reff_solve_diag(h, nodes, out_g, precision=prec, stream=s.cuda_stream, graphs=True)
        out_p = torch.empty(len(nodes), dtype=torch.float64, device="cuda")
        reff.reff_solve_diag(h, nodes, out_p, precision=prec, stream=s.cuda_stream, graphs=False)
    s.synchronize()
    assert torch.equal(out_g, out_p)


def test_batch_graph_replay_with_compaction():
    import torch
    reff = _reff()
    plans = gen.config3_plans(seed=91, n_plans=5, side_lo=40, side_hi=96)
    nodes = [gen.sample_free_nodes(p, 64, 900 + i) for i, p in enumerate(plans)]
    s = torch.cuda.Stream()
    _say("graphs batch")
    g, st_g = reff.reff_batch_plans(plans, nodes, precision=reff.REFF_PREC_MIXED,
                                    stream=s.cuda_stream, graphs=True)
    p, st_p = reff.reff_batch_plans(plans, nodes, precision=reff.REFF_PREC_MIXED,
                                    stream=s.cuda_stream, graphs=False)
    q, st_q = reff.reff_batch_plans(plans, nodes, precision=reff.REFF_PREC_MIXED)  # NULL stream
    for a, b in zip(q, p):
        assert np.array_equal(a, b)
    assert [x["iters_max"] for x in st_q] == [x["iters_max"] for x in st_p]
    iters = [x["iters_max"] for x in st_p]
    assert len(set(iters)) > 1  # blocks converged at different iterations
    for a, b in zip(g, p):
        assert np.array_equal(a, b)
