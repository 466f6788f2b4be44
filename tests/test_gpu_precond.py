"""The Chebyshev polynomial preconditioner is SPD and fixed, so every degree
gives PCG's answer: results stay within the parity bars of the oracle while
the block iterations fall with the degree (about proportionally)."""
import numpy as np
import pytest

from oracle import reff_oracle as ro
from paper_2607_05818_amd import gen

pytestmark = pytest.mark.gpu


def _reff():
    from paper_2607_05818_amd import reff
    return reff


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("prec,tol,rel", [(0, 1e-6, 1e-9), (1, 1e-3, 1e-5)], ids=["fp64", "mixed"])
def test_degrees_agree_with_oracle(prec, tol, rel):
    reff = _reff()
    d = gen.config2(side=128, n_tsv=64, sigma=10.0)
    nodes = gen.sample_free_nodes(d, 128, 77)
    want = ro.diag(d, nodes)
    h = reff.reff_build_pdn(d)
    iters = {}
    for k in (1, 2, 4, 8):
        _say("precond degree", k, "prec", prec)
        got, st = reff.reff_solve_diag(h, nodes, precision=prec, rel_tol=rel, precond_degree=k)
        err = float(np.max(np.abs(got - want) / want))
        iters[k] = st["iters_total"]
        print("degree", k, "iters", iters[k], "err", err, flush=True)
        assert err <= tol
    assert iters[4] < 0.5 * iters[1] and iters[8] < iters[4]


def test_degree_out_of_range_rejected():
    reff = _reff()
    h = reff.reff_build_pdn(gen.config1())
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_solve_diag(h, [5], precond_degree=33)
    assert ei.value.status == reff.REFF_ERR_INVALID_ARG


@pytest.mark.parametrize("kind", ["ragged_square", "ragged_rect"])
def test_fused_steps_on_ragged_strips(kind):
    """Degrees whose steps run as fused passes (3: two steps; 4: three; 5:
    three and one; 6: three and two; 7: two passes of three; 8: two of three
    and one; 9: two of three and two) on tiers whose width is not a multiple
    of the strip width, with TSVs: every result within the mixed bar.
    Float64 runs two steps per pass (3: one pass; 6: two passes and a single
    step)."""
    reff = _reff()
    if kind == "ragged_square":
        d = gen.config2(side=100, n_tsv=64, sigma=10.0)
    else:
        d = gen.small_random_desc(41, 3, 45, 37, 40, 4)
    nodes = gen.sample_free_nodes(d, 64, 5)
    want = ro.diag(d, nodes)
    h = reff.reff_build_pdn(d)
    for k in (3, 4, 5, 6, 7, 8, 9):
        _say("fused precond degree", k, kind)
        got, st = reff.reff_solve_diag(h, nodes, precision=1, rel_tol=1e-5, precond_degree=k)
        err = float(np.max(np.abs(got - want) / want))
        print("degree", k, "iters", st["iters_total"], "err", err, flush=True)
        assert err <= 1e-3
    for k in (3, 6):
        _say("float64 precond degree", k, kind)
        got, _ = reff.reff_solve_diag(h, nodes, precision=0, rel_tol=1e-9, precond_degree=k)
        assert float(np.max(np.abs(got - want) / want)) <= 1e-6


def test_eight_tiers_with_clustered_tsvs():
    """Eight tiers (the large stack's depth) on a small grid with many TSV
    columns close together, so that TSV nodes neighbour each other: the
    side-buffer values of the three-step passes at every tier, default
    degree, against the oracle in both precisions."""
    reff = _reff()
    d = gen.small_random_desc(57, 8, 40, 36, 60, 6)
    nodes = gen.sample_free_nodes(d, 64, 9)
    want = ro.diag(d, nodes)
    h = reff.reff_build_pdn(d)
    _say("eight tiers, mixed")
    got, st = reff.reff_solve_diag(h, nodes, precision=1, rel_tol=1e-5)
    assert float(np.max(np.abs(got - want) / want)) <= 1e-3
    _say("eight tiers, fp64")
    got, st = reff.reff_solve_diag(h, nodes, precision=0, rel_tol=1e-9)
    assert float(np.max(np.abs(got - want) / want)) <= 1e-6


def test_wide_tier_falls_back_to_two_step_passes():
    """A tier too wide for the three-step pass's 32-bit strip offsets (nine
    rows of 932,100 nodes x 256 B exceed 2^31 B): the host cuts one-row
    strips and runs two-step passes instead, and the float32 solve at the
    default degree meets the mixed bar.  A stack with TSVs solved after it
    on the same device (three-step passes again) does too."""
    reff = _reff()
    nx, ny = 932100, 2
    rng = np.random.default_rng(77)
    gx = rng.uniform(0.5, 2.0, size=(1, ny, nx - 1))
    gy = rng.uniform(0.5, 2.0, size=(1, ny - 1, nx))
    pads = [(x, 0) for x in range(0, nx, 50)]
    d = gen.make_desc(1, nx, ny, gx, gy, np.zeros((0, 2)), np.zeros((0, 0)), pads)
    nodes = gen.sample_free_nodes(d, 64, 78)
    want = ro.diag(d, nodes)
    _say("wide tier", nx, "x", ny)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_solve_diag(h, nodes, precision=1, rel_tol=1e-4)
    err = float(np.max(np.abs(got - want) / want))
    print("wide tier iters", st["iters_total"], "err", err, flush=True)
    assert err <= 1e-3
    del h
    d2 = gen.config2(side=96, n_tsv=48, sigma=8.0)
    nodes2 = gen.sample_free_nodes(d2, 64, 79)
    want2 = ro.diag(d2, nodes2)
    _say("stack after the wide tier")
    got2, _ = reff.reff_solve_diag(reff.reff_build_pdn(d2), nodes2, precision=1, rel_tol=1e-4)
    assert float(np.max(np.abs(got2 - want2) / want2)) <= 1e-3


@pytest.mark.parametrize("nx,ny,deg", [(96, 40, 19), (700, 24, 31)])
def test_automatic_degree_follows_the_grid(nx, ny, deg):
    """precond_degree 0 picks 19 up to 640 nodes a side and 31 above: the
    solves are deterministic, so the default call equals the explicit
    degree bit for bit (and stays within the mixed bar of the oracle)."""
    reff = _reff()
    d = gen.small_random_desc(900 + nx, 2, nx, ny, 12, 4)
    nodes = gen.sample_free_nodes(d, 64, 5)
    _say("automatic degree", nx, ny, "expects", deg)
    h = reff.reff_build_pdn(d)
    auto, st_a = reff.reff_solve_diag(h, nodes, precision=reff.REFF_PREC_MIXED, rel_tol=1e-4)
    expl, st_e = reff.reff_solve_diag(h, nodes, precision=reff.REFF_PREC_MIXED, rel_tol=1e-4,
                                      precond_degree=deg)
    assert np.array_equal(auto, expl)
    assert st_a["iters_total"] == st_e["iters_total"]
    want = ro.diag(d, nodes)
    assert float(np.max(np.abs(auto - want) / want)) <= 1e-3
    h.close()
