"""Pair resistances through the C ABI (reff_query_pairs) against the oracle
and against the paper's reduced-system method (Sec. III-C/D).

Tolerances: 1e-6 relative (float64 path), 1e-3 (mixed), on R(a, b) > 0;
R(a, a) = 0 exactly."""
import numpy as np
import pytest

from oracle import reff_oracle as ro
from paper_2607_05818_amd import gen
from tests import pins

pytestmark = pytest.mark.gpu


def _reff():
    from paper_2607_05818_amd import reff
    return reff


def _say(*a):
    print("[case]", *a, flush=True)


def _rel(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    zero = want == 0
    assert np.all(got[zero] == 0.0)
    m = ~zero
    return float(np.max(np.abs(got[m] - want[m]) / want[m])) if m.any() else 0.0


@pytest.mark.parametrize("mode", [0, 1], ids=["grounded", "floating"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-3)], ids=["fp64", "mixed"])
def test_config1_pairs_two_blocks(mode, prec, tol):
    """50 x 60 endpoints (about 110 distinct, so two solve blocks and the
    cross-block terms) including pads and a repeated node."""
    reff = _reff()
    d = gen.config1()
    rng = np.random.default_rng(17)
    a = rng.choice(2048, size=50, replace=False)
    b = rng.choice(2048, size=60, replace=False)
    a[0] = ro.pad_nodes(d)[0]
    b[1] = a[3]
    want = ro.pairs(d, a, b, mode)
    _say("config1 pairs mode", mode, "prec", prec)
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_query_pairs(h, a, b, mode, precision=prec,
                                    rel_tol=1e-9 if prec == 0 else 1e-5)
    err = _rel(got, want)
    print("max rel err", err, st, flush=True)
    assert err <= tol
    assert got[3, 1] == 0.0


def test_pairs_symmetry_and_device_output():
    import torch
    reff = _reff()
    d = gen.small_random_desc(55, 3, 14, 12, 8, 3)
    rng = np.random.default_rng(5)
    a = rng.choice(504, size=9, replace=False)
    b = rng.choice(504, size=7, replace=False)
    h = reff.reff_build_pdn(d)
    out = torch.zeros((9, 7), dtype=torch.float64, device="cuda")
    reff.reff_query_pairs(h, a, b, reff.REFF_PAIRS_FLOATING, out)
    torch.cuda.synchronize()
    ab = out.cpu().numpy()
    ba, _ = reff.reff_query_pairs(h, b, a, reff.REFF_PAIRS_FLOATING)
    assert np.allclose(ab, ba.T, rtol=1e-10, atol=0)
    assert _rel(ab, ro.pairs(d, a, b, ro.FLOATING)) <= 1e-6


@pytest.mark.parametrize("seed,d,nx,ny,p", [(21, 2, 6, 5, 4), (23, 4, 7, 4, 3), (24, 5, 6, 6, 6)])
def test_floating_pairs_match_paper_reduced_system(seed, d, nx, ny, p):
    """Uniform tiers, TSV columns, one bump on tier 0 and a load on the top
    tier: the GPU's floating pair resistance equals the paper's reduced
    saddle-point system built from Eq. 3 (Sec. III-C/D)."""
    reff = _reff()
    rng = np.random.default_rng(seed)
    r_t = rng.uniform(0.5, 2.0, size=d)
    s_t = rng.uniform(0.5, 2.0, size=d)
    flat = rng.choice(nx * ny, size=p + 2, replace=False)
    xy = [(int(f % nx), int(f // nx)) for f in flat]
    tsv, bump, load = xy[:p], xy[p], xy[p + 1]
    rt = rng.uniform(0.1, 1.0, size=(p, d - 1))
    gx = np.stack([np.full((ny, nx - 1), 1.0 / r_t[i]) for i in range(d)])
    gy = np.stack([np.full((ny - 1, nx), 1.0 / s_t[i]) for i in range(d)])
    desc = gen.make_desc(d, nx, ny, gx, gy, tsv, 1.0 / rt, [bump])
    want = pins.reduced_system_resistance(nx, ny, r_t, s_t, tsv, rt, bump, load)
    b_id = bump[1] * nx + bump[0]
    l_id = (d - 1) * nx * ny + load[1] * nx + load[0]
    h = reff.reff_build_pdn(desc)
    got, _ = reff.reff_query_pairs(h, [b_id], [l_id], reff.REFF_PAIRS_FLOATING)
    assert abs(got[0, 0] - want) / want <= 1e-6
    # with the bump as the only pad, the grounded diagonal is the same value
    gd, _ = reff.reff_solve_diag(h, [l_id])
    assert abs(gd[0] - want) / want <= 1e-6


def test_config2_recipe_pairs():
    """Grounded pairs on the mixed workload's recipe at side 128 (65,536
    nodes, block Krylov path)."""
    reff = _reff()
    d = gen.config2(side=128, n_tsv=64, sigma=10.0)
    nodes = gen.sample_free_nodes(d, 24, 9)
    a, b = nodes[:12], nodes[12:]
    want = ro.pairs(d, a, b, ro.GROUNDED)
    _say("config2 recipe pairs")
    h = reff.reff_build_pdn(d)
    got, st = reff.reff_query_pairs(h, a, b, reff.REFF_PAIRS_GROUNDED, rel_tol=1e-9)
    err = _rel(got, want)
    print("max rel err", err, st, flush=True)
    assert err <= 1e-6


def test_thousand_endpoints_recipe_side_256():
    """1,000 distinct endpoints (500 x 500 pairs, 16 solve blocks and 136
    block cross terms) on the mixed-precision recipe at side 256
    (4 x 256 x 256 = 262,144 nodes), float64, against the oracle at 1e-6;
    output in device memory, pads and coinciding endpoints included."""
    import time

    import torch
    reff = _reff()
    d = gen.config2(side=256, n_tsv=256, sigma=20.0)
    nodes = gen.sample_free_nodes(d, 1000, 77)
    a, b = nodes[:500].copy(), nodes[500:].copy()
    a[0] = gen.pad_ids(d)[0]
    b[1] = a[2]
    want = ro.pairs(d, a, b, mode=ro.GROUNDED)
    _say("1000 endpoints, side 256, fp64, device output")
    h = reff.reff_build_pdn(d)
    out = torch.full((500, 500), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reff.reff_query_pairs(h, a, b, mode=reff.REFF_PAIRS_GROUNDED, R_out=out,
                          precision=reff.REFF_PREC_FP64, rel_tol=1e-10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    got = out.cpu().numpy()
    err = _rel(got, want)
    print(f"max rel err {err:.3e}; {500 * 500 / dt:.3g} pairs/s ({dt:.2f} s)", flush=True)
    assert got[2, 1] == 0.0
    assert err <= 1e-6
    # bounded memory: four solution blocks on the device at a time (four
    # groups; cross-group terms first order after tighter solves)
    _say("1000 endpoints, side 256, fp64, groups of 4 resident blocks")
    t0 = time.perf_counter()
    grp, st = reff.reff_query_pairs(h, a, b, mode=reff.REFF_PAIRS_GROUNDED,
                                    precision=reff.REFF_PREC_FP64, rel_tol=1e-10,
                                    resident_blocks=4)
    dt = time.perf_counter() - t0
    err = _rel(grp, want)
    print(f"grouped: max rel err {err:.3e}; {500 * 500 / dt:.3g} pairs/s ({dt:.2f} s)", flush=True)
    assert grp[2, 1] == 0.0
    assert err <= 1e-6


@pytest.mark.parametrize("prec,tol,rel_tol", [(0, 1e-6, 1e-7), (1, 1e-3, 1e-4)],
                         ids=["fp64", "mixed"])
@pytest.mark.parametrize("resident", [1, 2])
def test_pairs_in_bounded_groups(prec, tol, rel_tol, resident):
    """100 x 100 endpoints on the 2 x 32 x 32 stack (about 200 distinct, four
    solve blocks) with one or two solution blocks on the device at a time:
    the grouped path against the oracle and beside the all-resident call."""
    reff = _reff()
    d = gen.config1()
    rng = np.random.default_rng(23)
    a = rng.choice(2048, size=100, replace=False)
    b = rng.choice(2048, size=100, replace=False)
    a[0] = ro.pad_nodes(d)[0]
    b[1] = a[3]
    want = ro.pairs(d, a, b, ro.GROUNDED)
    _say("bounded pairs, resident", resident, "prec", prec)
    h = reff.reff_build_pdn(d)
    full, _ = reff.reff_query_pairs(h, a, b, reff.REFF_PAIRS_GROUNDED, precision=prec,
                                    rel_tol=rel_tol)
    got, st = reff.reff_query_pairs(h, a, b, reff.REFF_PAIRS_GROUNDED, precision=prec,
                                    rel_tol=rel_tol, resident_blocks=resident)
    err, err_full = _rel(got, want), _rel(full, want)
    print("max rel err grouped", err, "all resident", err_full, st, flush=True)
    assert got[3, 1] == 0.0
    assert err <= tol and err_full <= tol
    with pytest.raises(reff.ReffError):
        reff.reff_query_pairs(h, a, b, reff.REFF_PAIRS_GROUNDED, resident_blocks=-1)
