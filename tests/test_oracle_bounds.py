"""Pins of oracle/bounds.py (Rayleigh window bounds on R_i) against what
the mathematics fixes: a chain's series and parallel closed forms, the exact
values of the independent oracle on small stacks (reff_oracle.diag, a dense
inverse or sparse LU), the whole-plane window (no cut, no merge: both bounds
exact) and the monotone closing-in of nested windows."""
import numpy as np
import pytest

from oracle import bounds as ob
from oracle import reff_oracle as ro
from paper_2607_05818_amd import gen

REL = 1e-11  # float64 solves of the same small systems, different orders


def _chain(g):
    """One tier, len(g) + 1 nodes in a row, edge j between x = j and j + 1,
    the pad at x = 0."""
    n = len(g) + 1
    return gen.make_desc(1, n, 1, np.asarray(g).reshape(1, 1, n - 1),
                         np.zeros((1, 0, n)), np.zeros((0, 2)), np.zeros((0, 0)),
                         np.array([[0, 0]]))


@pytest.mark.parametrize("i,half", [(5, 2), (5, 5), (5, 7), (9, 3), (1, 1), (11, 4)])
def test_chain_closed_forms(i, half):
    """Series resistances along the chain: the upper bound is the path to
    the pad when the window holds it (else infinite); the lower bound is the
    parallel combination of the paths to the pad or the left ring node and
    to the right ring node (none when the window reaches the chain's end)."""
    rng = np.random.default_rng(100 + i + half)
    g = rng.uniform(0.5, 2.0, size=12)
    d = _chain(g)
    n = len(g) + 1
    x0, x1 = max(0, i - half), min(n, i + half + 1)
    to_pad = float(np.sum(1.0 / g[:i]))
    up = to_pad if x0 == 0 else np.inf
    left = to_pad if x0 == 0 else float(np.sum(1.0 / g[x0 - 1:i]))
    right = float(np.sum(1.0 / g[i:x1])) if x1 < n else np.inf
    low = 1.0 / (1.0 / left + (0.0 if np.isinf(right) else 1.0 / right))
    lo, hi = ob.window_bounds(d, i, half)
    assert lo == pytest.approx(low, rel=REL)
    if np.isinf(up):
        assert np.isinf(hi)
    else:
        assert hi == pytest.approx(up, rel=REL)
    # the exact value lies between
    assert lo <= to_pad * (1 + REL) and to_pad <= hi * (1 + REL)


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", [(31, 2, 9, 7, 5, 2), (32, 3, 12, 5, 8, 3),
                                                     (33, 1, 10, 10, 0, 1), (34, 4, 6, 8, 6, 2)])
def test_bounds_bracket_exact_values_and_close_in(seed, nt, nx, ny, ntsv, npad):
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    exact = ro.diag(d)
    n = nt * nx * ny
    for v in range(0, n, 3):
        prev = (0.0, np.inf)
        for half in (1, 2, 3, 5, 8):
            lo, hi = ob.window_bounds(d, v, half)
            assert lo <= exact[v] * (1 + REL) + 1e-15
            assert exact[v] <= hi * (1 + REL)
            # nested windows: cut less, merge less
            assert lo >= prev[0] * (1 - REL) and hi <= prev[1] * (1 + REL)
            prev = (lo, hi)
        # a window holding the whole plane cuts and merges nothing
        lo, hi = ob.window_bounds(d, v, max(nx, ny))
        if exact[v] == 0.0:
            assert lo == 0.0 and hi == 0.0
        else:
            assert lo == pytest.approx(exact[v], rel=REL)
            assert hi == pytest.approx(exact[v], rel=REL)


def test_window_without_pad_on_upper_tier_has_no_upper_bound():
    """An upper-tier node whose window holds no TSV column cannot reach a
    pad inside the window: the upper bound is infinite, the lower finite."""
    d = gen.make_desc(2, 9, 9, np.ones((2, 9, 8)), np.ones((2, 8, 9)), np.array([[0, 0]]),
                      np.ones((1, 1)), np.array([[0, 0]]))
    v = 81 + 4 * 9 + 4  # tier 1, (4, 4)
    lo, hi = ob.window_bounds(d, v, 2)
    assert np.isinf(hi) and 0 < lo < np.inf
    assert lo <= ro.diag(d, [v])[0]


def test_planted_mistakes_are_caught():
    """Plausible mistakes in the bounds fail the pins above: merging the
    outside without keeping the resistors that reach it (the lower bound then
    loses its paths to the ring) breaks the chain's parallel form, and a
    window shifted by one column stops bracketing the exact values."""
    rng = np.random.default_rng(7)
    g = rng.uniform(0.5, 2.0, size=12)
    d = _chain(g)
    i, half = 6, 3  # window [3, 10) of 13 nodes: ring nodes at 2 and 10
    # correct lower bound: paths to both ring nodes
    left = float(np.sum(1.0 / g[i - half - 1:i]))
    right = float(np.sum(1.0 / g[i:i + half + 1]))
    want = 1.0 / (1.0 / left + 1.0 / right)
    lo, _ = ob.window_bounds(d, i, half)
    assert lo == pytest.approx(want, rel=REL)
    # planted: the ring grounded but the window's edges to it cut -> the
    # node has no path to ground inside the window
    w = ob.sub_desc(d, i - half, i + half + 1, 0, 1)
    L = ro.laplacian(w)
    assert np.isinf(ob._resistance(L, [], half))
    # planted: a window shifted one column away from the node's own column
    s = gen.small_random_desc(41, 2, 12, 9, 6, 2)
    exact = ro.diag(s)
    bad = 0
    for v in range(0, 2 * 12 * 9, 5):
        t, rem = divmod(v, 12 * 9)
        y, x = divmod(rem, 12)
        if x + 1 >= 12 or exact[v] == 0.0:
            continue
        lo, hi = ob.window_bounds(s, v + 1, 2)  # bounds of the neighbour, not of v
        bad += not (lo <= exact[v] * (1 + REL) and exact[v] <= hi * (1 + REL))
    assert bad > 0


def test_stored_large_stack_bounds_reproduce():
    """tests/golden/config5_bounds.json (the benchmark's check of the
    full-size large stack) holds what the oracle computes: its node sample
    and two of its bound pairs recomputed here."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config5_bounds.json")))
    d = gen.config5()
    nodes = gen.sample_free_nodes(d, 64, 5005)[:16]
    assert [int(v) for v in nodes] == g["nodes"]
    for j in (0, 5):
        lo, hi = ob.window_bounds(d, int(nodes[j]), 64)
        assert lo == pytest.approx(g["lo"][j], rel=1e-12)
        if g["hi"][j] is None:
            assert np.isinf(hi)
        else:
            assert hi == pytest.approx(g["hi"][j], rel=1e-12)
