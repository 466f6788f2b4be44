"""Pins of the CPU oracle against results fixed by the paper and by circuit
theory: a dense pseudo-inverse of the pad-merged Laplacian (Eq. 2),
closed-form chains and ladders, the paper's Eq. 3 on uniform grids, the
paper's reduced system (Sec. III-C/D), Foster's theorem, Rayleigh
monotonicity, metric properties and scaling.  A final group plants
plausible mistakes in a copy of the oracle's assembly and checks that a pin
catches each one."""
import numpy as np
import pytest

import oracle
from oracle import reff_oracle as ro
from paper_2607_05818_amd import gen
from tests import pins

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


SMALL = [
    (1, 1, 3, 4, 0, 1), (2, 1, 4, 3, 2, 1), (3, 2, 5, 4, 3, 2),
    (4, 3, 4, 4, 4, 3), (5, 2, 7, 2, 2, 1), (6, 1, 12, 12, 0, 5),
    (7, 3, 6, 6, 5, 4), (8, 2, 1, 9, 3, 1),
]


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL)
def test_diag_matches_merged_pad_pinv(seed, nt, nx, ny, ntsv, npad):
    """Eq. 2 with every pad contracted into one supply node g, evaluated by
    a dense pseudo-inverse, equals the oracle's (G^-1)_ii."""
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    L, idx, g = pins.merged_pad_laplacian_dense(d)
    Lp = np.linalg.pinv(L)
    n = nt * nx * ny
    want = np.zeros(n)
    for i in range(n):
        a = idx[i]
        if a == g:
            continue
        e = np.zeros(L.shape[0])
        e[a] += 1.0
        e[g] -= 1.0
        want[i] = e @ Lp @ e
    got = ro.diag(d)
    assert np.all(got[ro.pad_nodes(d)] == 0.0)
    free = want > 0
    assert _rel(got[free], want[free]) < 1e-10


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL[:5])
def test_sparse_path_matches_dense_path(seed, nt, nx, ny, ntsv, npad, monkeypatch):
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    dense = ro.diag(d)
    monkeypatch.setattr(ro, "DENSE_MAX", 0)
    sparse = ro.diag(d, chunk=3)
    assert _rel(sparse[dense > 0], dense[dense > 0]) < 1e-12
    a = np.arange(min(4, nt * nx * ny))
    pd_ = ro.pairs(d, a, a[::-1], ro.GROUNDED)
    monkeypatch.setattr(ro, "DENSE_MAX", 4096)
    pd2 = ro.pairs(d, a, a[::-1], ro.GROUNDED)
    assert np.allclose(pd_, pd2, rtol=1e-12, atol=1e-14)


def test_fast_assembly_matches_edge_by_edge():
    d = gen.small_random_desc(11, 3, 7, 5, 6, 3)
    A = ro.laplacian(d, fast=False).toarray()
    B = ro.laplacian(d, fast=True).toarray()
    assert np.array_equal(A, B)


def test_series_chain():
    """nt = ny = 1, pad at x = 0: R_x = sum of 1/gx over the edges left of x."""
    rng = np.random.default_rng(5)
    nx = 40
    gx = rng.uniform(0.5, 2.0, size=(1, 1, nx - 1))
    d = gen.make_desc(1, nx, 1, gx, np.zeros((1, 0, nx)), np.zeros((0, 2)),
                      np.zeros((0, 0)), [[0, 0]])
    want = np.concatenate([[0.0], np.cumsum(1.0 / gx.ravel())])
    got = ro.diag(d)
    assert got[0] == 0.0
    assert _rel(got[1:], want[1:]) < 1e-13


def test_vertical_tsv_chain():
    """nx = ny = 1, T tiers, one TSV column, pad on tier 0:
    R_t = sum of the segment resistances below tier t."""
    T = 9
    g = np.random.default_rng(6).uniform(1.0, 10.0, size=(1, T - 1))
    d = gen.make_desc(T, 1, 1, np.zeros((T, 1, 0)), np.zeros((T, 0, 1)),
                      [[0, 0]], g, [[0, 0]])
    want = np.concatenate([[0.0], np.cumsum(1.0 / g.ravel())])
    got = ro.diag(d)
    assert _rel(got[1:], want[1:]) < 1e-13


@pytest.mark.parametrize("L,g,h", [(12, 1.0, 0.3), (30, 2.0, 1.7), (7, 0.6, 4.0)])
def test_symmetric_ladder(L, g, h):
    d = gen.make_desc(1, L, 2, np.full((1, 2, L - 1), g), np.full((1, 1, L), h),
                      np.zeros((0, 2)), np.zeros((0, 0)), [[0, 0], [0, 1]])
    got = ro.diag(d)
    for k in range(1, L):
        want = pins.ladder_resistance(L, g, h, k)
        assert abs(got[k] - want) / want < 1e-11        # rail y = 0
        assert abs(got[L + k] - want) / want < 1e-11    # rail y = 1 (mirror)


@pytest.mark.parametrize("M,N,r,s,pad", [(9, 7, 0.8, 1.7, (3, 2)), (16, 16, 1.0, 1.0, (0, 0)),
                                         (5, 11, 2.5, 0.4, (4, 10))])
def test_wu_closed_form_single_tier(M, N, r, s, pad):
    """Uniform single tier with exactly one pad b: R_i = Wu(i, b), Eq. 3."""
    d = gen.make_desc(1, M, N, np.full((1, N, M - 1), 1.0 / r), np.full((1, N - 1, M), 1.0 / s),
                      np.zeros((0, 2)), np.zeros((0, 0)), [pad])
    got = ro.diag(d)
    for y in range(N):
        for x in range(M):
            if (x, y) == tuple(pad):
                continue
            want = pins.wu_two_point(M, N, r, s, x, y, pad[0], pad[1])
            assert abs(got[y * M + x] - want) / want < 1e-11


def test_wu_at_512_sampled():
    """Eq. 3 holds at the mixed-precision workload's tier size: a 512x512
    uniform tier with one pad, checked on a few sampled nodes."""
    M = N = 512
    r, s = 1.0, 1.3
    pad = (100, 317)
    d = gen.make_desc(1, M, N, np.full((1, N, M - 1), 1.0 / r), np.full((1, N - 1, M), 1.0 / s),
                      np.zeros((0, 2)), np.zeros((0, 0)), [pad])
    rng = np.random.default_rng(9)
    nodes = rng.choice(M * N, size=4, replace=False)
    got = ro.diag(d, nodes=nodes)
    for k, i in enumerate(nodes):
        want = pins.wu_two_point(M, N, r, s, i % M, i // M, pad[0], pad[1])
        assert abs(got[k] - want) / want < 1e-9


REDUCED = [
    # (seed, d, nx, ny, p)
    (21, 2, 6, 5, 4), (22, 3, 5, 6, 5), (23, 4, 7, 4, 3), (24, 5, 6, 6, 6),
]


@pytest.mark.parametrize("seed,d,nx,ny,p", REDUCED)
def test_paper_reduced_system(seed, d, nx, ny, p):
    """Uniform tiers joined by TSV columns, one bump on tier 0 and a load on
    the last tier: the paper's reduced system (Sec. III-C/D) gives the same
    pair resistance as the oracle in FLOATING mode, and as the oracle's
    grounded diagonal when the bump is the only pad."""
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
    fl = ro.pairs(desc, [b_id], [l_id], ro.FLOATING)[0, 0]
    gr = ro.diag(desc, nodes=[l_id])[0]
    assert abs(fl - want) / want < 1e-11
    assert abs(gr - want) / want < 1e-11
    # the same bump/load pair grounded at a different reference node
    fl2 = ro.pairs(desc, [l_id], [b_id], ro.FLOATING)[0, 0]
    assert abs(fl2 - want) / want < 1e-11


def test_foster_grounded_config1():
    """Pads merged into one ground: sum over edges of w_e * R_e equals the
    number of free nodes, where R_e of an edge touching a pad is the free
    endpoint's R, and pad-pad edges contribute nothing (Foster's theorem)."""
    d = gen.config1()
    R = ro.diag(d)
    u, v, w = ro.edge_list(d)
    pads = set(ro.pad_nodes(d).tolist())
    tot = 0.0
    K = ro.pairs(d, np.arange(len(R)), np.arange(len(R)), ro.GROUNDED)
    for a, b, ww in zip(u, v, w):
        if a in pads and b in pads:
            continue
        tot += ww * K[a, b]
    n_free = len(R) - len(pads)
    assert abs(tot - n_free) < 1e-8 * n_free


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL[1:6])
def test_foster_floating(seed, nt, nx, ny, ntsv, npad):
    """Foster on the ungrounded Laplacian: sum w_e R(u,v) = N - 1 when the
    graph is connected (with at least one TSV every tier is reachable)."""
    d = gen.small_random_desc(seed, nt, nx, ny, max(ntsv, 1), npad)
    n = nt * nx * ny
    u, v, w = ro.edge_list(d)
    K = ro.pairs(d, np.arange(n), np.arange(n), ro.FLOATING)
    tot = float(np.sum(w * K[u, v]))
    assert abs(tot - (n - 1)) < 1e-9 * n


def test_rayleigh_monotonicity():
    """Raising a conductance, adding a TSV column or adding a pad never
    raises any node's resistance to the supply."""
    d = gen.small_random_desc(31, 3, 6, 6, 3, 2)
    base = ro.diag(d)
    d2 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in d.items()}
    d2["gx"][1, 2, 3] *= 5.0
    r2 = ro.diag(d2)
    assert np.all(r2 <= base + 1e-13)
    assert np.any(r2 < base - 1e-6)
    d3 = dict(d2)
    d3["tsv_xy"] = np.vstack([d2["tsv_xy"], [[5, 5]]]).astype(np.int32)
    d3["tsv_g"] = np.vstack([d2["tsv_g"], [[3.0, 3.0]]])
    r3 = ro.diag(d3)
    assert np.all(r3 <= r2 + 1e-13)
    d4 = dict(d3)
    d4["pad_xy"] = np.vstack([d3["pad_xy"], [[0, 5]]]).astype(np.int32)
    r4 = ro.diag(d4)
    assert np.all(r4 <= r3 + 1e-13)
    assert r4[5 * 6 + 0] == 0.0


def test_metric_scaling_mirror():
    d = gen.small_random_desc(41, 2, 5, 4, 3, 2)
    n = 40
    nodes = np.arange(n)
    K = ro.pairs(d, nodes, nodes, ro.GROUNDED)
    F = ro.pairs(d, nodes, nodes, ro.FLOATING)
    R = ro.diag(d)
    for M in (K, F):
        assert np.allclose(M, M.T, rtol=1e-12, atol=1e-14)
        assert np.all(np.diag(M) == 0.0)
        # triangle inequality: R(a,c) <= R(a,b) + R(b,c)
        assert np.all(M[:, None, :] <= M[:, :, None] + M[None, :, :] + 1e-12)
    # grounded: R(a,b) <= R_a + R_b; pair with a pad equals the other's R
    assert np.all(K <= R[:, None] + R[None, :] + 1e-12)
    p = ro.pad_nodes(d)[0]
    assert np.allclose(K[p], R, rtol=1e-12, atol=1e-14)
    # scaling: G -> cG gives R -> R/c
    c = 3.7
    dc = dict(d, gx=d["gx"] * c, gy=d["gy"] * c, tsv_g=d["tsv_g"] * c)
    assert np.allclose(ro.diag(dc), R / c, rtol=1e-12, atol=0)
    # mirroring the instance in x mirrors the map
    nt, nx, ny = 2, 5, 4
    dm = dict(d)
    dm["gx"] = d["gx"][:, :, ::-1].copy()
    dm["gy"] = d["gy"][:, :, ::-1].copy()
    dm["tsv_xy"] = np.stack([nx - 1 - d["tsv_xy"][:, 0], d["tsv_xy"][:, 1]], 1).astype(np.int32)
    dm["pad_xy"] = np.stack([nx - 1 - d["pad_xy"][:, 0], d["pad_xy"][:, 1]], 1).astype(np.int32)
    Rm = ro.diag(dm).reshape(nt, ny, nx)[:, :, ::-1].ravel()
    assert np.allclose(Rm, R, rtol=1e-12, atol=0)


def test_config1_range():
    """Config-1 map: every free node positive, pads zero, and within the
    range a series bound allows (below the sum over any path to a pad)."""
    d = gen.config1()
    R = ro.diag(d)
    pads = ro.pad_nodes(d)
    assert np.all(R[pads] == 0.0)
    free = np.setdiff1d(np.arange(len(R)), pads)
    assert np.all(R[free] > 0.0)
    assert R[free].max() < 3.0


# --- planted mistakes: each variant of the assembly must fail a pin -------

def _planted(monkeypatch, kind):
    orig = ro.edge_list

    def bad(desc):
        u, v, w = orig(desc)
        nt, nx, ny = int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])
        if kind == "drop_tsv":
            keep = np.abs(v - u) != nx * ny
            return u[keep], v[keep], w[keep]
        if kind == "tsv_wrong_tier":
            same = np.abs(v - u) == nx * ny
            w = w.copy()
            w[same] = np.roll(w[same], 1)
            return u, v, w
        if kind == "gx_reversed":
            horiz = (v - u) == 1
            w = w.copy()
            w[horiz] = w[horiz][::-1]
            return u, v, w
        raise ValueError(kind)

    monkeypatch.setattr(ro, "edge_list", bad)


@pytest.mark.parametrize("kind", ["drop_tsv", "tsv_wrong_tier", "gx_reversed"])
def test_planted_mistakes_are_caught(kind, monkeypatch):
    _planted(monkeypatch, kind)
    caught = False
    # vertical chain pin (TSV segments) and series chain pin (x edges)
    T = 5
    g = np.array([[1.0, 2.0, 4.0, 8.0]])
    d = gen.make_desc(T, 1, 1, np.zeros((T, 1, 0)), np.zeros((T, 0, 1)), [[0, 0]], g, [[0, 0]])
    try:
        got = ro.diag(d)
        want = np.concatenate([[0.0], np.cumsum(1.0 / g.ravel())])
        caught |= _rel(got[1:], want[1:]) > 1e-9
    except Exception:
        caught = True
    gx = np.linspace(0.5, 2.0, 9).reshape(1, 1, 9)
    d = gen.make_desc(1, 10, 1, gx, np.zeros((1, 0, 10)), np.zeros((0, 2)), np.zeros((0, 0)), [[0, 0]])
    got = ro.diag(d)
    want = np.concatenate([[0.0], np.cumsum(1.0 / gx.ravel())])
    caught |= _rel(got[1:], want[1:]) > 1e-9
    assert caught
