"""Pins of the full-map oracle (oracle/selinv.py): sparse Cholesky with
nested-dissection ordering and selected inversion.

It is tied to results other than its own: the dense inverse of the
pad-merged Laplacian (Eq. 2) assembled independently in tests/pins.py, the
series-chain, vertical-chain and symmetric-ladder closed forms, the paper's
Eq. 3 on a uniform tier with one pad, the SuperLU path of the per-node
oracle on stacks of 10^4 - 10^5 nodes, and Foster's theorem on the full
maps of the plain and mixed-precision stacks, which checks the diagonal
and the off-diagonal entries of G^-1 on every edge together.  Planted
mistakes in the recurrence must fail a pin."""
import numpy as np
import pytest

from oracle import reff_oracle as ro
from oracle import selinv
from paper_2607_05818_amd import gen
from tests import pins

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")

SMALL = [
    (1, 1, 3, 4, 0, 1), (2, 1, 4, 3, 2, 1), (3, 2, 5, 4, 3, 2),
    (4, 3, 4, 4, 4, 3), (5, 2, 7, 2, 2, 1), (6, 1, 12, 12, 0, 5),
    (7, 3, 6, 6, 5, 4), (8, 2, 1, 9, 3, 1), (9, 3, 17, 13, 20, 4),
]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _pinv_diag(d):
    """R_i from Eq. 2 on the pad-merged Laplacian, dense pseudo-inverse."""
    L, idx, g = pins.merged_pad_laplacian_dense(d)
    Lp = np.linalg.pinv(L)
    n = int(d["n_tiers"]) * int(d["nx"]) * int(d["ny"])
    out = np.zeros(n)
    for i in range(n):
        a = idx[i]
        if a != g:
            out[i] = Lp[a, a] + Lp[g, g] - 2.0 * Lp[a, g]
    return out


@pytest.mark.parametrize("leaf", [1, 4, 64])
@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL)
def test_full_map_matches_merged_pad_pinv(seed, nt, nx, ny, ntsv, npad, leaf):
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    want = _pinv_diag(d)
    got = selinv.diag_full(d, leaf=leaf)
    pads = ro.pad_nodes(d)
    assert np.all(got[pads] == 0.0)
    free = np.setdiff1d(np.arange(len(got)), pads)
    assert _rel(got[free], want[free]) < 1e-10
    # the factor's substitutions give the same values (Sec. II-A)
    got2 = selinv.solve_nodes(d, np.arange(len(got)), leaf=leaf)
    assert _rel(got2[free], want[free]) < 1e-10
    assert np.all(got2[pads] == 0.0)


@pytest.mark.parametrize("seed,nt,nx,ny,ntsv,npad", SMALL)
def test_full_map_matches_dense_oracle(seed, nt, nx, ny, ntsv, npad):
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    want = ro.diag(d)
    got = selinv.diag_full(d)
    free = want > 0
    assert _rel(got[free], want[free]) < 1e-12
    assert np.array_equal(got == 0.0, want == 0.0)


def test_series_and_vertical_chains():
    rng = np.random.default_rng(5)
    nx = 40
    gx = rng.uniform(0.5, 2.0, size=(1, 1, nx - 1))
    d = gen.make_desc(1, nx, 1, gx, np.zeros((1, 0, nx)), np.zeros((0, 2)),
                      np.zeros((0, 0)), [[0, 0]])
    want = np.concatenate([[0.0], np.cumsum(1.0 / gx.ravel())])
    got = selinv.diag_full(d, leaf=2)
    assert got[0] == 0.0 and _rel(got[1:], want[1:]) < 1e-13
    T = 9
    g = rng.uniform(1.0, 10.0, size=(1, T - 1))
    d = gen.make_desc(T, 1, 1, np.zeros((T, 1, 0)), np.zeros((T, 0, 1)), [[0, 0]], g, [[0, 0]])
    want = np.concatenate([[0.0], np.cumsum(1.0 / g.ravel())])
    got = selinv.diag_full(d, leaf=2)
    assert _rel(got[1:], want[1:]) < 1e-13


@pytest.mark.parametrize("L,g,h", [(12, 1.0, 0.3), (30, 2.0, 1.7)])
def test_symmetric_ladder(L, g, h):
    d = gen.make_desc(1, L, 2, np.full((1, 2, L - 1), g), np.full((1, 1, L), h),
                      np.zeros((0, 2)), np.zeros((0, 0)), [[0, 0], [0, 1]])
    got = selinv.diag_full(d, leaf=3)
    for k in range(1, L):
        want = pins.ladder_resistance(L, g, h, k)
        assert abs(got[k] - want) / want < 1e-11
        assert abs(got[L + k] - want) / want < 1e-11


def test_wu_closed_form_single_tier():
    """One uniform tier (r, s) with one pad b: R_i = Eq. 3 between i and b."""
    M, N, r, s, pad = 24, 20, 0.8, 1.7, (7, 11)
    gx = np.full((1, N, M - 1), 1.0 / r)
    gy = np.full((1, N - 1, M), 1.0 / s)
    d = gen.make_desc(1, M, N, gx, gy, np.zeros((0, 2)), np.zeros((0, 0)), [pad])
    got = selinv.diag_full(d, leaf=16)
    for i in range(0, M * N, 37):
        y, x = divmod(i, M)
        want = pins.wu_two_point(M, N, r, s, x, y, pad[0], pad[1])
        if want > 0:
            assert abs(got[i] - want) / want < 1e-11


@pytest.mark.parametrize("kind", ["mixed_small", "surrogate_plan", "mixed_100k"])
def test_matches_superlu_path_on_larger_stacks(kind):
    if kind == "mixed_small":
        d = gen.config2(side=96, n_tsv=256, sigma=12.0)
    elif kind == "surrogate_plan":
        d = gen.config4_plan(np.random.default_rng(4004))
    else:
        d = gen.config2(side=160, n_tsv=400, sigma=16.0)
    nodes = gen.sample_free_nodes(d, 48, 77)
    want = ro.diag(d, nodes=nodes)
    got = selinv.diag_full(d)
    assert _rel(got[nodes], want) < 1e-12


def _foster_grounded(d, R, zedges):
    """Sum over the stack's resistors of w_e R_e with the pads merged into
    one supply node: R_e = Z_uu + Z_vv - 2 Z_uv for a free-free edge, the
    free end's R for an edge to a pad, nothing for pad-pad edges."""
    u, v, w = ro.edge_list_fast(d)
    zu, zv, z = zedges
    n = len(R)
    key = np.minimum(zu, zv) * n + np.maximum(zu, zv)
    order = np.argsort(key)
    key, z = key[order], z[order]
    ek = np.minimum(u, v) * n + np.maximum(u, v)
    pads = np.zeros(n, dtype=bool)
    pads[ro.pad_nodes(d)] = True
    both = ~pads[u] & ~pads[v]
    pos = np.searchsorted(key, ek[both])
    assert np.array_equal(key[pos], ek[both]), "an edge's entry is missing from Z"
    Re = np.zeros(len(u))
    Re[both] = R[u[both]] + R[v[both]] - 2.0 * z[pos]
    one = pads[u] ^ pads[v]
    Re[one] = np.where(pads[u[one]], R[v[one]], R[u[one]])
    return float(np.sum(w * Re)), int(n - pads.sum())


def test_foster_grounded_full_map_config1():
    d = gen.config1()
    R, zedges = selinv.diag_and_edges(d)
    tot, n_free = _foster_grounded(d, R, zedges)
    assert n_free == 2032
    assert abs(tot - n_free) < 1e-9 * n_free


@pytest.mark.slow
def test_foster_grounded_full_map_config2():
    """The whole 4 x 512 x 512 map (1,048,320 free nodes)."""
    d = gen.config2()
    R, zedges = selinv.diag_and_edges(d)
    tot, n_free = _foster_grounded(d, R, zedges)
    assert n_free == 1048320
    assert abs(tot - n_free) < 1e-9 * n_free
    assert np.all(R[ro.pad_nodes(d)] == 0.0) and np.all(R[R != 0] > 0)


# --- planted mistakes: each must fail a pin ---------------------------------

def _caught(d, want_pinv):
    try:
        R, zedges = selinv.diag_and_edges(d, leaf=4)
    except Exception:
        return True
    free = want_pinv > 0
    bad = _rel(R[free], want_pinv[free]) > 1e-9
    tot, n_free = _foster_grounded(d, R, zedges)
    return bad or abs(tot - n_free) > 1e-8 * n_free


@pytest.mark.parametrize("kind", ["gather_diagonal_blocks_only", "gather_lower_only",
                                  "drop_lhat_term", "skip_child_update"])
def test_planted_mistakes_are_caught(kind, monkeypatch):
    d = gen.small_random_desc(9, 3, 17, 13, 20, 4)
    want = _pinv_diag(d)
    assert not _caught(d, want)
    orig_gather = selinv.Factor._gather

    if kind == "gather_diagonal_blocks_only":
        def bad(self, Z, S):
            out = orig_gather(self, Z, S)
            sn = self.sn_of[S]
            return np.where(sn[:, None] == sn[None, :], out, 0.0)
        monkeypatch.setattr(selinv.Factor, "_gather", bad)
    elif kind == "gather_lower_only":
        def bad(self, Z, S):
            return np.tril(orig_gather(self, Z, S))
        monkeypatch.setattr(selinv.Factor, "_gather", bad)
    elif kind == "drop_lhat_term":
        orig_mm = selinv._mm
        calls = {"n": 0}

        def bad(a, b, ta=False, tb=False, alpha=1.0):
            # the Lhat^T Z_SJ product is the only ta=True call with alpha 1
            # during selected inversion whose left operand is tall
            if ta and not tb and alpha == 1.0 and a.shape[0] > a.shape[1] and calls["sel"]:
                return np.zeros((a.shape[1], b.shape[1]))
            return orig_mm(a, b, ta=ta, tb=tb, alpha=alpha)
        calls["sel"] = False
        orig_sel = selinv.Factor.selected_inverse

        def sel(self, pattern=False):
            calls["sel"] = True
            try:
                return orig_sel(self, pattern)
            finally:
                calls["sel"] = False
        monkeypatch.setattr(selinv, "_mm", bad)
        monkeypatch.setattr(selinv.Factor, "selected_inverse", sel)
    elif kind == "skip_child_update":
        orig_sym = selinv.Factor._symbolic

        def sym(self):
            orig_sym(self)
            # forget the first non-empty child list: its update matrices are
            # then never assembled into the parent's front
            for J in range(self.ns):
                if self.children[J]:
                    self.children[J] = self.children[J][1:]
                    break
        monkeypatch.setattr(selinv.Factor, "_symbolic", sym)
    assert _caught(d, want)
