"""Pins of the IR-drop / through-bump-current oracle (oracle/ir_drop.py)
against results fixed by circuit theory and by the paper's Eq. 4: Kirchhoff's
current law at the supply, Eq. 4 evaluated from effective resistances (with
the bumps merged into the supply node), a series chain in closed form, the
reciprocity between a pad's share of a unit load and the potential of a
Dirichlet problem with that pad at 1 V, and planted mistakes."""
import numpy as np
import pytest

from oracle import ir_drop as irl
from oracle import reff_oracle as ro
from paper_2607_05818_amd import gen

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")

STACKS = [(11, 2, 6, 5, 4, 3), (12, 3, 5, 7, 6, 2), (13, 1, 9, 4, 0, 4), (14, 4, 4, 4, 5, 1)]


def _scenario(d, seed, n_loads, n_scen, on_pad=False):
    rng = np.random.default_rng(seed)
    n = gen.n_nodes(d)
    loads = rng.choice(n, size=n_loads, replace=False).astype(np.int64)
    if on_pad:
        loads[0] = ro.pad_nodes(d)[0]
    amps = rng.uniform(0.1, 2.0, size=(n_scen, n_loads))
    return loads, amps


@pytest.mark.parametrize("case", STACKS)
def test_pad_currents_sum_to_the_load_current(case):
    seed, nt, nx, ny, ntsv, npad = case
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    loads, amps = _scenario(d, seed + 100, 5, 3, on_pad=True)
    pc = irl.pad_currents(d, loads, amps)
    assert np.allclose(pc.sum(axis=1), amps.sum(axis=1), rtol=1e-12, atol=0)
    assert np.all(pc >= -1e-12)     # no pad sinks current when every load draws


@pytest.mark.parametrize("case", STACKS)
def test_drop_matches_eq4_from_effective_resistances(case):
    """Eq. 4 with the bumps merged into the supply node:
    drop_j = 1/2 sum_k I_k (R_j + R_{l_k} - R(j, l_k))."""
    seed, nt, nx, ny, ntsv, npad = case
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    loads, amps = _scenario(d, seed + 200, 4, 2)
    n = gen.n_nodes(d)
    nodes = np.arange(n)
    Rd = ro.diag(d)
    Rp = ro.pairs(d, nodes, loads, mode=ro.GROUNDED)
    want = 0.5 * amps @ (Rd[:, None] + Rd[loads][None, :] - Rp).T
    got = irl.ir_drop(d, loads, amps)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-14)
    assert np.all(got[:, ro.pad_nodes(d)] == 0.0)


def test_series_chain_closed_form():
    """One row of nodes, pad at x = 0, load I at the far end: the whole
    current runs through every edge, drop_x = I sum_{e < x} 1 / g_e."""
    L = 9
    rng = np.random.default_rng(5)
    g = rng.uniform(0.5, 2.0, L - 1)
    d = gen.make_desc(1, L, 1, g, np.zeros(0), np.zeros((0, 2)), np.zeros((0, 0)),
                      np.array([[0, 0]]))
    I = 1.7
    got = irl.ir_drop(d, [L - 1], [[I]])[0]
    want = I * np.concatenate([[0.0], np.cumsum(1.0 / g)])
    assert np.allclose(got, want, rtol=1e-12)
    assert np.allclose(irl.pad_currents(d, [L - 1], [[I]]), [[I]], rtol=1e-12)


def _dirichlet_potential(d, pad_on):
    """Dense Laplacian of the stack built edge by edge; pad entry `pad_on`
    held at 1 V, every other pad at 0 V, no loads: potentials of all nodes."""
    nt, nx, ny = int(d["n_tiers"]), int(d["nx"]), int(d["ny"])
    n = nt * nx * ny
    Lp = np.zeros((n, n))

    def add(a, b, w):
        Lp[a, a] += w
        Lp[b, b] += w
        Lp[a, b] -= w
        Lp[b, a] -= w

    gx = np.asarray(d["gx"]).reshape(nt, ny, nx - 1)
    gy = np.asarray(d["gy"]).reshape(nt, ny - 1, nx)
    for t in range(nt):
        for y in range(ny):
            for x in range(nx - 1):
                add(t * nx * ny + y * nx + x, t * nx * ny + y * nx + x + 1, gx[t, y, x])
        for y in range(ny - 1):
            for x in range(nx):
                add(t * nx * ny + y * nx + x, t * nx * ny + (y + 1) * nx + x, gy[t, y, x])
    txy = np.asarray(d["tsv_xy"]).reshape(-1, 2)
    tg = np.asarray(d["tsv_g"]).reshape(len(txy), max(nt - 1, 0))
    for j, (x, y) in enumerate(txy):
        for t in range(nt - 1):
            add(t * nx * ny + y * nx + x, (t + 1) * nx * ny + y * nx + x, tg[j, t])
    pads = [int(p[1]) * nx + int(p[0]) for p in np.asarray(d["pad_xy"]).reshape(-1, 2)]
    fixed = np.zeros(n, dtype=bool)
    fixed[pads] = True
    vb = np.zeros(n)
    vb[pads[pad_on]] = 1.0
    fr = np.flatnonzero(~fixed)
    V = vb.copy()
    V[fr] = np.linalg.solve(Lp[np.ix_(fr, fr)], -Lp[np.ix_(fr, np.flatnonzero(fixed))] @ vb[fixed])
    return V


@pytest.mark.parametrize("case", STACKS[:3])
def test_pad_share_of_a_unit_load_is_the_dirichlet_potential(case):
    """Reciprocity: the current pad p delivers to a unit load at l equals the
    potential at l when p is held at 1 V and the other pads at 0 V."""
    seed, nt, nx, ny, ntsv, npad = case
    d = gen.small_random_desc(seed, nt, nx, ny, ntsv, npad)
    n = gen.n_nodes(d)
    free = np.setdiff1d(np.arange(n), ro.pad_nodes(d))
    loads = free[[0, len(free) // 2, len(free) - 1]]
    pc = irl.pad_currents(d, loads, np.eye(len(loads)))
    for p in range(len(np.asarray(d["pad_xy"]).reshape(-1, 2))):
        V = _dirichlet_potential(d, p)
        assert np.allclose(pc[:, p], V[loads], rtol=1e-10, atol=1e-13)


def test_share_statistic():
    assert irl.share_pads_for([10, 0, 0, 0]) == 0.25
    assert irl.share_pads_for([1, 1, 1, 1]) == 1.0
    assert irl.share_pads_for([50, 45, 4, 1]) == 0.5
    assert irl.share_pads_for([50, 44, 4, 2]) == 0.75


def test_planted_mistakes_are_caught(monkeypatch):
    """A pad current that forgets loads placed on the pad itself, or takes the
    edge currents with the wrong sign, fails Kirchhoff's law at the supply."""
    d = gen.small_random_desc(11, 2, 6, 5, 4, 3)
    loads, amps = _scenario(d, 111, 5, 2, on_pad=True)
    real_loads = irl._loads

    def no_pad_loads(desc, ln, la):
        I = real_loads(desc, ln, la)
        I[:, ro.pad_nodes(desc)] = 0.0
        return I

    monkeypatch.setattr(irl, "_loads", no_pad_loads)
    pc = irl.pad_currents(d, loads, amps)
    assert not np.allclose(pc.sum(axis=1), amps.sum(axis=1), rtol=1e-6)
    monkeypatch.setattr(irl, "_loads", real_loads)
    real_full = irl.drop_full
    monkeypatch.setattr(irl, "drop_full", lambda *a: -real_full(*a))
    pc = irl.pad_currents(d, loads, amps)
    assert not np.allclose(pc.sum(axis=1), amps.sum(axis=1), rtol=1e-6)


def test_band_plan_concentrates_bump_current():
    """Sec. IV-B's observation on the synthetic planning study: with every
    TSV in a central band a small fraction of the bumps carries 95 % of the
    current; spreading the same TSVs uniformly spreads it over many more."""
    st = gen.tsv_planning_study(side=64, n_tsv=64, bump_k=8, block_w=14, block_h=7)
    share = {}
    for plan in ("band", "uniform"):
        pc = irl.pad_currents(st[plan], st["loads"], st["amps"])
        assert np.allclose(pc.sum(), st["amps"].sum(), rtol=1e-10)
        share[plan] = irl.share_pads_for(pc[0])
    print(share)
    assert share["band"] < 0.6 * share["uniform"]
