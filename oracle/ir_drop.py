"""IR drop and through-bump currents of load scenarios (oracle).

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import
or call this module; only the tests and the benchmark use it.  It shares no
code with the HIP path.

What it computes (paper references are to arxiv 2607.05818): bumps (pads)
are ideal voltage sources at the supply voltage and loads are ideal current
sources drawing I_k at node l_k (Sec. III-B, assumption 1).  The DC model
G V = I (Sec. II-A, Eq. 1) on the free nodes, with the voltages measured as
drops below the supply, gives
    drop = G^{-1} I,   drop = 0 on pads,
the definition written out here (one sparse solve per scenario).  Eq. 4
(Sec. II-B) states the same voltages through effective resistances; with
every bump merged into the supply node it reads
    drop_j = 1/2 sum_k I_k (R_j + R_{l_k} - R(j, l_k)),
which tests/test_ir_drop_pins.py checks against this module.  The current a
pad delivers (the through-bump current of Sec. IV-B) is the sum over its
edges of g_pu (drop_u - drop_p) = g_pu drop_u, plus the current of any load
placed on the pad itself.

Parity unpinned: none.
"""
from __future__ import annotations

import numpy as np

from .reff_oracle import _dims, _Solver, edge_list, edge_list_fast, grounded


def _loads(desc, load_nodes, load_amps):
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    load_nodes = np.asarray(load_nodes, dtype=np.int64)
    A = np.atleast_2d(np.asarray(load_amps, dtype=np.float64))
    assert A.shape[1] == len(load_nodes)
    I = np.zeros((A.shape[0], n))
    for k, v in enumerate(load_nodes):
        I[:, v] += A[:, k]
    return I


def drop_full(desc, load_nodes, load_amps):
    """(n_scen, n) IR drop at every node id for each load scenario; row c of
    load_amps gives the currents drawn at load_nodes."""
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    I = _loads(desc, load_nodes, load_amps)
    G, free = grounded(desc)
    V = _Solver(G).solve(I[:, free].T)
    out = np.zeros((I.shape[0], n))
    out[:, free] = V.T
    return out


def ir_drop(desc, load_nodes, load_amps, nodes=None):
    """IR drop at the requested node ids (all if None), (n_scen, len)."""
    D = drop_full(desc, load_nodes, load_amps)
    return D if nodes is None else D[:, np.asarray(nodes, dtype=np.int64)]


def pad_currents(desc, load_nodes, load_amps):
    """(n_scen, n_pads) current delivered by each pad entry of the
    descriptor, in descriptor order; a pad position listed twice reports its
    current at its first entry and 0 at the later ones."""
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    D = drop_full(desc, load_nodes, load_amps)
    I = _loads(desc, load_nodes, load_amps)
    u, v, w = edge_list_fast(desc) if n > 20000 else edge_list(desc)
    flow = np.zeros((D.shape[0], n))
    # current leaving node a towards node b along edge (a, b): w (V_a - V_b)
    # = w (drop_b - drop_a); a pad's outflow sums it over its edges
    np.add.at(flow.T, u, (w * (D[:, v] - D[:, u])).T)
    np.add.at(flow.T, v, (w * (D[:, u] - D[:, v])).T)
    pxy = np.asarray(desc["pad_xy"], dtype=np.int64).reshape(-1, 2)
    ids = pxy[:, 1] * nx + pxy[:, 0]
    out = np.zeros((D.shape[0], len(ids)))
    seen = set()
    for k, p in enumerate(ids):
        if int(p) in seen:
            continue
        seen.add(int(p))
        out[:, k] = flow[:, p] + I[:, p]
    return out


def share_pads_for(currents, frac=0.95):
    """Fraction of the pads that carry `frac` of the total current: pads
    sorted by current, largest first, counted until their sum reaches frac
    of the total (the through-bump current statistic of Sec. IV-B)."""
    c = np.sort(np.asarray(currents, dtype=np.float64))[::-1]
    tot = c.sum()
    k = int(np.searchsorted(np.cumsum(c), frac * tot - 1e-12 * abs(tot))) + 1
    return min(k, len(c)) / len(c)
