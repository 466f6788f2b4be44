"""Two-sided bounds on R_i for stacks too large for an exact oracle solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import
or call this module; only the tests and the benchmark's checks use it.  It
shares no code with the HIP path.

R_i is node i's effective resistance to the supply with every pad grounded
(paper Sec. II-B, Eq. 2, bumps merged into one grounded node, Sec. III-B):
R_i = (G^-1)_ii.  Rayleigh's monotonicity law says that an effective
resistance cannot fall when a resistor's conductance is lowered (to zero:
the resistor is cut) and cannot rise when it is raised (to infinity: its two
ends are merged).  For a window W of the (x, y) plane around node i, taken
through every tier (TSV segments are vertical, so each one lies inside or
outside W as a whole):

* upper bound: cut every resistor with an end outside W.  What is left is
  the stack restricted to W with the pads inside W grounded; its R_i is
  >= the true one (infinite when no pad is reachable from i inside W).
* lower bound: merge every node outside W with the grounded supply.  Only
  the ring of nodes just outside W touches W, so this is the stack
  restricted to W plus that ring, with the ring and the pads grounded; its
  R_i is <= the true one.

Both are exact float64 solves of small systems (reff_oracle's Laplacian and
SciPy's sparse LU, as in reff_oracle.diag), so they hold at any stack size,
and they close in on R_i as the window grows; with the whole plane as the
window both equal the exact value.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .reff_oracle import laplacian, pad_nodes


def sub_desc(desc, x0, x1, y0, y1):
    """The stack restricted to columns x0 <= x < x1, rows y0 <= y < y1 (all
    tiers): the resistors with both ends inside, the TSV columns and the
    pads inside, coordinates shifted to the window's origin."""
    nt, nx, ny = int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])
    gx = np.asarray(desc["gx"], dtype=np.float64).reshape(nt, ny, nx - 1)
    gy = np.asarray(desc["gy"], dtype=np.float64).reshape(nt, ny - 1, nx)
    txy = np.asarray(desc["tsv_xy"], dtype=np.int64).reshape(-1, 2)
    tg = np.asarray(desc["tsv_g"], dtype=np.float64).reshape(len(txy), max(nt - 1, 0))
    pxy = np.asarray(desc["pad_xy"], dtype=np.int64).reshape(-1, 2)

    def inside(xy):
        return (xy[:, 0] >= x0) & (xy[:, 0] < x1) & (xy[:, 1] >= y0) & (xy[:, 1] < y1)

    mt, mp = inside(txy), inside(pxy)
    return {"n_tiers": nt, "nx": x1 - x0, "ny": y1 - y0,
            "gx": gx[:, y0:y1, x0:x1 - 1].copy(), "gy": gy[:, y0:y1 - 1, x0:x1].copy(),
            "tsv_xy": (txy[mt] - [x0, y0]).astype(np.int32),
            "tsv_g": tg[mt].copy(),
            "pad_xy": (pxy[mp] - [x0, y0]).astype(np.int32)}


def _resistance(L, ground, i):
    """(G^-1)_ii of the Laplacian L with the nodes `ground` grounded; inf
    when i has no path to a grounded node."""
    n = L.shape[0]
    keep = np.ones(n, dtype=bool)
    keep[np.asarray(ground, dtype=np.int64)] = False
    if not keep[i]:
        return 0.0
    free = np.flatnonzero(keep)
    # nodes of i's connected component among the free ones: a component
    # with no grounded neighbour makes G singular (i's R is then infinite,
    # or unaffected when i is elsewhere)
    A = L[free][:, free].tocsr()
    pos = np.full(n, -1, dtype=np.int64)
    pos[free] = np.arange(len(free))
    from scipy.sparse.csgraph import connected_components
    _, lab = connected_components(A, directed=False)
    comp = np.flatnonzero(lab == lab[pos[i]])
    # grounded neighbours show up as a diagonal larger than the row's
    # off-diagonal sum inside the component
    sub = A[comp][:, comp].tocsc()
    excess = np.asarray(sub.sum(axis=1)).ravel()
    if not np.any(excess > 1e-12 * np.abs(sub.diagonal()).max()):
        return np.inf
    b = np.zeros(len(comp))
    k = int(np.searchsorted(comp, pos[i]))
    b[k] = 1.0
    x = spla.spsolve(sub, b)
    return float(x[k])


def window_bounds(desc, node, half):
    """(lower, upper) bounds on R_node from the window of half-width `half`
    around the node's (x, y) (clipped to the plane), by Rayleigh's
    monotonicity law (module docstring).  Pads give (0, 0)."""
    nt, nx, ny = int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])
    t, rem = divmod(int(node), nx * ny)
    y, x = divmod(rem, nx)
    x0, x1 = max(0, x - half), min(nx, x + half + 1)
    y0, y1 = max(0, y - half), min(ny, y + half + 1)
    # upper: the window alone, its own pads grounded
    w = sub_desc(desc, x0, x1, y0, y1)
    wnx, wny = x1 - x0, y1 - y0
    wi = (t * wny + (y - y0)) * wnx + (x - x0)
    wp = pad_nodes(w) if len(w["pad_xy"]) else np.zeros(0, dtype=np.int64)
    hi = _resistance(laplacian(w), wp, wi) if len(wp) else np.inf
    # lower: the window and the ring around it, ring and pads grounded
    ex0, ex1 = max(0, x0 - 1), min(nx, x1 + 1)
    ey0, ey1 = max(0, y0 - 1), min(ny, y1 + 1)
    e = sub_desc(desc, ex0, ex1, ey0, ey1)
    enx, eny = ex1 - ex0, ey1 - ey0
    ids = np.arange(nt * enx * eny, dtype=np.int64).reshape(nt, eny, enx)
    X = np.arange(ex0, ex1)[None, None, :]
    Y = np.arange(ey0, ey1)[None, :, None]
    ring = np.broadcast_to((X < x0) | (X >= x1) | (Y < y0) | (Y >= y1), ids.shape)
    ep = pad_nodes(e) if len(e["pad_xy"]) else np.zeros(0, dtype=np.int64)
    ground = np.union1d(ep, ids[ring])
    ei = (t * eny + (y - ey0)) * enx + (x - ex0)
    lo = _resistance(laplacian(e), ground, ei) if len(ground) else np.inf
    return lo, hi
