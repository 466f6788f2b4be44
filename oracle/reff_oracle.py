"""CPU oracle for node-to-supply and pairwise effective resistance.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import
or call this module; only the tests, the package's smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
it reads the same plain descriptor dict (arrays of edge conductances, TSV
columns and pad positions) and does everything else on its own, in float64,
the slow and obvious way.

What it computes (paper references are to arxiv 2607.05818):

* The stacked PDN is a resistive network: each tier is a 2D mesh, tiers are
  joined only by TSV segments (Sec. III-B, assumption 2).  Its DC model is
  G V = I with G sparse, symmetric and positive definite (Sec. II-A, Eq. 1).
* Supply bumps are ideal voltage sources (Sec. III-B, assumption 1), so they
  are Dirichlet nodes: with all pads merged into one supply node g, the
  effective resistance of Eq. 2 (Sec. II-B) between node i and the supply is
  R(i, g) = (e_i - e_g)^T L'^+ (e_i - e_g) = (G^{-1})_{ii}, where
  G = L[F, F] is the Laplacian restricted to the free (non-pad) nodes.
  That grounded-Laplacian identity is the definition the oracle writes out:
  R_i = e_i^T G^{-1} e_i, and R_i = 0 on pads.
* Pairwise resistance (Eq. 2) between two nodes a, b:
    GROUNDED: pads stay merged into the grounded supply; with K = G^{-1}
              padded by zero rows/columns on pads,
              R(a,b) = K_aa + K_bb - 2 K_ab.
    FLOATING: pads are ordinary nodes of the un-grounded Laplacian L of the
              whole stack, exactly Eq. 2; computed by grounding one
              reference node r, K = (L[-r,-r])^{-1} padded with zero,
              R(a,b) = K_aa + K_bb - 2 K_ab (independent of r).
  Solving only for the m + n columns K e_a, K e_b mirrors the paper's use of
  linearity to get m x n pairs from m + n solves (Sec. III-D).

Solves use a dense inverse for small systems and SciPy's sparse LU
(SuperLU) as a library primitive for larger ones.  Full maps of large
stacks come from oracle/selinv.py (sparse Cholesky + selected inversion),
which is pinned against this module.  Parity unpinned: none.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GROUNDED = 0
FLOATING = 1

DENSE_MAX = 4096


def _dims(desc):
    return int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])


def node_id(desc, t, x, y):
    nt, nx, ny = _dims(desc)
    return (t * ny + y) * nx + x


def edge_list(desc):
    """All resistors of the stack as (u, v, conductance) arrays.

    In-plane x edges join (t,x,y)-(t,x+1,y), y edges join (t,x,y)-(t,x,y+1),
    and every TSV column at (x,y) contributes one segment per adjacent tier
    pair (t,x,y)-(t+1,x,y) with its own conductance (the per-segment Rt of
    the paper's notation table, Sec. III-C)."""
    nt, nx, ny = _dims(desc)
    us, vs, ws = [], [], []
    gx = np.asarray(desc["gx"], dtype=np.float64).reshape(nt, ny, nx - 1)
    gy = np.asarray(desc["gy"], dtype=np.float64).reshape(nt, ny - 1, nx)
    for t in range(nt):
        for y in range(ny):
            for x in range(nx - 1):
                us.append(node_id(desc, t, x, y))
                vs.append(node_id(desc, t, x + 1, y))
                ws.append(gx[t, y, x])
        for y in range(ny - 1):
            for x in range(nx):
                us.append(node_id(desc, t, x, y))
                vs.append(node_id(desc, t, x, y + 1))
                ws.append(gy[t, y, x])
    tsv_xy = np.asarray(desc["tsv_xy"]).reshape(-1, 2)
    tsv_g = np.asarray(desc["tsv_g"], dtype=np.float64).reshape(len(tsv_xy), max(nt - 1, 0))
    for j, (x, y) in enumerate(tsv_xy):
        for t in range(nt - 1):
            us.append(node_id(desc, t, int(x), int(y)))
            vs.append(node_id(desc, t + 1, int(x), int(y)))
            ws.append(tsv_g[j, t])
    return (np.asarray(us, dtype=np.int64), np.asarray(vs, dtype=np.int64),
            np.asarray(ws, dtype=np.float64))


def edge_list_fast(desc):
    """The same edges as edge_list, built with array operations so that
    million-node stacks assemble in seconds.  A test checks that the two
    agree edge for edge."""
    nt, nx, ny = _dims(desc)
    ids = np.arange(nt * nx * ny, dtype=np.int64).reshape(nt, ny, nx)
    gx = np.asarray(desc["gx"], dtype=np.float64).reshape(nt, ny, nx - 1)
    gy = np.asarray(desc["gy"], dtype=np.float64).reshape(nt, ny - 1, nx)
    u = [ids[:, :, :-1].ravel(), ids[:, :-1, :].ravel()]
    v = [ids[:, :, 1:].ravel(), ids[:, 1:, :].ravel()]
    w = [gx.ravel(), gy.ravel()]
    tsv_xy = np.asarray(desc["tsv_xy"], dtype=np.int64).reshape(-1, 2)
    tsv_g = np.asarray(desc["tsv_g"], dtype=np.float64).reshape(len(tsv_xy), max(nt - 1, 0))
    for t in range(nt - 1):
        u.append(ids[t, tsv_xy[:, 1], tsv_xy[:, 0]])
        v.append(ids[t + 1, tsv_xy[:, 1], tsv_xy[:, 0]])
        w.append(tsv_g[:, t])
    return np.concatenate(u), np.concatenate(v), np.concatenate(w)


def laplacian(desc, fast=None):
    """Weighted Laplacian L of the whole stack (pads not grounded), CSR."""
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    if fast is None:
        fast = n > 20000
    u, v, w = edge_list_fast(desc) if fast else edge_list(desc)
    rows = np.concatenate([u, v, u, v])
    cols = np.concatenate([v, u, u, v])
    vals = np.concatenate([-w, -w, w, w])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def pad_nodes(desc):
    nx = int(desc["nx"])
    p = np.asarray(desc["pad_xy"], dtype=np.int64).reshape(-1, 2)
    return np.unique(p[:, 1] * nx + p[:, 0])


def grounded(desc, fast=None):
    """G = L[F, F] with F the free (non-pad) nodes; returns (G, free ids)."""
    L = laplacian(desc, fast)
    n = L.shape[0]
    is_pad = np.zeros(n, dtype=bool)
    is_pad[pad_nodes(desc)] = True
    free = np.flatnonzero(~is_pad)
    G = L[free][:, free].tocsc()
    return G, free


class _Solver:
    """Solves G X = B for the grounded (or reference-grounded) matrix."""

    def __init__(self, M):
        self.n = M.shape[0]
        if self.n <= DENSE_MAX:
            self.dense_inv = np.linalg.inv(M.toarray())
            self.lu = None
        else:
            self.dense_inv = None
            self.lu = spla.splu(M.tocsc(), permc_spec="MMD_AT_PLUS_A")

    def solve(self, B):
        if self.dense_inv is not None:
            return self.dense_inv @ B
        return self.lu.solve(np.asarray(B, dtype=np.float64))


def _unit_columns(n, rows):
    E = np.zeros((n, len(rows)), dtype=np.float64)
    E[rows, np.arange(len(rows))] = 1.0
    return E


def diag(desc, nodes=None, chunk=64, fast=None):
    """R_i = (G^{-1})_ii for the requested node ids (all nodes if None);
    pads give 0.  One unit-current solve per free node (Sec. II-B, Eq. 2,
    with the pads merged into the grounded supply)."""
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    nodes = np.arange(n, dtype=np.int64) if nodes is None else np.asarray(nodes, dtype=np.int64)
    G, free = grounded(desc, fast)
    pos = np.full(n, -1, dtype=np.int64)
    pos[free] = np.arange(len(free))
    out = np.zeros(len(nodes), dtype=np.float64)
    want = np.flatnonzero(pos[nodes] >= 0)
    if len(want) == 0:
        return out
    S = _Solver(G)
    if S.dense_inv is not None:
        out[want] = S.dense_inv[pos[nodes[want]], pos[nodes[want]]]
        return out
    for c0 in range(0, len(want), chunk):
        sel = want[c0:c0 + chunk]
        rows = pos[nodes[sel]]
        X = S.solve(_unit_columns(G.shape[0], rows))
        out[sel] = X[rows, np.arange(len(rows))]
    return out


def pairs(desc, a, b, mode=GROUNDED, fast=None):
    """m x n matrix of R(a_i, b_j) (Eq. 2); see the module docstring for
    the two modes.  Solves m + n unit-current systems."""
    nt, nx, ny = _dims(desc)
    n = nt * nx * ny
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    if mode == GROUNDED:
        M, keep = grounded(desc, fast)
    elif mode == FLOATING:
        L = laplacian(desc, fast)
        r = 0
        keep = np.arange(1, n, dtype=np.int64)
        M = L[keep][:, keep].tocsc()
    else:
        raise ValueError("mode must be GROUNDED or FLOATING")
    pos = np.full(n, -1, dtype=np.int64)
    pos[keep] = np.arange(len(keep))
    S = _Solver(M)
    ends = np.unique(np.concatenate([a, b]))
    live = ends[pos[ends] >= 0]
    # K restricted to the columns of the requested endpoints (zero on the
    # grounded nodes, whose potential is fixed at 0).
    Kcols = {}
    if len(live):
        X = S.solve(_unit_columns(M.shape[0], pos[live]))
        for j, node in enumerate(live):
            Kcols[int(node)] = X[:, j]

    def K(u, v):
        if pos[u] < 0 or pos[v] < 0:
            return 0.0
        return Kcols[int(v)][pos[u]]

    R = np.empty((len(a), len(b)), dtype=np.float64)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            R[i, j] = K(u, u) + K(v, v) - 2.0 * K(u, v)
    return R
