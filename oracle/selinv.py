"""Full-map oracle: every diagonal entry of G^{-1} by sparse Cholesky
factorisation and selected inversion.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import
or call this module; only the tests, the package's smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

What it computes (paper references are to arxiv 2607.05818): the same
R_i = (G^{-1})_ii as reff_oracle.diag, for every node at once, where G is
the pad-grounded conductance matrix of the stack (Sec. II-A, Eq. 1: G sparse
symmetric positive definite; Sec. II-B, Eq. 2 with all ideal supply bumps
merged into the grounded node, Sec. III-B), and R_i = 0 on pads.  The paper
names Cholesky factorisation with forward/backward substitution as the
direct way to solve G V = I (Sec. II-A).  n substitutions would give the map
at n times the cost of one; the selected-inversion recurrences instead give
every entry of Z = G^{-1} that lies inside the factor's pattern (the whole
diagonal among them) at about the cost of the factorisation.

Steps, each a published method restated here:

1. Ordering: geometric nested dissection (George, 1973) on the (x, y)
   plane.  A rectangle of the plane is split at its middle column (or row)
   along its longer side; the nodes of that line, on every tier, form the
   separator.  TSV segments are vertical, so a line through all tiers
   separates the two halves of the stack.  Rectangles holding at most
   ``leaf`` free nodes are not split.  Subdomains come before their
   separator (post-order), and each separator or leaf is one supernode
   (a contiguous range of columns held as one dense block).
2. Symbolic factorisation: the row structure S_J below supernode J is the
   union of the rows of G's columns in J and of its children's structures,
   restricted to rows after J; J's parent is the supernode owning the first
   row of S_J (the elimination / assembly tree, Liu 1990).
3. Numeric factorisation, multifrontal (Duff & Reid, 1983): the frontal
   matrix of J holds G's entries of J's columns plus its children's update
   matrices (extend-add); then L_JJ = chol(F_JJ), L_SJ = F_SJ L_JJ^{-T}
   and the update F_SS - L_SJ L_SJ^T goes to the parent.
4. Selected inversion: the block form of the Takahashi / Erisman-Tinney
   recurrences (Takahashi, Fagan & Chen, 1973; Erisman & Tinney, 1975; in
   supernodal form as in SelInv, Lin et al., 2011).  From G = L L^T,
   Z = L^{-T} L^{-1}, so L^T Z is lower triangular; its block rows give,
   supernode by supernode from the last to the first, with
   Lhat = L_SJ L_JJ^{-1}:
       Z_SJ = -Z_SS Lhat
       Z_JJ = L_JJ^{-T} L_JJ^{-1} - Lhat^T Z_SJ
   Z_SS is needed only on S_J x S_J, and every such entry lies in the block
   column of an ancestor supernode (S_J is a clique of the filled graph),
   computed before J.

Dense blocks use SciPy's LAPACK / BLAS wrappers as library primitives (all
of them from one library, so that one BLAS thread pool serves every call);
the tree is walked in plain Python.  Parity is pinned by
tests/test_selinv_pins.py: against the dense inverse and SuperLU paths of
reff_oracle.diag, against the scalar recurrence, and against Foster's
theorem on the full maps of the plain and mixed-precision stacks (which
uses the off-diagonal entries of Z on G's pattern as well).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .reff_oracle import grounded

LEAF = 64


def _mm(a, b, ta=False, tb=False, alpha=1.0):
    """alpha op(a) op(b) by SciPy's dgemm."""
    return sla.blas.dgemm(alpha, a, b, trans_a=ta, trans_b=tb)


def nd_order(x, y, nx, ny, leaf=LEAF):
    """Nested-dissection elimination order of nodes with plane coordinates
    (x, y).  Returns (perm, sn_ptr): perm lists node indices in elimination
    order and supernode J owns positions sn_ptr[J] .. sn_ptr[J+1]-1."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    blocks = []

    def split(nodes, x0, x1, y0, y1):
        if len(nodes) == 0:
            return
        if len(nodes) <= leaf or (x1 - x0 <= 1 and y1 - y0 <= 1):
            blocks.append(nodes)
            return
        if x1 - x0 >= y1 - y0:
            mid = (x0 + x1) // 2
            c = x[nodes]
            split(nodes[c < mid], x0, mid, y0, y1)
            split(nodes[c > mid], mid + 1, x1, y0, y1)
        else:
            mid = (y0 + y1) // 2
            c = y[nodes]
            split(nodes[c < mid], x0, x1, y0, mid)
            split(nodes[c > mid], x0, x1, mid + 1, y1)
        sep = nodes[c == mid]
        if len(sep):
            blocks.append(sep)

    split(np.arange(len(x), dtype=np.int64), 0, nx, 0, ny)
    perm = np.concatenate(blocks) if blocks else np.zeros(0, dtype=np.int64)
    sn_ptr = np.concatenate([[0], np.cumsum([len(b) for b in blocks])]).astype(np.int64)
    return perm, sn_ptr


class Factor:
    """Supernodal Cholesky factor G[perm][:, perm] = L L^T (steps 1-3)."""

    def __init__(self, G, x, y, nx, ny, leaf=LEAF):
        G = sp.csc_matrix(G)
        self.n = G.shape[0]
        self.perm, self.sn_ptr = nd_order(x, y, nx, ny, leaf)
        self.iperm = np.empty(self.n, dtype=np.int64)
        self.iperm[self.perm] = np.arange(self.n)
        A = G[self.perm][:, self.perm].tocsc()
        A.sort_indices()
        self.A = A
        self._symbolic()
        self._numeric()

    def cols(self, J):
        return self.sn_ptr[J], self.sn_ptr[J + 1]

    def rows(self, J):
        """Row indices of supernode J's block column: its own columns, then
        S_J (ascending)."""
        c0, c1 = self.cols(J)
        return np.concatenate([np.arange(c0, c1, dtype=np.int64), self.struct[J]])

    def _symbolic(self):
        A, ptr = self.A, self.sn_ptr
        ns = len(ptr) - 1
        self.ns = ns
        self.sn_of = np.repeat(np.arange(ns, dtype=np.int64), np.diff(ptr))
        self.struct = [None] * ns
        self.parent = np.full(ns, -1, dtype=np.int64)
        self.children = [[] for _ in range(ns)]
        for J in range(ns):
            c0, c1 = ptr[J], ptr[J + 1]
            r = A.indices[A.indptr[c0]:A.indptr[c1]]
            parts = [r[r >= c1]]
            for C in self.children[J]:
                s = self.struct[C]
                parts.append(s[s >= c1])
            S = np.unique(np.concatenate(parts)).astype(np.int64)
            self.struct[J] = S
            if len(S):
                P = int(self.sn_of[S[0]])
                self.parent[J] = P
                self.children[P].append(J)

    def _numeric(self):
        A, ptr = self.A, self.sn_ptr
        pos = np.empty(self.n, dtype=np.int64)
        upd = [None] * self.ns
        self.L = [None] * self.ns
        for J in range(self.ns):
            c0, c1 = ptr[J], ptr[J + 1]
            nJ = c1 - c0
            idx = self.rows(J)
            k = len(idx)
            pos[idx] = np.arange(k)
            F = np.zeros((k, k))
            lo, hi = A.indptr[c0], A.indptr[c1]
            r = A.indices[lo:hi]
            v = A.data[lo:hi]
            c = np.repeat(np.arange(nJ), np.diff(A.indptr[c0:c1 + 1]))
            keep = r >= c0
            F[pos[r[keep]], c[keep]] = v[keep]
            for C in self.children[J]:
                pc = pos[self.struct[C]]
                F[np.ix_(pc, pc)] += upd[C]
                upd[C] = None
            LJJ = sla.cholesky(F[:nJ, :nJ], lower=True, check_finite=False)
            LSJ = sla.solve_triangular(LJJ, F[nJ:, :nJ].T, lower=True, check_finite=False).T
            if k > nJ:
                upd[J] = F[nJ:, nJ:] - _mm(LSJ, LSJ, tb=True)
            self.L[J] = np.vstack([LJJ, LSJ])

    def solve(self, B):
        """G X = B by forward and backward substitution with the factor
        (B in the original, unpermuted node order)."""
        B = np.asarray(B, dtype=np.float64)
        one = B.ndim == 1
        Y = (B[:, None] if one else B)[self.perm].copy()
        for J in range(self.ns):
            c0, c1 = self.cols(J)
            nJ = c1 - c0
            L = self.L[J]
            Y[c0:c1] = sla.solve_triangular(L[:nJ], Y[c0:c1], lower=True, check_finite=False)
            S = self.struct[J]
            if len(S):
                Y[S] -= _mm(L[nJ:], Y[c0:c1])
        for J in range(self.ns - 1, -1, -1):
            c0, c1 = self.cols(J)
            nJ = c1 - c0
            L = self.L[J]
            S = self.struct[J]
            if len(S):
                Y[c0:c1] -= _mm(L[nJ:], Y[S], ta=True)
            Y[c0:c1] = sla.solve_triangular(L[:nJ], Y[c0:c1], lower=True, trans="T",
                                            check_finite=False)
        X = Y[self.iperm]
        return X[:, 0] if one else X

    def selected_inverse(self, pattern=False):
        """Step 4.  Returns diag(Z) in the original order and, with
        pattern=True, Z on the lower-triangular pattern of G as
        (row, col, value) arrays in the original order."""
        ptr = self.sn_ptr
        # Z's block column of K is needed until its last descendant is done.
        first_desc = np.arange(self.ns, dtype=np.int64)
        for J in range(self.ns):
            for C in self.children[J]:
                first_desc[J] = min(first_desc[J], first_desc[C])
        release = [[] for _ in range(self.ns)]
        for K in range(self.ns):
            release[first_desc[K]].append(K)
        Z = [None] * self.ns
        dz = np.empty(self.n)
        pr_all, pc_all, pv_all = [], [], []
        A = self.A
        for J in range(self.ns - 1, -1, -1):
            c0, c1 = ptr[J], ptr[J + 1]
            nJ = c1 - c0
            LJJ = self.L[J][:nJ]
            LSJ = self.L[J][nJ:]
            S = self.struct[J]
            Linv = sla.solve_triangular(LJJ, np.eye(nJ), lower=True, check_finite=False)
            ZJJ = _mm(Linv, Linv, ta=True)
            if len(S):
                Lhat = _mm(LSJ, Linv)
                ZSJ = _mm(self._gather(Z, S), Lhat, alpha=-1.0)
                ZJJ -= _mm(Lhat, ZSJ, ta=True)
                ZJ = np.vstack([ZJJ, ZSJ])
            else:
                ZJ = ZJJ
            Z[J] = ZJ
            dz[c0:c1] = np.diag(ZJJ)
            if pattern:
                lo, hi = A.indptr[c0], A.indptr[c1]
                r = A.indices[lo:hi]
                c = c0 + np.repeat(np.arange(nJ), np.diff(A.indptr[c0:c1 + 1]))
                keep = r > c
                r, c = r[keep], c[keep]
                idx = self.rows(J)
                pr_all.append(r)
                pc_all.append(c)
                pv_all.append(ZJ[np.searchsorted(idx, r), c - c0])
            for K in release[J]:
                Z[K] = None
        diag = dz[self.iperm]
        if not pattern:
            return diag
        r = np.concatenate(pr_all) if pr_all else np.zeros(0, dtype=np.int64)
        c = np.concatenate(pc_all) if pc_all else np.zeros(0, dtype=np.int64)
        v = np.concatenate(pv_all) if pv_all else np.zeros(0)
        return diag, (self.perm[r], self.perm[c], v)

    def _gather(self, Z, S):
        """Z[S, S] from the block columns of the supernodes owning S."""
        k = len(S)
        out = np.empty((k, k))
        sn = self.sn_of[S]
        starts = np.flatnonzero(np.r_[True, sn[1:] != sn[:-1]])
        ends = np.r_[starts[1:], k]
        for a, b in zip(starts, ends):
            K = int(sn[a])
            idx = self.rows(K)
            pr = np.searchsorted(idx, S[a:])
            if pr[-1] >= len(idx) or not np.array_equal(idx[pr], S[a:]):
                raise RuntimeError("selected inversion: a needed entry lies outside the factor")
            blk = Z[K][np.ix_(pr, S[a:b] - self.sn_ptr[K])]
            out[a:, a:b] = blk
            out[a:b, a:] = blk.T
        return out


def _free_xy(desc, free):
    nx, ny = int(desc["nx"]), int(desc["ny"])
    rem = free % (nx * ny)
    return rem % nx, rem // nx


def factor(desc, leaf=LEAF):
    """(Factor of the grounded G, free node ids) for a descriptor."""
    G, free = grounded(desc, fast=True)
    x, y = _free_xy(desc, free)
    return Factor(G, x, y, int(desc["nx"]), int(desc["ny"]), leaf), free


def diag_full(desc, leaf=LEAF):
    """R_i = (G^{-1})_ii for every node id of the stack, 0 on pads."""
    F, free = factor(desc, leaf)
    n = int(desc["n_tiers"]) * int(desc["nx"]) * int(desc["ny"])
    out = np.zeros(n)
    out[free] = F.selected_inverse()
    return out


def diag_and_edges(desc, leaf=LEAF):
    """diag_full plus Z = G^{-1} on every in-stack edge: returns
    (R per node id, (u, v, Z_uv) over the free-free edges, in node ids)."""
    F, free = factor(desc, leaf)
    n = int(desc["n_tiers"]) * int(desc["nx"]) * int(desc["ny"])
    d, (r, c, v) = F.selected_inverse(pattern=True)
    out = np.zeros(n)
    out[free] = d
    return out, (free[r], free[c], v)


def solve_nodes(desc, nodes, leaf=LEAF):
    """R_i for the requested node ids by one factorisation and one unit
    solve per free requested node (forward/backward substitution, Sec.
    II-A); pads give 0."""
    F, free = factor(desc, leaf)
    n = int(desc["n_tiers"]) * int(desc["nx"]) * int(desc["ny"])
    nodes = np.asarray(nodes, dtype=np.int64)
    pos = np.full(n, -1, dtype=np.int64)
    pos[free] = np.arange(len(free))
    out = np.zeros(len(nodes))
    want = np.flatnonzero(pos[nodes] >= 0)
    if len(want):
        rows = pos[nodes[want]]
        E = np.zeros((len(free), len(rows)))
        E[rows, np.arange(len(rows))] = 1.0
        X = F.solve(E)
        out[want] = X[rows, np.arange(len(rows))]
    return out
