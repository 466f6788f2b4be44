"""Closed forms and independent reformulations used to pin the CPU oracle.

Each helper is written from its mathematical source, not from the oracle:

* wu_two_point: the closed-form two-point resistance of a uniform M x N
  resistor grid, the paper's Eq. 3 (Sec. II-B), with x in [0, M) along the
  r-routed (x) direction, y in [0, N) along the s-routed direction.
* reduced_system_resistance: the paper's divide-and-conquer pair resistance
  for uniformly meshed tiers joined by TSVs (Sec. III-C and III-D): intra-die
  resistances from Eq. 3, the transformed saddle-point system C x = b of
  size (p+1)(d-1), and R = -x^T b.  Three printed details are read as
  follows (each reading is checked by the tests against a dense
  pseudo-inverse):
    - A^i = Atilde^i + (M^i + M^i^T)/2, the split of a^i_{s,j,k} =
      (R_{s,j} + R_{s,k} - R_{j,k})/2;
    - the constraint block of b is 1_{d-1} (one unit per tier interface);
    - b's TSV blocks are -R^1_{s,.}/2 in the first and -R^d_{s,.}/2 in the
      last interface block and zero in between (their sum when d = 2).
* ladder_resistance: symmetric-ladder closed form from the symmetric /
  antisymmetric mode split (derivation in the docstring).
"""
from __future__ import annotations

import numpy as np


def wu_two_point(M, N, r, s, x1, y1, x2, y2):
    """Eq. 3 of the paper: two-point resistance on a uniform M x N grid."""
    R = r / N * abs(x1 - x2) + s / M * abs(y1 - y2)
    m = np.arange(1, M)[:, None]
    n = np.arange(1, N)[None, :]
    th = m * np.pi / M
    ph = n * np.pi / N
    num = (np.cos((x1 + 0.5) * th) * np.cos((y1 + 0.5) * ph)
           - np.cos((x2 + 0.5) * th) * np.cos((y2 + 0.5) * ph)) ** 2
    den = (1.0 - np.cos(th)) / r + (1.0 - np.cos(ph)) / s
    if M > 1 and N > 1:
        R += 2.0 / (M * N) * float(np.sum(num / den))
    return R


def reduced_system_resistance(nx, ny, r_t, s_t, tsv_xy, rt_seg, bump_xy, load_xy):
    """Pair resistance between a bump on tier 0 (die_1) and a load on the
    last tier (die_d) of d = len(r_t) uniform tiers, by the paper's reduced
    system.  rt_seg[k][i] is the resistance of TSV k between tiers i, i+1."""
    d = len(r_t)
    p = len(tsv_xy)
    assert d >= 2 and p >= 1

    def Rintra(i, a, b):
        return wu_two_point(nx, ny, r_t[i], s_t[i], a[0], a[1], b[0], b[1])

    RT = np.zeros((d, p, p))
    for i in range(d):
        for j in range(p):
            for k in range(j + 1, p):
                RT[i, j, k] = RT[i, k, j] = Rintra(i, tsv_xy[j], tsv_xy[k])
    Rs1 = np.array([Rintra(0, bump_xy, tsv_xy[k]) for k in range(p)])
    Rsd = np.array([Rintra(d - 1, load_xy, tsv_xy[k]) for k in range(p)])
    At = [-0.5 * RT[i] for i in range(d)]          # Atilde^i
    nI = p * (d - 1)
    C = np.zeros((nI + d - 1, nI + d - 1))
    for i in range(d - 1):                          # interface i: tiers i,i+1
        sl = slice(i * p, (i + 1) * p)
        C[sl, sl] = At[i] + At[i + 1] + np.diag([rt_seg[k][i] for k in range(p)])
        if i + 1 < d - 1:
            sl2 = slice((i + 1) * p, (i + 2) * p)
            C[sl, sl2] = -At[i + 1]
            C[sl2, sl] = -At[i + 1]
        C[sl, nI + i] = 1.0
        C[nI + i, sl] = 1.0
    b = np.zeros(nI + d - 1)
    b[0:p] += -0.5 * Rs1
    b[(d - 2) * p:(d - 1) * p] += -0.5 * Rsd
    b[nI:] = 1.0
    x = np.linalg.solve(C, b)
    return float(-x @ b)


def ladder_resistance(L, g, h, k):
    """Two-rail ladder, nx = L nodes per rail, rails of conductance g, rungs
    of conductance h, both rail nodes at x = 0 grounded.  Resistance from
    rail node x = k to ground.

    Inject 1/2 at both rail nodes (symmetric mode: rungs idle, each rail a
    series chain, voltage k/(2g)) plus +-1/2 (antisymmetric mode: rung
    midpoints at 0 V, so each rail is a chain leaking 2h to ground at every
    node; with cosh(theta) = 1 + h/g its Green's function is
    sinh(k theta) cosh((L - 1/2 - k) theta) / (g sinh(theta) cosh((L - 1/2) theta))).
    """
    th = np.arccosh(1.0 + h / g)
    anti = (np.sinh(k * th) * np.cosh((L - 0.5 - k) * th)
            / (g * np.sinh(th) * np.cosh((L - 0.5) * th)))
    return 0.5 * (k / g + anti)


def merged_pad_laplacian_dense(desc):
    """Dense Laplacian of the stack with every pad contracted into one
    supply node (last index).  Built edge by edge from the descriptor
    arrays, independently of the oracle's assembly."""
    nt, nx, ny = int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])
    n = nt * nx * ny
    pads = set(int(p[1]) * nx + int(p[0]) for p in np.asarray(desc["pad_xy"]).reshape(-1, 2))
    free = [i for i in range(n) if i not in pads]
    idx = {v: k for k, v in enumerate(free)}
    g_node = len(free)
    for p in pads:
        idx[p] = g_node
    L = np.zeros((len(free) + 1, len(free) + 1))

    def add(u, v, w):
        a, b = idx[u], idx[v]
        if a == b:
            return
        L[a, a] += w
        L[b, b] += w
        L[a, b] -= w
        L[b, a] -= w

    gx = np.asarray(desc["gx"]).reshape(nt, ny, nx - 1)
    gy = np.asarray(desc["gy"]).reshape(nt, ny - 1, nx)
    for t in range(nt):
        base = t * nx * ny
        for y in range(ny):
            for x in range(nx - 1):
                add(base + y * nx + x, base + y * nx + x + 1, gx[t, y, x])
        for y in range(ny - 1):
            for x in range(nx):
                add(base + y * nx + x, base + (y + 1) * nx + x, gy[t, y, x])
    txy = np.asarray(desc["tsv_xy"]).reshape(-1, 2)
    tg = np.asarray(desc["tsv_g"]).reshape(len(txy), max(nt - 1, 0))
    for j, (x, y) in enumerate(txy):
        for t in range(nt - 1):
            add(t * nx * ny + y * nx + x, (t + 1) * nx * ny + y * nx + x, tg[j, t])
    return L, idx, g_node
