"""Seeded synthetic 3D power-delivery-network instances.

This module only draws random inputs.  It holds none of the method's
arithmetic (no conductance assembly, no solve), so the CPU oracle and the
HIP path can both consume what it produces without sharing any code.

A descriptor is a plain dict of numpy arrays, matching the C ABI layout:

    n_tiers, nx, ny    ints; node id = t*nx*ny + y*nx + x, tier 0 holds pads
    gx   float64 [n_tiers][ny][nx-1]  edge (t,x,y)-(t,x+1,y) conductance, S
    gy   float64 [n_tiers][ny-1][nx]  edge (t,x,y)-(t,x,y+1) conductance, S
    tsv_xy int32 [n_tsv][2]           (x, y) of a vertical TSV column
    tsv_g  float64 [n_tsv][n_tiers-1] segment conductance between tiers t, t+1
    pad_xy int32 [n_pads][2]          (x, y) of an ideal supply bump on tier 0

The stack follows the early-stage model of Sec. III-B of the paper: each
tier is a 2D resistive mesh, tiers are joined only through TSV segments,
and the bumps are ideal voltage sources (grounded, i.e. Dirichlet nodes).

Draw order within one instance is fixed: gx, gy, TSVs, pads, sampled nodes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "cell_centred", "make_desc", "config1", "config2", "config3_plans",
    "config4_plan", "config5", "sample_free_nodes", "pad_ids", "n_nodes",
    "CONFIG_SEEDS", "small_random_desc", "config3_samples", "tsv_planning_study",
    "uniform_tier_stack",
]

CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}


def n_nodes(desc) -> int:
    return int(desc["n_tiers"]) * int(desc["nx"]) * int(desc["ny"])


def pad_ids(desc) -> np.ndarray:
    """Global ids of the pad nodes (all on tier 0)."""
    p = np.asarray(desc["pad_xy"], dtype=np.int64).reshape(-1, 2)
    return np.unique(p[:, 1] * int(desc["nx"]) + p[:, 0])


def cell_centred(n: int, k: int) -> np.ndarray:
    """k positions centred in k equal cells of an axis of n nodes."""
    a = np.arange(k, dtype=np.int64)
    return (2 * a + 1) * n // (2 * k)


def _grid_xy(nx: int, ny: int, kx: int, ky: int) -> np.ndarray:
    xs = cell_centred(nx, kx)
    ys = cell_centred(ny, ky)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.int32)


def make_desc(n_tiers, nx, ny, gx, gy, tsv_xy, tsv_g, pad_xy) -> dict:
    d = {
        "n_tiers": int(n_tiers), "nx": int(nx), "ny": int(ny),
        "gx": np.ascontiguousarray(gx, dtype=np.float64).reshape(n_tiers, ny, nx - 1),
        "gy": np.ascontiguousarray(gy, dtype=np.float64).reshape(n_tiers, ny - 1, nx),
        "tsv_xy": np.ascontiguousarray(tsv_xy, dtype=np.int32).reshape(-1, 2),
        "tsv_g": np.ascontiguousarray(tsv_g, dtype=np.float64).reshape(
            np.asarray(tsv_xy).reshape(-1, 2).shape[0], max(n_tiers - 1, 0)),
        "pad_xy": np.ascontiguousarray(pad_xy, dtype=np.int32).reshape(-1, 2),
    }
    return d


def _clustered_xy(rng, nx, ny, count, n_clusters, sigma) -> np.ndarray:
    """Distinct (x,y) drawn around n_clusters Gaussian centres, clipped to
    the grid; duplicates are rejected and redrawn."""
    centres = rng.uniform(0.0, 1.0, size=(n_clusters, 2)) * np.array([nx, ny])
    seen = set()
    out = []
    while len(out) < count:
        c = centres[rng.integers(0, n_clusters)]
        x = int(np.clip(np.rint(c[0] + sigma * rng.standard_normal()), 0, nx - 1))
        y = int(np.clip(np.rint(c[1] + sigma * rng.standard_normal()), 0, ny - 1))
        if (x, y) in seen:
            continue
        seen.add((x, y))
        out.append((x, y))
    return np.asarray(out, dtype=np.int32)


def _uniform_distinct_xy(rng, nx, ny, count) -> np.ndarray:
    flat = rng.choice(nx * ny, size=count, replace=False)
    return np.stack([flat % nx, flat // nx], axis=1).astype(np.int32)


def config1(seed: int = CONFIG_SEEDS[1]) -> dict:
    """Plain FP64 workload: 2 tiers of 32x32, i.i.d. U[0.5,2] S edges,
    16 TSV columns (10 S) and 16 pads on a cell-centred 4x4 array."""
    rng = np.random.default_rng(seed)
    nt, nx, ny = 2, 32, 32
    gx = rng.uniform(0.5, 2.0, size=(nt, ny, nx - 1))
    gy = rng.uniform(0.5, 2.0, size=(nt, ny - 1, nx))
    tsv_xy = _grid_xy(nx, ny, 4, 4)
    tsv_g = np.full((len(tsv_xy), nt - 1), 10.0)
    pad_xy = _grid_xy(nx, ny, 4, 4)
    return make_desc(nt, nx, ny, gx, gy, tsv_xy, tsv_g, pad_xy)


def config2(seed: int = CONFIG_SEEDS[2], side: int = 512, n_tiers: int = 4,
            n_tsv: int = 1024, sigma: float = 40.0, pad_pitch: int = 32) -> dict:
    """Mixed-precision workload: 4 tiers of 512x512, lognormal(0,0.3) S
    edges, 1024 TSV columns (5 S) in 8 Gaussian clusters (sigma 40 nodes),
    256 pads cell-centred at pitch 32 on tier 0.  The keyword arguments
    shrink the same recipe for tests."""
    rng = np.random.default_rng(seed)
    nt, nx, ny = n_tiers, side, side
    gx = rng.lognormal(0.0, 0.3, size=(nt, ny, nx - 1))
    gy = rng.lognormal(0.0, 0.3, size=(nt, ny - 1, nx))
    tsv_xy = _clustered_xy(rng, nx, ny, n_tsv, 8, sigma)
    tsv_g = np.full((len(tsv_xy), nt - 1), 5.0)
    k = max(1, side // pad_pitch)
    pad_xy = _grid_xy(nx, ny, k, k)
    return make_desc(nt, nx, ny, gx, gy, tsv_xy, tsv_g, pad_xy)


def config3_plans(seed: int = CONFIG_SEEDS[3], n_plans: int = 256,
                  side_lo: int = 64, side_hi: int = 256):
    """Batching workload: n_plans candidate TSV plans with 2-4 tiers,
    square sides U{side_lo..side_hi}, U[0.5,2] S edges, 16-512 TSV columns
    (10 S) at distinct uniform positions, pads cell-centred at pitch 32
    (at least 2x2) on tier 0.  Each plan has its own child seed."""
    children = np.random.SeedSequence(seed).spawn(n_plans)
    plans = []
    for ss in children:
        rng = np.random.default_rng(ss)
        nt = int(rng.integers(2, 5))
        side = int(rng.integers(side_lo, side_hi + 1))
        gx = rng.uniform(0.5, 2.0, size=(nt, side, side - 1))
        gy = rng.uniform(0.5, 2.0, size=(nt, side - 1, side))
        n_tsv = int(rng.integers(16, 513))
        n_tsv = min(n_tsv, side * side)
        tsv_xy = _uniform_distinct_xy(rng, side, side, n_tsv)
        tsv_g = np.full((n_tsv, nt - 1), 10.0)
        k = max(2, side // 32)
        pad_xy = _grid_xy(side, side, k, k)
        plans.append(make_desc(nt, side, side, gx, gy, tsv_xy, tsv_g, pad_xy))
    return plans


def config4_plan(rng) -> dict:
    """One surrogate-training plan: 3 tiers of 128x128, U[0.5,2] S edges,
    TSV-column mask density U[0.5%,3%] (10 S), pad mask density
    U[0.2%,1%] on tier 0."""
    nt, side = 3, 128
    gx = rng.uniform(0.5, 2.0, size=(nt, side, side - 1))
    gy = rng.uniform(0.5, 2.0, size=(nt, side - 1, side))
    n_tsv = int(round(rng.uniform(0.005, 0.03) * side * side))
    tsv_xy = _uniform_distinct_xy(rng, side, side, n_tsv)
    tsv_g = np.full((n_tsv, nt - 1), 10.0)
    n_pad = max(1, int(round(rng.uniform(0.002, 0.01) * side * side)))
    pad_xy = _uniform_distinct_xy(rng, side, side, n_pad)
    return make_desc(nt, side, side, gx, gy, tsv_xy, tsv_g, pad_xy)


def config5(seed: int = CONFIG_SEEDS[5], side: int = 2048, n_tiers: int = 8) -> dict:
    """Large workload: 8 tiers of 2048x2048, anisotropic x U[0.5,2] /
    y U[1,4] S edges, 16384 TSV columns (5 S) in 8 clusters (sigma 160),
    4096 pads cell-centred at pitch 32 on tier 0."""
    rng = np.random.default_rng(seed)
    nt, nx, ny = n_tiers, side, side
    gx = rng.uniform(0.5, 2.0, size=(nt, ny, nx - 1))
    gy = rng.uniform(1.0, 4.0, size=(nt, ny - 1, nx))
    n_tsv = 16384 * side * side // (2048 * 2048)
    tsv_xy = _clustered_xy(rng, nx, ny, n_tsv, 8, 160.0 * side / 2048)
    tsv_g = np.full((len(tsv_xy), nt - 1), 5.0)
    k = max(1, side // 32)
    pad_xy = _grid_xy(nx, ny, k, k)
    return make_desc(nt, nx, ny, gx, gy, tsv_xy, tsv_g, pad_xy)


def config3_samples(plans, per_plan: int = 64, seed: int = CONFIG_SEEDS[3]) -> list:
    """One seeded block of per_plan free nodes for each batching plan
    (plan i draws with the seed sequence [seed, i])."""
    return [sample_free_nodes(d, per_plan, np.random.SeedSequence([seed, i]))
            for i, d in enumerate(plans)]


def sample_free_nodes(desc, count: int, seed) -> np.ndarray:
    """count distinct non-pad node ids drawn uniformly (seeded), in draw
    order, so that every prefix is itself a uniform sample."""
    rng = np.random.default_rng(seed)
    n = n_nodes(desc)
    pads = pad_ids(desc)
    free = np.setdiff1d(np.arange(n, dtype=np.int64), pads, assume_unique=True)
    count = min(count, len(free))
    return rng.choice(free, size=count, replace=False).astype(np.int64)


def small_random_desc(seed: int, n_tiers: int, nx: int, ny: int,
                      n_tsv: int, n_pads: int, glo: float = 0.5,
                      ghi: float = 2.0) -> dict:
    """A tiny random stack for brute-force checks: U[glo,ghi] S edges,
    n_tsv distinct uniform TSV columns with U[1,10] S segments, n_pads
    distinct uniform pads on tier 0."""
    rng = np.random.default_rng(seed)
    gx = rng.uniform(glo, ghi, size=(n_tiers, ny, max(nx - 1, 0)))
    gy = rng.uniform(glo, ghi, size=(n_tiers, max(ny - 1, 0), nx))
    tsv_xy = _uniform_distinct_xy(rng, nx, ny, min(n_tsv, nx * ny))
    tsv_g = rng.uniform(1.0, 10.0, size=(len(tsv_xy), max(n_tiers - 1, 0)))
    pad_xy = _uniform_distinct_xy(rng, nx, ny, min(n_pads, nx * ny))
    return make_desc(n_tiers, nx, ny, gx, gy, tsv_xy, tsv_g, pad_xy)


def tsv_planning_study(seed: int = 1006, side: int = 128, n_tiers: int = 3, n_tsv: int = 256,
                       bump_k: int = 16, block_w: int = 30, block_h: int = 15,
                       amps_per_block: float = 6.1) -> dict:
    """A synthetic analog of the TSV-planning comparison of Sec. IV-B: one
    stack with two TSV plans of the same TSV count, band-like (every TSV
    in a central vertical band, as in HBM-style stacks) and uniformly
    distributed (a cell-centred array), bumps cell-centred bump_k x bump_k on
    tier 0, and four functional blocks of block_w x block_h nodes on the last
    tier, one per quadrant, each drawing amps_per_block spread evenly over
    its nodes (the paper's blocks draw 220 A/cm^2 over 2.35 x 1.18 mm^2,
    about 6.1 A).  Edges lognormal(0, 0.3) S, TSV segments 5 S.  Returns
    {"band": desc, "uniform": desc, "loads": node ids, "amps": (1, n)}."""
    rng = np.random.default_rng(seed)
    nt, nx, ny = n_tiers, side, side
    gx = rng.lognormal(0.0, 0.3, size=(nt, ny, nx - 1))
    gy = rng.lognormal(0.0, 0.3, size=(nt, ny - 1, nx))
    pad_xy = _grid_xy(nx, ny, bump_k, bump_k)
    # uniform plan: a cell-centred array of about n_tsv columns
    ku = max(1, int(round(np.sqrt(n_tsv))))
    uni = _grid_xy(nx, ny, ku, max(1, n_tsv // ku))
    # band plan: the same count packed in a band of columns at the centre
    bw = max(1, int(np.ceil(len(uni) / ny)))
    bx = np.arange(nx // 2 - bw // 2, nx // 2 - bw // 2 + bw)
    band_all = np.stack(np.meshgrid(bx, np.arange(ny), indexing="xy"), axis=-1).reshape(-1, 2)
    pick = np.sort(rng.choice(len(band_all), size=len(uni), replace=False))
    band = band_all[pick].astype(np.int32)
    tg = np.full((len(uni), nt - 1), 5.0)
    loads, amps = [], []
    plane = nx * ny
    for qx, qy in ((0, 0), (1, 0), (0, 1), (1, 1)):
        x0 = (2 * qx + 1) * nx // 4 - block_w // 2
        y0 = (2 * qy + 1) * ny // 4 - block_h // 2
        xs, ys = np.meshgrid(np.arange(x0, x0 + block_w), np.arange(y0, y0 + block_h),
                             indexing="xy")
        ids = (nt - 1) * plane + ys.ravel() * nx + xs.ravel()
        loads.append(ids)
        amps.append(np.full(len(ids), amps_per_block / len(ids)))
    return {
        "band": make_desc(nt, nx, ny, gx, gy, band, tg, pad_xy),
        "uniform": make_desc(nt, nx, ny, gx, gy, uni, tg, pad_xy),
        "loads": np.concatenate(loads).astype(np.int64),
        "amps": np.concatenate(amps)[None, :],
    }


def uniform_tier_stack(seed: int, n_tiers: int, side: int, n_tsv: int, m: int, n: int) -> dict:
    """Inputs of the paper's pair method (Sec. III-C/D): n_tiers uniform
    tiers of side x side nodes (per-tier edge resistances U[0.5, 2] Ohm along
    x and y), n_tsv distinct uniform TSV columns with U[0.05, 1] Ohm segments,
    m bumps on tier 0 and n loads on the last tier at distinct uniform
    positions."""
    rng = np.random.default_rng(seed)
    r_t = rng.uniform(0.5, 2.0, n_tiers)
    s_t = rng.uniform(0.5, 2.0, n_tiers)
    tsv = _uniform_distinct_xy(rng, side, side, n_tsv)
    tsv_r = rng.uniform(0.05, 1.0, (n_tsv, n_tiers - 1))
    bumps = _uniform_distinct_xy(rng, side, side, m)
    loads = _uniform_distinct_xy(rng, side, side, n)
    return {"side": side, "r_t": r_t, "s_t": s_t, "tsv_xy": tsv, "tsv_r": tsv_r,
            "bump_xy": bumps, "load_xy": loads}
