#!/usr/bin/env python3
"""Throughput benchmark of the effective-resistance hot path on one MI355X.

Workload: the mixed-precision stack (4 tiers of 512 x 512 = 1,048,576 nodes,
lognormal(0, 0.3) S edges, 1024 TSV columns in 8 Gaussian clusters, 256
pads), synthetic and seeded.  One step solves R_i = (G^-1)_ii for a batch of
sampled nodes (default 128 = two 64-column blocks) with the float32 block
PCG inside float64 refinement, writing the results to a device buffer.
`value` counts only nodes whose result is within 1e-3 relative error of the
stored float64 oracle values for that batch.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # dense matrix-core peaks
S = 64


def cheb_passes(cheb, fp32=True):
    """The Chebyshev passes of one preconditioner application, in order:
    (steps, has z_{j-1}) per pass.  Steps run three per pass while three
    remain (float32; two in float64), then two, then one."""
    left, first, out = cheb - 1, True, []
    top = 3 if fp32 else 2
    while left > 0:
        k = min(top, left)
        out.append((k, not first))
        left -= k
        first = False
    return out


def cheb_folds_z1(cheb, fp32=True):
    """The first pass is a three-step pass that forms z_1 = D^-1 R / theta
    from R itself (nothing writes z_1)."""
    return fp32 and cheb > 3


def cheb_words(cheb, fp32=True):
    """S-wide vector words per node that the Chebyshev passes of one
    application read and write, and the number of passes: a pass reads z_j,
    R (and z_{j-1} after the first; a first pass that forms z_1 from R reads
    R alone) and writes its last two iterates (one for a single step; a last
    three-step pass writes only its last)."""
    passes = cheb_passes(cheb, fp32)
    words = 0
    for n, (k, prev) in enumerate(passes):
        last = n == len(passes) - 1
        reads = 3 if prev else (1 if cheb_folds_z1(cheb, fp32) else 2)
        words += reads + (1 if k == 1 or (k == 3 and last) else 2)
    return words, len(passes)


def kernel_bytes(n, fp32=True, mixed_with_d=True, cheb=1):
    """Algorithmic HBM bytes per launch of the block kernels for an n-node
    stack and S right-hand sides (w = bytes per word):
      stencil+Gram (K1): read Y, R; write P = Y T, Q = (G Y) T -> 4 S w per node
                         + coefficients d, cE, cN (w each) and the TSV slot (4)
      residual update (K2): read Q, R (P, D); write R (D)       -> 3 (6) S w
                         + Dinv; with the polynomial preconditioner it also
                         writes z_1 = D^-1 R / theta            -> + S w
                         unless the first pass forms z_1 itself
      search block (K3): read P, R (or Z); write Y              -> 3 S w + d, Dinv
      Chebyshev passes (degree k > 1), all passes of one application: the
                         vector words of cheb_words, each pass also reading
                         d, cE, cN, Dinv and the slot
      Q^T Z Gram (degree k > 1): read Q, Z                     -> 2 S w
    """
    w = 4 if fp32 else 8
    k1 = n * (4 * S * w + 3 * w + 4)
    z1 = cheb > 1 and not cheb_folds_z1(cheb, fp32)
    k2 = n * ((6 if mixed_with_d else 3) * S * w + w + (S * w if z1 else 0))
    k3 = n * (3 * S * w + 2 * w)
    kp = kg = 0
    if cheb > 1:
        words, passes = cheb_words(cheb, fp32)
        kp = n * (words * S * w + passes * (4 * w + 4))
        kg = n * 2 * S * w
    return [k1, k2, k3, kp, kg]


def kernel_flops(cheb=1):
    """Matrix-core flops per 64-column block row of the block kernels
    (2 S^2 per S x S product or Gram): K1 = P = Y T and Q = (G Y) T with T
    upper triangular (10 of the 16 16 x 16 blocks of T are nonzero) plus the
    Grams P^T Q and P^T R; K2 = Q A, P A and (Jacobi) Q^T Z; K3 = P B and
    Y^T D Y; the Chebyshev passes are stencil arithmetic (no matrix-core
    work); the preconditioner's Q^T Z Gram."""
    g = 2 * S * S
    if cheb > 1:
        return [2 * g * 10 // 16 + 2 * g, 2 * g, 2 * g, 0, g]
    return [2 * g * 10 // 16 + 2 * g, 3 * g, 2 * g, 0, 0]


def cpu_baseline(desc, batch_nodes, n_timed=2):
    """The CPU oracle as it stands, on a bounded sample: assembly + sparse
    LU factorisation of G, then n_timed single-column solves; the time for
    the whole batch is extrapolated as fixed + len(batch) * per-solve."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import reff_oracle as ro
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        G, free = ro.grounded(desc)
        t1 = time.perf_counter()
        solver = ro._Solver(G)
        t2 = time.perf_counter()
        pos = np.full(int(desc["n_tiers"]) * int(desc["nx"]) * int(desc["ny"]), -1)
        pos[free] = np.arange(len(free))
        ts = []
        for v in batch_nodes[:n_timed]:
            e = np.zeros(G.shape[0])
            e[pos[v]] = 1.0
            a = time.perf_counter()
            solver.solve(e[:, None])
            ts.append(time.perf_counter() - a)
    per_solve = sum(ts) / len(ts)
    fixed = (t1 - t0) + (t2 - t1)
    t_batch = fixed + len(batch_nodes) * per_solve
    return {
        "value": len(batch_nodes) / t_batch,
        "unit": "nodes/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"float64 sparse-LU oracle on the same stack: assembly {t1 - t0:.1f} s + "
                   f"factorisation {t2 - t1:.1f} s, {n_timed} timed unit-current solves "
                   f"({per_solve:.2f} s each); batch of {len(batch_nodes)} nodes "
                   f"extrapolated to {t_batch:.0f} s; BLAS limited to 1 thread"),
    }


def grid_pairs_compare(reff, log, M=512, N=512, P=256, reps=3):
    """Eq. 3 on one uniform tier (the intra-die step of the paper's pair
    method, Sec. III-C/D): every pair of P seeded points on an M x N grid,
    output to device memory, checked on sampled pairs against the closed form
    summed directly in float64.  The work is counted in the direct form:
    each pair is a double sum over (M-1)(N-1) terms of 6 float64 flops (two
    products and their difference, the square, the weight, the
    accumulation); the library evaluates it as a float64 matrix-core product
    (T = X diag(W) X^T)."""
    import numpy as np
    import torch
    from tests import pins
    rng = np.random.default_rng(3001)
    r, s = (float(v) for v in rng.uniform(0.5, 2.0, size=2))
    flat = rng.choice(M * N, size=P, replace=False)
    xy = np.stack([flat % M, flat // M], axis=1).astype(np.int32)
    out = torch.empty((P, P), dtype=torch.float64, device="cuda:0")
    reff.reff_grid_pairs(M, N, r, s, xy, out)  # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        reff.reff_grid_pairs(M, N, r, s, xy, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    R = out.cpu().numpy()
    pairs = P * (P - 1) // 2
    terms = pairs * (M - 1) * (N - 1)
    err = 0.0
    for i, j in [(0, 1), (7, 200), (100, 255), (31, 32)]:
        w = pins.wu_two_point(M, N, r, s, *xy[i], *xy[j])
        err = max(err, abs(R[i, j] - w) / w)
    tflops = 6.0 * terms / dt / 1e12
    log(f"grid pairs (Eq. 3): {pairs / dt:.3g} pairs/s, {tflops:.1f} TFLOP/s float64, err {err:.1e}")
    return {"workload": f"Eq. 3, all pairs of {P} seeded points on a uniform {M} x {N} grid",
            "pairs_per_s": pairs / dt, "seconds": dt, "terms_per_s": terms / dt,
            "fp64_tflops": tflops, "fp64_vector_peak_tflops": 78.6,
            "frac": tflops / 78.6, "bound": "mfma", "max_rel_err_sampled": err}


def batched_compare(reff, gen, log, rel_tol, n_seq=16):
    """The batching workload: 256 candidate TSV plans (2-4 tiers, sides
    64-256, about 22M nodes in total) with one seeded 64-node block per
    plan, solved in one reff_batch_plans call (mixed precision), against
    one reff_build_pdn + reff_solve_diag per plan on the first n_seq plans
    (extrapolated).  Accuracy is checked on the plans the stored oracle
    fixture covers."""
    import numpy as np
    import torch
    plans = gen.config3_plans()
    nodes = gen.config3_samples(plans)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "config3_sample.json")))
    total = sum(len(x) for x in nodes)
    prec = reff.REFF_PREC_MIXED
    # first call on a few plans: lazy runtime initialisation
    reff.reff_batch_plans(plans[:4], nodes[:4], precision=prec, rel_tol=rel_tol)
    torch.cuda.synchronize()
    a = time.perf_counter()
    outs, stats = reff.reff_batch_plans(plans, nodes, precision=prec, rel_tol=rel_tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    errs = []
    for i in range(len(gold["nodes"])):
        assert list(nodes[i]) == gold["nodes"][i], "batching sample drifted from the fixture"
        want = np.array(gold["R"][i])
        errs.append(float(np.max(np.abs(outs[i] - want) / want)))
    a = time.perf_counter()
    for i in range(n_seq):
        h = reff.reff_build_pdn(plans[i])
        reff.reff_solve_diag(h, nodes[i], precision=prec, rel_tol=rel_tol)
        h.close()
    torch.cuda.synchronize()
    dseq = time.perf_counter() - a
    seq_nodes = sum(len(nodes[i]) for i in range(n_seq))
    rec = {
        "workload": "256 TSV plans, 2-4 tiers x side 64-256 (%d nodes), 64 seeded nodes per plan"
                    % sum(gen.n_nodes(d) for d in plans),
        "nodes_per_s": total / dt, "seconds": dt, "nodes": total,
        "iters_max": max(x["iters_max"] for x in stats),
        "checked_plans": len(errs), "max_rel_err_checked": max(errs),
        "est_max_rel_err": max(x["est_max_rel_err"] for x in stats),
        "sequential_nodes_per_s": seq_nodes / dseq, "sequential_plans_timed": n_seq,
        "rel_tol": rel_tol,
    }
    log(f"batched: {total / dt:.1f} nodes/s ({dt:.2f} s), sequential {seq_nodes / dseq:.1f} "
        f"nodes/s, checked err {max(errs):.2e}")
    return rec


def measured_traffic():
    """The committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (HBM bytes per
    node row of the block kernels, and the preconditioner degree it was
    taken with), or None when the kernel sources have changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "block_pcg_mixed_4x512x512_hbm_traffic.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return rec


def surrogate_compare(reff, gen, log, rel_tol, n_train=512, n_test=16, per_test=640,
                      n_full=2, epochs=20):
    """The surrogate workload (3 tiers of 128 x 128, TSV and pad densities
    drawn per plan): labels for 64 seeded nodes of each of n_train plans
    from one batched mixed-precision solve, Adam training of the BF16 U-Net,
    then screening of n_test held-out plans (per_test requested nodes each,
    1 % checked by the solver, fallback above 1e-2) against solving every
    requested node.  The model's own contract is 1e-2: its errors are
    reported as a distribution over the held-out requested nodes and over
    the full maps of n_full held-out plans."""
    import numpy as np
    import torch
    rng = np.random.default_rng(gen.CONFIG_SEEDS[4])
    plans = [gen.config4_plan(rng) for _ in range(n_train + n_test)]
    train, test = plans[:n_train], plans[n_train:]
    prec = reff.REFF_PREC_MIXED
    lab_nodes = [gen.sample_free_nodes(d, 64, np.random.SeedSequence([4, i]))
                 for i, d in enumerate(train)]
    a = time.perf_counter()
    lab_R, _ = reff.reff_batch_plans(train, lab_nodes, precision=prec, rel_tol=1e-5)
    t_label = time.perf_counter() - a
    s = reff.reff_surrogate_create(3, 128, 128, 32, seed=gen.CONFIG_SEEDS[4])
    a = time.perf_counter()
    hist = reff.reff_surrogate_train(s, train, list(zip(lab_nodes, lab_R)), epochs=epochs,
                                     batch=16, lr=1e-3, seed=1)
    t_train = time.perf_counter() - a
    req = [gen.sample_free_nodes(d, per_test, np.random.SeedSequence([44, i]))
           for i, d in enumerate(test)]
    torch.cuda.synchronize()
    a = time.perf_counter()
    ref, _ = reff.reff_batch_plans(test, req, precision=prec, rel_tol=rel_tol)
    t_solver = time.perf_counter() - a
    a = time.perf_counter()
    scr, st = reff.reff_batch_plans(test, req, precision=prec, rel_tol=rel_tol, surrogate=s,
                                    spot_frac=0.01, fallback_rel_err=1e-2)
    t_screen = time.perf_counter() - a
    a = time.perf_counter()
    pred = reff.reff_surrogate_predict(s, test)
    t_pred = time.perf_counter() - a
    e_req = np.concatenate([np.abs(pred[i][req[i]] - ref[i]) / ref[i] for i in range(n_test)])
    e_scr = np.concatenate([np.abs(scr[i] - ref[i]) / ref[i] for i in range(n_test)])
    full = reff.reff_batch_plans(test[:n_full], None, precision=prec, rel_tol=rel_tol)[0]
    e_full = np.concatenate([np.abs(pred[i] - full[i])[full[i] > 0] / full[i][full[i] > 0]
                             for i in range(n_full)])
    total = n_test * per_test
    q = lambda e: {"median": float(np.median(e)), "p90": float(np.quantile(e, 0.9)),
                   "p99": float(np.quantile(e, 0.99)), "max": float(e.max()),
                   "frac_le_1e-2": float(np.mean(e <= 1e-2))}
    rec = {
        "workload": ("3 tiers x 128 x 128 plans (TSV density U[0.5%,3%], pad density "
                     f"U[0.2%,1%]); {n_train} training plans x 64 labelled nodes, {n_test} "
                     f"held-out plans x {per_test} requested nodes"),
        "label_seconds": t_label, "train_seconds": t_train, "epochs": epochs,
        "train_loss_first_last": [float(hist[0]), float(hist[-1])],
        "screened_nodes_per_s": total / t_screen,
        "n_ok_1e-2": int(np.sum(e_scr <= 1e-2)), "nodes": total,
        "solver_nodes_per_s": total / t_solver,
        "predict_nodes_per_s": n_test * 3 * 128 * 128 / t_pred,
        "plans_screened": int(sum(x["screened"] for x in st)), "plans": n_test,
        "model_err_requested": q(e_req), "model_err_full_maps": q(e_full),
        "screened_err": q(e_scr),
    }
    log(f"surrogate: train {t_train:.1f} s (labels {t_label:.1f} s), loss {hist[0]:.3g} -> "
        f"{hist[-1]:.3g}; screened {rec['plans_screened']}/{n_test} plans, "
        f"{total / t_screen:.0f} nodes/s vs solver {total / t_solver:.0f}; model median err "
        f"{rec['model_err_requested']['median']:.3g}")
    s.close()
    return rec


def large_run(args, reff, gen, log):
    """The large stack (8 tiers of 2048 x 2048, 33,554,432 nodes): a full
    map is out of reach on one GPU, so the first `large_blocks` 64-node
    blocks of a seeded sample are solved (mixed precision), the 1M-node
    wall time is projected from that rate, and the first block is checked
    against the float64 block PCG on the same GPU at rel_tol 1e-8."""
    import numpy as np
    import torch
    desc = gen.config5()
    n = gen.n_nodes(desc)
    nodes = gen.sample_free_nodes(desc, S * args.large_blocks, 5005)
    log(f"large stack n={n}, {len(nodes)} nodes")
    h = reff.reff_build_pdn(desc, device=0)
    log("stack built and uploaded")
    stream = torch.cuda.current_stream()
    out = torch.empty(len(nodes), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    a = time.perf_counter()
    st = reff.reff_solve_diag(h, nodes, out, precision=reff.REFF_PREC_MIXED, rel_tol=args.rel_tol,
                              stream=stream.cuda_stream, timing=True, progress=True)[1]
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    log(f"mixed: {len(nodes) / dt:.2f} nodes/s, {st['iters_total']} block iterations, {dt:.1f} s")
    a = time.perf_counter()
    ref, st64 = reff.reff_solve_diag(h, nodes[:S], precision=reff.REFF_PREC_FP64, rel_tol=1e-8,
                                     progress=True)
    dt64 = time.perf_counter() - a
    got = out.cpu().numpy()[:S]
    err = float(np.max(np.abs(got - ref) / ref))
    log(f"float64 check: {S / dt64:.2f} nodes/s, {st64['iters_total']} iterations, max rel diff {err:.2e}")
    kms = np.array(st["kernel_ms"])
    kl = np.array(st["kernel_launches"])
    rec = {
        "metric": "R_eff nodes/sec at <=1e-3 max rel err (large stack, measured subset)",
        "value": len(nodes) / dt, "unit": "nodes/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "large stack: 8 tiers x 2048 x 2048 (33,554,432 nodes), x edges "
                               "U[0.5,2] S, y edges U[1,4] S, 16384 clustered TSVs at 5 S, 4096 "
                               f"pads; first {len(nodes)} nodes of a seeded sample",
                   "precision": "mixed", "rel_tol": args.rel_tol, "block_rhs": S},
        "iters_total": st["iters_total"], "iters_max": st["iters_max"],
        "kernel_avg_us": (kms / np.maximum(kl, 1) * 1e3).tolist(),
        "projected_hours_for_1M_nodes": 1e6 / (len(nodes) / dt) / 3600,
        "fp64_check": {"nodes": S, "max_rel_diff": err, "iters": st64["iters_total"],
                       "nodes_per_s": S / dt64, "rel_tol": 1e-8},
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--rel-tol", type=float, default=1e-3,
                    help="solver tolerance (default: the metric's 1e-3 bar; every node is "
                         "still checked against the oracle values)")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--krylov", choices=["block", "indep"], default="block")
    ap.add_argument("--precond-degree", type=int, default=19,
                    help="Chebyshev preconditioner degree (1 = Jacobi)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--large", action="store_true",
                    help="only the large-stack subset measurement (8 x 2048 x 2048)")
    ap.add_argument("--large-blocks", type=int, default=1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy kernel 4 times (the "
                         "reference point for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                          "launches": 4}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(solves shard by node blocks; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_05818_amd import gen, reff

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.large:
        large_run(args, reff, gen, log)
        return
    desc = gen.config2()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "config2_sample.json")))
    sample = gen.sample_free_nodes(desc, 16384, 2002)
    B = args.batch
    assert B <= len(gold["nodes"]), "batch larger than the stored oracle sample"
    batch = sample[:B]
    assert np.array_equal(batch, np.array(gold["nodes"][:B])), "sample drifted from the fixture"
    want = np.array(gold["R"][:B])
    n = gen.n_nodes(desc)
    log(f"building stack n={n}")
    h = reff.reff_build_pdn(desc, device=0)
    prec = reff.REFF_PREC_MIXED if args.precision == "mixed" else reff.REFF_PREC_FP64
    kry = reff.REFF_KRYLOV_BLOCK if args.krylov == "block" else reff.REFF_KRYLOV_INDEPENDENT
    out = torch.empty(B, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step(timing):
        return reff.reff_solve_diag(h, batch, out, precision=prec, krylov=kry,
                                    rel_tol=args.rel_tol, stream=stream.cuda_stream,
                                    timing=timing, precond_degree=args.precond_degree)[1]

    for w in range(args.warmup):
        st = step(False)
        log(f"warmup {w}: {st['iters_total']} iterations, {st['seconds']:.2f} s")
    torch.cuda.synchronize()
    kms = np.zeros(5)
    kl = np.zeros(5, dtype=np.int64)
    krows = np.zeros(5, dtype=np.int64)
    iters = 0
    worst = 0.0
    n_ok = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step(True)
        kms += np.array(st["kernel_ms"])
        kl += np.array(st["kernel_launches"], dtype=np.int64)
        krows += np.array(st["kernel_rows"], dtype=np.int64)
        iters += st["iters_total"]
        log(f"step {k}: {st['iters_total']} iterations, {st['seconds']:.2f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    got = out.cpu().numpy()
    rel = np.abs(got - want) / want
    worst = float(rel.max())
    n_ok = int(np.sum(rel <= 1e-3))
    elapsed = t1 - t0
    value = n_ok * args.steps / elapsed

    fp32 = args.precision == "mixed"
    cheb = args.precond_degree if args.krylov == "block" else 1
    kb = kernel_bytes(1, fp32=fp32, mixed_with_d=fp32, cheb=cheb)
    kf = kernel_flops(cheb)
    mpeak = MFMA_PEAK_TFLOPS["f32" if fp32 else "f64"]
    names = ["stencil_gram", "update_r", "update_y", "cheb_pass", "precond_gram"]
    # one timed span of the Chebyshev entry covers all passes of an iteration
    passes = cheb_words(cheb, fp32)[1] if cheb > 1 else 0
    kern = {}
    for i, nm in enumerate(names):
        if kl[i] == 0 or kms[i] == 0:
            continue
        per_span = passes if i == 3 else 1
        launches = kl[i] * per_span
        avg_ms = kms[i] / launches
        # A launch streams every unconverged block of the group: bytes (and
        # flops) per launch = per node row x rows streamed / launches.
        rows = krows[i] / max(kl[i], 1)
        per_launch = kb[i] / per_span * rows
        flops = kf[i] / per_span * rows
        # the binding ceiling: the larger of the two times at peak
        t_hbm = per_launch / (HBM_PEAK_GBS * 1e9)
        t_mfma = flops / (mpeak * 1e12)
        kern[nm] = {"avg_us": avg_ms * 1e3, "launches": int(launches), "rows_per_launch": rows,
                    "alg_bytes_per_row": kb[i] / per_span, "alg_bytes_per_launch": per_launch,
                    "alg_flops_per_row": kf[i] / per_span,
                    "GBps": per_launch / (avg_ms * 1e-3) / 1e9,
                    "TFLOPs": flops / (avg_ms * 1e-3) / 1e12,
                    "hbm_frac": t_hbm / (avg_ms * 1e-3), "mfma_frac": t_mfma / (avg_ms * 1e-3),
                    "bound": "mfma" if t_mfma > t_hbm else "hbm"}
    dom = max(range(5), key=lambda i: kms[i])
    dk = kern[names[dom]]
    mt = measured_traffic() if fp32 else None
    traffic = None
    if (mt is not None and names[dom] in mt["hbm_bytes_per_row"]
            and mt.get("precond_degree", 1) == cheb):
        traffic = mt["hbm_bytes_per_row"][names[dom]] * krows[dom] / max(kl[dom], 1)
    if dk["bound"] == "mfma":
        roofline = {"bound": "mfma", "achieved": dk["TFLOPs"], "peak": mpeak, "unit": "TFLOP/s",
                    "frac": dk["TFLOPs"] / mpeak, "traffic": traffic, "kernel": names[dom],
                    "hbm_frac": dk["hbm_frac"]}
    else:
        roofline = {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": dk["GBps"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": names[dom],
                    "mfma_frac": dk["mfma_frac"]}

    compare = {}
    if not args.no_compare and args.precision == "mixed":
        # The plain float64 block-PCG and the independent-column variant on
        # one 64-node block of the same batch, same GPU.
        for tag, p, kk, tol in (("plain_fp64_block", reff.REFF_PREC_FP64, reff.REFF_KRYLOV_BLOCK, 1e-6),
                                ("mixed_independent", reff.REFF_PREC_MIXED,
                                 reff.REFF_KRYLOV_INDEPENDENT, args.rel_tol)):
            o2 = torch.empty(S, dtype=torch.float64, device="cuda:0")
            torch.cuda.synchronize()
            a = time.perf_counter()
            st2 = reff.reff_solve_diag(h, batch[:S], o2, precision=p, krylov=kk, rel_tol=tol,
                                       stream=stream.cuda_stream)[1]
            torch.cuda.synchronize()
            dt = time.perf_counter() - a
            e2 = float(np.max(np.abs(o2.cpu().numpy() - want[:S]) / want[:S]))
            compare[tag] = {"nodes_per_s": S / dt, "iters": st2["iters_total"],
                            "max_rel_err": e2, "rel_tol": tol}
            log(f"{tag}: {S / dt:.1f} nodes/s, {st2['iters_total']} iterations, err {e2:.2e}")

    if not args.no_compare:
        compare["grid_pairs"] = grid_pairs_compare(reff, log)
    if not args.no_batched and args.precision == "mixed":
        compare["batched_plans"] = batched_compare(reff, gen, log, args.rel_tol)
    if not args.no_surrogate and args.precision == "mixed":
        compare["surrogate_screened"] = surrogate_compare(reff, gen, log, args.rel_tol)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(desc, batch)
        log(f"cpu baseline {cpu['value']:.4f} nodes/s")

    rec = {
        "metric": "R_eff nodes/sec at <=1e-3 max rel err, plain vs mixed/batched/surrogate; %HBM",
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": "mixed-precision stack: 4 tiers x 512 x 512 (1,048,576 nodes), "
                               "lognormal(0,0.3) S edges, 1024 clustered TSVs at 5 S, 256 pads; "
                               f"{B} seeded sampled nodes per step",
                   "precision": args.precision, "krylov": args.krylov, "rel_tol": args.rel_tol,
                   "block_rhs": S, "precond_degree": cheb},
        "accuracy": {"max_rel_err": worst, "n_ok": n_ok, "n": B},
        "iters_per_step": iters / args.steps,
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "compare": compare,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
