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
S = 64


def kernel_bytes(n, fp32=True, mixed_with_d=True):
    """Algorithmic HBM bytes per launch of the three block kernels for an
    n-node stack and S right-hand sides (w = bytes per word):
      stencil+Gram (K1): read Y, R; write P = Y T, Q = (G Y) T -> 4 S w per node
                         + coefficients d, cE, cN (w each) and the TSV slot (4)
      residual update (K2): read Q, R (P, D); write R (D)       -> 3 (6) S w
                         + Dinv
      search block (K3): read P, R; write Y                     -> 3 S w + d, Dinv
    """
    w = 4 if fp32 else 8
    k1 = n * (4 * S * w + 3 * w + 4)
    k2 = n * ((6 if mixed_with_d else 3) * S * w + w)
    k3 = n * (3 * S * w + 2 * w)
    return [k1, k2, k3]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--rel-tol", type=float, default=1e-4)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--krylov", choices=["block", "indep"], default="block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(solves shard by node blocks; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_05818_amd import gen, reff

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

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
                                    timing=timing)[1]

    for w in range(args.warmup):
        st = step(False)
        log(f"warmup {w}: {st['iters_total']} iterations, {st['seconds']:.2f} s")
    torch.cuda.synchronize()
    kms = np.zeros(3)
    kl = np.zeros(3, dtype=np.int64)
    iters = 0
    worst = 0.0
    n_ok = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step(True)
        kms += np.array(st["kernel_ms"])
        kl += np.array(st["kernel_launches"], dtype=np.int64)
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
    kb = kernel_bytes(n, fp32=fp32, mixed_with_d=fp32)
    names = ["stencil_gram", "update_r", "update_y"]
    kern = {}
    for i, nm in enumerate(names):
        avg_ms = kms[i] / max(kl[i], 1)
        kern[nm] = {"avg_us": avg_ms * 1e3, "launches": int(kl[i]),
                    "alg_bytes": int(kb[i]), "GBps": kb[i] / (avg_ms * 1e-3) / 1e9}
    dom = max(range(3), key=lambda i: kms[i])
    dk = kern[names[dom]]
    roofline = {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["GBps"] / HBM_PEAK_GBS, "traffic": None,
                "kernel": names[dom]}

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
                   "block_rhs": S},
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
