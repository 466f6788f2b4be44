"""The benchmark's algorithmic byte and flop model (bench.py), against the
counts written out by hand from the kernels' reads and writes: S = 64
right-hand sides, float32 words (4 bytes) in the mixed path."""
import bench

S, W = 64, 4


def test_chebyshev_pass_words_degree_19():
    """Degree 19 = 18 steps = six three-step passes: the first forms z_1 from
    R (reads R, writes two iterates), four middle passes read z_j, z_{j-1},
    R and write two, the last writes one."""
    words, passes = bench.cheb_words(19, fp32=True)
    assert passes == 6
    assert words == (1 + 2) + 4 * (3 + 2) + (3 + 1)


def test_block_kernel_bytes_with_the_solution_update_in_k3():
    n = 1000
    k1, k2, k3, kp, kg = bench.kernel_bytes(n, fp32=True, mixed_with_d=True, cheb=19)
    assert k1 == n * (4 * S * W + 3 * W + 4)          # Y, R in; P, Q out; d, cE, cN, slot
    assert k2 == n * (3 * S * W + W)                  # Q, R in; R out; Dinv
    assert k3 == n * (5 * S * W + 2 * W)              # P, Z, D in; Y, D out; d, Dinv
    assert kg == n * 2 * S * W                        # Q, Z
    words, passes = bench.cheb_words(19, fp32=True)
    assert kp == n * (words * S * W + passes * (4 * W + 4))
    # per row of one iteration: 1040 + 772 + 7032 + 512 + 1288 bytes
    assert (k1 + k2 + kp + kg + k3) // n == 1040 + 772 + 7032 + 512 + 1288
    # the Jacobi variant keeps the update in K2
    j1, j2, j3, _, _ = bench.kernel_bytes(n, fp32=True, mixed_with_d=True, cheb=1)
    assert j2 == n * (6 * S * W + W) and j3 == n * (3 * S * W + 2 * W)


def test_block_kernel_flops():
    g = 2 * S * S
    k1, k2, k3, kp, kg = bench.kernel_flops(cheb=19)
    assert k1 == 2 * g * 10 // 16 + 2 * g            # P = Y T, Q = (G Y) T (10 of 16 blocks of T), 2 Grams
    assert (k2, k3, kp, kg) == (g, 3 * g, 0, g)        # Q A; P B, P A, Y^T D Y; none; Q^T Z
    assert bench.kernel_flops(cheb=1)[1:3] == [3 * g, 2 * g]


def test_stored_bounds_check():
    """The large-stack check reads the stored oracle bounds: values at the
    lower bounds count as inside, values 1 % above a finite upper bound do
    not, and another node sample is not checked at all."""
    import json
    import os

    import numpy as np
    g = json.load(open(os.path.join(bench.ROOT, "tests", "golden", "config5_bounds.json")))
    nodes = np.array(g["nodes"] + [0] * 48)
    lo = np.array(g["lo"] + [0.0] * 48)
    rec = bench.stored_bounds_check(nodes, lo)
    assert rec["inside_within_1e-3"] == 16
    finite = [j for j, h in enumerate(g["hi"]) if h is not None]
    assert rec["finite_upper"] == len(finite) > 0
    over = lo.copy()
    for j in finite:
        over[j] = 1.01 * g["hi"][j]
    assert bench.stored_bounds_check(nodes, over)["inside_within_1e-3"] == 16 - len(finite)
    assert bench.stored_bounds_check(nodes[::-1].copy(), lo) is None
