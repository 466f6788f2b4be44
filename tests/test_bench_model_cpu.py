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
