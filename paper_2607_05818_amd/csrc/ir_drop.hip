// Superposition of unit-load responses (Eq. 4, Sec. II-B) for IR drop and
// through-bump currents (Sec. IV-B).
//
// A solved block holds x_l = G^-1 e_l for up to S load nodes l (column k of
// an n x S float64 array, RHS-interleaved).  With the bumps merged into the
// supply node, Eq. 4's 1/2 (R_j + R_l - R(j, l)) is exactly x_l[j], so a
// scenario c drawing I_c,l at the loads has
//     drop_c[j] = sum_l I_c,l x_l[j],
// and a pad delivers sum_u g_pu drop_c[u] over its edges.  Both are a
// weighted node row of the block times the block's S x n_scen load matrix;
// k_rows_times_loads evaluates them for a list of weighted rows (CSR: one
// row per requested node with weight 1, one per pad with its edge
// conductances) and adds the result into out[c * ld + r].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "reff_internal.h"

namespace reff {
namespace {

constexpr int RW = 4;  // waves per workgroup, one output row per wave at a time

__global__ __launch_bounds__(64 * RW) void k_rows_times_loads(
    const double* __restrict__ X, const int32_t* __restrict__ rptr,
    const int64_t* __restrict__ rnode, const double* __restrict__ rw, int64_t nrows,
    const double* __restrict__ amps, int n_scen, double* __restrict__ out, int64_t ld) {
  __shared__ double A[S][S + 1];   // amps[k][c] of one 64-scenario chunk
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < n_scen; c0 += S) {
    const int nc = min(S, n_scen - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
      const int k = e / S, c = e % S;
      A[k][c] = c < nc ? amps[(size_t)k * n_scen + c0 + c] : 0.0;
    }
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * RW + w; r < nrows; r += (int64_t)gridDim.x * RW) {
      double x = 0.0;
      for (int e = rptr[r]; e < rptr[r + 1]; ++e) x += rw[e] * X[rnode[e] * S + lane];
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < S; ++k) acc += __shfl(x, k) * A[k][lane];
      if (lane < nc) out[(size_t)(c0 + lane) * ld + r] += acc;
    }
  }
}

}  // namespace

hipError_t launch_rows_times_loads(const double* X, const int32_t* rptr, const int64_t* rnode,
                                   const double* rw, int64_t nrows, const double* amps,
                                   int n_scen, double* out, int64_t ld, hipStream_t st) {
  if (nrows <= 0 || n_scen <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((nrows + RW - 1) / RW, 4096);
  hipLaunchKernelGGL(k_rows_times_loads, dim3((unsigned)blocks), dim3(64 * RW), 0, st, X, rptr,
                     rnode, rw, nrows, amps, n_scen, out, ld);
  return hipGetLastError();
}

}  // namespace reff
