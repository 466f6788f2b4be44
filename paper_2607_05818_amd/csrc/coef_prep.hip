// Derived stencil coefficient arrays, formed on the device from the float64
// ones the host uploads: the Jacobi scaling D^-1 (float64) and the float32
// copies of d, D^-1, cE and cN that the mixed-precision kernels read.  The
// host then moves three float64 arrays per node instead of four float64 and
// four float32 ones.  Division and rounding are IEEE (correctly rounded
// float64 reciprocal, round-to-nearest float32 conversion), so the arrays
// equal what the same operations give on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reff {

__global__ __launch_bounds__(256) void k_coef_derived(const double* __restrict__ d,
                                                      const double* __restrict__ cE,
                                                      const double* __restrict__ cN, int64_t n,
                                                      double* __restrict__ dinv64,
                                                      float* __restrict__ d32,
                                                      float* __restrict__ dinv32,
                                                      float* __restrict__ cE32,
                                                      float* __restrict__ cN32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = d[i];
    const double r = 1.0 / v;
    dinv64[i] = r;
    d32[i] = (float)v;
    dinv32[i] = (float)r;
    cE32[i] = (float)cE[i];
    cN32[i] = (float)cN[i];
  }
}

// Forms dinv64, d32, dinv32, cE32 and cN32 (n entries each) from d, cE, cN
// on `st`.  All pointers are device memory of n entries.
hipError_t launch_coef_derived(const double* d, const double* cE, const double* cN, int64_t n,
                               double* dinv64, float* d32, float* dinv32, float* cE32,
                               float* cN32, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(k_coef_derived, dim3(grid), dim3(256), 0, st, d, cE, cN, n, dinv64, d32,
                     dinv32, cE32, cN32);
  return hipGetLastError();
}

}  // namespace reff
