// Two-point resistances on a uniform M x N resistor grid by the closed form
// of Eq. 3 (Sec. II-B), for every pair of a point set: the intra-die
// resistances of the paper's divide-and-conquer pair method (Sec. III-C/D).
//
// For points (x1, y1), (x2, y2), with xh = x + 1/2, yh = y + 1/2,
//   R = r |x1 - x2| / N + s |y1 - y2| / M
//       + 2 / (M N) sum_{m=1}^{M-1} sum_{n=1}^{N-1}
//           (cos(m t xh1) cos(n u yh1) - cos(m t xh2) cos(n u yh2))^2
//           / ((1 - cos(m t)) / r + (1 - cos(n u)) / s),
// t = pi / M, u = pi / N.  One wave per pair (i < j; the mirror is written
// by the same wave): lanes own n (WN values each per chunk of 64 WN), the m
// loop runs in order and takes cos(m t xh) from the multiple-angle recurrence
// cos((m+1) a) = 2 cos(a) cos(m a) - cos((m-1) a), as the paper's GPU
// evaluation does (Sec. III-D); the m-dependent part of the denominator is a
// per-workgroup LDS table.
#include <hip/hip_runtime.h>
#include <cmath>
#include <stdint.h>

#include <string>
#include <vector>

#include "reff_internal.h"

namespace reff {
namespace {

constexpr int GP_WAVES = 4;      // pairs per workgroup (one wave each)
constexpr int GP_WN = 8;         // n values per lane and chunk
constexpr int GP_MMAX = 4096;    // LDS table of (1 - cos(m t)) / r

// 1/x for x > 0: hardware estimate and two Newton steps (float64 accuracy).
__device__ __forceinline__ double grid_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// Grid (ceil(P / GP_WAVES), P): row i = blockIdx.y, column j = blockIdx.x *
// GP_WAVES + wave; waves with j < i exit (their pair is the mirror of one
// evaluated by another wave), j == i writes the zero diagonal.
__global__ __launch_bounds__(64 * GP_WAVES) void k_grid_pairs(int M, int N, double r, double s,
                                                             const int32_t* __restrict__ xy,
                                                             int64_t P, double* __restrict__ out) {
  __shared__ double dm[GP_MMAX];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double t = M_PI / M, u = M_PI / N;
  for (int m = threadIdx.x; m < M && m < GP_MMAX; m += blockDim.x) dm[m] = (1.0 - cos(m * t)) / r;
  __syncthreads();
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * GP_WAVES + w;
  if (j < i || j >= P) return;  // the whole wave
  if (j == i) {
    if (lane == 0) out[i * P + i] = 0.0;
    return;
  }
  const int x1 = xy[2 * i], y1 = xy[2 * i + 1], x2 = xy[2 * j], y2 = xy[2 * j + 1];
  const double xh1 = x1 + 0.5, xh2 = x2 + 0.5, yh1 = y1 + 0.5, yh2 = y2 + 0.5;
  const double c1 = cos(xh1 * t), c2 = cos(xh2 * t);  // cos(a) of the two recurrences
  double acc = 0.0;
  for (int n0 = 1; n0 < N; n0 += 64 * GP_WN) {
    double b1[GP_WN], b2[GP_WN], e[GP_WN];
#pragma unroll
    for (int k = 0; k < GP_WN; ++k) {
      const int n = n0 + lane + 64 * k;
      const bool ok = n < N;
      b1[k] = ok ? cos(n * u * yh1) : 0.0;  // a lane past N - 1 adds 0
      b2[k] = ok ? cos(n * u * yh2) : 0.0;
      e[k] = ok ? (1.0 - cos(n * u)) / s : 1.0;
    }
    // cos(m a) for m = 1 (a1, a2) and m = 0 (p1, p2)
    double a1 = c1, a2 = c2, p1 = 1.0, p2 = 1.0;
    for (int m = 1; m < M; ++m) {
      const double d = m < GP_MMAX ? dm[m] : (1.0 - cos(m * t)) / r;
#pragma unroll
      for (int k = 0; k < GP_WN; ++k) {
        const double num = fma(a1, b1[k], -a2 * b2[k]);
        acc = fma(num * num, grid_rcp(d + e[k]), acc);
      }
      const double q1 = fma(2.0 * c1, a1, -p1), q2 = fma(2.0 * c2, a2, -p2);
      p1 = a1, p2 = a2, a1 = q1, a2 = q2;
    }
  }
  // sum over the lanes
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    const double R = r * fabs((double)(x1 - x2)) / N + s * fabs((double)(y1 - y2)) / M +
                     2.0 / ((double)M * N) * acc;
    out[i * P + j] = R;
    out[j * P + i] = R;
  }
}

}  // namespace
}  // namespace reff

extern "C" reff_status reff_grid_pairs(int32_t M, int32_t N, double r, double s,
                                       const int32_t* xy, int64_t P, double* R_out,
                                       int32_t out_on_device, void* stream) {
  using namespace reff;
  if (M < 1 || N < 1) return host_fail(REFF_ERR_INVALID_ARG, "grid size must be at least 1 x 1");
  if (!std::isfinite(r) || !(r > 0.0) || !std::isfinite(s) || !(s > 0.0))
    return host_fail(REFF_ERR_INVALID_ARG, "edge resistances must be finite and positive");
  if (P < 0) return host_fail(REFF_ERR_INVALID_ARG, "negative point count");
  if (P == 0) return REFF_OK;
  if (!xy || !R_out) return host_fail(REFF_ERR_INVALID_ARG, "NULL points or output");
  if (P > 65535) return host_fail(REFF_ERR_INVALID_ARG, "at most 65535 points per call");
  for (int64_t k = 0; k < P; ++k)
    if (xy[2 * k] < 0 || xy[2 * k] >= M || xy[2 * k + 1] < 0 || xy[2 * k + 1] >= N)
      return host_fail(REFF_ERR_INVALID_ARG, "point " + std::to_string(k) + " is off the grid");
  hipStream_t st = (hipStream_t)stream;
  auto dev_fail = [&](hipError_t e, const char* what) {
    return host_fail(e == hipErrorOutOfMemory ? REFF_ERR_OUT_OF_MEMORY : REFF_ERR_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
  };
  int32_t* dxy = nullptr;
  double* dout = nullptr;
  hipError_t e = hipMalloc((void**)&dxy, (size_t)P * 2 * sizeof(int32_t));
  if (e != hipSuccess) return dev_fail(e, "hipMalloc");
  const size_t obytes = (size_t)P * P * sizeof(double);
  if (!out_on_device) {
    e = hipMalloc((void**)&dout, obytes);
    if (e != hipSuccess) {
      (void)hipFree(dxy);
      return dev_fail(e, "hipMalloc");
    }
  }
  double* o = out_on_device ? R_out : dout;
  e = hipMemcpyAsync(dxy, xy, (size_t)P * 2 * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)((P + GP_WAVES - 1) / GP_WAVES), (unsigned)P);
    hipLaunchKernelGGL(k_grid_pairs, grid, dim3(64 * GP_WAVES), 0, st, (int)M, (int)N, r, s, dxy,
                       P, o);
    e = hipGetLastError();
  }
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(R_out, dout, obytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dxy);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return dev_fail(e, "grid pairs");
  return REFF_OK;
}
