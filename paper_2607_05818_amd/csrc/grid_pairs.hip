// Two-point resistances on a uniform M x N resistor grid by the closed form
// of Eq. 3 (Sec. II-B), for every pair of a point set: the intra-die
// resistances of the paper's divide-and-conquer pair method (Sec. III-C/D).
//
// For points (x1, y1), (x2, y2), with xh = x + 1/2, yh = y + 1/2,
//   R = r |x1 - x2| / N + s |y1 - y2| / M
//       + 2 / (M N) sum_{m=1}^{M-1} sum_{n=1}^{N-1}
//           (cos(m t xh1) cos(n u yh1) - cos(m t xh2) cos(n u yh2))^2
//           / ((1 - cos(m t)) / r + (1 - cos(n u)) / s),
// t = pi / M, u = pi / N.  The denominator does not depend on the pair:
// k_grid_weights stores its reciprocal W[m][n] once per call ((M-1)(N-1)
// float64, cache-resident at the sizes of a tier).  k_grid_pairs then gives
// each wave GP_PW pairs (i, j) with one i: lanes own n (GP_WN values each
// per chunk of 64 GP_WN), the m loop runs in order and takes cos(m t xh)
// from the multiple-angle recurrence cos((m+1) a) = 2 cos(a) cos(m a) -
// cos((m-1) a), as the paper's GPU evaluation does (Sec. III-D), and each
// W entry loaded serves the wave's GP_PW pairs.
#include <hip/hip_runtime.h>
#include <cmath>
#include <stdint.h>

#include <string>
#include <vector>

#include "reff_internal.h"

namespace reff {
namespace {

constexpr int GP_WAVES = 4;   // waves per workgroup
constexpr int GP_PW = 4;      // pairs per wave (one row point i, GP_PW columns j)
constexpr int GP_WN = 8;      // n values per lane and chunk

// W[(m-1)(N-1) + n-1] = 1 / ((1 - cos(m t)) / r + (1 - cos(n u)) / s).
__global__ __launch_bounds__(256) void k_grid_weights(int M, int N, double r, double s,
                                                      double* __restrict__ W) {
  const int64_t total = (int64_t)(M - 1) * (N - 1);
  const double t = M_PI / M, u = M_PI / N;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(q / (N - 1)) + 1, n = (int)(q % (N - 1)) + 1;
    W[q] = 1.0 / ((1.0 - cos(m * t)) / r + (1.0 - cos(n * u)) / s);
  }
}

// Grid (ceil(P / (GP_WAVES GP_PW)), P): row point i = blockIdx.y; wave w
// takes the columns j = (blockIdx.x GP_WAVES + w) GP_PW + q, q < GP_PW.
// Pairs with j <= i or j >= P are formed with a valid stand-in column and
// not written (their values come from the mirror pair); a wave with no
// pair to write exits.  The diagonal is written as 0 by the wave of j = i.
__global__ __launch_bounds__(64 * GP_WAVES) void k_grid_pairs(int M, int N, double r, double s,
                                                             const int32_t* __restrict__ xy,
                                                             const double* __restrict__ W,
                                                             int64_t P, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = blockIdx.y;
  const int64_t j0 = ((int64_t)blockIdx.x * GP_WAVES + w) * GP_PW;
  if (j0 + GP_PW - 1 < i || j0 >= P) return;  // the whole wave: nothing to write
  const double t = M_PI / M, u = M_PI / N;
  const int x1 = xy[2 * i], y1 = xy[2 * i + 1];
  const double xh1 = x1 + 0.5, yh1 = y1 + 0.5;
  int x2[GP_PW], y2[GP_PW];
  double xh2[GP_PW], yh2[GP_PW], c2[GP_PW];
#pragma unroll
  for (int q = 0; q < GP_PW; ++q) {
    const int64_t j = min(j0 + q, P - 1);
    x2[q] = xy[2 * j];
    y2[q] = xy[2 * j + 1];
    xh2[q] = x2[q] + 0.5;
    yh2[q] = y2[q] + 0.5;
    c2[q] = cos(xh2[q] * t);
  }
  const double c1 = cos(xh1 * t);
  double acc[GP_PW];
#pragma unroll
  for (int q = 0; q < GP_PW; ++q) acc[q] = 0.0;
  for (int n0 = 1; n0 < N; n0 += 64 * GP_WN) {
    double b1[GP_WN], b2[GP_PW][GP_WN];
    int nw[GP_WN];  // column of this lane's n in W (clamped; b = 0 past N - 1)
#pragma unroll
    for (int k = 0; k < GP_WN; ++k) {
      const int n = n0 + lane + 64 * k;
      const bool ok = n < N;
      nw[k] = ok ? n - 1 : 0;
      b1[k] = ok ? cos(n * u * yh1) : 0.0;
#pragma unroll
      for (int q = 0; q < GP_PW; ++q) b2[q][k] = ok ? cos(n * u * yh2[q]) : 0.0;
    }
    // cos(m a) at m = 1 (a*) and m = 0 (p*) for the row point and the columns
    double a1 = c1, p1 = 1.0, a2[GP_PW], p2[GP_PW];
#pragma unroll
    for (int q = 0; q < GP_PW; ++q) a2[q] = c2[q], p2[q] = 1.0;
    // W row m - 1, loaded one m ahead (the last row is loaded again at the end)
    double wn[GP_WN];
#pragma unroll
    for (int k = 0; k < GP_WN; ++k) wn[k] = M > 1 ? W[nw[k]] : 0.0;
    for (int m = 1; m < M; ++m) {
      double wc[GP_WN];
      const double* Wn = W + (int64_t)min(m, M - 2) * (N - 1);  // row of m + 1
#pragma unroll
      for (int k = 0; k < GP_WN; ++k) {
        wc[k] = wn[k];
        wn[k] = Wn[nw[k]];
      }
#pragma unroll
      for (int k = 0; k < GP_WN; ++k) {
        const double wt = wc[k];
        const double f1 = a1 * b1[k];
#pragma unroll
        for (int q = 0; q < GP_PW; ++q) {
          const double num = fma(-a2[q], b2[q][k], f1);
          acc[q] = fma(num * num, wt, acc[q]);
        }
      }
      const double q1 = fma(2.0 * c1, a1, -p1);
      p1 = a1, a1 = q1;
#pragma unroll
      for (int q = 0; q < GP_PW; ++q) {
        const double qq = fma(2.0 * c2[q], a2[q], -p2[q]);
        p2[q] = a2[q], a2[q] = qq;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < GP_PW; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int64_t j = j0 + q;
    if (lane == 0 && j < P) {
      if (j == i) {
        out[i * P + i] = 0.0;
      } else if (j > i) {
        const double R = r * fabs((double)(x1 - x2[q])) / N + s * fabs((double)(y1 - y2[q])) / M +
                         2.0 / ((double)M * N) * v;
        out[i * P + j] = R;
        out[j * P + i] = R;
      }
    }
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
  double* dW = nullptr;
  const size_t nw = (size_t)(M - 1) * (N - 1);
  hipError_t e = hipMalloc((void**)&dxy, (size_t)P * 2 * sizeof(int32_t));
  if (e != hipSuccess) return dev_fail(e, "hipMalloc");
  e = hipMalloc((void**)&dW, std::max<size_t>(nw, 1) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipFree(dxy);
    return dev_fail(e, "hipMalloc");
  }
  const size_t obytes = (size_t)P * P * sizeof(double);
  if (!out_on_device) {
    e = hipMalloc((void**)&dout, obytes);
    if (e != hipSuccess) {
      (void)hipFree(dxy);
      (void)hipFree(dW);
      return dev_fail(e, "hipMalloc");
    }
  }
  double* o = out_on_device ? R_out : dout;
  e = hipMemcpyAsync(dxy, xy, (size_t)P * 2 * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nw > 0) {
    const int64_t blocks = std::min<int64_t>((int64_t)((nw + 255) / 256), 4096);
    hipLaunchKernelGGL(k_grid_weights, dim3((unsigned)blocks), dim3(256), 0, st, (int)M, (int)N,
                       r, s, dW);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int64_t per = (int64_t)GP_WAVES * GP_PW;
    const dim3 grid((unsigned)((P + per - 1) / per), (unsigned)P);
    hipLaunchKernelGGL(k_grid_pairs, grid, dim3(64 * GP_WAVES), 0, st, (int)M, (int)N, r, s, dxy,
                       (const double*)dW, P, o);
    e = hipGetLastError();
  }
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(R_out, dout, obytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dxy);
  (void)hipFree(dW);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return dev_fail(e, "grid pairs");
  return REFF_OK;
}
