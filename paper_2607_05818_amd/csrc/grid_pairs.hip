// Two-point resistances on a uniform M x N resistor grid by the closed form
// of Eq. 3 (Sec. II-B), for every pair of a point set: the intra-die
// resistances of the paper's divide-and-conquer pair method (Sec. III-C/D).
//
// For points (x1, y1), (x2, y2), with xh = x + 1/2, yh = y + 1/2,
//   R = r |x1 - x2| / N + s |y1 - y2| / M
//       + 2 / (M N) sum_{m=1}^{M-1} sum_{n=1}^{N-1}
//           (cos(m t xh1) cos(n u yh1) - cos(m t xh2) cos(n u yh2))^2
//           / ((1 - cos(m t)) / r + (1 - cos(n u)) / s),
// t = pi / M, u = pi / N.  The denominator does not depend on the pair, so
// k_grid_weights stores its reciprocal W[m][n] once per call ((M-1)(N-1)
// float64, cache-resident at the sizes of a tier).  With X_i[m][n] =
// cos(m t xh_i) cos(n u yh_i) the double sum of a pair is T_ii + T_jj -
// 2 T_ij, T = X diag(W) X^T: a float64 product over K = (M-1)(N-1) that
// runs on the matrix cores (k_grid_gram), its m factors from the
// multiple-angle recurrence cos((m+1) a) = 2 cos(a) cos(m a) - cos((m-1) a)
// as in the paper's GPU evaluation (Sec. III-D); k_grid_finish forms R.
#include <hip/hip_runtime.h>
#include <cmath>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "reff_internal.h"

namespace reff {
namespace {

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

// k_grid_gram computes 64 x 64 blocks of T (upper block pairs only) on the
// float64 matrix cores (16x16x4), the K range split over workgroups by m
// segment; its operands are formed on the fly: the n factor from a table C[p][n-1] =
// cos(n u yh_p) staged in LDS per 64-wide chunk of n, the m factor from the
// multiple-angle recurrence per lane, W from the weight table.  Each
// segment writes its partial block; k_grid_finish sums them and forms R.
constexpr int GG_B = 64;    // points per block
constexpr int GG_NC = 64;   // n values per staged chunk

__global__ __launch_bounds__(256) void k_grid_ncos(int N, const int32_t* __restrict__ xy,
                                                   int64_t P, double* __restrict__ Cn) {
  const int64_t total = P * (N - 1);
  const double u = M_PI / N;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = q / (N - 1);
    const int n = (int)(q % (N - 1)) + 1;
    Cn[q] = cos(n * u * (xy[2 * p + 1] + 0.5));
  }
}

// Grid (block pairs, m segments).  Tpart[seg][i][j] for the block pair's
// i, j (rows of block bi, columns of block bj, bi <= bj); points past P
// are stand-ins (the last point) whose entries are not written.
__global__ __launch_bounds__(256) void k_grid_gram(int M, int N, const int32_t* __restrict__ xy,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ Cn, int64_t P,
                                                   int nb, int mseg, double* __restrict__ Tpart) {
  __shared__ double BI[GG_B][GG_NC + 1], BJ[GG_B][GG_NC + 1];
  int q = blockIdx.x, bi = 0;
  while (q >= nb - bi) q -= nb - bi, ++bi;
  const int bj = bi + q;
  const int seg = blockIdx.y;
  const int mlen = (M - 1 + mseg - 1) / mseg;
  const int m0 = 1 + seg * mlen, m1 = min(M, m0 + mlen);  // m in [m0, m1)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cc = lane & 15, kr = lane >> 4;
  const double t = M_PI / M;
  const int64_t ia = min((int64_t)bi * GG_B + w * 16 + cc, P - 1);
  int64_t jb[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) jb[tt] = min((int64_t)bj * GG_B + tt * 16 + cc, P - 1);
  const double xi = xy[2 * ia] + 0.5;
  double xj[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) xj[tt] = xy[2 * jb[tt]] + 0.5;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) acc[tt] = d4{0.0, 0.0, 0.0, 0.0};
  for (int n0 = 1; n0 < N; n0 += GG_NC) {
    __syncthreads();  // the previous chunk is no longer read
    for (int e = threadIdx.x; e < GG_B * GG_NC; e += blockDim.x) {
      const int pt = e / GG_NC, k = e % GG_NC, n = n0 + k;
      const int64_t pi = min((int64_t)bi * GG_B + pt, P - 1), pj = min((int64_t)bj * GG_B + pt, P - 1);
      const bool ok = n < N;
      BI[pt][k] = ok ? Cn[pi * (N - 1) + (n - 1)] : 0.0;
      BJ[pt][k] = ok ? Cn[pj * (N - 1) + (n - 1)] : 0.0;
    }
    __syncthreads();
    if (m0 >= m1) continue;
    // cos(m a) at m = m0 and m0 - 1, then the recurrence
    double ai = cos(m0 * t * xi), pi_ = cos((m0 - 1) * t * xi), ki = 2.0 * cos(t * xi);
    double aj[4], pj_[4], kj[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      aj[tt] = cos(m0 * t * xj[tt]);
      pj_[tt] = cos((m0 - 1) * t * xj[tt]);
      kj[tt] = 2.0 * cos(t * xj[tt]);
    }
    for (int m = m0; m < m1; ++m) {
      const double* Wm = W + (int64_t)(m - 1) * (N - 1);
#pragma unroll 4  // (full unrolling needs 305 registers: one wave per SIMD)
      for (int ks = 0; ks < GG_NC / 4; ++ks) {
        const int k = 4 * ks + kr, n = n0 + k;
        const double wv = Wm[min(n, N - 1) - 1];
        const double A = ai * BI[w * 16 + cc][k];
        const double wk = n < N ? wv : 0.0;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const double B = wk * aj[tt] * BJ[tt * 16 + cc][k];
          acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B, acc[tt], 0, 0, 0);
        }
      }
      const double qi = fma(ki, ai, -pi_);
      pi_ = ai, ai = qi;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const double qj = fma(kj[tt], aj[tt], -pj_[tt]);
        pj_[tt] = aj[tt], aj[tt] = qj;
      }
    }
  }
  double* Ts = Tpart + (int64_t)seg * P * P;
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = (int64_t)bi * GG_B + w * 16 + kr + 4 * r;
      const int64_t j = (int64_t)bj * GG_B + tt * 16 + cc;
      if (i < P && j < P) Ts[i * P + j] = acc[tt][r];
    }
}

// R(i,j) from the summed partial T (its upper blocks): r |dx| / N + s |dy| / M
// + 2 / (M N) (T_ii + T_jj - 2 T_ij), i != j; R(i,i) = 0.  T_ij is read at
// (min, max), so both halves of R are the same value.
__global__ __launch_bounds__(256) void k_grid_finish(int M, int N, double r, double s,
                                                     const int32_t* __restrict__ xy,
                                                     const double* __restrict__ Tpart,
                                                     int mseg, int64_t P,
                                                     double* __restrict__ out) {
  const int64_t total = P * P;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / P, j = q % P;
    if (i == j) {
      out[q] = 0.0;
      continue;
    }
    const int64_t lo = min(i, j), hi = max(i, j);
    double tii = 0.0, tjj = 0.0, tij = 0.0;
    for (int g = 0; g < mseg; ++g) {
      const double* Ts = Tpart + (int64_t)g * P * P;
      tii += Ts[lo * P + lo];
      tjj += Ts[hi * P + hi];
      tij += Ts[lo * P + hi];
    }
    const int dx = xy[2 * lo] - xy[2 * hi], dy = xy[2 * lo + 1] - xy[2 * hi + 1];
    out[q] = r * fabs((double)dx) / N + s * fabs((double)dy) / M +
             2.0 / ((double)M * N) * (tii + tjj - 2.0 * tij);
  }
}

// The four launches of one call: weights, cosine table, Gram blocks, R.
hipError_t grid_pairs_launch(int M, int N, double r, double s, const int32_t* dxy, int64_t P,
                             double* dW, double* dC, double* dT, int mseg, double* o,
                             hipStream_t st) {
  const int64_t nb = (P + GG_B - 1) / GG_B;
  const int64_t nbp = nb * (nb + 1) / 2;
  const size_t nw = (size_t)(M - 1) * (N - 1);
  const size_t ncos = (size_t)P * (N - 1);
  auto grid1 = [](size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)); };
  hipError_t e = hipSuccess;
  if (nw > 0) {
    hipLaunchKernelGGL(k_grid_weights, grid1(nw), dim3(256), 0, st, M, N, r, s, dW);
    e = hipGetLastError();
  }
  if (e == hipSuccess && ncos > 0) {
    hipLaunchKernelGGL(k_grid_ncos, grid1(ncos), dim3(256), 0, st, N, dxy, P, dC);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_grid_gram, dim3((unsigned)nbp, (unsigned)mseg), dim3(256), 0, st, M, N,
                       dxy, (const double*)dW, (const double*)dC, P, (int)nb, mseg, dT);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_grid_finish, grid1((size_t)P * P), dim3(256), 0, st, M, N, r, s, dxy,
                       (const double*)dT, mseg, P, o);
    e = hipGetLastError();
  }
  return e;
}

// Segments of the m range: about 2048 workgroups per launch.
int grid_pairs_mseg(int M, int64_t P) {
  const int64_t nb = (P + GG_B - 1) / GG_B;
  const int64_t nbp = nb * (nb + 1) / 2;
  return (int)std::max<int64_t>(1, std::min<int64_t>(std::max(M - 1, 1), (2048 + nbp - 1) / nbp));
}

reff_status grid_pairs_validate(int32_t M, int32_t N, double r, double s, const int32_t* xy,
                                int64_t P, const double* R_out) {
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
  return REFF_OK;
}

reff_status grid_dev_fail(hipError_t e, const char* what) {
  return host_fail(e == hipErrorOutOfMemory ? REFF_ERR_OUT_OF_MEMORY : REFF_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

// Work memory of reff_grid_pairs_noalloc: one array per GPU, resident until
// the process ends.  Host code never passes `scratch` itself to a kernel or
// a copy (on the host it is only a stand-in for the symbol); it uses the
// device address looked up once per device below.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace reff

namespace reff {

// All-pairs Eq. 3 resistances of P points already in device memory, into
// device out[P * P]; the work memory is allocated here and released after
// the stream has run the kernels (the call returns with them complete).
hipError_t grid_pairs_device(int M, int N, double r, double s, const int32_t* dxy, int64_t P,
                             double* dout, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  const int mseg = grid_pairs_mseg(M, P);
  double *dW = nullptr, *dC = nullptr, *dT = nullptr;
  hipError_t e = hipMalloc((void**)&dW, std::max<size_t>((size_t)(M - 1) * (N - 1), 1) * sizeof(double));
  if (e == hipSuccess)
    e = hipMalloc((void**)&dC, std::max<size_t>((size_t)P * (N - 1), 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dT, (size_t)mseg * P * P * sizeof(double));
  if (e == hipSuccess) e = grid_pairs_launch(M, N, r, s, dxy, P, dW, dC, dT, mseg, dout, st);
  const hipError_t e2 = hipStreamSynchronize(st);
  if (e == hipSuccess) e = e2;
  if (dW) (void)hipFree(dW);
  if (dC) (void)hipFree(dC);
  if (dT) (void)hipFree(dT);
  return e;
}

}  // namespace reff

extern "C" reff_status reff_grid_pairs(int32_t M, int32_t N, double r, double s,
                                       const int32_t* xy, int64_t P, double* R_out,
                                       int32_t out_on_device, void* stream) {
  using namespace reff;
  const reff_status v = grid_pairs_validate(M, N, r, s, xy, P, R_out);
  if (v != REFF_OK || P == 0) return v;
  hipStream_t st = (hipStream_t)stream;
  const int mseg = grid_pairs_mseg(M, P);
  const size_t nw = (size_t)(M - 1) * (N - 1);
  const size_t ncos = (size_t)P * (N - 1);
  const size_t tbytes = (size_t)mseg * P * P * sizeof(double);
  const size_t obytes = (size_t)P * P * sizeof(double);
  int32_t* dxy = nullptr;
  double *dW = nullptr, *dC = nullptr, *dT = nullptr, *dout = nullptr;
  auto release = [&]() {
    if (dxy) (void)hipFree(dxy);
    if (dW) (void)hipFree(dW);
    if (dC) (void)hipFree(dC);
    if (dT) (void)hipFree(dT);
    if (dout) (void)hipFree(dout);
  };
  hipError_t e = hipMalloc((void**)&dxy, (size_t)P * 2 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&dW, std::max<size_t>(nw, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dC, std::max<size_t>(ncos, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dT, tbytes);
  if (e == hipSuccess && !out_on_device) e = hipMalloc((void**)&dout, obytes);
  if (e != hipSuccess) {
    release();
    return grid_dev_fail(e, "hipMalloc");
  }
  double* o = out_on_device ? R_out : dout;
  e = hipMemcpyAsync(dxy, xy, (size_t)P * 2 * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = grid_pairs_launch(M, N, r, s, dxy, P, dW, dC, dT, mseg, o, st);
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(R_out, dout, obytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  release();
  if (e != hipSuccess) return grid_dev_fail(e, "grid pairs");
  return REFF_OK;
}

extern "C" reff_status reff_grid_pairs_noalloc(int32_t M, int32_t N, double r, double s,
                                               const int32_t* xy, int64_t P, double* R_out,
                                               int32_t out_on_device, void* stream) {
  using namespace reff;
  const reff_status v = grid_pairs_validate(M, N, r, s, xy, P, R_out);
  if (v != REFF_OK || P == 0) return v;
  // Layout of the work memory: points, weights, cosine table, host staging
  // of R (host output only), then as many m segments of partial Gram blocks
  // as fit, up to the count the allocating entry point uses.
  const size_t b_xy = round256((size_t)P * 2 * sizeof(int32_t));
  const size_t b_w = round256((size_t)(M - 1) * (N - 1) * sizeof(double));
  const size_t b_c = round256((size_t)P * (N - 1) * sizeof(double));
  const size_t b_o = out_on_device ? 0 : round256((size_t)P * P * sizeof(double));
  const size_t b_seg = (size_t)P * P * sizeof(double);
  const size_t fixed = b_xy + b_w + b_c + b_o;
  if (fixed + b_seg > kScratchBytes)
    return host_fail(REFF_ERR_INVALID_ARG,
                     "grid pairs without allocation: " + std::to_string(M) + " x " +
                         std::to_string(N) + " with " + std::to_string(P) + " points needs " +
                         std::to_string(fixed + b_seg) + " bytes of work memory, more than the " +
                         std::to_string(kScratchBytes) + " bytes it holds");
  const int mseg = (int)std::min<size_t>(grid_pairs_mseg(M, P), (kScratchBytes - fixed) / b_seg);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return grid_dev_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return host_fail(REFF_ERR_UNSUPPORTED, "device index too large");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return grid_dev_fail(e, "hipGetSymbolAddress(scratch)");
      g_scratch_ptr[dev] = ptr;
    }
    base = (unsigned char*)g_scratch_ptr[dev];
  }
  hipStream_t st = (hipStream_t)stream;
  int32_t* dxy = (int32_t*)base;
  double* dW = (double*)(base + b_xy);
  double* dC = (double*)(base + b_xy + b_w);
  double* dout = (double*)(base + b_xy + b_w + b_c);
  double* dT = (double*)(base + fixed);
  double* o = out_on_device ? R_out : dout;
  e = hipMemcpyAsync(dxy, xy, (size_t)P * 2 * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = grid_pairs_launch(M, N, r, s, dxy, P, dW, dC, dT, mseg, o, st);
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(R_out, dout, (size_t)P * P * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return grid_dev_fail(e, "grid pairs (no allocation)");
  return REFF_OK;
}
