// Bump-to-load pair resistances of a stack of uniformly meshed tiers by the
// paper's divide-and-conquer method (Sec. III-C, III-D):
//
//  1. intra-die resistances from the closed form of Eq. 3: TSV-TSV on every
//     tier (d x p x p), bump-TSV on tier 0 (m x p), load-TSV on the last
//     tier (n x p) -- one all-pairs evaluation per tier (grid_pairs.hip);
//  2. the reduced saddle-point system C x = b of size (p+1)(d-1): unknowns
//     are the p TSV currents of each of the d-1 tier interfaces and the d-1
//     supply-voltage differences.  With Atilde^i = -R^i_TT / 2 (TSV-TSV
//     resistances of tier i) the TSV block H is block tridiagonal: diagonal
//     block of interface a = Atilde^a + Atilde^{a+1} + diag(Rt_{., a}),
//     off-diagonal block between interfaces a and a+1 = -Atilde^{a+1}; the
//     constraint block B holds one row of ones per interface (each
//     interface carries the unit current);
//  3. C depends on neither bump nor load, so it is factorised once; each
//     bump i contributes b^1_i = [-R^1_{s_i,.}/2 in interface 0; 1_{d-1}/2]
//     and each load j b^d_j = [-R^d_{s_j,.}/2 in interface d-2; 1_{d-1}/2],
//     so that m + n solves give x^1_i, x^d_j (linearity of Sec. III-D);
//  4. R(i, j) = -(x^1_i + x^d_j)^T (b^1_i + b^d_j)
//            = -x^1_i^T b^1_i - x^d_j^T b^d_j - (x^1_i^T b^d_j + x^d_j^T b^1_i),
//     the m x n cross term as one product.
//
// C is symmetric but indefinite (a saddle point): H alone is indefinite,
// positive definite only on the currents that satisfy the constraints.
// The factorisation works on that subspace (null-space method): per
// interface the last TSV's current is eliminated, I^a = Z u^a + g_a e_p with
// Z = [I_{p-1}; -1^T], so H_Z = Z^T H Z ((p-1)(d-1) square, symmetric
// positive definite) takes a Cholesky factorisation, u = H_Z^-1 Z^T
// (f - H E g), and the voltage differences follow from the last row of each
// interface, y_a = f_(a,p-1) - (H I)_(a,p-1).  The paper decomposes C by LU
// (its Sec. IV); the answer is the same, the symmetric positive definite
// form needs no pivoting.
//
// The dense float64 work (Cholesky, triangular solves with many right-hand
// sides, the cross-term product) runs as 64 x 64 tiles on the float64
// matrix cores (v_mfma_f64_16x16x4).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "reff_internal.h"

namespace reff {
namespace {

constexpr int TB = 64;  // tile edge of the dense kernels

typedef double d4v __attribute__((ext_vector_type(4)));

// C[M x N] = alpha op(A) op(B) + beta C (float64, row-major, leading
// dimensions lda / ldb / ldc); op(A)(i, k) = ta ? A[k lda + i] : A[i lda + k],
// op(B)(k, j) = tb ? B[j ldb + k] : B[k ldb + j].  With `lower`, only tiles
// whose first row is at or below their first column are computed (the lower
// triangle of a square update).  One workgroup (four waves) per 64 x 64 tile
// of C; wave w owns rows 16 w .. 16 w + 15, as four 16 x 16 matrix-core
// accumulators; the K range is staged through LDS 16 at a time.
__global__ __launch_bounds__(256) void k_gemm64(int M, int N, int K, double alpha,
                                                const double* __restrict__ A, int64_t lda, int ta,
                                                const double* __restrict__ B, int64_t ldb, int tb,
                                                double beta, double* __restrict__ Cm, int64_t ldc,
                                                int lower) {
  const int i0 = blockIdx.y * TB, j0 = blockIdx.x * TB;
  if (lower && i0 + TB - 1 < j0) return;
  __shared__ double sA[TB][17], sB[16][TB + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int cc = lane & 15, kr = lane >> 4;
  d4v acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = d4v{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + 256 * e;   // 0 .. 1023
      // A tile: 64 rows x 16 k (k fastest for the row-major case)
      const int ar = ta ? idx % TB : idx / 16, ak = ta ? idx / TB : idx % 16;
      const int gi = i0 + ar, gk = k0 + ak;
      double va = 0.0;
      if (gi < M && gk < K) va = ta ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      sA[ar][ak] = va;
      // B tile: 16 k x 64 columns
      const int bk = tb ? idx % 16 : idx / TB, bc = tb ? idx / 16 : idx % TB;
      const int gj = j0 + bc, gk2 = k0 + bk;
      double vb = 0.0;
      if (gj < N && gk2 < K) vb = tb ? B[(int64_t)gj * ldb + gk2] : B[(int64_t)gk2 * ldb + gj];
      sB[bk][bc] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = sA[16 * w + cc][4 * ks + kr];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sB[4 * ks + kr][16 * q + cc], acc[q], 0,
                                                      0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = i0 + 16 * w + kr + 4 * r, gj = j0 + 16 * q + cc;
      if (gi < M && gj < N) {
        double* c = &Cm[(int64_t)gi * ldc + gj];
        *c = alpha * acc[q][r] + (beta != 0.0 ? beta * *c : 0.0);
      }
    }
}

// Cholesky factor of the diagonal tile kt of A (n x n, row-major, lda), in
// LDS: L_kk (written into L, zero above the diagonal) and its inverse
// (Linv[kt][64][64]).  Rows and columns past n are padded with the
// identity.  A pivot that is not positive sets *bad.
__global__ __launch_bounds__(256) void k_potrf_tile(int n, int kt, const double* __restrict__ A,
                                                    int64_t lda, double* __restrict__ L,
                                                    double* __restrict__ Linv, int* bad) {
  __shared__ double T[TB][TB + 1], X[TB][TB + 1];
  const int t = threadIdx.x, o = kt * TB;
  const int nb = min(TB, n - o);
  for (int e = t; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    T[i][j] = (i < nb && j < nb) ? A[(int64_t)(o + i) * lda + (o + j)] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < TB; ++j) {
    const double piv = T[j][j];
    __syncthreads();
    if (t == 0) {
      if (!(piv > 0.0) || !std::isfinite(piv)) atomicOr(bad, 1);
      T[j][j] = sqrt(fmax(piv, 1e-300));
    }
    __syncthreads();
    const double djj = T[j][j];
    for (int i = j + 1 + t; i < TB; i += 256) T[i][j] /= djj;
    __syncthreads();
    for (int e = t; e < TB * TB; e += 256) {
      const int i = e / TB, k = e % TB;
      if (k > j && i >= k) T[i][k] -= T[i][j] * T[k][j];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular factor, one column per thread:
  // forward substitution L X = I
  if (t < TB) {
    const int c = t;
    for (int i = 0; i < TB; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= T[i][k] * X[k][c];
      X[i][c] = (i < c) ? 0.0 : v / T[i][i];
    }
  }
  __syncthreads();
  double* Li = Linv + (size_t)kt * TB * TB;
  for (int e = t; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    Li[e] = X[i][j];
    if (i < nb && j < nb) L[(int64_t)(o + i) * lda + (o + j)] = (j <= i) ? T[i][j] : 0.0;
  }
}

// H entry between TSV k of interface b and TSV j of interface a (0-based
// interfaces a, b in [0, d-1), interface a joining tiers a and a+1):
// RT[t][j][k] = TSV-TSV resistance on tier t, rt[k][a] = segment resistance.
__device__ __forceinline__ double h_entry(const double* __restrict__ RT,
                                          const double* __restrict__ rt, int d, int p, int a,
                                          int j, int b, int k) {
  const size_t pp = (size_t)p * p;
  if (a == b) {
    double v = -0.5 * (RT[a * pp + (size_t)j * p + k] + RT[(a + 1) * pp + (size_t)j * p + k]);
    if (j == k) v += rt[(size_t)k * (d - 1) + a];
    return v;
  }
  if (b == a + 1 || a == b + 1) return 0.5 * RT[max(a, b) * pp + (size_t)j * p + k];
  return 0.0;
}

// H_Z = Z^T H Z: entry ((a, j), (b, k)), j, k < p-1, is
// H(aj, bk) - H(aj, b p-1) - H(a p-1, bk) + H(a p-1, b p-1).
__global__ __launch_bounds__(256) void k_assemble_hz(int d, int p, const double* __restrict__ RT,
                                                     const double* __restrict__ rt,
                                                     double* __restrict__ HZ) {
  const int q = p - 1, nz = q * (d - 1);
  const int64_t total = (int64_t)nz * nz;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / nz), c = (int)(e % nz);
    const int a = r / q, j = r % q, b = c / q, k = c % q;
    HZ[e] = h_entry(RT, rt, d, p, a, j, b, k) - h_entry(RT, rt, d, p, a, j, b, p - 1) -
            h_entry(RT, rt, d, p, a, p - 1, b, k) + h_entry(RT, rt, d, p, a, p - 1, b, p - 1);
  }
}

// Endpoint e (bumps first, then loads): f_e is -R_{s_e,.}/2 in interface
// 0 (bump) or d-2 (load), g_e = 1/2 per interface.  Reduced right-hand side
// rhs[(a,j)][e] = v(a,j) - v(a,p-1), v = f_e - H E g_e with
// (H E g)(a,j) = sum_b H(aj, b p-1) / 2.
__device__ __forceinline__ double f_entry(const double* __restrict__ Rs1,
                                          const double* __restrict__ Rsd, int d, int p, int m,
                                          int e, int a, int j) {
  if (e < m) return a == 0 ? -0.5 * Rs1[(size_t)e * p + j] : 0.0;
  return a == d - 2 ? -0.5 * Rsd[(size_t)(e - m) * p + j] : 0.0;
}

__global__ __launch_bounds__(256) void k_reduced_rhs(int d, int p, int m, int ne,
                                                     const double* __restrict__ RT,
                                                     const double* __restrict__ rt,
                                                     const double* __restrict__ Rs1,
                                                     const double* __restrict__ Rsd,
                                                     double* __restrict__ rhs) {
  const int q = p - 1, nz = q * (d - 1);
  const int64_t total = (int64_t)nz * ne;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(x / ne), e = (int)(x % ne);
    const int a = row / q, j = row % q;
    double hj = 0.0, hl = 0.0;
    for (int b = max(a - 1, 0); b <= min(a + 1, d - 2); ++b) {
      hj += h_entry(RT, rt, d, p, a, j, b, p - 1);
      hl += h_entry(RT, rt, d, p, a, p - 1, b, p - 1);
    }
    const double vj = f_entry(Rs1, Rsd, d, p, m, e, a, j) - 0.5 * hj;
    const double vl = f_entry(Rs1, Rsd, d, p, m, e, a, p - 1) - 0.5 * hl;
    rhs[x] = vj - vl;
  }
}

// From u (nz x ne): the TSV currents I_e (interface-major, p per
// interface; the last one is 1/2 - sum of the others), the voltage
// differences y_a = f(a,p-1) - (H I)(a,p-1), and per endpoint
//   selfv[e] = -x_e^T b_e - (sum_a y_e,a) / 2
// (the part of R(i,j) that depends on one endpoint only), plus the two
// operands of the cross term: crossA[i] = [I_i in interface d-2, f_i in
// interface 0] for bumps, crossB[j] = [f_j in interface d-2, I_j in
// interface 0] for loads, so that crossA_i . crossB_j = x_i^T b_j minus its
// y part + x_j^T b_i minus its y part.  One workgroup per endpoint.
__global__ __launch_bounds__(256) void k_reduced_post(int d, int p, int m, int ne,
                                                      const double* __restrict__ RT,
                                                      const double* __restrict__ rt,
                                                      const double* __restrict__ Rs1,
                                                      const double* __restrict__ Rsd,
                                                      const double* __restrict__ U,
                                                      double* __restrict__ Icur,
                                                      double* __restrict__ selfv,
                                                      double* __restrict__ crossA,
                                                      double* __restrict__ crossB) {
  const int e = blockIdx.x, t = threadIdx.x;
  const int q = p - 1, K = p * (d - 1);
  double* I = Icur + (size_t)e * K;
  __shared__ double red[256];
  __shared__ double ysum_s, self_s;
  // currents
  for (int a = 0; a < d - 1; ++a) {
    double s = 0.0;
    for (int j = t; j < q; j += 256) {
      const double u = U[(size_t)(a * q + j) * ne + e];
      I[a * p + j] = u;
      s += u;
    }
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) red[t] += red[t + h];
      __syncthreads();
    }
    if (t == 0) I[a * p + q] = 0.5 - red[0];
    __syncthreads();
  }
  __threadfence_block();
  __syncthreads();
  if (t == 0) ysum_s = 0.0, self_s = 0.0;
  __syncthreads();
  // y_a and the two dot products of x_e^T b_e
  for (int a = 0; a < d - 1; ++a) {
    double s = 0.0;
    for (int b = max(a - 1, 0); b <= min(a + 1, d - 2); ++b)
      for (int k = t; k < p; k += 256) s += h_entry(RT, rt, d, p, a, q, b, k) * I[b * p + k];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) red[t] += red[t + h];
      __syncthreads();
    }
    if (t == 0) {
      const double y = f_entry(Rs1, Rsd, d, p, m, e, a, q) - red[0];
      ysum_s += y;
    }
    __syncthreads();
  }
  {
    double s = 0.0;
    for (int a = 0; a < d - 1; ++a)
      for (int k = t; k < p; k += 256) s += I[a * p + k] * f_entry(Rs1, Rsd, d, p, m, e, a, k);
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) red[t] += red[t + h];
      __syncthreads();
    }
  }
  if (t == 0) {
    // x_e^T b_e = I^T f + y^T g, g = 1/2 per interface
    const double xb = red[0] + 0.5 * ysum_s;
    selfv[e] = -xb - 0.5 * ysum_s;
  }
  for (int k = t; k < p; k += 256) {
    if (e < m) {
      double* A = crossA + (size_t)e * 2 * p;
      A[k] = I[(d - 2) * p + k];
      A[p + k] = f_entry(Rs1, Rsd, d, p, m, e, 0, k);
    } else {
      double* B = crossB + (size_t)(e - m) * 2 * p;
      B[k] = f_entry(Rs1, Rsd, d, p, m, e, d - 2, k);
      B[p + k] = I[k];
    }
  }
}

// R(i, j) = selfv[i] + selfv[m + j] - G[i][j].
__global__ __launch_bounds__(256) void k_reduced_finish(int m, int n,
                                                        const double* __restrict__ selfv,
                                                        const double* __restrict__ G,
                                                        double* __restrict__ out) {
  const int64_t total = (int64_t)m * n;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(x / n), j = (int)(x % n);
    out[x] = selfv[i] + selfv[m + j] - G[x];
  }
}

dim3 rgrid(int64_t n) { return dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)); }

hipError_t gemm(hipStream_t st, int M, int N, int K, double alpha, const double* A, int64_t lda,
                int ta, const double* B, int64_t ldb, int tb, double beta, double* C, int64_t ldc,
                int lower = 0) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)((N + TB - 1) / TB), (unsigned)((M + TB - 1) / TB)),
                     dim3(256), 0, st, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, lower);
  return hipGetLastError();
}

// Device buffers of one call, released together.
struct Bufs {
  std::vector<void*> ptrs;
  ~Bufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t get(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(p);
    *out = (T*)p;
    return e;
  }
};

}  // namespace
}  // namespace reff

extern "C" reff_status reff_reduced_pairs(int32_t n_tiers, int32_t nx, int32_t ny,
                                          const double* r_t, const double* s_t, int32_t p,
                                          const int32_t* tsv_xy, const double* tsv_r, int64_t m,
                                          const int32_t* bump_xy, int64_t n,
                                          const int32_t* load_xy, double* R_out,
                                          int32_t out_on_device, void* stream) {
  using namespace reff;
  const int d = n_tiers;
  if (d < 2) return host_fail(REFF_ERR_INVALID_ARG, "the reduced system needs at least 2 tiers");
  if (nx < 1 || ny < 1) return host_fail(REFF_ERR_INVALID_ARG, "tier size must be at least 1 x 1");
  if (p < 1) return host_fail(REFF_ERR_INVALID_ARG, "at least one TSV column is needed");
  if (m < 0 || n < 0) return host_fail(REFF_ERR_INVALID_ARG, "negative bump or load count");
  if (!r_t || !s_t || !tsv_xy || !tsv_r)
    return host_fail(REFF_ERR_INVALID_ARG, "NULL tier or TSV array");
  if (m * n == 0) return REFF_OK;
  if (!bump_xy || !load_xy || !R_out) return host_fail(REFF_ERR_INVALID_ARG, "NULL bump, load or output");
  for (int t = 0; t < d; ++t)
    if (!std::isfinite(r_t[t]) || !(r_t[t] > 0.0) || !std::isfinite(s_t[t]) || !(s_t[t] > 0.0))
      return host_fail(REFF_ERR_INVALID_ARG, "tier edge resistances must be finite and positive");
  for (int64_t k = 0; k < (int64_t)p * (d - 1); ++k)
    if (!std::isfinite(tsv_r[k]) || !(tsv_r[k] > 0.0))
      return host_fail(REFF_ERR_INVALID_ARG, "TSV segment resistances must be finite and positive");
  auto on_grid = [&](const int32_t* xy, int64_t cnt) {
    for (int64_t k = 0; k < cnt; ++k)
      if (xy[2 * k] < 0 || xy[2 * k] >= nx || xy[2 * k + 1] < 0 || xy[2 * k + 1] >= ny) return false;
    return true;
  };
  if (!on_grid(tsv_xy, p) || !on_grid(bump_xy, m) || !on_grid(load_xy, n))
    return host_fail(REFF_ERR_INVALID_ARG, "a TSV, bump or load is off the tier grid");
  {
    std::vector<int64_t> ids(p);
    for (int k = 0; k < p; ++k) ids[k] = (int64_t)tsv_xy[2 * k + 1] * nx + tsv_xy[2 * k];
    std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
      return host_fail(REFF_ERR_INVALID_ARG, "duplicate TSV column");
  }
  const int64_t P0 = p + m, Pd = p + n;
  if (P0 > 65535 || Pd > 65535)
    return host_fail(REFF_ERR_INVALID_ARG, "at most 65535 TSVs plus bumps (or loads) per call");
  hipStream_t st = (hipStream_t)stream;
  auto dev_fail = [&](hipError_t e, const char* what) {
    return host_fail(e == hipErrorOutOfMemory ? REFF_ERR_OUT_OF_MEMORY : REFF_ERR_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
  };
  const int q = p - 1, nz = q * (d - 1), ne = (int)(m + n);
  const int ntile = (nz + TB - 1) / TB;
  Bufs bufs;
  int32_t* dxy = nullptr;
  double *dR = nullptr, *RT = nullptr, *rt = nullptr, *Rs1 = nullptr, *Rsd = nullptr;
  double *HZ = nullptr, *L = nullptr, *Linv = nullptr, *rhs = nullptr, *Y = nullptr;
  double *Icur = nullptr, *selfv = nullptr, *cA = nullptr, *cB = nullptr, *G = nullptr;
  double* dout = nullptr;
  int* bad = nullptr;
  hipError_t e = bufs.get(&dxy, 2 * (size_t)std::max(P0, Pd));
  if (e == hipSuccess) e = bufs.get(&dR, (size_t)std::max(P0, Pd) * std::max(P0, Pd));
  if (e == hipSuccess) e = bufs.get(&RT, (size_t)d * p * p);
  if (e == hipSuccess) e = bufs.get(&rt, (size_t)p * (d - 1));
  if (e == hipSuccess) e = bufs.get(&Rs1, (size_t)m * p);
  if (e == hipSuccess) e = bufs.get(&Rsd, (size_t)n * p);
  if (e == hipSuccess) e = bufs.get(&HZ, (size_t)nz * nz);
  if (e == hipSuccess) e = bufs.get(&L, (size_t)nz * nz);
  if (e == hipSuccess) e = bufs.get(&Linv, (size_t)ntile * TB * TB);
  if (e == hipSuccess) e = bufs.get(&rhs, (size_t)nz * ne);
  if (e == hipSuccess) e = bufs.get(&Y, (size_t)nz * ne);
  if (e == hipSuccess) e = bufs.get(&Icur, (size_t)ne * p * (d - 1));
  if (e == hipSuccess) e = bufs.get(&selfv, (size_t)ne);
  if (e == hipSuccess) e = bufs.get(&cA, (size_t)m * 2 * p);
  if (e == hipSuccess) e = bufs.get(&cB, (size_t)n * 2 * p);
  if (e == hipSuccess) e = bufs.get(&G, (size_t)m * n);
  if (e == hipSuccess) e = bufs.get(&bad, 1);
  if (e == hipSuccess && !out_on_device) e = bufs.get(&dout, (size_t)m * n);
  if (e != hipSuccess) return dev_fail(e, "hipMalloc");
  double* out = out_on_device ? R_out : dout;
  e = hipMemsetAsync(bad, 0, sizeof(int), st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rt, tsv_r, sizeof(double) * p * (d - 1), hipMemcpyHostToDevice, st);
  // 1. intra-die resistances, tier by tier: TSVs first, then the tier's
  //    bumps (tier 0) or loads (last tier)
  std::vector<int32_t> pts;
  for (int t = 0; t < d && e == hipSuccess; ++t) {
    pts.assign(tsv_xy, tsv_xy + 2 * (size_t)p);
    int64_t extra = 0;
    if (t == 0) pts.insert(pts.end(), bump_xy, bump_xy + 2 * m), extra = m;
    if (t == d - 1) pts.insert(pts.end(), load_xy, load_xy + 2 * n), extra = n;
    const int64_t P = p + extra;
    e = hipMemcpyAsync(dxy, pts.data(), sizeof(int32_t) * 2 * P, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = grid_pairs_device(nx, ny, r_t[t], s_t[t], dxy, P, dR, st);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(RT + (size_t)t * p * p, sizeof(double) * p, dR, sizeof(double) * P,
                           sizeof(double) * p, p, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && extra > 0)
      e = hipMemcpy2DAsync(t == 0 ? Rs1 : Rsd, sizeof(double) * p, dR + (size_t)p * P,
                           sizeof(double) * P, sizeof(double) * p, extra,
                           hipMemcpyDeviceToDevice, st);
    // the staged points are read by the next tier's upload only after
    // this tier's kernels have run
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  // 2.-3. H_Z, its Cholesky factor, and the reduced solves for all endpoints
  if (e == hipSuccess && nz > 0) {
    hipLaunchKernelGGL(k_assemble_hz, rgrid((int64_t)nz * nz), dim3(256), 0, st, d, p,
                       (const double*)RT, (const double*)rt, HZ);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_reduced_rhs, rgrid((int64_t)nz * ne), dim3(256), 0, st, d, p,
                         (int)m, ne, (const double*)RT, (const double*)rt, (const double*)Rs1,
                         (const double*)Rsd, rhs);
      e = hipGetLastError();
    }
    for (int kt = 0; kt < ntile && e == hipSuccess; ++kt) {
      const int o = kt * TB, nb = std::min(TB, nz - o), rest = nz - o - nb;
      hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, st, nz, kt, (const double*)HZ,
                         (int64_t)nz, L, Linv, bad);
      e = hipGetLastError();
      // panel: L(rest, k) = A(rest, k) L_kk^-T
      if (e == hipSuccess && rest > 0)
        e = gemm(st, rest, nb, nb, 1.0, HZ + (size_t)(o + nb) * nz + o, nz, 0,
                 Linv + (size_t)kt * TB * TB, TB, 1, 0.0, L + (size_t)(o + nb) * nz + o, nz);
      // trailing update (lower tiles): A(rest, rest) -= L(rest, k) L(rest, k)^T
      if (e == hipSuccess && rest > 0)
        e = gemm(st, rest, rest, nb, -1.0, L + (size_t)(o + nb) * nz + o, nz, 0,
                 L + (size_t)(o + nb) * nz + o, nz, 1, 1.0, HZ + (size_t)(o + nb) * nz + o + nb, nz,
                 1);
    }
    // forward: L Y = rhs (rhs is consumed), tile row by tile row
    for (int kt = 0; kt < ntile && e == hipSuccess; ++kt) {
      const int o = kt * TB, nb = std::min(TB, nz - o), rest = nz - o - nb;
      e = gemm(st, nb, ne, nb, 1.0, Linv + (size_t)kt * TB * TB, TB, 0, rhs + (size_t)o * ne, ne,
               0, 0.0, Y + (size_t)o * ne, ne);
      if (e == hipSuccess && rest > 0)
        e = gemm(st, rest, ne, nb, -1.0, L + (size_t)(o + nb) * nz + o, nz, 0,
                 Y + (size_t)o * ne, ne, 0, 1.0, rhs + (size_t)(o + nb) * ne, ne);
    }
    // backward: L^T U = Y (U written into rhs), last tile row first
    for (int kt = ntile - 1; kt >= 0 && e == hipSuccess; --kt) {
      const int o = kt * TB, nb = std::min(TB, nz - o);
      e = gemm(st, nb, ne, nb, 1.0, Linv + (size_t)kt * TB * TB, TB, 1, Y + (size_t)o * ne, ne, 0,
               0.0, rhs + (size_t)o * ne, ne);
      if (e == hipSuccess && o > 0)
        e = gemm(st, o, ne, nb, -1.0, L + (size_t)o * nz, nz, 1, rhs + (size_t)o * ne, ne, 0, 1.0,
                 Y, ne);
    }
  }
  // 4. currents, voltage differences, self terms, cross-term operands
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_reduced_post, dim3((unsigned)ne), dim3(256), 0, st, d, p, (int)m, ne,
                       (const double*)RT, (const double*)rt, (const double*)Rs1,
                       (const double*)Rsd, (const double*)rhs, Icur, selfv, cA, cB);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm(st, (int)m, (int)n, 2 * p, 1.0, cA, 2 * p, 0, cB, 2 * p, 1, 0.0, G, n);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_reduced_finish, rgrid(m * n), dim3(256), 0, st, (int)m, (int)n,
                       (const double*)selfv, (const double*)G, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(R_out, dout, sizeof(double) * m * n, hipMemcpyDeviceToHost, st);
  int hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return dev_fail(e, "reduced pairs");
  if (hbad)
    return host_fail(REFF_ERR_DEVICE,
                     "reduced system: a Cholesky pivot of Z^T H Z was not positive");
  return REFF_OK;
}
