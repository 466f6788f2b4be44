// gfx950 kernels of the screening model: one BF16 matrix-core GEMM that
// carries every convolution (im2col + GEMM; the 2x2 transposed convolution
// is a 1x1 GEMM into a space-to-depth layout), plus the pooling, layout,
// loss and optimiser kernels around it.  Activations are NHWC BF16 (stored
// as uint16_t), accumulation is FP32.
#include <hip/hip_runtime.h>
#include <math.h>

#include "surrogate_internal.h"

namespace reffsg {

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDT = BK + 8;

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Eight consecutive bf16 of one tile row, from global memory: one 16-byte
// load when the run is in range and 16-byte aligned, element loads (zero
// outside [0, lim)) otherwise.
__device__ __forceinline__ u4v load8(const uint16_t* __restrict__ base, int64_t first,
                                     int64_t stride, int idx0, int lim, bool vec_ok) {
  if (vec_ok && idx0 + 8 <= lim) return *reinterpret_cast<const u4v*>(base + first);
  uint16_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = idx0 + e < lim ? base[first + e * stride] : (uint16_t)0;
  return u4v{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
             (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
}

// 64 x 64 output tile (blockIdx.x along M, blockIdx.y along N, blockIdx.z
// the K slice) per 256-thread workgroup; wave w owns the 32 x 32
// quarter (w / 2, w % 2) as 2 x 2 tiles of v_mfma_f32_16x16x16bf16 (A lane
// l holds A[l%16][4(l/16) .. +3], B lane l holds B[4(l/16) .. +3][l%16],
// result row 4(l/16) + r, column l%16 in register r).  Every thread moves
// eight consecutive bf16 of A and of B per 32-wide K step with one 16-byte
// global load each; the next step's loads are in flight while the current
// step's products run, and the LDS tiles are double-buffered, so one
// barrier per step suffices.  A with unit K stride (im2col rows) lands in
// LDS as one 16-byte store; the K-strided A (weight gradients) and B are
// scattered into the transposed [n][k] layout the matrix-core operands read.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t sA[2][BM][LDT];
  __shared__ __align__(16) uint16_t sB[2][BN][LDT];  // transposed: sB[n][k]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const bool arow = g.sAk == 1;
  // this thread's slice of a K step: A row-major: row t/4, k (t%4)*8;
  // A K-strided: k t/8, rows (t%8)*8; B: k t/8, columns (t%8)*8
  const int ar = arow ? t >> 2 : (t & 7) * 8, ak = arow ? (t & 3) * 8 : t >> 3;
  const int bk = t >> 3, bn = (t & 7) * 8;
  const bool a_vec = arow ? (g.sAm % 8 == 0 && ((uintptr_t)g.A & 15) == 0)
                          : (g.sAm == 1 && g.sAk % 8 == 0 && ((uintptr_t)g.A & 15) == 0);
  const bool b_vec = g.sBk % 8 == 0 && ((uintptr_t)g.B & 15) == 0;
  auto load_step = [&](int k0, u4v& va, u4v& vb) {
    if (arow) {
      const int gm = m0 + ar;
      va = gm < g.M ? load8(g.A, (int64_t)gm * g.sAm + k0 + ak, 1, k0 + ak, kend, a_vec)
                    : u4v{0u, 0u, 0u, 0u};
    } else {
      const int gk = k0 + ak;
      va = gk < kend ? load8(g.A, (int64_t)(m0 + ar) * g.sAm + (int64_t)gk * g.sAk, g.sAm, m0 + ar,
                             g.M, a_vec)
                     : u4v{0u, 0u, 0u, 0u};
    }
    const int gk = k0 + bk;
    vb = gk < kend ? load8(g.B, (int64_t)gk * g.sBk + n0 + bn, 1, n0 + bn, g.N, b_vec)
                   : u4v{0u, 0u, 0u, 0u};
  };
  auto store_step = [&](int buf, const u4v& va, const u4v& vb) {
    if (arow) {
      *reinterpret_cast<u4v*>(&sA[buf][ar][ak]) = va;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) sA[buf][ar + e][ak] = (uint16_t)(va[e >> 1] >> (16 * (e & 1)));
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) sB[buf][bn + e][bk] = (uint16_t)(vb[e >> 1] >> (16 * (e & 1)));
  };
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  u4v va, vb;
  if (kbeg < kend) {
    load_step(kbeg, va, vb);
    store_step(0, va, vb);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load_step(k0 + BK, va, vb);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      s4v af[2], bfr[2];
      const int kc = kk + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = *reinterpret_cast<const s4v*>(&sA[buf][wm + 16 * i + (lane & 15)][kc]);
        bfr[i] = *reinterpret_cast<const s4v*>(&sB[buf][wn + 16 * i + (lane & 15)][kc]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    if (more) store_step(buf ^ 1, va, vb);
    __syncthreads();
    buf ^= 1;
  }
  const bool split = gridDim.z > 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        if (split) {
          ((float*)g.C)[(int64_t)blockIdx.z * g.M * g.ldc + (int64_t)m * g.ldc + n] = v;
          continue;
        }
        if (g.bias) v += g.bias[n];
        if (g.relu) v = fmaxf(v, 0.f);
        if (g.c_fp32)
          ((float*)g.C)[(int64_t)m * g.ldc + n] = v;
        else
          ((uint16_t*)g.C)[(int64_t)m * g.ldc + n] = f2bf(v);
      }
}

hipError_t gemm(const GemmArgs& g, int nsplit, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN, nsplit);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

__global__ void k_splitk_reduce(const float* part, int nsplit, int64_t len, float* out,
                                int accumulate) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * len + i];
    out[i] = accumulate ? out[i] + s : s;
  }
}

static int blocks_for(int64_t n, int per = 256, int cap = 16384) {
  const int64_t b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t splitk_reduce(const float* part, int nsplit, int64_t len, float* out, int accumulate,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks_for(len)), dim3(256), 0, st, part, nsplit, len,
                     out, accumulate);
  return hipGetLastError();
}

__global__ void k_im2col(const uint16_t* X, int64_t ldx, int C, int B, int H, int W, int K,
                         uint16_t* col) {
  const int KK = K * K;
  const int64_t total = (int64_t)B * H * W * KK * C;
  const int h = (K - 1) / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t q = e / C;
    const int kk = (int)(q % KK);
    const int64_t p = q / KK;
    const int x = (int)(p % W);
    const int y = (int)((p / W) % H);
    const int64_t b = p / ((int64_t)W * H);
    const int sy = y + kk / K - h, sx = x + kk % K - h;
    uint16_t v = 0;
    if (sy >= 0 && sy < H && sx >= 0 && sx < W) v = X[((b * H + sy) * W + sx) * ldx + c];
    col[e] = v;
  }
}

// The same with eight channels (16 bytes) per thread and 32-bit index
// arithmetic: for C and ldx multiples of 8, 16-byte aligned buffers and
// fewer than 2^31 groups.
__global__ void k_im2col8(const uint16_t* __restrict__ X, int ldx, int C8, int B, int H, int W,
                          int K, uint16_t* __restrict__ col) {
  const int KK = K * K;
  const int total = B * H * W * KK * C8;
  const int h = (K - 1) / 2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int cg = e % C8;
    const int q = e / C8;
    const int kk = q % KK;
    const int p = q / KK;
    const int x = p % W;
    const int py = p / W;
    const int y = py % H;
    const int b = py / H;
    const int sy = y + kk / K - h, sx = x + kk % K - h;
    u4v v = u4v{0u, 0u, 0u, 0u};
    if (sy >= 0 && sy < H && sx >= 0 && sx < W)
      v = *reinterpret_cast<const u4v*>(X + ((int64_t)(b * H + sy) * W + sx) * ldx + cg * 8);
    *reinterpret_cast<u4v*>(col + (int64_t)e * 8) = v;
  }
}

hipError_t im2col(const uint16_t* X, int64_t ldx, int C, int B, int H, int W, int K,
                  uint16_t* col, hipStream_t st) {
  const int64_t total = (int64_t)B * H * W * K * K * C;
  if (C % 8 == 0 && ldx % 8 == 0 && ldx < ((int64_t)1 << 30) && total / 8 < ((int64_t)1 << 31) &&
      ((uintptr_t)X & 15) == 0 && ((uintptr_t)col & 15) == 0) {
    hipLaunchKernelGGL(k_im2col8, dim3(blocks_for(total / 8)), dim3(256), 0, st, X, (int)ldx,
                       C / 8, B, H, W, K, col);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_im2col, dim3(blocks_for(total)), dim3(256), 0, st, X, ldx, C, B, H, W, K,
                     col);
  return hipGetLastError();
}

__global__ void k_pool_fwd(const uint16_t* X, int64_t ldx, int C, int B, int H, int W,
                           uint16_t* Y) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)B * Ho * Wo * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int x = (int)(p % Wo);
    const int y = (int)((p / Wo) % Ho);
    const int64_t b = p / ((int64_t)Wo * Ho);
    const int64_t base = (b * H + 2 * y) * W + 2 * x;
    float m = bf2f(X[base * ldx + c]);
    m = fmaxf(m, bf2f(X[(base + 1) * ldx + c]));
    m = fmaxf(m, bf2f(X[(base + W) * ldx + c]));
    m = fmaxf(m, bf2f(X[(base + W + 1) * ldx + c]));
    Y[e] = f2bf(m);
  }
}

hipError_t pool_fwd(const uint16_t* X, int64_t ldx, int C, int B, int H, int W, uint16_t* Y,
                    hipStream_t st) {
  const int64_t total = (int64_t)B * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_pool_fwd, dim3(blocks_for(total)), dim3(256), 0, st, X, ldx, C, B, H, W,
                     Y);
  return hipGetLastError();
}

__global__ void k_pool_bwd(const uint16_t* X, int64_t ldx, const uint16_t* dY, int C, int B,
                           int H, int W, uint16_t* dX) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)B * Ho * Wo * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int x = (int)(p % Wo);
    const int y = (int)((p / Wo) % Ho);
    const int64_t b = p / ((int64_t)Wo * Ho);
    const int64_t base = (b * H + 2 * y) * W + 2 * x;
    const int64_t cand[4] = {base, base + 1, base + W, base + W + 1};
    int arg = 0;
    float m = bf2f(X[cand[0] * ldx + c]);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      const float v = bf2f(X[cand[q] * ldx + c]);
      if (v > m) {
        m = v;
        arg = q;
      }
    }
    uint16_t* d = &dX[cand[arg] * ldx + c];
    *d = f2bf(bf2f(*d) + bf2f(dY[e]));
  }
}

hipError_t pool_bwd(const uint16_t* X, int64_t ldx, const uint16_t* dY, int C, int B, int H,
                    int W, uint16_t* dX, hipStream_t st) {
  const int64_t total = (int64_t)B * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for(total)), dim3(256), 0, st, X, ldx, dY, C, B, H,
                     W, dX);
  return hipGetLastError();
}

// One element per (low-res pixel, a, c, channel); forward gathers from S and
// scatters to Y, the adjoint does the reverse.
template <bool TO_Y>
__global__ void k_d2s(const uint16_t* src, uint16_t* dst, int C, int B, int H, int W,
                      int64_t ldy) {
  const int64_t total = (int64_t)B * H * W * 4 * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(e % C);
    const int64_t q = e / C;
    const int ac = (int)(q % 4);
    const int64_t p = q / 4;
    const int x = (int)(p % W);
    const int y = (int)((p / W) % H);
    const int64_t b = p / ((int64_t)W * H);
    const int a = ac >> 1, c = ac & 1;
    const int64_t py = (b * 2 * H + 2 * y + a) * (2 * W) + 2 * x + c;
    if (TO_Y)
      dst[py * ldy + ch] = src[e];
    else
      dst[e] = src[py * ldy + ch];
  }
}

hipError_t d2s(const uint16_t* S, int C, int B, int H, int W, uint16_t* Y, int64_t ldy,
               hipStream_t st) {
  const int64_t total = (int64_t)B * H * W * 4 * C;
  hipLaunchKernelGGL(k_d2s<true>, dim3(blocks_for(total)), dim3(256), 0, st, S, Y, C, B, H, W,
                     ldy);
  return hipGetLastError();
}

hipError_t s2d(const uint16_t* Y, int64_t ldy, int C, int B, int H, int W, uint16_t* S,
               hipStream_t st) {
  const int64_t total = (int64_t)B * H * W * 4 * C;
  hipLaunchKernelGGL(k_d2s<false>, dim3(blocks_for(total)), dim3(256), 0, st, Y, S, C, B, H, W,
                     ldy);
  return hipGetLastError();
}

__global__ void k_relu_bwd(uint16_t* dY, int64_t lddy, const uint16_t* Y, int64_t ldy, int C,
                           int64_t P) {
  const int64_t total = P * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    if (!(bf2f(Y[p * ldy + c]) > 0.f)) dY[p * lddy + c] = 0;
  }
}

hipError_t relu_bwd(uint16_t* dY, int64_t lddy, const uint16_t* Y, int64_t ldy, int C, int64_t P,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(P * C)), dim3(256), 0, st, dY, lddy, Y, ldy, C,
                     P);
  return hipGetLastError();
}

// Block (cx, r): channels 64 cx .. +63, rows r, r + nblk, ... ; 4 row
// groups of 64 lanes, combined in LDS.
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* dY, int64_t ld, int C, int64_t P,
                                                float* part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int grp = threadIdx.x >> 6;
  float s = 0.f;
  if (c < C)
    for (int64_t p = (int64_t)blockIdx.y * 4 + grp; p < P; p += (int64_t)gridDim.y * 4)
      s += bf2f(dY[p * ld + c]);
  red[grp][threadIdx.x & 63] = s;
  __syncthreads();
  if (grp == 0 && c < C)
    part[(int64_t)blockIdx.y * C + c] = red[0][threadIdx.x] + red[1][threadIdx.x] +
                                        red[2][threadIdx.x] + red[3][threadIdx.x];
}

hipError_t colsum(const uint16_t* dY, int64_t ld, int C, int64_t P, float* part, int nblk,
                  float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((C + 63) / 64, nblk), dim3(256), 0, st, dY, ld, C, P, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return splitk_reduce(part, nblk, C, db, 0, st);
}

__global__ void k_weight_copies(const float* W, int Cin, int Cout, int K, uint16_t* Wb,
                                uint16_t* Wt) {
  const int KK = K * K;
  const int64_t total = (int64_t)KK * Cin * Cout;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(e % Cout);
    const int64_t q = e / Cout;
    const int ci = (int)(q % Cin);
    const int kk = (int)(q / Cin);
    const uint16_t v = f2bf(W[e]);
    Wb[e] = v;
    const int kh = kk / K, kw = kk % K;
    const int kf = (K - 1 - kh) * K + (K - 1 - kw);
    Wt[((int64_t)kf * Cout + co) * Cin + ci] = v;
  }
}

hipError_t weight_copies(const float* W, int Cin, int Cout, int K, uint16_t* Wb, uint16_t* Wt,
                         hipStream_t st) {
  const int64_t total = (int64_t)K * K * Cin * Cout;
  hipLaunchKernelGGL(k_weight_copies, dim3(blocks_for(total)), dim3(256), 0, st, W, Cin, Cout, K,
                     Wb, Wt);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_masked_loss(const float* pred, int nt,
                                                     const LabelRec* lab, int n, float inv_n,
                                                     uint16_t* dpred, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const LabelRec L = lab[i];
    const int64_t at = (int64_t)L.pix * nt + L.t;
    const float d = pred[at] - L.logR;
    dpred[at] = f2bf(2.f * d * inv_n);
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

hipError_t masked_loss(const float* pred, int nt, const LabelRec* lab, int n, float inv_n,
                       uint16_t* dpred, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_masked_loss, dim3(nblk), dim3(256), 0, st, pred, nt, lab, n, inv_n, dpred,
                     part);
  return hipGetLastError();
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2,
                     eps, bc1, bc2);
  return hipGetLastError();
}

__global__ void k_fill16(uint16_t* a, int64_t n, uint16_t val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = val;
}

hipError_t fill16(uint16_t* a, int64_t n, uint16_t val, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill16, dim3(blocks_for(n)), dim3(256), 0, st, a, n, val);
  return hipGetLastError();
}

__global__ void k_predict_out(const float* pred, const uint8_t* padm, int B, int nt, int H, int W,
                              double* R) {
  const int64_t HW = (int64_t)H * W;
  const int64_t total = (int64_t)B * nt * HW;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pix = e % HW;
    const int t = (int)((e / HW) % nt);
    const int64_t b = e / (HW * nt);
    R[e] = padm[b * HW + pix] && t == 0 ? 0.0 : exp((double)pred[(b * HW + pix) * nt + t]);
  }
}

hipError_t predict_out(const float* pred, const uint8_t* padm, int B, int nt, int H, int W,
                       double* R, hipStream_t st) {
  const int64_t total = (int64_t)B * nt * H * W;
  hipLaunchKernelGGL(k_predict_out, dim3(blocks_for(total)), dim3(256), 0, st, pred, padm, B, nt,
                     H, W, R);
  return hipGetLastError();
}

}  // namespace reffsg
