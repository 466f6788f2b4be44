// Full maps R_i = (G^-1)_ii by sparse-direct selected inversion.
//
// Block PCG pays one block solve per 64 nodes; a full map of a large stack
// needs every diagonal entry of G^-1, which a sparse Cholesky factorisation
// and the Takahashi recurrence give at the cost of a few factorisations.
// The symbolic part (nested dissection of the stacked grid, fronts, maps)
// is host code (selinv_plan.cpp); everything numeric runs here, in float64,
// level by level of the dissection tree (all fronts of one depth together).
//
// Factorisation (deepest level first): each front is a dense F x F
// column-major block over [pivots, update set Q].  It is cleared, receives
// the entries of G in its pivot columns, and the update matrices of its
// children (extend-add, children of rank 0 then 1, so no two writers meet).
// Its k pivot columns are then factored 64 at a time, right-looking:
//   L_jj = chol(A_jj), L_Rj = A_Rj L_jj^-T, A_RR -= L_Rj L_Rj^T  (lower),
// where R is every front row after the panel; after the last panel the
// trailing Q x Q block is the update matrix passed to the parent.
//
// Selected inversion (roots first; Z = G^-1): a front first gathers Z_QQ
// from its parent's finished block, then takes its panels last to first.
// For a panel P with the rows R after it (the later pivots of the front and
// Q, all of whose Z entries are known by then):
//   Lhat = L_RP L_PP^-1,  Z_RP = -Z_RR Lhat,
//   Z_PP = L_PP^-T L_PP^-1 - Lhat^T Z_RP,
// the block form of the Takahashi identities (L^T Z = L^-1, whose upper
// part is known and whose lower part is the identity's inverse on the
// diagonal), written over Z_RP / Z_PR / Z_PP in place.  The dense front
// makes the structure of every column the whole of R, so the supernodal
// block form applies to any panel split.  diag(Z_PP) is R_i for the panel's
// nodes.
//
// The dense work is 64 x 64 output tiles on the float64 matrix cores
// (v_mfma_f64_16x16x4); tiles of all fronts of a level share one launch
// (grid.y walks the fronts).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "reff_internal.h"
#include "selinv_plan.h"

namespace reff {
namespace {

constexpr int PT = 64;  // panel width and output tile edge
constexpr int LEAF_AREA = 16;
constexpr unsigned MAX_GY = 65535;

typedef double d4v __attribute__((ext_vector_type(4)));

// Device copy of a front (see SnFront), plus its per-level scratch slots.
struct DFront {
  int64_t off;   // arena offset of the F x F block
  int64_t poff;  // parent's arena offset, -1 at a root
  int64_t rel;   // into rel[]: F - k parent positions of Q
  int64_t piv;   // into piv_node[]: k node ids
  int64_t ybuf;  // offset of its F x 64 block in the level's Y buffer
  int64_t part;  // offset of its nsplit x 64 x 64 partial products
  int32_t F, k, pF, rank, nsplit, pad_;
};

constexpr int KS = 32;  // K slice staged through LDS

// C(i, j) = alpha sum_{kk in [kb, ke)} A(i, kk) B(kk, j) [+ beta C(i, j)] on the
// 64 x 64 tile at (i0, j0) of an M x N column-major C (ldc).
//   A(i, kk) = ta ? A[i lda + kk] : A[kk lda + i]
//   B(kk, j) = tb ? B[kk ldb + j] : B[j ldb + kk]
// With `lower`, entries above the diagonal are not written.  Four waves;
// wave w owns tile rows 16 w .. 16 w + 15 as four 16 x 16 accumulators.
// K goes through LDS 32 at a time, the next slice's loads in flight (in
// registers) while the matrix cores work on the current one.  The whole K
// range is read before the tile is written, so C may alias the rows of A
// it covers.
__device__ __forceinline__ void gemm_tile(int i0, int j0, int M, int N, int kb, int ke,
                                          double alpha, const double* A, int64_t lda, bool ta,
                                          const double* B, int64_t ldb, bool tb, double beta,
                                          double* C, int64_t ldc, bool lower,
                                          double (*sA)[KS + 1], double (*sB)[PT + 1]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int cc = lane & 15, kr = lane >> 4;
  d4v acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = d4v{0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;  // 0 .. 2047
      const int ai = ta ? idx >> 5 : idx & 63, ak = ta ? idx & 31 : idx >> 6;
      const int gi = i0 + ai, gk = k0 + ak;
      ra[e] = (gi < M && gk < ke) ? (ta ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi])
                                  : 0.0;
      const int bj = tb ? idx & 63 : idx >> 5, bk = tb ? idx >> 6 : idx & 31;
      const int gj = j0 + bj, gk2 = k0 + bk;
      rb[e] = (gj < N && gk2 < ke) ? (tb ? B[(int64_t)gk2 * ldb + gj] : B[(int64_t)gj * ldb + gk2])
                                   : 0.0;
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KS) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      sA[ta ? idx >> 5 : idx & 63][ta ? idx & 31 : idx >> 6] = ra[e];
      sB[tb ? idx >> 6 : idx & 31][tb ? idx & 63 : idx >> 5] = rb[e];
    }
    __syncthreads();
    if (k0 + KS < ke) load(k0 + KS);
#pragma unroll
    for (int ks = 0; ks < KS / 4; ++ks) {
      const double av = sA[16 * w + cc][4 * ks + kr];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sB[4 * ks + kr][16 * q + cc], acc[q],
                                                      0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = i0 + 16 * w + kr + 4 * r, gj = j0 + 16 * q + cc;
      if (gi < M && gj < N && (!lower || gi >= gj)) {
        double* c = &C[(int64_t)gj * ldc + gi];
        *c = alpha * acc[q][r] + (beta != 0.0 ? beta * *c : 0.0);
      }
    }
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Entries of G into the cleared fronts (each position occurs once).
__global__ void k_scatter(const int64_t* __restrict__ idx, const double* __restrict__ val,
                          int64_t n, double* __restrict__ ar) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    ar[idx[e]] = val[e];
}

// Extend-add: the lower triangle of each rank-`rank` child's update matrix
// (its trailing (F-k) x (F-k) block) into its parent at rel x rel.  One wave
// per column b of the update matrix (four per workgroup, blockIdx.x walks
// the columns), its lanes down the rows a >= b: the child's column is read
// contiguously and the parent's rows rel[a] are increasing.
__global__ __launch_bounds__(256) void k_extend_add(const DFront* __restrict__ fr,
                                                    const int32_t* __restrict__ list, int nf,
                                                    int rank, const int32_t* __restrict__ rel,
                                                    double* ar) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
    const DFront f = fr[list[fi]];
    if (f.poff < 0 || f.rank != rank) continue;
    const int q = f.F - f.k;
    const int32_t* rl = rel + f.rel;
    for (int b = blockIdx.x * 4 + w; b < q; b += gridDim.x * 4) {
      const double* src = ar + f.off + (int64_t)(f.k + b) * f.F + f.k;
      double* dst = ar + f.poff + (int64_t)rl[b] * f.pF;
      for (int a = b + lane; a < q; a += 64) dst[rl[a]] += src[a];
    }
  }
}

// Z_QQ of each front (full square) from its parent's finished block; one
// wave per column as in k_extend_add.
__global__ __launch_bounds__(256) void k_gather(const DFront* __restrict__ fr,
                                                const int32_t* __restrict__ list, int nf,
                                                const int32_t* __restrict__ rel, double* ar) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
    const DFront f = fr[list[fi]];
    if (f.poff < 0) continue;
    const int q = f.F - f.k;
    const int32_t* rl = rel + f.rel;
    for (int b = blockIdx.x * 4 + w; b < q; b += gridDim.x * 4) {
      double* dst = ar + f.off + (int64_t)(f.k + b) * f.F + f.k;
      const double* src = ar + f.poff + (int64_t)rl[b] * f.pF;
      for (int a = lane; a < q; a += 64) dst[a] = src[rl[a]];
    }
  }
}

// Diagonal tile of panel jp of every front.  FACTOR: Cholesky of A_jj in
// place (lower) and L_jj^-1 into Li; a pivot that is not positive sets
// *bad.  Otherwise (selected inversion): L_jj^-1 into Li and
// L_jj^-T L_jj^-1 into Z0.  Li, Z0: 64 x 64 column-major per list slot,
// identity-padded past the panel width.
//
// The tile lives in registers: lane r of wave g holds row r of columns
// g, g+4, .., g+60 (Cholesky), then column r of rows g, g+4, .. of the
// inverse (forward elimination); one LDS tile holds L for the elimination
// and then the inverse.  Each of the 64 steps publishes one
// column (one row) through a double-buffered LDS vector, so a step costs
// one barrier, a few LDS broadcasts and 16 fused multiply-adds per lane.
template <bool FACTOR>
__global__ __launch_bounds__(256) void k_tile(const DFront* __restrict__ fr,
                                              const int32_t* __restrict__ list, int nf, int jp,
                                              double* ar, double* __restrict__ Li,
                                              double* __restrict__ Z0, int* bad) {
  __shared__ double T[PT][PT + 1];  // the tile, then its inverse
  __shared__ double buf[2][PT];
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  for (int fi = blockIdx.x; fi < nf; fi += gridDim.x) {
    const DFront f = fr[list[fi]];
    const int j0 = PT * jp;
    if (f.k <= j0) continue;
    const int w = min(PT, f.k - j0);
    double* a = ar + f.off + (int64_t)j0 * f.F + j0;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int cc = g + 4 * j;
      v[j] = (r < w && cc < w) ? (r >= cc ? a[(int64_t)cc * f.F + r] : 0.0) : (r == cc ? 1.0 : 0.0);
    }
    __syncthreads();  // the previous front's LDS reads are done
    if (FACTOR) {
#pragma unroll
      for (int c = 0; c < PT; ++c) {
        if (c >= w) break;  // the rest of the tile is identity padding
        double* bf = buf[c & 1];
        if (g == (c & 3)) bf[r] = v[c >> 2];
        __syncthreads();
        const double piv = bf[c];
        if (t == 0 && !(piv > 0.0 && std::isfinite(piv))) atomicOr(bad, 1);
        const double sq = sqrt(fmax(piv, 1e-300)), inv = 1.0 / sq;
        const double lr = bf[r] * inv;
        if (g == (c & 3)) v[c >> 2] = r > c ? lr : (r == c ? sq : 0.0);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int cc = g + 4 * j;
          if (cc > c && r >= cc) v[j] -= lr * (bf[cc] * inv);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int cc = g + 4 * j;
        if (r < w && cc < w && r >= cc) a[(int64_t)cc * f.F + r] = v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) T[r][g + 4 * j] = v[j];
    __syncthreads();
    // X = L^-1: lane r holds column r of rows g + 4 j
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = (g + 4 * j == r) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      if (k >= w) break;  // rows past the panel width keep the identity
      double* bk = buf[k & 1];
      if (g == (k & 3)) {
        v[k >> 2] /= T[k][k];
        bk[r] = v[k >> 2];
      }
      __syncthreads();
      const double xk = bk[r];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = g + 4 * j;
        if (i > k) v[j] -= T[i][k] * xk;
      }
    }
    __syncthreads();  // every step's reads of L are done
#pragma unroll
    for (int j = 0; j < 16; ++j) T[g + 4 * j][r] = v[j];
    __syncthreads();
    double* li = Li + (size_t)fi * PT * PT;
    for (int e = t; e < PT * PT; e += 256) li[e] = T[e & 63][e >> 6];
    if (!FACTOR) {
      // Z0(r, b) = sum_k X(k, r) X(k, b), b = g + 4 j
      double z[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) z[j] = 0.0;
      for (int k = 0; k < w; ++k) {  // the inverse is block diagonal past w
        const double xr = T[k][r];
#pragma unroll
        for (int j = 0; j < 16; ++j) z[j] += xr * T[k][g + 4 * j];
      }
      double* z0 = Z0 + (size_t)fi * PT * PT;
#pragma unroll
      for (int j = 0; j < 16; ++j) z0[(g + 4 * j) * PT + r] = z[j];
    }
  }
}

enum GemmOp { OP_TRSM = 0, OP_SYRK = 1, OP_LHAT = 2, OP_Y = 3, OP_PART = 4 };

__device__ __forceinline__ void lower_tile(int t, int& ti, int& tj) {
  ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  tj = t - ti * (ti + 1) / 2;
}

// The panel products of step jp for every front of a level (see the file
// comment); blockIdx.x is the tile (or, for OP_PART, the K split).
template <int OP>
__global__ __launch_bounds__(256) void k_front_gemm(const DFront* __restrict__ fr,
                                                    const int32_t* __restrict__ list, int nf,
                                                    int jp, double* ar,
                                                    const double* __restrict__ Li,
                                                    double* __restrict__ Ybuf,
                                                    double* __restrict__ part, int tiles,
                                                    int ysplit, double* __restrict__ Ysp,
                                                    int64_t ylev) {
  __shared__ double sA[PT][KS + 1], sB[KS][PT + 1];
  for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
    const DFront f = fr[list[fi]];
    const int j0 = PT * jp;
    if (f.k <= j0) continue;
    const int w = min(PT, f.k - j0), r0 = j0 + w, m = f.F - r0;
    const int64_t F = f.F;
    double* base = ar + f.off;
    const double* li = Li + (size_t)fi * PT * PT;
    const int ntile = (m + PT - 1) / PT;
    if (OP == OP_TRSM || OP == OP_LHAT) {
      // rows R of the panel, in place: times L_jj^-T (factor) or L_jj^-1
      if ((int)blockIdx.x >= ntile) continue;
      double* c = base + (int64_t)j0 * F + r0;
      gemm_tile(blockIdx.x * PT, 0, m, w, 0, w, 1.0, c, F, false, li, PT, OP == OP_TRSM, 0.0, c,
                F, false, sA, sB);
    } else if (OP == OP_SYRK) {
      if ((int)blockIdx.x >= ntile * (ntile + 1) / 2) continue;
      int ti, tj;
      lower_tile(blockIdx.x, ti, tj);
      const double* l = base + (int64_t)j0 * F + r0;
      gemm_tile(ti * PT, tj * PT, m, m, 0, w, -1.0, l, F, false, l, F, true, 1.0,
                base + (int64_t)r0 * F + r0, F, true, sA, sB);
    } else if (OP == OP_Y) {
      // Y = -Z_RR Lhat; with ysplit > 1, the K range in ysplit parts, each
      // into its own copy of the level's Y buffer (summed by k_ysum)
      const int tile = (int)blockIdx.x % tiles, sp = (int)blockIdx.x / tiles;
      if (tile >= ntile) continue;
      int kb = 0, ke = m;
      double* y = Ybuf + f.ybuf;
      if (ysplit > 1) {
        const int ks = ((m + ysplit - 1) / ysplit + KS - 1) / KS * KS;
        kb = min(m, sp * ks);
        ke = min(m, kb + ks);
        y = Ysp + (size_t)sp * ylev + f.ybuf;
      }
      gemm_tile(tile * PT, 0, m, w, kb, ke, -1.0, base + (int64_t)r0 * F + r0, F, false,
                base + (int64_t)j0 * F + r0, F, false, 0.0, y, F, false, sA, sB);
    } else {
      // partial -Lhat^T Y over split blockIdx.x of the rows R
      if ((int)blockIdx.x >= f.nsplit) continue;
      const int ks = (m + f.nsplit - 1) / f.nsplit;
      const int kb = min(m, (int)blockIdx.x * ks), ke = min(m, kb + ks);
      gemm_tile(0, 0, w, w, kb, ke, -1.0, base + (int64_t)j0 * F + r0, F, true, Ybuf + f.ybuf, F,
                false, 0.0, part + f.part + (size_t)blockIdx.x * PT * PT, PT, false, sA, sB);
    }
  }
}

// Y = sum of the ysplit partial products (rows of row tile blockIdx.x).
__global__ __launch_bounds__(256) void k_ysum(const DFront* __restrict__ fr,
                                              const int32_t* __restrict__ list, int nf, int jp,
                                              int ysplit, const double* __restrict__ Ysp,
                                              int64_t ylev, double* __restrict__ Ybuf) {
  for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
    const DFront f = fr[list[fi]];
    const int j0 = PT * jp;
    if (f.k <= j0) continue;
    const int w = min(PT, f.k - j0), m = f.F - j0 - w;
    const int i0 = blockIdx.x * PT;
    if (i0 >= m) continue;
    for (int e = threadIdx.x; e < PT * PT; e += 256) {
      const int c = e >> 6, i = i0 + (e & 63);
      if (i >= m || c >= w) continue;
      const int64_t o = f.ybuf + (int64_t)c * f.F + i;
      double v = 0.0;
      for (int s = 0; s < ysplit; ++s) v += Ysp[(size_t)s * ylev + o];
      Ybuf[o] = v;
    }
  }
}

// End of a selected-inversion panel step: Z_PP = Z0 + sum of the partials
// (blockIdx.x == 0, also writing diag(Z_PP) to Rfull), and Z_RP = Y,
// Z_PR = Y^T (blockIdx.x = 1 + row tile).
__global__ __launch_bounds__(256) void k_finish(const DFront* __restrict__ fr,
                                                const int32_t* __restrict__ list, int nf, int jp,
                                                double* ar, const double* __restrict__ Z0,
                                                const double* __restrict__ Ybuf,
                                                const double* __restrict__ part,
                                                const int64_t* __restrict__ piv_node,
                                                double* __restrict__ Rfull) {
  __shared__ double Ts[PT][PT + 1];
  const int t = threadIdx.x;
  for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
    const DFront f = fr[list[fi]];
    const int j0 = PT * jp;
    if (f.k <= j0) continue;
    const int w = min(PT, f.k - j0), r0 = j0 + w, m = f.F - r0;
    const int64_t F = f.F;
    double* base = ar + f.off;
    if (blockIdx.x == 0) {
      const double* z0 = Z0 + (size_t)fi * PT * PT;
      const int ns = m > 0 ? f.nsplit : 0;
      for (int e = t; e < PT * PT; e += 256) {
        const int c = e >> 6, r = e & 63;
        if (r >= w || c >= w) continue;
        double v = z0[e];
        for (int s = 0; s < ns; ++s) v += part[f.part + (size_t)s * PT * PT + e];
        base[(int64_t)(j0 + c) * F + j0 + r] = v;
        if (r == c) Rfull[piv_node[f.piv + j0 + r]] = v;
      }
      continue;
    }
    const int rt = (int)blockIdx.x - 1;
    if (rt * PT >= m) continue;
    const int rows = min(PT, m - rt * PT);
    const double* y = Ybuf + f.ybuf + rt * PT;
    __syncthreads();
    for (int e = t; e < PT * PT; e += 256) {
      const int c = e >> 6, r = e & 63;
      if (r < rows && c < w) {
        const double v = y[(int64_t)c * F + r];
        base[(int64_t)(j0 + c) * F + r0 + rt * PT + r] = v;  // Z_RP
        Ts[c][r] = v;
      }
    }
    __syncthreads();
    for (int e = t; e < PT * PT; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (r < rows && c < w) base[(int64_t)(r0 + rt * PT + r) * F + j0 + c] = Ts[c][r];  // Z_PR
    }
  }
}

__global__ void k_pick(const double* __restrict__ Rfull, const int64_t* __restrict__ nodes,
                       int64_t n, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = Rfull[nodes[i]];
}

dim3 flat(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192))); }

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

template <typename T>
hipError_t put(Bufs& b, T** out, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = b.get(out, v.size());
  if (e == hipSuccess && !v.empty())
    e = hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
  return e;
}

// The fronts of a level are launched in groups of at most GROUP fronts, so
// that the per-front scratch of a panel step (tile inverses, Y blocks,
// partial products) is sized by a group, not by a level of a large forest.
constexpr size_t GROUP = 16384;

// One launch group: a contiguous range of a level's front list.
struct GroupDev {
  int64_t list_off = 0;  // into the device front lists
  int nf = 0;
  int max_panels = 0;
  int ysplit = 1;        // K parts of the Y product
  int64_t ylev = 0;      // doubles of the group's Y buffer
  int64_t part = 0;      // doubles of its partial products
  int64_t maxq = 0;      // largest update set
  std::vector<int> mt, ms;  // per panel: row tiles after it, K parts of its partials
};

struct LevelDev {
  int64_t ent_off = 0, ent_n = 0;
  int nf = 0;
  std::vector<GroupDev> groups;
};

reff_status dev_status(hipError_t e, const char* what) {
  return host_fail(e == hipErrorOutOfMemory ? REFF_ERR_OUT_OF_MEMORY : REFF_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

std::shared_ptr<SelinvPlan> selinv_plan_of(reff_pdn_t* p, reff_status& s) {
  s = REFF_OK;
  if (p->sel_plan) return p->sel_plan;
  auto plan = std::make_shared<SelinvPlan>();
  std::string err;
  if (!build_selinv_plan(p->nt, p->nx, p->ny, p->gx.data(), p->gy.data(),
                         (int32_t)(p->tsv_xy.size() / 2), p->tsv_xy.data(), p->tsv_g.data(),
                         (int32_t)(p->pad_xy.size() / 2), p->pad_xy.data(), LEAF_AREA, *plan,
                         err)) {
    s = host_fail(REFF_ERR_DEVICE, "selected inversion plan: " + err);
    return nullptr;
  }
  p->sel_plan = plan;
  return plan;
}

// Parts the K range of a group's Y products is split into: enough
// workgroups to fill the chip where a group has few fronts, at least 128
// rows of K per part, and at most 1 GiB of partial products.
int group_ysplit(const SelinvPlan& P, const int32_t* fronts, size_t nf, int64_t yb) {
  int64_t tiles0 = 0, maxm = 0;
  for (size_t j = 0; j < nf; ++j) {
    const SnFront& f = P.fronts[(size_t)fronts[j]];
    if (f.k == 0) continue;
    const int64_t m0 = f.F - std::min(PT, f.k);
    tiles0 += (m0 + PT - 1) / PT;
    maxm = std::max(maxm, m0);
  }
  if (tiles0 == 0) return 1;
  int64_t sp = std::min<int64_t>((2048 + tiles0 - 1) / tiles0, 16);
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, maxm / 128));
  while (sp > 1 && sp * yb > ((int64_t)1 << 27)) --sp;
  return (int)std::max<int64_t>(1, sp);
}

int front_nsplit(const SnFront& f) { return std::min(16, std::max(1, (f.F + 255) / 256)); }

// The launch groups of every level, with their scratch sizes.
std::vector<std::vector<GroupDev>> plan_groups(const SelinvPlan& P) {
  std::vector<std::vector<GroupDev>> out(P.levels.size());
  for (size_t d = 0; d < P.levels.size(); ++d) {
    const SelinvLevel& L = P.levels[d];
    for (size_t b = 0; b < L.fronts.size(); b += GROUP) {
      GroupDev g;
      g.list_off = (int64_t)b;  // within the level; made absolute by the device build
      g.nf = (int)std::min(GROUP, L.fronts.size() - b);
      for (int j = 0; j < g.nf; ++j) {
        const SnFront& f = P.fronts[(size_t)L.fronts[b + (size_t)j]];
        g.max_panels = std::max(g.max_panels, (f.k + PT - 1) / PT);
        g.ylev += (int64_t)f.F * PT;
        g.part += (int64_t)front_nsplit(f) * PT * PT;
        g.maxq = std::max<int64_t>(g.maxq, (int64_t)(f.F - f.k));
      }
      g.mt.assign((size_t)g.max_panels, 0);
      g.ms.assign((size_t)g.max_panels, 0);
      for (int j = 0; j < g.nf; ++j) {
        const SnFront& f = P.fronts[(size_t)L.fronts[b + (size_t)j]];
        for (int jp = 0; PT * jp < f.k; ++jp) {
          const int m = f.F - PT * jp - std::min(PT, f.k - PT * jp);
          g.mt[(size_t)jp] = std::max(g.mt[(size_t)jp], (m + PT - 1) / PT);
          g.ms[(size_t)jp] = std::max(g.ms[(size_t)jp], front_nsplit(f));
        }
      }
      g.ysplit = group_ysplit(P, L.fronts.data() + b, (size_t)g.nf, g.ylev);
      out[d].push_back(std::move(g));
    }
  }
  return out;
}

// Scratch sizes of a plan on the device, in doubles / bytes.
struct SelinvSizes {
  int64_t tiles = 0, ybuf = 0, part = 0, ysp = 0;
  int64_t bytes = 0;
};

SelinvSizes selinv_sizes(const SelinvPlan& P) {
  SelinvSizes z;
  for (const auto& lev : plan_groups(P))
    for (const GroupDev& g : lev) {
      z.tiles = std::max<int64_t>(z.tiles, (int64_t)g.nf * PT * PT);
      z.ybuf = std::max(z.ybuf, g.ylev);
      z.part = std::max(z.part, g.part);
      if (g.ysplit > 1) z.ysp = std::max(z.ysp, g.ysplit * g.ylev);
    }
  int64_t ent = 0;
  for (const SelinvLevel& L : P.levels) ent += (int64_t)L.ent_idx.size();
  z.bytes = 8 * (P.arena + 2 * z.tiles + z.ybuf + z.part + z.ysp + P.n) + 16 * ent +
            (int64_t)sizeof(DFront) * (int64_t)P.fronts.size() + 4 * (int64_t)P.rel.size() +
            8 * (int64_t)P.piv_node.size();
  return z;
}

// Device state of a handle's plan: the uploaded tables and every work
// buffer, allocated on the first call and kept with the handle.
// A batch of plans can need 100 GB of fronts, and mapping that much device
// memory afresh costs up to seconds per call; the batch path therefore
// carves its buffers from one workspace per device that is kept between
// calls (grown when a call needs more; reff_release_cached_memory frees
// it).  A call that finds it in use allocates its own.
struct WorkspaceCache {
  std::mutex mu;
  void* p = nullptr;
  size_t bytes = 0;
  bool busy = false;
};
WorkspaceCache g_ws[64];

constexpr size_t ALIGN = 256;
size_t aligned(size_t b) { return (std::max<size_t>(b, 1) + ALIGN - 1) / ALIGN * ALIGN; }

struct SelinvDevice {
  std::vector<LevelDev> lv;
  SelinvSizes sz;
  double *ar = nullptr, *Li = nullptr, *Z0 = nullptr, *Yb = nullptr, *part = nullptr;
  double *Ysp = nullptr, *Rfull = nullptr, *vals = nullptr;
  int64_t *idx = nullptr, *piv = nullptr;
  int32_t *rel = nullptr, *dl = nullptr;
  DFront* dF = nullptr;
  int* bad = nullptr;
  std::vector<void*> ptrs;       // own allocations
  WorkspaceCache* ws = nullptr;  // or buffers carved from a cached workspace
  char* carve = nullptr;
  size_t carve_left = 0;
  ~SelinvDevice() {
    for (void* q : ptrs) (void)hipFree(q);
    if (ws) {
      std::lock_guard<std::mutex> lk(ws->mu);
      ws->busy = false;
    }
  }
  // Take `total` bytes from the device's cached workspace for the buffers
  // that follow (false: use own allocations).
  hipError_t reserve(size_t total, bool& from_cache) {
    from_cache = false;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) return e;
    WorkspaceCache& c = g_ws[dev];
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.busy) return hipSuccess;
    if (c.bytes < total) {
      if (c.p) (void)hipFree(c.p);
      c.p = nullptr;
      c.bytes = 0;
      e = hipMalloc(&c.p, total);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c.p = nullptr;
        return hipSuccess;  // fall back to own allocations
      }
      c.bytes = total;
    }
    c.busy = true;
    ws = &c;
    carve = (char*)c.p;
    carve_left = c.bytes;
    from_cache = true;
    return hipSuccess;
  }
  template <typename T>
  hipError_t get(T** out, size_t count) {
    const size_t b = aligned(count * sizeof(T));
    if (ws && b <= carve_left) {
      *out = (T*)carve;
      carve += b;
      carve_left -= b;
      return hipSuccess;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e == hipSuccess) ptrs.push_back(q);
    *out = (T*)q;
    return e;
  }
  template <typename T>
  hipError_t put(T** out, const std::vector<T>& v) {
    hipError_t e = get(out, v.size());
    if (e == hipSuccess && !v.empty())
      e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
  }
};

std::shared_ptr<SelinvDevice> selinv_device_build(const SelinvPlan& P, reff_status& s,
                                                  bool use_cache = false) {
  s = REFF_OK;
  auto D = std::make_shared<SelinvDevice>();
  std::vector<DFront> dfr(P.fronts.size());
  std::vector<int32_t> lists;
  int64_t n_ent = 0;
  D->sz = selinv_sizes(P);
  auto groups = plan_groups(P);
  D->lv.resize(P.levels.size());
  for (size_t d = 0; d < P.levels.size(); ++d) {
    const SelinvLevel& L = P.levels[d];
    LevelDev& V = D->lv[d];
    V.nf = (int)L.fronts.size();
    V.ent_off = n_ent;
    V.ent_n = (int64_t)L.ent_idx.size();
    n_ent += V.ent_n;
    const int64_t lbase = (int64_t)lists.size();
    for (GroupDev& g : groups[d]) {
      int64_t yb = 0, pa = 0;
      for (int j = 0; j < g.nf; ++j) {
        const int32_t i = L.fronts[(size_t)(g.list_off + j)];
        const SnFront& f = P.fronts[(size_t)i];
        DFront& x = dfr[(size_t)i];
        x.off = f.off;
        x.poff = f.parent >= 0 ? P.fronts[(size_t)f.parent].off : -1;
        x.rel = f.rel;
        x.piv = f.piv;
        x.F = f.F;
        x.k = f.k;
        x.pF = f.parent >= 0 ? P.fronts[(size_t)f.parent].F : 0;
        x.rank = f.rank;
        x.nsplit = front_nsplit(f);
        x.pad_ = 0;
        x.ybuf = yb;
        x.part = pa;
        yb += (int64_t)f.F * PT;
        pa += (int64_t)x.nsplit * PT * PT;
      }
      g.list_off += lbase;
    }
    lists.insert(lists.end(), L.fronts.begin(), L.fronts.end());
    V.groups = std::move(groups[d]);
  }
  hipError_t e = hipSuccess;
  if (use_cache) {
    const SelinvSizes& z = D->sz;
    const size_t total = aligned(8 * (size_t)P.arena) + 2 * aligned(8 * (size_t)z.tiles) +
                         aligned(8 * (size_t)z.ybuf) + aligned(8 * (size_t)z.part) +
                         aligned(8 * (size_t)z.ysp) + aligned(8 * (size_t)P.n) + aligned(4) +
                         2 * aligned(8 * (size_t)n_ent) + aligned(8 * P.piv_node.size()) +
                         aligned(4 * P.rel.size()) + aligned(4 * lists.size()) +
                         aligned(sizeof(DFront) * dfr.size());
    bool cached = false;
    e = D->reserve(total, cached);
  }
  if (e == hipSuccess) e = D->get(&D->ar, (size_t)P.arena);
  if (e == hipSuccess) e = D->get(&D->Li, (size_t)D->sz.tiles);
  if (e == hipSuccess) e = D->get(&D->Z0, (size_t)D->sz.tiles);
  if (e == hipSuccess) e = D->get(&D->Yb, (size_t)D->sz.ybuf);
  if (e == hipSuccess) e = D->get(&D->part, (size_t)D->sz.part);
  if (e == hipSuccess) e = D->get(&D->Ysp, (size_t)D->sz.ysp);
  if (e == hipSuccess) e = D->get(&D->Rfull, (size_t)P.n);
  if (e == hipSuccess) e = D->get(&D->bad, 1);
  // G's entries, level by level straight from the plan
  if (e == hipSuccess) e = D->get(&D->idx, (size_t)n_ent);
  if (e == hipSuccess) e = D->get(&D->vals, (size_t)n_ent);
  for (size_t d = 0; d < P.levels.size() && e == hipSuccess; ++d) {
    const SelinvLevel& L = P.levels[d];
    const LevelDev& V = D->lv[d];
    if (V.ent_n == 0) continue;
    e = hipMemcpy(D->idx + V.ent_off, L.ent_idx.data(), sizeof(int64_t) * V.ent_n,
                  hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(D->vals + V.ent_off, L.ent_val.data(), sizeof(double) * V.ent_n,
                    hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = D->put(&D->piv, P.piv_node);
  if (e == hipSuccess) e = D->put(&D->rel, P.rel);
  if (e == hipSuccess) e = D->put(&D->dl, lists);
  if (e == hipSuccess) e = D->put(&D->dF, dfr);
  if (e != hipSuccess) {
    s = dev_status(e, "selected inversion: allocation / upload");
    return nullptr;
  }
  return D;
}

std::shared_ptr<SelinvDevice> selinv_device_of(reff_pdn_t* p, const SelinvPlan& P,
                                               reff_status& s) {
  s = REFF_OK;
  if (p->sel_dev) return p->sel_dev;
  auto D = selinv_device_build(P, s);
  if (D) p->sel_dev = D;
  return D;
}

// The numeric work of a plan on its device state, on `st`: factorisation
// (deepest level first) then selected inversion (roots first); D.Rfull
// receives R for every pivot node (0 elsewhere).  t_fact: when the
// factorisation finished (the call synchronises there to read the pivot
// flag).
reff_status selinv_run(const SelinvPlan& P, const SelinvDevice& D, hipStream_t st_,
                       std::chrono::steady_clock::time_point& t_fact,
                       const std::vector<uint8_t>* need = nullptr) {
  double *ar = D.ar, *Li = D.Li, *Z0 = D.Z0, *Yb = D.Yb, *part = D.part, *Ysp = D.Ysp;
  double* Rfull = D.Rfull;
  const int32_t *rel = D.rel, *dl = D.dl;
  const DFront* dF = D.dF;
  int* bad = D.bad;
  hipLaunchKernelGGL(k_zero, flat(P.n), dim3(256), 0, st_, Rfull, P.n);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), st_);
  auto gy = [](int nf) { return (unsigned)std::min<int64_t>(nf, MAX_GY); };
  const int nlev = (int)P.levels.size();
  // factorisation, deepest level first
  for (int d = nlev - 1; d >= 0 && e == hipSuccess; --d) {
    const SelinvLevel& L = P.levels[(size_t)d];
    const LevelDev& V = D.lv[(size_t)d];
    if (V.nf == 0) continue;
    const int64_t span = L.arena_end - L.arena_begin;
    if (span > 0) hipLaunchKernelGGL(k_zero, flat(span), dim3(256), 0, st_, ar + L.arena_begin, span);
    if (V.ent_n > 0)
      hipLaunchKernelGGL(k_scatter, flat(V.ent_n), dim3(256), 0, st_, D.idx + V.ent_off,
                         D.vals + V.ent_off, V.ent_n, ar);
    if (d + 1 < nlev)
      for (int rank = 0; rank < 2; ++rank)
        for (const GroupDev& C : D.lv[(size_t)d + 1].groups) {
          const unsigned gx = (unsigned)std::max<int64_t>(1, (C.maxq + 3) / 4);
          hipLaunchKernelGGL(k_extend_add, dim3(gx, gy(C.nf)), dim3(256), 0, st_, dF,
                             dl + C.list_off, C.nf, rank, rel, ar);
        }
    for (const GroupDev& G : V.groups) {
      const int32_t* l = dl + G.list_off;
      for (int jp = 0; jp < G.max_panels; ++jp) {
        hipLaunchKernelGGL(k_tile<true>, dim3(gy(G.nf)), dim3(256), 0, st_, dF, l, G.nf, jp, ar,
                           Li, Z0, bad);
        const int mt = G.mt[(size_t)jp];
        if (mt == 0) continue;
        hipLaunchKernelGGL(k_front_gemm<OP_TRSM>, dim3((unsigned)mt, gy(G.nf)), dim3(256), 0,
                           st_, dF, l, G.nf, jp, ar, Li, Yb, part, mt, 1, Ysp, (int64_t)0);
        hipLaunchKernelGGL(k_front_gemm<OP_SYRK>, dim3((unsigned)(mt * (mt + 1) / 2), gy(G.nf)),
                           dim3(256), 0, st_, dF, l, G.nf, jp, ar, Li, Yb, part, mt, 1, Ysp,
                           (int64_t)0);
      }
    }
    e = hipGetLastError();
  }
  int hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return dev_status(e, "selected inversion: factorisation");
  if (hbad) return host_fail(REFF_ERR_DEVICE, "sparse Cholesky: a pivot was not positive");
  t_fact = std::chrono::steady_clock::now();
  // With a request, the selected inversion visits only the needed fronts:
  // each launch group runs over the compacted list of its needed fronts
  // (their scratch slots and Y offsets are those of the full group).
  Bufs lb;
  int32_t* dact = nullptr;
  std::vector<std::vector<std::pair<int64_t, int>>> act_rng(P.levels.size());
  if (need) {
    std::vector<int32_t> act;
    for (size_t d = 0; d < P.levels.size(); ++d) {
      const SelinvLevel& L = P.levels[d];
      for (const GroupDev& G : D.lv[d].groups) {
        const int64_t lbase = G.list_off - D.lv[d].groups.front().list_off;
        const int64_t a0 = (int64_t)act.size();
        for (int j = 0; j < G.nf; ++j) {
          const int32_t fi = L.fronts[(size_t)(lbase + j)];
          if ((*need)[(size_t)fi]) act.push_back(fi);
        }
        act_rng[d].push_back({a0, (int)((int64_t)act.size() - a0)});
      }
    }
    e = put(lb, &dact, act, st_);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    if (e != hipSuccess) return dev_status(e, "selected inversion: request lists");
  }
  // selected inversion, roots first
  for (int d = 0; d < nlev && e == hipSuccess; ++d) {
    const LevelDev& V = D.lv[(size_t)d];
    for (size_t gi = 0; gi < V.groups.size(); ++gi) {
      const GroupDev& G = V.groups[gi];
      const int32_t* l = dl + G.list_off;
      int nfa = G.nf;
      if (need) {
        l = dact + act_rng[(size_t)d][gi].first;
        nfa = act_rng[(size_t)d][gi].second;
        if (nfa == 0) continue;
      }
      if (d > 0 && G.maxq > 0) {
        const unsigned gx = (unsigned)std::max<int64_t>(1, (G.maxq + 3) / 4);
        hipLaunchKernelGGL(k_gather, dim3(gx, gy(nfa)), dim3(256), 0, st_, dF, l, nfa, rel, ar);
      }
      for (int jp = G.max_panels - 1; jp >= 0; --jp) {
        const int mt = G.mt[(size_t)jp], ms = G.ms[(size_t)jp];
        hipLaunchKernelGGL(k_tile<false>, dim3(gy(nfa)), dim3(256), 0, st_, dF, l, nfa, jp, ar,
                           Li, Z0, bad);
        if (mt > 0) {
          hipLaunchKernelGGL(k_front_gemm<OP_LHAT>, dim3((unsigned)mt, gy(nfa)), dim3(256), 0,
                             st_, dF, l, nfa, jp, ar, Li, Yb, part, mt, 1, Ysp, (int64_t)0);
          hipLaunchKernelGGL(k_front_gemm<OP_Y>, dim3((unsigned)(mt * G.ysplit), gy(nfa)),
                             dim3(256), 0, st_, dF, l, nfa, jp, ar, Li, Yb, part, mt, G.ysplit,
                             Ysp, G.ylev);
          if (G.ysplit > 1)
            hipLaunchKernelGGL(k_ysum, dim3((unsigned)mt, gy(nfa)), dim3(256), 0, st_, dF, l,
                               nfa, jp, G.ysplit, (const double*)Ysp, G.ylev, Yb);
          hipLaunchKernelGGL(k_front_gemm<OP_PART>, dim3((unsigned)ms, gy(nfa)), dim3(256), 0,
                             st_, dF, l, nfa, jp, ar, Li, Yb, part, mt, 1, Ysp, (int64_t)0);
        }
        hipLaunchKernelGGL(k_finish, dim3((unsigned)(1 + mt), gy(nfa)), dim3(256), 0, st_, dF,
                           l, nfa, jp, ar, Z0, Yb, part, D.piv, Rfull);
      }
    }
    e = hipGetLastError();
  }
  if (e != hipSuccess) return dev_status(e, "selected inversion");
  return REFF_OK;
}

}  // namespace reff

extern "C" {

reff_status reff_selinv_info(const reff_pdn_desc* d, reff_selinv_stats* info) {
  using namespace reff;
  if (!d || !info) return host_fail(REFF_ERR_INVALID_ARG, "NULL descriptor or info");
  reff_status s = host_validate_desc(d);
  if (s != REFF_OK) return s;
  SelinvPlan plan;
  std::string err;
  bool dis = false;
  if (!build_selinv_plan(d->n_tiers, d->nx, d->ny, d->gx, d->gy, d->n_tsv, d->tsv_xy, d->tsv_g,
                         d->n_pads, d->pad_xy, LEAF_AREA, plan, err, &dis))
    return host_fail(dis ? REFF_ERR_DISCONNECTED : REFF_ERR_INVALID_ARG,
                     "selected inversion plan: " + err);
  std::memset(info, 0, sizeof(*info));
  info->n_fronts = (int64_t)plan.fronts.size();
  info->n_levels = (int32_t)plan.levels.size();
  for (const SnFront& f : plan.fronts) info->max_front = std::max<int64_t>(info->max_front, f.F);
  info->device_bytes = selinv_sizes(plan).bytes;
  info->flops_factor = plan.flops_factor;
  info->flops_selinv = plan.flops_selinv;
  return REFF_OK;
}

reff_status reff_selinv_diag(reff_pdn p, const int64_t* nodes, int64_t n_nodes, double* R_out,
                             const reff_solve_opts* opts, reff_selinv_stats* st) {
  using namespace reff;
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return host_fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  if (nodes && n_nodes < 0) return host_fail(REFF_ERR_INVALID_ARG, "n_nodes < 0");
  const int64_t count = nodes ? n_nodes : p->n;
  if (count > 0 && !R_out) return host_fail(REFF_ERR_INVALID_ARG, "R_out is NULL");
  for (int64_t i = 0; nodes && i < count; ++i)
    if (nodes[i] < 0 || nodes[i] >= p->n)
      return host_fail(REFF_ERR_INVALID_ARG, "node id " + std::to_string(nodes[i]) + " out of range");
  hipStream_t st_ = opts ? (hipStream_t)opts->stream : nullptr;
  const bool out_dev = opts && opts->out_on_device;
  if (opts && opts->out_on_device != 0 && opts->out_on_device != 1)
    return host_fail(REFF_ERR_INVALID_ARG, "out_on_device must be 0 or 1");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return dev_status(e, "hipSetDevice");
  reff_status s;
  auto plan_sp = selinv_plan_of(p, s);
  if (!plan_sp) return s;
  const SelinvPlan& P = *plan_sp;
  const auto t_plan = std::chrono::steady_clock::now();

  auto dev_sp = selinv_device_of(p, P, s);
  if (!dev_sp) return s;
  const SelinvDevice& D = *dev_sp;
  const auto t_setup = std::chrono::steady_clock::now();
  double* Rfull = D.Rfull;
  Bufs b;
  double* dout = nullptr;
  int64_t* dnodes = nullptr;
  if (nodes && count > 0) {
    std::vector<int64_t> nv(nodes, nodes + count);
    e = put(b, &dnodes, nv, st_);
    // the staged host vector must outlive the copy
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
  }
  if (e == hipSuccess && !out_dev && count > 0) e = b.get(&dout, (size_t)count);
  if (e != hipSuccess) return dev_status(e, "selected inversion: output buffers");
  // a node list needs only its fronts and their ancestors inverted
  double fl_sel = P.flops_selinv;
  std::vector<uint8_t> need;
  if (nodes) need = needed_fronts(P, std::vector<int64_t>(nodes, nodes + count), &fl_sel);
  std::chrono::steady_clock::time_point t_fact;
  s = selinv_run(P, D, st_, t_fact, nodes ? &need : nullptr);
  if (s != REFF_OK) return s;
  // output
  if (e == hipSuccess && count > 0) {
    double* out = out_dev ? R_out : dout;
    if (nodes) {
      hipLaunchKernelGGL(k_pick, flat(count), dim3(256), 0, st_, Rfull, dnodes, count, out);
      e = hipGetLastError();
    } else {
      e = hipMemcpyAsync(out, Rfull, sizeof(double) * count, hipMemcpyDeviceToDevice, st_);
    }
    if (e == hipSuccess && !out_dev)
      e = hipMemcpyAsync(R_out, dout, sizeof(double) * count, hipMemcpyDeviceToHost, st_);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return dev_status(e, "selected inversion");
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->n_fronts = (int64_t)P.fronts.size();
    st->n_levels = (int32_t)P.levels.size();
    for (const SnFront& f : P.fronts) st->max_front = std::max<int64_t>(st->max_front, f.F);
    st->device_bytes = D.sz.bytes;
    st->flops_factor = P.flops_factor;
    st->flops_selinv = fl_sel;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->seconds_plan = std::chrono::duration<double>(t_plan - t0).count();
    st->seconds_factor = std::chrono::duration<double>(t_fact - t_plan).count();
    st->seconds_selinv = std::chrono::duration<double>(t1 - t_fact).count();
    st->seconds_setup = std::chrono::duration<double>(t_setup - t_plan).count();
  }
  return REFF_OK;
}

reff_status reff_release_cached_memory(int32_t device) {
  using namespace reff;
  if (device < 0 || device >= 64) return host_fail(REFF_ERR_INVALID_ARG, "bad device");
  WorkspaceCache& c = g_ws[device];
  std::lock_guard<std::mutex> lk(c.mu);
  if (!c.p || c.busy) return REFF_OK;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipFree(c.p);
  c.p = nullptr;
  c.bytes = 0;
  if (e != hipSuccess) return dev_status(e, "releasing cached memory");
  return REFF_OK;
}

reff_status reff_selinv_batch(const reff_pdn_desc* plans, int32_t n_plans,
                              const int64_t* const* nodes, const int64_t* n_nodes,
                              double* const* R_out, const reff_solve_opts* opts,
                              reff_selinv_stats* st) {
  using namespace reff;
  const auto t0 = std::chrono::steady_clock::now();
  if (st) std::memset(st, 0, sizeof(*st));
  if (n_plans < 0) return host_fail(REFF_ERR_INVALID_ARG, "n_plans < 0");
  if (n_plans == 0) return REFF_OK;
  if (!plans || !R_out) return host_fail(REFF_ERR_INVALID_ARG, "NULL plans or R_out");
  if (opts && opts->out_on_device != 0 && opts->out_on_device != 1)
    return host_fail(REFF_ERR_INVALID_ARG, "out_on_device must be 0 or 1");
  const bool out_dev = opts && opts->out_on_device;
  hipStream_t st_ = opts ? (hipStream_t)opts->stream : nullptr;
  const size_t np = (size_t)n_plans;
  std::vector<int64_t> cnt(np);
  // descriptors checked on host threads; the first bad plan is reported
  std::vector<reff_status> vs(np, REFF_OK);
  std::vector<std::string> vm(np);
  selinv_parallel_for(np, [&](size_t i) {
    vs[i] = host_validate_desc(&plans[i]);
    if (vs[i] != REFF_OK) vm[i] = reff_last_error();  // this thread's message
  });
  for (size_t i = 0; i < np; ++i) {
    const std::string who = "plan " + std::to_string(i) + ": ";
    if (vs[i] != REFF_OK) return host_fail(vs[i], who + vm[i]);
    const int64_t n = (int64_t)plans[i].n_tiers * plans[i].nx * plans[i].ny;
    const bool given = nodes && nodes[i];
    if (given && (!n_nodes || n_nodes[i] < 0)) return host_fail(REFF_ERR_INVALID_ARG, who + "bad n_nodes");
    cnt[i] = given ? n_nodes[i] : n;
    if (cnt[i] > 0 && !R_out[i]) return host_fail(REFF_ERR_INVALID_ARG, who + "R_out NULL");
    for (int64_t k = 0; given && k < cnt[i]; ++k)
      if (nodes[i][k] < 0 || nodes[i][k] >= n)
        return host_fail(REFF_ERR_INVALID_ARG,
                         who + "node id " + std::to_string(nodes[i][k]) + " out of range");
  }
  // Plans are taken in chunks of consecutive plans with about equal node
  // counts (one chunk below 4M nodes, at most four): the host analysis of
  // chunk c + 1 runs on host threads while the device factors and inverts
  // chunk c, and each chunk is one forest (the plans' trees merged by
  // depth) on the device workspace.
  int64_t tot_n = 0;
  std::vector<int64_t> pn(np);
  for (size_t i = 0; i < np; ++i) {
    pn[i] = (int64_t)plans[i].n_tiers * plans[i].nx * plans[i].ny;
    tot_n += pn[i];
  }
  const int64_t nch = std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)4, (int64_t)np, tot_n / (int64_t(4) << 20)}));
  std::vector<size_t> cb{0};
  {
    const int64_t share = (tot_n + nch - 1) / nch;
    int64_t acc = 0;
    for (size_t i = 0; i < np; ++i) {
      acc += pn[i];
      if (acc >= share * (int64_t)cb.size() && (int64_t)cb.size() < nch && i + 1 < np)
        cb.push_back(i + 1);
    }
    cb.push_back(np);
  }
  struct Chunk {
    SelinvPlan P;
    std::vector<int64_t> base;
    reff_status s = REFF_OK;
    std::string err;
  };
  auto analyse = [&](size_t c, Chunk& out) {
    const size_t p0 = cb[c], p1 = cb[c + 1];
    std::vector<SelinvPlan> sp(p1 - p0);
    std::vector<std::string> err(p1 - p0);
    std::vector<char> ok(p1 - p0, 0), disc(p1 - p0, 0);
    selinv_parallel_for(p1 - p0, [&](size_t k) {
      const reff_pdn_desc& d = plans[p0 + k];
      bool dis = false;
      ok[k] = build_selinv_plan(d.n_tiers, d.nx, d.ny, d.gx, d.gy, d.n_tsv, d.tsv_xy, d.tsv_g,
                                d.n_pads, d.pad_xy, LEAF_AREA, sp[k], err[k], &dis);
      disc[k] = dis;
    });
    for (size_t k = 0; k < p1 - p0; ++k)
      if (!ok[k]) {
        out.s = disc[k] ? REFF_ERR_DISCONNECTED : REFF_ERR_INVALID_ARG;
        out.err = "plan " + std::to_string(p0 + k) + ": " + err[k];
        return;
      }
    out.P = merge_selinv_plans(sp, out.base);
  };
  // requested nodes of every plan, in plan order, into one device array
  int64_t total = 0;
  std::vector<int64_t> out_at(np + 1, 0);
  for (size_t i = 0; i < np; ++i) out_at[i + 1] = out_at[i] + cnt[i];
  total = out_at[np];
  double t_plan = 0.0, t_setup = 0.0, t_factor = 0.0, t_selinv = 0.0;
  int64_t n_fronts = 0, max_front = 0, dev_bytes = 0;
  int32_t n_levels = 0;
  double fl_fact = 0.0, fl_sel = 0.0;
  auto tp = std::chrono::steady_clock::now();
  auto cur = std::make_unique<Chunk>();
  analyse(0, *cur);
  t_plan += std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
  // a plan of the first chunk that fails its analysis is refused before any
  // device work; later chunks' failures come after earlier chunks' device
  // work, with nothing written to R_out either way
  if (cur->s != REFF_OK) return host_fail(cur->s, cur->err);
  Bufs b;
  double* dres = nullptr;
  hipError_t e = b.get(&dres, (size_t)total);
  if (e != hipSuccess) return dev_status(e, "selected inversion batch: output");
  for (size_t c = 0; c + 1 < cb.size(); ++c) {
    if (cur->s != REFF_OK) return host_fail(cur->s, cur->err);
    auto next = std::make_unique<Chunk>();
    std::thread ahead;
    if (c + 2 < cb.size()) ahead = std::thread([&, c] { analyse(c + 1, *next); });
    struct Join {
      std::thread& t;
      ~Join() {
        if (t.joinable()) t.join();
      }
    } join{ahead};
    const SelinvPlan& P = cur->P;
    const size_t p0 = cb[c], p1 = cb[c + 1];
    const auto t0c = std::chrono::steady_clock::now();
    reff_status s;
    auto dev_sp = selinv_device_build(P, s, true);
    if (!dev_sp) return s;
    const SelinvDevice& D = *dev_sp;
    const auto t_set = std::chrono::steady_clock::now();
    std::vector<int64_t> ids;
    ids.reserve((size_t)(out_at[p1] - out_at[p0]));
    bool every = true;
    for (size_t i = p0; i < p1; ++i) {
      const bool given = nodes && nodes[i];
      every = every && !given;
      for (int64_t k = 0; k < cnt[i]; ++k)
        ids.push_back(cur->base[i - p0] + (given ? nodes[i][k] : k));
    }
    // with node lists, only their fronts and ancestors are inverted
    double fl = P.flops_selinv;
    std::vector<uint8_t> need;
    if (!every) need = needed_fronts(P, ids, &fl);
    std::chrono::steady_clock::time_point t_fact;
    s = selinv_run(P, D, st_, t_fact, every ? nullptr : &need);
    if (s != REFF_OK) return s;
    Bufs bc;
    int64_t* dids = nullptr;
    e = put(bc, &dids, ids, st_);
    const int64_t nc = (int64_t)ids.size();
    if (e == hipSuccess && nc > 0) {
      hipLaunchKernelGGL(k_pick, flat(nc), dim3(256), 0, st_, D.Rfull, dids, nc,
                         dres + out_at[p0]);
      e = hipGetLastError();
    }
    // the workspace and the staged ids are reused or freed after this
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    if (e != hipSuccess) return dev_status(e, "selected inversion batch");
    const auto t_end = std::chrono::steady_clock::now();
    t_setup += std::chrono::duration<double>(t_set - t0c).count();
    t_factor += std::chrono::duration<double>(t_fact - t_set).count();
    t_selinv += std::chrono::duration<double>(t_end - t_fact).count();
    n_fronts += (int64_t)P.fronts.size();
    n_levels = std::max<int32_t>(n_levels, (int32_t)P.levels.size());
    for (const SnFront& f : P.fronts) max_front = std::max<int64_t>(max_front, f.F);
    dev_bytes = std::max<int64_t>(dev_bytes, D.sz.bytes);
    fl_fact += P.flops_factor;
    fl_sel += fl;
    dev_sp.reset();
    // the next chunk's analysis: whatever of it the device work did not hide
    const auto tw = std::chrono::steady_clock::now();
    if (ahead.joinable()) ahead.join();
    t_plan += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count();
    cur = std::move(next);
  }
  std::vector<double> host;
  if (!out_dev) {
    host.resize((size_t)total);
    if (total > 0)
      e = hipMemcpyAsync(host.data(), dres, sizeof(double) * total, hipMemcpyDeviceToHost, st_);
  }
  for (size_t i = 0; i < np && e == hipSuccess; ++i)
    if (cnt[i] > 0 && out_dev)
      e = hipMemcpyAsync(R_out[i], dres + out_at[i], sizeof(double) * cnt[i],
                         hipMemcpyDeviceToDevice, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return dev_status(e, "selected inversion batch");
  if (!out_dev)
    for (size_t i = 0; i < np; ++i)
      if (cnt[i] > 0) std::memcpy(R_out[i], host.data() + out_at[i], sizeof(double) * cnt[i]);
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    st->n_fronts = n_fronts;
    st->n_levels = n_levels;
    st->max_front = max_front;
    st->device_bytes = dev_bytes;
    st->flops_factor = fl_fact;
    st->flops_selinv = fl_sel;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->seconds_plan = t_plan;
    st->seconds_setup = t_setup;
    st->seconds_factor = t_factor + t_setup;
    st->seconds_selinv = t_selinv;
  }
  return REFF_OK;
}

}  // extern "C"
