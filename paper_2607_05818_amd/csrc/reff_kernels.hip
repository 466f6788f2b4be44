// gfx950 kernels of the block-PCG effective-resistance solver.
//
// Vectors are n x S blocks stored node-major with the S = 64 right-hand
// sides contiguous (V[v*S + k]).  One wavefront owns one node at a time and
// lane k owns column k, so every vector access of a wave is one coalesced
// 64-element row and a node's stencil coefficients are wave-uniform (scalar
// loads).
//
// Block PCG with rank-revealing orthonormalised search directions.  The
// search block arrives as Y (any basis) plus an S x S upper-triangular map T
// such that P = Y T has D-orthonormal kept columns (D = diag G) and zero
// dropped ones.  One iteration for all S columns:
//   K1  Qt = G Y (stencil); P = Y T; Q = Qt T;  W1 = P^T Q, W2 = P^T R
//   Ks1 W1^+ by a guarded sweep;  A = W1^+ W2;
//       psi_k += sum_j P[tgt_k, j] A[j, k]  (= change of x_k at node tgt_k)
//   K2  R -= Q A;  (D += P A);  Z = Dinv R;  W3 = Q^T Z
//   Ks2 B = W1^+ W3
//   K3  Y = Z - P B;  W4 = Y^T D Y
//   Ks3 T from the guarded sweep of W4: directions whose pivot falls below
//       eps are numerically dependent and are dropped
// The S x S products and Grams of K1-K3 run on the matrix cores.
// (the per-workgroup Gram partials are reduced by Kr first).  With x0 = 0
// and R0 = e_i, psi_k = e_i^T x_k is the Galerkin estimate of
// R_i = (G^-1)_ii and rises to it from below.  The "independent" variant
// keeps only the diagonals: S ordinary PCGs side by side.
#include "reff_internal.h"

#include <math.h>

#include <algorithm>

namespace reff {

// Hardware dispatches workgroup b to XCD (b mod 8).  Give each XCD a
// contiguous range of logical blocks so that neighbouring node ranges, which
// share stencil halo rows, are served by the same L2.
__device__ __forceinline__ int logical_block(int b, int nb) {
  if ((nb & 7) != 0) return b;
  const int per = nb >> 3;
  return (b & 7) * per + (b >> 3);
}

struct Range {
  int64_t begin, end;
};

__device__ __forceinline__ Range block_range(int64_t n, int grid) {
  const int lb = logical_block(blockIdx.x, grid);
  const int64_t nch = (n + CH - 1) / CH;
  const int64_t cpb = (nch + grid - 1) / grid;
  Range r;
  r.begin = (int64_t)lb * cpb * CH;
  const int64_t e = (int64_t)(lb + 1) * cpb * CH;
  r.end = e < n ? e : n;
  return r;
}

int grid_for(int64_t n) {
  const int64_t nch = (n + CH - 1) / CH;
  return (int)(nch < MAX_GRID ? nch : MAX_GRID);
}

// (G y)_v for the lane's column.
template <typename T, typename U>
__device__ __forceinline__ T stencil_row(const Coef<T>& c, const U* __restrict__ Y, int64_t v,
                                         int lane) {
  const int64_t n = c.n;
  const T ce = c.cE[v];
  const T cn = c.cN[v];
  const T cw = v >= 1 ? c.cE[v - 1] : T(0);
  const T cs = v >= c.nx ? c.cN[v - c.nx] : T(0);
  // Clamped indices keep every load in range; the matching coefficient is
  // zero whenever the neighbour does not exist (grid edge or pad).
  const int64_t ve = v + 1 < n ? v + 1 : n - 1;
  const int64_t vw = v >= 1 ? v - 1 : 0;
  const int64_t vn = v + c.nx < n ? v + c.nx : n - 1;
  const int64_t vs = v >= c.nx ? v - c.nx : 0;
  const T y = (T)Y[v * S + lane];
  const T ye = (T)Y[ve * S + lane];
  const T yw = (T)Y[vw * S + lane];
  const T yn = (T)Y[vn * S + lane];
  const T ys = (T)Y[vs * S + lane];
  T q = c.d[v] * y - ce * ye - cw * yw - cn * yn - cs * ys;
  const int sl = c.slot[v];
  if (sl >= 0) {
    const T gu = c.up[sl];
    const T gd = c.dn[sl];
    if (gu != T(0)) q -= gu * (T)Y[(v + c.plane) * S + lane];
    if (gd != T(0)) q -= gd * (T)Y[(v - c.plane) * S + lane];
  }
  return q;
}

// Partial Grams of one workgroup: part[g][m][S*S] (or the first S entries
// for diagonal-only Grams).
constexpr int NGRAM = 4;
// Padded LDS row (words).  A row offset of 4 words spreads the 16 rows read
// by one product operand over distinct banks.
constexpr int LDW = S + 4;

__device__ __forceinline__ double* part_of(double* part, int m) {
  return part + ((size_t)blockIdx.x * NGRAM + m) * S * S;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

// Matrix-core primitives.  v_mfma_{f32,f64}_16x16x4 multiply A (16x4, lane l
// holds element (l%16, l/16)) by B (4x16, lane l holds (l/16, l%16)); the
// 16x16 result holds column l%16 of rows tile_row(l, r) in register r
// (float32: 4*(l/16)+r, float64: (l/16)+4*r).
template <typename T>
__device__ __forceinline__ int tile_row(int lane, int r) {
  return sizeof(T) == 4 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

__device__ __forceinline__ f4v mma(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4v mma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<float> { typedef f4v type; };
template <> struct Acc<double> { typedef d4v type; };

// Product tile: rows [16 nb, 16 nb + 16) of the CH x S block staged in sA
// times an S x S matrix B, of which the lane holds column block cb as
// breg[ks] = B[4 ks + l/16][16 cb + l%16].  Result as described above.
template <typename T>
__device__ __forceinline__ typename Acc<T>::type prod_tile(const T (*sA)[LDW], int nb,
                                                           const T* breg, int lane) {
  typename Acc<T>::type c = {0, 0, 0, 0};
  const int rr = nb * 16 + (lane & 15), kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < S / 4; ++ks) c = mma(sA[rr][4 * ks + kq], breg[ks], c);
  return c;
}

template <typename T>
__device__ __forceinline__ void load_bcol(const T* __restrict__ B, int cb, int lane, T* breg) {
#pragma unroll
  for (int ks = 0; ks < S / 4; ++ks) breg[ks] = B[(4 * ks + (lane >> 4)) * S + 16 * cb + (lane & 15)];
}

// Gram tile (ti, tj) of A^T B over the CH staged rows, added to acc (float64).
// float32 products are summed over one chunk in float32 first.
template <typename T>
__device__ __forceinline__ void gram_tile(const T (*sA)[LDW], const T (*sB)[LDW], int ti, int tj,
                                          int lane, double* acc) {
  typename Acc<T>::type c = {0, 0, 0, 0};
  const int kr = lane >> 4, cc = lane & 15;
#pragma unroll
  for (int kb = 0; kb < CH; kb += 4) c = mma(sA[kb + kr][ti * 16 + cc], sB[kb + kr][tj * 16 + cc], c);
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] += (double)c[r];
}

// Wave w owns Gram tiles 2w and 2w+1 of the 4 x 4 tiles of an S x S Gram.
template <typename T>
__device__ __forceinline__ void gram_chunk(const T (*sA)[LDW], const T (*sB)[LDW], int w,
                                           int lane, double (&acc)[2][4]) {
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = 2 * w + tt;
    gram_tile<T>(sA, sB, t >> 2, t & 3, lane, acc[tt]);
  }
}

template <typename T>
__device__ __forceinline__ void gram_store(double* dst, int w, int lane,
                                           const double (&acc)[2][4]) {
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = 2 * w + tt;
    const int i0 = (t >> 2) * 16, j = (t & 3) * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(i0 + tile_row<T>(lane, r)) * S + j] = acc[tt][r];
  }
}

__device__ __forceinline__ void zero_acc(double (&acc)[2][4]) {
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[tt][r] = 0.0;
}

// Sum over the waves of per-lane diagonal partials -> dst[lane].
__device__ __forceinline__ void diag_store(double* dst, double v, int w, int lane) {
  __shared__ double red[WG / 64][S];
  red[w][lane] = v;
  __syncthreads();
  if (w == 0) {
    double s = 0.0;
    for (int u = 0; u < WG / 64; ++u) s += red[u][lane];
    dst[lane] = s;
  }
}

// In the block kernels each wave owns product tile (nb, cb) = (w / 4, w % 4)
// of the CH x S chunk, and stages/streams the CH/8 rows w*4 .. w*4+3.
static_assert(CH == 32 && WG == 512, "tile ownership assumes 32-node chunks, 8 waves");

// ---------------------------------------------------------------- K1
// Qt = G Y;  P = Y T;  Q = Qt T;  W1 = P^T Q,  W2 = P^T R.
template <typename T, bool DIAG>
__global__ __launch_bounds__(WG, 4) void k_stencil_gram(Coef<T> c, const T* __restrict__ Y,
                                                     const T* __restrict__ Tm,
                                                     const T* __restrict__ R, T* __restrict__ P,
                                                     T* __restrict__ Q, double* __restrict__ part) {
  __shared__ T sA[DIAG ? 1 : CH][LDW];  // Y rows, then P rows
  __shared__ T sB[DIAG ? 1 : CH][LDW];  // G Y rows, then Q rows
  __shared__ T sR[DIAG ? 1 : CH][LDW];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nb = w >> 2, cb = w & 3;
  const Range rg = block_range(c.n, gridDim.x);
  T breg[DIAG ? 1 : S / 4];
  if (!DIAG) load_bcol<T>(Tm, cb, lane, breg);
  double a1[2][4], a2[2][4];
  zero_acc(a1);
  zero_acc(a2);
  double d1 = 0.0, d2 = 0.0;
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) {
          const T y = Y[v * S + lane];
          const T q = stencil_row<T, T>(c, Y, v, lane);
          const T r = R[v * S + lane];
          P[v * S + lane] = y;
          Q[v * S + lane] = q;
          d1 += (double)y * (double)q;
          d2 += (double)y * (double)r;
        }
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      T y = 0, q = 0, r = 0;
      if (v < rg.end) {
        y = Y[v * S + lane];
        r = R[v * S + lane];
        q = stencil_row<T, T>(c, Y, v, lane);
      }
      sA[row][lane] = y;
      sB[row][lane] = q;
      sR[row][lane] = r;
    }
    __syncthreads();
    const auto pt = prod_tile<T>(sA, nb, breg, lane);
    const auto qt = prod_tile<T>(sB, nb, breg, lane);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sA[row][col] = pt[r];
      sB[row][col] = qt[r];
    }
    __syncthreads();
    gram_chunk<T>(sA, sB, w, lane, a1);
    gram_chunk<T>(sA, sR, w, lane, a2);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < rg.end) {
        P[v * S + lane] = sA[row][lane];
        Q[v * S + lane] = sB[row][lane];
      }
    }
    __syncthreads();
  }
  if (DIAG) {
    diag_store(part_of(part, 0), d1, w, lane);
    __syncthreads();
    diag_store(part_of(part, 1), d2, w, lane);
  } else {
    gram_store<T>(part_of(part, 0), w, lane, a1);
    gram_store<T>(part_of(part, 1), w, lane, a2);
  }
}

// ---------------------------------------------------------------- K2
// R -= Q A;  (D += P A);  Z = Dinv R;  W3 = Q^T Z.
template <typename T, bool DIAG, bool WITH_D>
__global__ __launch_bounds__(WG, 4) void k_update_r(Coef<T> c, const T* __restrict__ alpha,
                                                 const T* __restrict__ Q,
                                                 const T* __restrict__ P, T* __restrict__ R,
                                                 T* __restrict__ D, double* __restrict__ part) {
  __shared__ T sQ[DIAG ? 1 : CH][LDW];
  __shared__ T sP[DIAG ? 1 : CH][LDW];  // P rows, then Z rows
  __shared__ T sR[DIAG ? 1 : CH][LDW];
  __shared__ T sD[(WITH_D && !DIAG) ? CH : 1][LDW];
  __shared__ T sDinv[CH];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nb = w >> 2, cb = w & 3;
  const Range rg = block_range(c.n, gridDim.x);
  T breg[DIAG ? 1 : S / 4];
  if (DIAG)
    breg[0] = alpha[lane];
  else
    load_bcol<T>(alpha, cb, lane, breg);
  double a3[2][4];
  zero_acc(a3);
  double d3 = 0.0;
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) {
          const T q = Q[v * S + lane];
          const T r = R[v * S + lane] - breg[0] * q;
          R[v * S + lane] = r;
          if (WITH_D) D[v * S + lane] += breg[0] * P[v * S + lane];
          d3 += (double)q * (double)(c.dinv[v] * r);
        }
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      const bool ok = v < rg.end;
      sQ[row][lane] = ok ? Q[v * S + lane] : T(0);
      sR[row][lane] = ok ? R[v * S + lane] : T(0);
      if (WITH_D) {
        sP[row][lane] = ok ? P[v * S + lane] : T(0);
        sD[row][lane] = ok ? D[v * S + lane] : T(0);
      }
    }
    if (threadIdx.x < CH) {
      const int64_t v = base + threadIdx.x;
      sDinv[threadIdx.x] = v < rg.end ? c.dinv[v] : T(0);
    }
    __syncthreads();
    const auto qa = prod_tile<T>(sQ, nb, breg, lane);
    typename Acc<T>::type pa = {0, 0, 0, 0};
    if (WITH_D) pa = prod_tile<T>(sP, nb, breg, lane);
    T rn[4], zn[4], dn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      rn[r] = sR[row][col] - qa[r];
      zn[r] = sDinv[row] * rn[r];
      if (WITH_D) dn[r] = sD[row][col] + pa[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sR[row][col] = rn[r];
      sP[row][col] = zn[r];
      if (WITH_D) sD[row][col] = dn[r];
    }
    __syncthreads();
    gram_chunk<T>(sQ, sP, w, lane, a3);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < rg.end) {
        R[v * S + lane] = sR[row][lane];
        if (WITH_D) D[v * S + lane] = sD[row][lane];
      }
    }
    __syncthreads();
  }
  if (DIAG)
    diag_store(part_of(part, 2), d3, w, lane);
  else
    gram_store<T>(part_of(part, 2), w, lane, a3);
}

// ---------------------------------------------------------------- K3
// Y = Dinv R - P B;  W4 = Y^T D Y (block variant).
template <typename T, bool DIAG>
__global__ __launch_bounds__(WG, 4) void k_update_y(Coef<T> c, const T* __restrict__ delta,
                                                 const T* __restrict__ R,
                                                 const T* __restrict__ P, T* __restrict__ Y,
                                                 double* __restrict__ part) {
  __shared__ T sP[DIAG ? 1 : CH][LDW];  // P rows, then Y rows
  __shared__ T sR[DIAG ? 1 : CH][LDW];  // R rows, then D Y rows
  __shared__ T sDv[CH][2];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nb = w >> 2, cb = w & 3;
  const Range rg = block_range(c.n, gridDim.x);
  T breg[DIAG ? 1 : S / 4];
  if (DIAG)
    breg[0] = delta[lane];
  else
    load_bcol<T>(delta, cb, lane, breg);
  double a4[2][4];
  zero_acc(a4);
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) Y[v * S + lane] = c.dinv[v] * R[v * S + lane] - breg[0] * P[v * S + lane];
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      const bool ok = v < rg.end;
      sP[row][lane] = ok ? P[v * S + lane] : T(0);
      sR[row][lane] = ok ? R[v * S + lane] : T(0);
    }
    if (threadIdx.x < CH) {
      const int64_t v = base + threadIdx.x;
      const bool ok = v < rg.end;
      sDv[threadIdx.x][0] = ok ? c.dinv[v] : T(0);
      sDv[threadIdx.x][1] = ok ? c.d[v] : T(0);
    }
    __syncthreads();
    const auto pd = prod_tile<T>(sP, nb, breg, lane);
    T yn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      yn[r] = sDv[row][0] * sR[row][col] - pd[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sP[row][col] = yn[r];
      sR[row][col] = sDv[row][1] * yn[r];
    }
    __syncthreads();
    gram_chunk<T>(sP, sR, w, lane, a4);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < rg.end) Y[v * S + lane] = sP[row][lane];
    }
    __syncthreads();
  }
  if (!DIAG) gram_store<T>(part_of(part, 3), w, lane, a4);
}

// W4 = Y^T D Y alone (used when a refinement step restarts from a new Y).
template <typename T>
__global__ __launch_bounds__(WG) void k_gram_dy(Coef<T> c, const T* __restrict__ Y,
                                                double* __restrict__ part) {
  __shared__ T sY[CH][LDW];
  __shared__ T sDY[CH][LDW];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  double a4[2][4];
  zero_acc(a4);
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      const T y = v < rg.end ? Y[v * S + lane] : T(0);
      sY[row][lane] = y;
      sDY[row][lane] = v < rg.end ? c.d[v] * y : T(0);
    }
    __syncthreads();
    gram_chunk<T>(sY, sDY, w, lane, a4);
    __syncthreads();
  }
  gram_store<T>(part_of(part, 3), w, lane, a4);
}

// ---------------------------------------------------------------- Kr
// W[m][e] = sum_g part[g][m][e] for m in [m0, m0+nmat), e < len, summed in
// a fixed order (deterministic).  Eight independent partial sums per thread
// keep many loads in flight.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part,
                                                double* __restrict__ W, int G, int m0,
                                                int nmat, int len) {
  __shared__ double red[4][64];
  const int el = threadIdx.x & 63;
  const int grp = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  const int total = nmat * len;
  const int m = m0 + (e < total ? e / len : 0);
  const int off = e % len;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  if (e < total) {
    int g = grp;
    for (; g + 28 < G; g += 32) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += part[((size_t)(g + 4 * u) * NGRAM + m) * S * S + off];
    }
    for (; g < G; g += 4) acc[0] += part[((size_t)g * NGRAM + m) * S * S + off];
  }
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < total)
    W[(size_t)m * S * S + off] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

// ---------------------------------------------------------------- small
// Dense S x S work in one workgroup, float64 throughout.
constexpr int SM_THREADS = 256;
typedef double Mat[S][S + 1];





__device__ void convergence_update(BlockState* st, const double* dpsi, double tol) {
  // Column k (thread k < S) adds its increment, keeps the last HIST
  // increments and extrapolates what is left geometrically from the sums A,
  // B of |increment| over the older and the newer half of that window:
  //   tail ~= B * rho / (1 - rho),  rho = B / A,
  // reported relative to max(psi, ref).  Krylov convergence speeds up
  // rather than slows down, so the geometric tail tends to over-estimate.
  __shared__ int nconv;
  const int k = threadIdx.x;
  const int it = st->it;
  if (k == 0) nconv = 0;
  __syncthreads();
  if (k < S) {
    const double d = dpsi[k];
    const double psi = st->psi[k] + d;
    st->psi[k] = psi;
    st->hist[it % HIST][k] = d;
    const int itn = it + 1;
    double est = INFINITY;
    if (itn >= 2 * HIST) {
      double A = 0.0, B = 0.0;
      for (int h = 0; h < HIST; ++h) {
        const double val = fabs(st->hist[(itn - HIST + h) % HIST][k]);
        if (h < HIST / 2)
          A += val;
        else
          B += val;
      }
      const double ref = fmax(fabs(psi), st->ref[k]);
      if (B == 0.0) {
        est = 0.0;
      } else if (A > B && ref > 0.0) {
        const double rho = B / A;
        est = (B * rho / (1.0 - rho)) / ref;
      }
    }
    st->est_rel[k] = est;
    if (est <= CONV_SAFETY * tol) atomicAdd(&nconv, 1);
  }
  __syncthreads();
  if (k == 0) {
    st->it = it + 1;
    if (nconv == S) st->all_conv = 1;
  }
}

// Register-resident S x S matrices for the small kernels: wave w (0..3)
// holds rows 16w .. 16w+15 and lane k holds column k, so a[r] = M[16w+r][k].
__device__ __forceinline__ void load_sym_regs(const double* __restrict__ M, Mat& tmp,
                                              double (&a)[16]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 16; ++r) tmp[16 * w + r][lane] = M[(16 * w + r) * S + lane];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    a[r] = 0.5 * (tmp[i][lane] + tmp[lane][i]);
  }
  __syncthreads();
}

// Jacobi scaling: sc[i] = 1/sqrt(M_ii) for live columns, 0 otherwise (empty,
// non-finite, or not above floor_[i]); a is scaled in place.
__device__ void scale_regs(double (&a)[16], double* sc, const double* floor_) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ double dg[S];
  __shared__ double maxd;
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if (16 * w + r == lane) dg[lane] = a[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int j = 0; j < S; ++j) m = fmax(m, dg[j]);
    maxd = m;
  }
  __syncthreads();
  if (threadIdx.x < S) {
    const double d = dg[threadIdx.x];
    const bool live = isfinite(d) && d > 1e-300 && d > 1e-28 * maxd &&
                      (floor_ == nullptr || d > floor_[threadIdx.x]);
    sc[threadIdx.x] = live ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  const double sk = sc[lane];
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] *= sc[16 * w + r] * sk;
}

// Symmetric sweep of the Jacobi-scaled matrix held in registers, over every
// index in order.  Index j is swept only if its current pivot (the Schur
// complement with respect to the indices swept before it) is above eps;
// otherwise it is dropped as numerically dependent.  Afterwards a holds
// -(A_KK)^-1 on the kept set K.  If Tl is given, column j of the upper
// triangular T = Sc (e_j - beta)/sqrt(pivot) is written to it (beta: the
// coefficients of j on the kept earlier indices), so that T^T M T = I on K
// and T has zero columns for dropped j.
__device__ void sweep_regs(double (&a)[16], double eps, int* drop, const double* sc,
                           Mat* Tl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ double cjb[2][S];
  for (int j = 0; j < S; ++j) {
    double* cj = cjb[j & 1];
    if (lane == j) {
#pragma unroll
      for (int r = 0; r < 16; ++r) cj[16 * w + r] = a[r];
    }
    __syncthreads();
    const double piv = cj[j];
    const bool dj = !(piv > eps);
    if (threadIdx.x == 0) drop[j] = dj ? 1 : 0;
    if (Tl != nullptr && lane == j) {
      const double rs = dj ? 0.0 : 1.0 / sqrt(piv);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 16 * w + r;
        double t = 0.0;
        if (!dj) t = i < j ? (drop[i] ? 0.0 : -cj[i] * rs) : (i == j ? rs : 0.0);
        (*Tl)[i][j] = sc[i] * t;
      }
    }
    if (!dj) {
      const double inv = 1.0 / piv;
      const double ck = cj[lane];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 16 * w + r;
        const double ci = cj[i];
        if (i == j)
          a[r] = (lane == j) ? -inv : ck * inv;
        else if (lane == j)
          a[r] = ci * inv;
        else
          a[r] -= ci * ck * inv;
      }
    }
  }
  __syncthreads();
}

// C[16w+r][lane] = sum_j A[16w+r][j] * B[j][lane] with A, B in LDS.
__device__ __forceinline__ void mm_rows(const Mat& A, const Mat& B, double (&c)[16]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 16; ++r) c[r] = 0.0;
  for (int j = 0; j < S; ++j) {
    const double b = B[j][lane];
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] += A[16 * w + r][j] * b;
  }
}

// Ks1: W1^+ by the guarded sweep (kept in winv), A = W1^+ W2, psi update
// from the target rows of P, convergence.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small1(const double* __restrict__ W,
                                                       const T* __restrict__ P,
                                                       const int64_t* __restrict__ tgt,
                                                       double* __restrict__ winv,
                                                       T* __restrict__ alpha_out,
                                                       BlockState* __restrict__ st, double tol,
                                                       double eps, int diag) {
  __shared__ Mat Wi, B, PT;
  __shared__ double sc[S], dpsi[S];
  __shared__ int drop[S];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const bool frozen = st->frozen != 0;
  // outputs are written at the end so that no barrier waits on global stores
  const double* W1 = W;
  const double* W2 = W + S * S;
  if (diag) {
    if (tid < S) {
      const double w1 = W1[tid];
      const double a = (w1 > 0.0 && !frozen) ? W2[tid] / w1 : 0.0;
      winv[tid] = w1 > 0.0 ? 1.0 / w1 : 0.0;
      alpha_out[tid] = (T)a;
      const int64_t v = tgt[tid];
      dpsi[tid] = v >= 0 ? a * (double)P[v * S + tid] : 0.0;
    }
    __syncthreads();
    if (!frozen) convergence_update(st, dpsi, tol);
    __syncthreads();
    if (tid == 0 && st->all_conv) st->frozen = 1;
    return;
  }
  double a[16];
  load_sym_regs(W1, Wi, a);
  // Stage W2 and the target rows of P while the sweep runs.
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    B[i][lane] = W2[i * S + lane];
    const int64_t v = tgt[i];
    PT[i][lane] = v >= 0 ? (double)P[v * S + lane] : 0.0;
  }
  scale_regs(a, sc, nullptr);
  sweep_regs(a, eps, drop, sc, nullptr);
  const double sk = sc[lane];
  const bool dk = drop[lane] != 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    Wi[i][lane] = (drop[i] || dk) ? 0.0 : -a[r] * sc[i] * sk;
  }
  __syncthreads();
  double c[16];
  mm_rows(Wi, B, c);  // alpha = W1^+ W2
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) B[16 * w + r][lane] = frozen ? 0.0 : c[r];
  __syncthreads();
  // psi_k increment: row tgt_k of P times column k of alpha.
  if (tid < S) {
    double acc = 0.0;
    for (int j = 0; j < S; ++j) acc += PT[tid][j] * B[j][tid];
    dpsi[tid] = acc;
  }
  if (tid == 0) {
    int nd = 0;
    for (int j = 0; j < S; ++j) nd += drop[j];
    st->n_drop = nd;
  }
  __syncthreads();
  if (!frozen) convergence_update(st, dpsi, tol);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    winv[i * S + lane] = Wi[i][lane];
    alpha_out[i * S + lane] = (T)B[i][lane];
  }
  __syncthreads();
  if (tid == 0 && st->all_conv) st->frozen = 1;
}

// Ks2: B = W1^+ W3.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small2(const double* __restrict__ W,
                                                       const double* __restrict__ winv,
                                                       T* __restrict__ delta_out,
                                                       const BlockState* __restrict__ st,
                                                       int diag) {
  __shared__ Mat A, B;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const double* W3 = W + 2 * S * S;
  const bool frozen = st->frozen != 0;
  if (diag) {
    if (tid < S) delta_out[tid] = frozen ? (T)0 : (T)(W3[tid] * winv[tid]);
    return;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    A[i][lane] = winv[i * S + lane];
    B[i][lane] = W3[i * S + lane];
  }
  __syncthreads();
  double c[16];
  mm_rows(A, B, c);
#pragma unroll
  for (int r = 0; r < 16; ++r) delta_out[(16 * w + r) * S + lane] = frozen ? (T)0 : (T)c[r];
}

// Ks3: T from the guarded sweep of W4 = Y^T D Y, so that the kept columns
// of Y T are D-orthonormal.  A column whose squared D-norm has fallen below
// tau times its value at the start of the solve carries only rounding noise
// (its residual has converged) and is dropped as well; the first call after
// a (re)start records those reference norms.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small3(const double* __restrict__ W,
                                                       T* __restrict__ Tg,
                                                       BlockState* __restrict__ st, double eps,
                                                       double tau) {
  __shared__ Mat tmp, Tl;
  __shared__ double sc[S], floor_[S];
  __shared__ int drop[S];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* W4 = W + 3 * S * S;
  const bool first = st->it == 0;
  double djj = 0.0;
  if (threadIdx.x < S) {
    djj = W4[threadIdx.x * S + threadIdx.x];
    floor_[threadIdx.x] = first ? 0.0 : tau * st->scale0[threadIdx.x];
  }
  double a[16];
  load_sym_regs(W4, tmp, a);
  scale_regs(a, sc, floor_);
  sweep_regs(a, eps, drop, sc, &Tl);
#pragma unroll
  for (int r = 0; r < 16; ++r) Tg[(16 * w + r) * S + lane] = (T)Tl[16 * w + r][lane];
  if (first && threadIdx.x < S) st->scale0[threadIdx.x] = djj;
}

// ---------------------------------------------------------------- init
template <typename T>
__global__ void k_zero(T* __restrict__ a, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = T(0);
}

__device__ void reset_columns(BlockState* st, int k, bool clear_ref) {
  st->psi[k] = 0.0;
  st->est_rel[k] = INFINITY;
  if (clear_ref) st->ref[k] = 0.0;
  for (int h = 0; h < HIST; ++h) st->hist[h][k] = 0.0;
  if (k == 0) {
    st->it = 0;
    st->all_conv = 0;
    st->frozen = 0;
    st->n_drop = 0;
  }
}

// R = E (unit column k at node tgt[k]), Y = Dinv E, T = diag(sqrt(d_tgt))
// (so that P = Y T is D-orthonormal), state cleared.  R, Y (and D) were
// zeroed before.
template <typename T>
__global__ void k_set_targets(const T* __restrict__ d, const T* __restrict__ dinv,
                              const int64_t* __restrict__ tgt, T* __restrict__ R,
                              T* __restrict__ Y, T* __restrict__ Tm, BlockState* st,
                              int diag) {
  const int k = threadIdx.x;
  if (k < S) {
    const int64_t v = tgt[k];
    if (v >= 0) {
      R[v * S + k] = T(1);
      Y[v * S + k] = dinv[v];
    }
    for (int j = 0; j < S; ++j)
      Tm[j * S + k] = (T)((j == k && v >= 0) ? (diag ? 1.0 : sqrt((double)d[v])) : 0.0);
    reset_columns(st, k, true);
    st->scale0[k] = v >= 0 ? (double)dinv[v] : 0.0;
  }
}

// ---------------------------------------------------------------- mixed path
// X += D (float64 accumulation of the float32 correction).
__global__ void k_accum(double* __restrict__ X, const float* __restrict__ D, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    X[i] += (double)D[i];
}

// r = E - G X in float64; partial sums of x_k . r_k per column.  r is also
// stored (as float) into R for a further refinement step, with Y = Dinv r
// and D = 0.
__global__ __launch_bounds__(WG) void k_resid(Coef<double> c, Coef<float> cf,
                                              const double* __restrict__ X,
                                              const int64_t* __restrict__ tgt,
                                              float* __restrict__ Rf, float* __restrict__ Yf,
                                              float* __restrict__ Df,
                                              double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  const int64_t my_t = tgt[lane];
  double acc = 0.0;
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = base + w * NODES_PER_WAVE + i;
      if (v < rg.end) {
        const double gx = stencil_row<double, double>(c, X, v, lane);
        const double r = (v == my_t ? 1.0 : 0.0) - gx;
        acc += X[v * S + lane] * r;
        Rf[v * S + lane] = (float)r;
        Yf[v * S + lane] = cf.dinv[v] * (float)r;
        Df[v * S + lane] = 0.0f;
      }
    }
  }
  __shared__ double red[WG / 64][S];
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    double s = 0;
    for (int u = 0; u < WG / 64; ++u) s += red[u][lane];
    part_of(part, 0)[lane] = s;
  }
}

// Variational estimate R_k = e^T x + x^T r = 2 e^T x - x^T G x (float64),
// whose error is the energy norm of the solution error (>= 0).
__global__ void k_finalize_mixed(const double* __restrict__ X, const int64_t* __restrict__ tgt,
                                 const double* __restrict__ W, BlockState* st,
                                 double* __restrict__ out, const int64_t* __restrict__ pos) {
  const int k = threadIdx.x;
  if (k < S) {
    const int64_t v = tgt[k];
    double val = 0.0;
    if (v >= 0) val = X[v * S + k] + W[k];
    st->ref[k] = val;
    if (pos[k] >= 0) out[pos[k]] = val;
  }
}

__global__ void k_finalize_plain(const BlockState* st, double* __restrict__ out,
                                 const int64_t* __restrict__ pos) {
  const int k = threadIdx.x;
  if (k < S && pos[k] >= 0) out[pos[k]] = st->psi[k];
}

__global__ void k_reset_state(BlockState* st) {
  const int k = threadIdx.x;
  if (k < S) reset_columns(st, k, false);
}

// out_user[i] = res[map[i]] (map < 0 -> 0.0): solved values scattered into
// the caller's order on the device.
__global__ void k_gather_out(const double* __restrict__ res, const int64_t* __restrict__ map,
                             double* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = map[i];
    out[i] = m >= 0 ? res[m] : 0.0;
  }
}

// ---------------------------------------------------------------- launchers
template <typename T>
static hipError_t iteration_t(bool indep, bool with_d, const Coef<T>& c, const SolveBuffers& b,
                              double tol, hipStream_t st, hipEvent_t* ev) {
  const int G = grid_for(c.n);
  T* Y = (T*)b.Y;
  T* P = (T*)b.P;
  T* Q = (T*)b.Q;
  T* R = (T*)b.R;
  T* D = (T*)b.D;
  // Rank guards (relative pivots of the Jacobi-scaled Grams) and the
  // converged-column floor, per precision.
  const double eps1 = sizeof(T) == 8 ? 1e-10 : 1e-7;
  const double eps4 = sizeof(T) == 8 ? 1e-14 : 1e-6;
  const double tau = sizeof(T) == 8 ? 1e-26 : 1e-12;
  const int len = indep ? S : S * S;
  const int di = indep ? 1 : 0;
  const dim3 g(G), blk(WG);
  const T* Tm = (const T*)b.Tm;
  if (ev) hipEventRecord(ev[0], st);
  if (indep)
    hipLaunchKernelGGL((k_stencil_gram<T, true>), g, blk, 0, st, c, Y, Tm, R, P, Q, b.part);
  else
    hipLaunchKernelGGL((k_stencil_gram<T, false>), g, blk, 0, st, c, Y, Tm, R, P, Q, b.part);
  if (ev) hipEventRecord(ev[1], st);
  hipLaunchKernelGGL(k_reduce, dim3((2 * len + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 0,
                     2, len);
  hipLaunchKernelGGL((k_small1<T>), dim3(1), dim3(SM_THREADS), 0, st, b.W, (const T*)P, b.tgt,
                     b.winv, (T*)b.alpha, b.state, tol, eps1, di);
  if (ev) hipEventRecord(ev[2], st);
  const T* al = (const T*)b.alpha;
  if (indep) {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, true, true>), g, blk, 0, st, c, al, Q, P, R, D, b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, true, false>), g, blk, 0, st, c, al, Q, P, R, D, b.part);
  } else {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, false, true>), g, blk, 0, st, c, al, Q, P, R, D, b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, false, false>), g, blk, 0, st, c, al, Q, P, R, D,
                         b.part);
  }
  if (ev) hipEventRecord(ev[3], st);
  hipLaunchKernelGGL(k_reduce, dim3((len + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 2, 1,
                     len);
  hipLaunchKernelGGL((k_small2<T>), dim3(1), dim3(SM_THREADS), 0, st, b.W, b.winv,
                     (T*)b.delta, b.state, di);
  if (ev) hipEventRecord(ev[4], st);
  const T* de = (const T*)b.delta;
  if (indep) {
    hipLaunchKernelGGL((k_update_y<T, true>), g, blk, 0, st, c, de, R, P, Y, b.part);
    if (ev) hipEventRecord(ev[5], st);
  } else {
    hipLaunchKernelGGL((k_update_y<T, false>), g, blk, 0, st, c, de, R, P, Y, b.part);
    if (ev) hipEventRecord(ev[5], st);
    hipLaunchKernelGGL(k_reduce, dim3((len + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 3, 1,
                       len);
    hipLaunchKernelGGL((k_small3<T>), dim3(1), dim3(SM_THREADS), 0, st, b.W, (T*)b.Tm, b.state,
                       eps4, tau);
  }
  return hipGetLastError();
}

hipError_t launch_iteration(bool fp32, bool indep, bool with_d, const void* coef,
                            const SolveBuffers& b, int64_t n, double tol, hipStream_t st,
                            hipEvent_t* ev) {
  (void)n;
  if (fp32) return iteration_t<float>(indep, with_d, *(const Coef<float>*)coef, b, tol, st, ev);
  return iteration_t<double>(indep, with_d, *(const Coef<double>*)coef, b, tol, st, ev);
}

template <typename T>
static hipError_t init_t(const Coef<T>& c, const SolveBuffers& b, bool indep, hipStream_t st) {
  const int64_t cnt = c.n * S;
  const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
  hipLaunchKernelGGL((k_zero<T>), dim3(blocks), dim3(256), 0, st, (T*)b.R, cnt);
  hipLaunchKernelGGL((k_zero<T>), dim3(blocks), dim3(256), 0, st, (T*)b.Y, cnt);
  if (b.D) hipLaunchKernelGGL((k_zero<T>), dim3(blocks), dim3(256), 0, st, (T*)b.D, cnt);
  hipLaunchKernelGGL((k_set_targets<T>), dim3(1), dim3(S), 0, st, c.d, c.dinv, b.tgt, (T*)b.R,
                     (T*)b.Y, (T*)b.Tm, b.state, indep ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_init_block(bool fp32, bool indep, const void* coef, const SolveBuffers& b,
                             hipStream_t st) {
  if (fp32) return init_t<float>(*(const Coef<float>*)coef, b, indep, st);
  return init_t<double>(*(const Coef<double>*)coef, b, indep, st);
}

hipError_t launch_zero_x(double* X, int64_t cnt, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
  hipLaunchKernelGGL((k_zero<double>), dim3(blocks), dim3(256), 0, st, X, cnt);
  return hipGetLastError();
}

hipError_t launch_mixed_residual(const Coef<double>& c, const Coef<float>& cf,
                                 const SolveBuffers& b, double* out, const int64_t* pos,
                                 hipStream_t st) {
  const int64_t cnt = c.n * S;
  const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
  hipLaunchKernelGGL(k_accum, dim3(blocks), dim3(256), 0, st, b.X, (const float*)b.D, cnt);
  const int G = grid_for(c.n);
  hipLaunchKernelGGL(k_resid, dim3(G), dim3(WG), 0, st, c, cf, b.X, b.tgt, (float*)b.R,
                     (float*)b.Y, (float*)b.D, b.part);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, b.part, b.W, G, 0, 1, S);
  hipLaunchKernelGGL(k_finalize_mixed, dim3(1), dim3(S), 0, st, b.X, b.tgt, b.W, b.state, out,
                     pos);
  return hipGetLastError();
}

__global__ void k_set_identity(float* __restrict__ Tm) {
  for (int e = threadIdx.x; e < S * S; e += blockDim.x) Tm[e] = (e / S == e % S) ? 1.0f : 0.0f;
}

hipError_t launch_restart(const Coef<float>& cf, const SolveBuffers& b, bool indep,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(S), 0, st, b.state);
  const int G = grid_for(cf.n);
  if (indep) {
    // T = I: the independent variant needs no orthonormalisation.
    hipLaunchKernelGGL(k_set_identity, dim3(1), dim3(256), 0, st, (float*)b.Tm);
  } else {
    hipLaunchKernelGGL((k_gram_dy<float>), dim3(G), dim3(WG), 0, st, cf, (const float*)b.Y,
                       b.part);
    hipLaunchKernelGGL(k_reduce, dim3((S * S + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 3,
                       1, S * S);
    hipLaunchKernelGGL((k_small3<float>), dim3(1), dim3(SM_THREADS), 0, st, b.W, (float*)b.Tm,
                       b.state, 1e-6, 1e-12);
  }
  return hipGetLastError();
}

hipError_t launch_finalize_plain(const SolveBuffers& b, double* out, const int64_t* pos,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_plain, dim3(1), dim3(S), 0, st, b.state, out, pos);
  return hipGetLastError();
}

hipError_t launch_gather_out(const double* res, const int64_t* map, double* out, int64_t count,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gather_out, dim3(blocks), dim3(256), 0, st, res, map, out, count);
  return hipGetLastError();
}

}  // namespace reff
