// gfx950 kernels of the block-PCG effective-resistance solver.
//
// Vectors are rows x S blocks stored row-major with the S = 64 right-hand
// sides contiguous (V[v*S + k]).  One wavefront owns one node at a time and
// lane k owns column k, so every vector access of a wave is one coalesced
// 64-element row and a node's stencil coefficients are wave-uniform (scalar
// loads).  Several solve blocks (one per stack of a batch, each with its own
// S right-hand sides) run in the same launches: the vector kernels walk a
// table of work units (node ranges of one block each), the small S x S
// kernels run one workgroup per block.
//
// Block PCG with rank-revealing orthonormalised search directions.  The
// search block arrives as Y (any basis) plus an S x S upper-triangular map T
// such that P = Y T has D-orthonormal kept columns (D = diag G) and zero
// dropped ones.  One iteration for all S columns of every block:
//   K1  Qt = G Y (stencil); P = Y T; Q = Qt T;  W1 = P^T Q, W2 = P^T R
//   Ks1 W1^+ by a guarded sweep;  A = W1^+ W2;
//       psi_k += sum_j P[tgt_k, j] A[j, k]  (= change of x_k at node tgt_k)
//   K2  R -= Q A;  (D += P A);  Z = Dinv R;  W3 = Q^T Z
//   Ks2 B = W1^+ W3
//   K3  Y = Z - P B;  W4 = Y^T D Y
//   Ks3 T from the guarded sweep of W4: directions whose pivot falls below
//       eps are numerically dependent and are dropped
// (the per-unit Gram partials are reduced per block by Kr first).  The
// S x S products and Grams of K1-K3 run on the matrix cores.  With x0 = 0
// and R0 = e_i, psi_k = e_i^T x_k is the Galerkin estimate of
// R_i = (G^-1)_ii and rises to it from below.  The "independent" variant
// keeps only the diagonals: S ordinary PCGs side by side.
#include "reff_internal.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace reff {

// Hardware dispatches workgroup b to XCD (b mod 8).  Give each XCD a
// contiguous range of logical units so that neighbouring node ranges, which
// share stencil halo rows, are served by the same L2.
__device__ __forceinline__ int logical_block(int b, int nb) {
  if ((nb & 7) != 0) return b;
  const int per = nb >> 3;
  return (b & 7) * per + (b >> 3);
}

// This workgroup's logical item among the n active ones of a kind (0 units,
// 1 strips; n read from device memory), or -1 when it has none.  With a grid
// that is a multiple of 8 the active items are spread evenly over the XCDs,
// each XCD taking a contiguous range.
__device__ __forceinline__ int active_item(const Work& wk, int kind) {
  const int n = wk.cnt[kind];
  const int b = (int)blockIdx.x;
  if ((gridDim.x & 7) != 0) return b < n ? b : -1;
  const int np = (n + 7) & ~7;
  if (b >= np) return -1;
  const int l = logical_block(b, np);
  return l < n ? l : -1;
}

// The unit, its block and the block's S x S matrices of this workgroup.
struct UnitCtx {
  int64_t begin, end;  // vector rows
  PlanDesc pd;
  int plan;
};

__device__ __forceinline__ UnitCtx unit_ctx(const Work& wk, int lu) {
  const Unit u = wk.units[wk.uid[lu]];
  UnitCtx c;
  c.begin = u.begin;
  c.end = u.end;
  c.plan = u.plan;
  c.pd = wk.plans[u.plan];
  return c;
}

int grid_for(int64_t n) {
  const int64_t nch = (n + CH - 1) / CH;
  return (int)(nch < MAX_GRID ? nch : MAX_GRID);
}

// (G y)_v for the lane's column; v is a vector row of block pd.
template <typename T, typename U>
__device__ __forceinline__ T stencil_row(const Coef<T>& c, const U* __restrict__ Y,
                                         const PlanDesc& pd, int64_t v, int lane) {
  const int64_t lv = v - pd.vbase;      // node of the stack
  const int64_t ci = pd.cbase + lv;     // its coefficient index
  const int64_t nx = pd.nx;
  const T ce = c.cE[ci];
  const T cn = c.cN[ci];
  const T cw = lv >= 1 ? c.cE[ci - 1] : T(0);
  const T cs = lv >= nx ? c.cN[ci - nx] : T(0);
  // Neighbour rows that do not exist fall back to v itself; their
  // coefficient is zero (grid edge or grounded node).
  const int64_t ve = lv + 1 < pd.n ? v + 1 : v;
  const int64_t vw = lv >= 1 ? v - 1 : v;
  const int64_t vn = lv + nx < pd.n ? v + nx : v;
  const int64_t vs = lv >= nx ? v - nx : v;
  const T y = (T)Y[v * S + lane];
  const T ye = (T)Y[ve * S + lane];
  const T yw = (T)Y[vw * S + lane];
  const T yn = (T)Y[vn * S + lane];
  const T ys = (T)Y[vs * S + lane];
  // TSV segments: the rows above / below exist only where the coupling is
  // nonzero; elsewhere the load repeats row v (an L1 hit) and is multiplied
  // by zero, so that no load sits behind a branch.
  const int sl = c.slot[ci];
  const int sc = sl >= 0 ? sl : 0;
  const T gu = sl >= 0 ? c.up[sc] : T(0);
  const T gd = sl >= 0 ? c.dn[sc] : T(0);
  const int64_t vu = gu != T(0) ? v + pd.plane : v;
  const int64_t vd = gd != T(0) ? v - pd.plane : v;
  const T yu = (T)Y[vu * S + lane];
  const T yd = (T)Y[vd * S + lane];
  return c.d[ci] * y - ce * ye - cw * yw - cn * yn - cs * ys - gu * yu - gd * yd;
}

// Partial Grams of unit u: part[u][m][S*S] (or the first S entries for
// diagonal-only Grams).
// Padded LDS row (words).  A row offset of 4 words spreads the 16 rows read
// by one product operand over distinct banks.
constexpr int LDW = S + 4;

__device__ __forceinline__ double* part_of(double* part, int unit, int m) {
  return part + ((size_t)unit * NGRAM + m) * S * S;
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

// Product tiles: rows [16 nb, 16 nb + 16) of CH x S blocks staged in LDS
// times an S x S matrix B, of which the lane holds column block cb.  The
// 64-term contraction runs over k-blocks kb of 16 and steps st of 4, taking
// k = 16 kb + 4 (l/16) + st at step (kb, st): a lane's A operands of one
// k-block are 4 consecutive words of its row (one wide LDS read), and
// breg[4 kb + st] = B[16 kb + 4 (l/16) + st][16 cb + l%16].  Only the first
// kbn k-blocks are taken (B upper triangular: kbn = cb + 1).
template <typename T>
__device__ __forceinline__ void load_arow(const T (*sA)[LDW], int nb, int lane, int kbn,
                                          T (&a)[S / 4]) {
  const T* row = &sA[nb * 16 + (lane & 15)][4 * (lane >> 4)];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    if (kb >= kbn) break;
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(row + 16 * kb);
      a[4 * kb] = v.x;
      a[4 * kb + 1] = v.y;
      a[4 * kb + 2] = v.z;
      a[4 * kb + 3] = v.w;
    } else {
      const double2 v0 = *reinterpret_cast<const double2*>(row + 16 * kb);
      const double2 v1 = *reinterpret_cast<const double2*>(row + 16 * kb + 2);
      a[4 * kb] = v0.x;
      a[4 * kb + 1] = v0.y;
      a[4 * kb + 2] = v1.x;
      a[4 * kb + 3] = v1.y;
    }
  }
}

template <typename T>
__device__ __forceinline__ typename Acc<T>::type prod_tile(const T (*sA)[LDW], int nb,
                                                           const T* breg, int lane, int kbn = 4) {
  typename Acc<T>::type c = {0, 0, 0, 0};
  if constexpr (sizeof(T) == 8) {  // float64: operands read step by step (registers)
    const T* row = &sA[nb * 16 + (lane & 15)][4 * (lane >> 4)];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      if (kb >= kbn) break;
#pragma unroll
      for (int st = 0; st < 4; ++st) c = mma(row[16 * kb + st], breg[4 * kb + st], c);
    }
  } else {
    T a[S / 4];
    load_arow<T>(sA, nb, lane, kbn, a);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      if (kb >= kbn) break;
#pragma unroll
      for (int st = 0; st < 4; ++st) c = mma(a[4 * kb + st], breg[4 * kb + st], c);
    }
  }
  return c;
}

// Two products with the same B, their matrix-core chains interleaved
// (float64: one after the other, to stay within the register budget).
template <typename T>
__device__ __forceinline__ void prod_tile2(const T (*sA1)[LDW], const T (*sA2)[LDW], int nb,
                                           const T* breg, int lane, typename Acc<T>::type& c1,
                                           typename Acc<T>::type& c2, int kbn = 4) {
  if constexpr (sizeof(T) == 8) {
    c1 = prod_tile<T>(sA1, nb, breg, lane, kbn);
    c2 = prod_tile<T>(sA2, nb, breg, lane, kbn);
  } else {
    // one k-block of both operands at a time (8 registers)
    const float* r1 = &sA1[nb * 16 + (lane & 15)][4 * (lane >> 4)];
    const float* r2 = &sA2[nb * 16 + (lane & 15)][4 * (lane >> 4)];
    c1 = typename Acc<T>::type{0, 0, 0, 0};
    c2 = typename Acc<T>::type{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      if (kb >= kbn) break;
      const float4 v1 = *reinterpret_cast<const float4*>(r1 + 16 * kb);
      const float4 v2 = *reinterpret_cast<const float4*>(r2 + 16 * kb);
      const float x1[4] = {v1.x, v1.y, v1.z, v1.w}, x2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        c1 = mma(x1[st], breg[4 * kb + st], c1);
        c2 = mma(x2[st], breg[4 * kb + st], c2);
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void load_bcol(const T* __restrict__ B, int cb, int lane, T* breg) {
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int st = 0; st < 4; ++st)
      breg[4 * kb + st] = B[(16 * kb + 4 * (lane >> 4) + st) * S + 16 * cb + (lane & 15)];
}

// Wave w owns Gram tiles 2w and 2w+1 of the 4 x 4 tiles of an S x S Gram
// (same tile row ti = w / 2, columns 2 (w % 2) and 2 (w % 2) + 1): one A
// operand read serves both, and the two matrix-core chains interleave.
template <typename T>
__device__ __forceinline__ void gram_chunk(const T (*sA)[LDW], const T (*sB)[LDW], int w,
                                           int lane, double (&acc)[2][4]) {
  typename Acc<T>::type c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
  const int kr = lane >> 4, cc = lane & 15;
  const int ti = (2 * w) >> 2, tj = (2 * w) & 3;
#pragma unroll
  for (int kb = 0; kb < CH; kb += 4) {
    const T a = sA[kb + kr][ti * 16 + cc];
    c0 = mma(a, sB[kb + kr][tj * 16 + cc], c0);
    c1 = mma(a, sB[kb + kr][(tj + 1) * 16 + cc], c1);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    acc[0][r] += (double)c0[r];
    acc[1][r] += (double)c1[r];
  }
}

// Two Grams A^T B1 and A^T B2 with the same tiles: four interleaved chains.
template <typename T>
__device__ __forceinline__ void gram_chunk2(const T (*sA)[LDW], const T (*sB1)[LDW],
                                            const T (*sB2)[LDW], int w, int lane,
                                            double (&acc1)[2][4], double (&acc2)[2][4]) {
  if constexpr (sizeof(T) == 8) {  // float64: within the register budget
    gram_chunk<T>(sA, sB1, w, lane, acc1);
    gram_chunk<T>(sA, sB2, w, lane, acc2);
    return;
  }
  typename Acc<T>::type c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0}, d0 = {0, 0, 0, 0},
                        d1 = {0, 0, 0, 0};
  const int kr = lane >> 4, cc = lane & 15;
  const int ti = (2 * w) >> 2, tj = (2 * w) & 3;
#pragma unroll
  for (int kb = 0; kb < CH; kb += 4) {
    const T a = sA[kb + kr][ti * 16 + cc];
    c0 = mma(a, sB1[kb + kr][tj * 16 + cc], c0);
    c1 = mma(a, sB1[kb + kr][(tj + 1) * 16 + cc], c1);
    d0 = mma(a, sB2[kb + kr][tj * 16 + cc], d0);
    d1 = mma(a, sB2[kb + kr][(tj + 1) * 16 + cc], d1);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    acc1[0][r] += (double)c0[r];
    acc1[1][r] += (double)c1[r];
    acc2[0][r] += (double)d0[r];
    acc2[1][r] += (double)d1[r];
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
__global__ __launch_bounds__(WG, 4) void k_stencil_gram(Coef<T> c, Work wk,
                                                        const T* __restrict__ Y,
                                                        const T* __restrict__ Tm,
                                                        const T* __restrict__ R,
                                                        T* __restrict__ P, T* __restrict__ Q,
                                                        double* __restrict__ part) {
  __shared__ __align__(16) T sA[DIAG ? 1 : CH][LDW];  // Y rows, then P rows
  __shared__ __align__(16) T sB[DIAG ? 1 : CH][LDW];  // G Y rows, then Q rows
  __shared__ __align__(16) T sR[DIAG ? 1 : CH][LDW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  // Product tile (nb, cb) of wave w; T is upper triangular, so tile column
  // cb needs cb + 1 k-blocks: the two waves sharing a SIMD (w, w + 4) take
  // cb and 3 - cb, five k-blocks per SIMD.
  const int nb = w >> 2, cb = nb == 0 ? (w & 3) : 3 - (w & 3);
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  T breg[DIAG ? 1 : S / 4];
  if (!DIAG) load_bcol<T>(Tm + (size_t)u.plan * S * S, cb, lane, breg);
  double a1[2][4], a2[2][4];
  zero_acc(a1);
  zero_acc(a2);
  double d1 = 0.0, d2 = 0.0;
  for (int64_t base = u.begin; base < u.end; base += CH) {
    if (DIAG) {
      T yv[NODES_PER_WAVE], rv[NODES_PER_WAVE], qv[NODES_PER_WAVE];
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
        yv[i] = Y[v * S + lane];
        rv[i] = R[v * S + lane];
        qv[i] = stencil_row<T, T>(c, Y, u.pd, v, lane);
      }
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < u.end) {
          P[v * S + lane] = yv[i];
          Q[v * S + lane] = qv[i];
          d1 += (double)yv[i] * (double)qv[i];
          d2 += (double)yv[i] * (double)rv[i];
        }
      }
      continue;
    }
    // All loads of the chunk first (rows past the unit's end are clamped to
    // its last row and zeroed afterwards), so none waits behind a branch.
    T yv[NODES_PER_WAVE], rv[NODES_PER_WAVE], qv[NODES_PER_WAVE];
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
      yv[i] = Y[v * S + lane];
      rv[i] = R[v * S + lane];
      qv[i] = stencil_row<T, T>(c, Y, u.pd, v, lane);
    }
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const bool ok = base + row < u.end;
      sA[row][lane] = ok ? yv[i] : T(0);
      sB[row][lane] = ok ? qv[i] : T(0);
      sR[row][lane] = ok ? rv[i] : T(0);
    }
    __syncthreads();
    typename Acc<T>::type pt, qt;
    prod_tile2<T>(sA, sB, nb, breg, lane, pt, qt, cb + 1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sA[row][col] = pt[r];
      sB[row][col] = qt[r];
    }
    __syncthreads();
    gram_chunk2<T>(sA, sB, sR, w, lane, a1, a2);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < u.end) {
        P[v * S + lane] = sA[row][lane];
        Q[v * S + lane] = sB[row][lane];
      }
    }
    __syncthreads();
  }
  if (DIAG) {
    diag_store(part_of(part, uidx, 0), d1, w, lane);
    __syncthreads();
    diag_store(part_of(part, uidx, 1), d2, w, lane);
  } else {
    gram_store<T>(part_of(part, uidx, 0), w, lane, a1);
    gram_store<T>(part_of(part, uidx, 1), w, lane, a2);
  }
}

// Read of an array that no kernel writes while a solve runs (stencil
// coefficients): through the constant address space, so that a
// wave-uniform index becomes a scalar-cache load that no vector store in
// the kernel can be taken to clobber.
template <typename T>
__device__ __forceinline__ T ldc(const T* p, int64_t i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}

// K1 over strips (block variant): the same products and Grams, with the
// stencil read from an on-chip window.  The workgroup marches its strip in
// +y; the ring win[3] holds the Y rows y-1, y, y+1 of the strip plus one
// halo node on each side (column 0 = x0-1, column j+1 = node x0+j), so
// every Y row comes from HBM once.  The loads of row y+2, of R row y+1 and
// of the coefficients of row y+1 are issued before row y's work and written
// to LDS after its products, in the same iteration: every load reads a
// clamped, valid address, values outside the tier or the strip become zero
// only when written to LDS, and no load or store sits under a data-dependent
// branch, so no instruction waits for the next row before that point.
template <typename T>
__global__ __launch_bounds__(WG, 4) void k_stencil_gram_strip(Coef<T> c, Work wk,
                                                              const T* __restrict__ Y,
                                                              const T* __restrict__ Tm,
                                                              const T* __restrict__ R,
                                                              T* __restrict__ P,
                                                              T* __restrict__ Q,
                                                              double* __restrict__ part) {
  constexpr int HWW = CH + 2;
  constexpr int NPW = NODES_PER_WAVE;
  __shared__ __align__(16) T win[3][HWW][LDW];
  __shared__ __align__(16) T sR[2][CH][LDW];  // R rows of row y in buffer s % 2
  __shared__ __align__(16) T sQ[CH][LDW];     // G Y rows
  __shared__ __align__(16) T sQo[CH][LDW];    // Q rows
  __shared__ __align__(16) T sP[CH][LDW];
  // Stencil coefficients of row y (buffer s % 2): d, cE from node x0-1 on,
  // cN (buffer s % 2 = row y, the other = row y-1), TSV slot.
  __shared__ T cd[2][CH], ce[2][CH + 1], cn[2][CH];
  __shared__ int cslot[2][CH];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  // Product tile (nb, cb): T is upper triangular (see k_stencil_gram).
  const int nb = w >> 2, cb = nb == 0 ? (w & 3) : 3 - (w & 3);
  const int ls = active_item(wk, 1);
  if (ls < 0) return;
  const int sidx = wk.sid[ls];
  const Strip st = wk.strips[sidx];
  const PlanDesc pd = wk.plans[st.plan];
  const int64_t nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  const int wdt = st.wdt;
  const bool has_w = st.x0 > 0;
  const bool has_e = st.x0 + wdt < pd.nx;
  T breg[S / 4];
  load_bcol<T>(Tm + (size_t)st.plan * S * S, cb, lane, breg);
  double a1[2][4], a2[2][4];
  zero_acc(a1);
  zero_acc(a2);
  // Window row yy of the strip: this thread's nodes are j = 4w + i, plus the
  // west halo (wave 0) and east halo (wave 1; a strip narrower than CH ends
  // at the east edge of the tier).  Rows outside the tier are 0.
  const int hoff = w == 0 ? (has_w ? -1 : 0) : (has_e ? wdt : 0);
  auto load_row = [&](int yy, T (&v)[NPW], T& halo) {
    const bool in = yy >= 0 && yy < ny;
    const int64_t base = pd.vbase + st.lrow0 + (int64_t)((in ? yy : st.y0) - st.y0) * nx;
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = Y[(base + min(w * NPW + i, wdt - 1)) * S + lane];
    if (w < 2) halo = Y[(base + hoff) * S + lane];
  };
  auto store_row = [&](int slot, const T (&v)[NPW], T halo, int yy) {
    const bool in = yy >= 0 && yy < ny;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      win[slot][j + 1][lane] = (in && j < wdt) ? v[i] : T(0);
    }
    if (w == 0) win[slot][0][lane] = (in && has_w) ? halo : T(0);
    if (w == 1 && wdt == CH) win[slot][CH + 1][lane] = (in && has_e) ? halo : T(0);
  };
  auto load_r = [&](int s, T (&v)[NPW]) {
    const int64_t base = pd.vbase + st.lrow0 + (int64_t)min(s, st.nrows - 1) * nx;
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = R[(base + min(w * NPW + i, wdt - 1)) * S + lane];
  };
  auto store_r = [&](int b, const T (&v)[NPW]) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      sR[b][j][lane] = j < wdt ? v[i] : T(0);
    }
  };
  // Coefficients of strip row s, one value per thread t <= 3 CH of waves
  // 0 - 1 (t < CH: d;  CH <= t <= 2 CH: cE of node x0 - 1 + (t - CH);
  // 2 CH < t <= 3 CH: cN), and one slot entry per thread t of waves 0 - 2
  // (used by 3 CH < t <= 4 CH).
  const int t = threadIdx.x;
  const int kc = t < CH ? t : t <= 2 * CH ? t - CH - 1 : t - 2 * CH - 1;
  const int klo = (t == CH && has_w) ? -1 : 0;
  const T* csrc = t < CH ? c.d : t <= 2 * CH ? c.cE : c.cN;
  const int ks = t - 3 * CH - 1;
  auto load_coef = [&](int srow, T& val, int& sl) {
    if (w < 3) {
      const int64_t base = pd.cbase + st.lrow0 + (int64_t)min(srow, st.nrows - 1) * nx;
      val = csrc[base + min(max(kc, klo), wdt - 1)];
      sl = c.slot[base + min(max(ks, 0), wdt - 1)];
    }
  };
  auto store_coef = [&](int b, T val, int sl) {
    if (t < CH) {
      cd[b][t] = val;
    } else if (t <= 2 * CH) {
      const int e = t - CH;  // node x0 - 1 + e
      ce[b][e] = ((e > 0 || has_w) && e <= wdt) ? val : T(0);
    } else if (t <= 3 * CH) {
      cn[b][t - 2 * CH - 1] = val;
    } else if (t <= 4 * CH) {
      cslot[b][t - 3 * CH - 1] = sl;
    }
  };
  // Prologue: rows y0-1, y0, y0+1 into slots 0, 1, 2; R row y0 and the
  // coefficients of row y0 into buffer 0; cN of row y0-1 into buffer 1.
  {
    T v[NPW], h = T(0), cv = T(0);
    int csl = -1;
    load_row(st.y0 - 1, v, h);
    store_row(0, v, h, st.y0 - 1);
    load_row(st.y0, v, h);
    store_row(1, v, h, st.y0);
    load_row(st.y0 + 1, v, h);
    store_row(2, v, h, st.y0 + 1);
    load_r(0, v);
    store_r(0, v);
    load_coef(0, cv, csl);
    store_coef(0, cv, csl);
    if (t > 2 * CH && t <= 3 * CH) {
      const int j = t - 2 * CH - 1;
      const int64_t ci = pd.cbase + st.lrow0 + min(j, wdt - 1) - nx;  // row y0 - 1
      cn[1][j] = st.y0 > 0 ? c.cN[st.y0 > 0 ? ci : ci + nx] : T(0);
    }
  }
  __syncthreads();
  for (int s = 0; s < st.nrows; ++s) {
    const int y = st.y0 + s;
    const int ss = s % 3, sc = (s + 1) % 3, sn = (s + 2) % 3;  // rows y-1, y, y+1
    const int b = s & 1;
    const int64_t obase = pd.vbase + st.lrow0 + (int64_t)s * nx;
    // TSV partners (tiers above / below) of this row's nodes, read before
    // the next row so that waiting for them does not wait for that row.
    int sl[NPW];
    bool any = false;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      sl[i] = __builtin_amdgcn_readfirstlane(cslot[b][min(w * NPW + i, wdt - 1)]);
      any |= sl[i] >= 0;
    }
    T gu[NPW], gd[NPW], yu[NPW], yd[NPW];
    if (any) {  // wave-uniform
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int64_t v = obase + min(w * NPW + i, wdt - 1);
        // slot 0 exists: some node of this wave has a TSV
        const int q = max(sl[i], 0);
        gu[i] = sl[i] >= 0 ? ldc(c.up, q) : T(0);
        gd[i] = sl[i] >= 0 ? ldc(c.dn, q) : T(0);
        yu[i] = Y[(gu[i] != T(0) ? v + pd.plane : v) * S + lane];
        yd[i] = Y[(gd[i] != T(0) ? v - pd.plane : v) * S + lane];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NPW; ++i) gu[i] = gd[i] = yu[i] = yd[i] = T(0);
    }
    // next row (the last iteration reads valid rows again and discards them)
    T ny_v[NPW], ny_h = T(0), r_v[NPW], c_v = T(0);
    int c_sl = -1;
    load_row(y + 2, ny_v, ny_h);
    load_r(s + 1, r_v);
    load_coef(s + 1, c_v, c_sl);
    // (G Y)_v for this wave's nodes of row y.
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      const int jc = min(j, wdt - 1);
      T q = cd[b][jc] * win[sc][jc + 1][lane] - ce[b][jc + 1] * win[sc][jc + 2][lane] -
            ce[b][jc] * win[sc][jc][lane] - cn[b][jc] * win[sn][jc + 1][lane] -
            cn[b ^ 1][jc] * win[ss][jc + 1][lane];
      q -= gu[i] * yu[i] + gd[i] * yd[i];
      sQ[j][lane] = j < wdt ? q : T(0);
    }
    __syncthreads();
    typename Acc<T>::type pt, qt;
    prod_tile2<T>(&win[sc][1], sQ, nb, breg, lane, pt, qt, cb + 1);
    // Two barriers per row.  sP, sQo and sR[b ^ 1] were last read by the
    // previous row's Grams, which precede the barrier after this row's
    // stencil; so were the window slot of row y - 1 and the coefficients of
    // row y - 1 (read by this row's stencil).  Row y + 2, R of row y + 1 and
    // the coefficients of row y + 1 go there now, before the barrier that
    // opens the Grams and makes them visible to the next row's stencil.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sP[row][col] = pt[r];
      sQo[row][col] = qt[r];
    }
    store_row(ss, ny_v, ny_h, y + 2);
    store_r(b ^ 1, r_v);
    store_coef(b ^ 1, c_v, c_sl);
    __syncthreads();
    gram_chunk2<T>(sP, sQo, sR[b], w, lane, a1, a2);
    // nodes past a ragged strip's width store the last node's row again
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int jc = min(w * NPW + i, wdt - 1);
      P[(obase + jc) * S + lane] = sP[jc][lane];
      Q[(obase + jc) * S + lane] = sQo[jc][lane];
    }
  }
  gram_store<T>(part_of(part, sidx, 0), w, lane, a1);
  gram_store<T>(part_of(part, sidx, 1), w, lane, a2);
}

// ---------------------------------------------------------------- K2
// R -= Q A;  (D += P A);  Z = Dinv R;  W3 = Q^T Z.
// With CHEB (polynomial preconditioner, block variant) the kernel does not
// form W3 (a Gram kernel takes it from the finished Z) and writes z_1 =
// D^-1 R / theta, the Chebyshev steps' start, to Z1 unless Z1 is null (the
// first Chebyshev pass then forms z_1 from R itself).
template <typename T, bool DIAG, bool WITH_D, bool CHEB = false>
__global__ __launch_bounds__(WG, 4) void k_update_r(Coef<T> c, Work wk,
                                                    const T* __restrict__ alpha,
                                                    const T* __restrict__ Q,
                                                    const T* __restrict__ P, T* __restrict__ R,
                                                    T* __restrict__ D,
                                                    double* __restrict__ part,
                                                    T* __restrict__ Z1 = nullptr,
                                                    T inv_theta = T(1)) {
  __shared__ __align__(16) T sQ[DIAG ? 1 : CH][LDW];
  __shared__ __align__(16) T sP[DIAG ? 1 : CH][LDW];  // P rows, then Z rows
  __shared__ __align__(16) T sR[DIAG ? 1 : CH][LDW];
  __shared__ __align__(16) T sD[(WITH_D && !DIAG) ? CH : 1][LDW];
  __shared__ __align__(16) T sDinv[CH];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int nb = w >> 2, cb = w & 3;
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  const T* al = alpha + (size_t)u.plan * S * S;
  T breg[DIAG ? 1 : S / 4];
  if (DIAG)
    breg[0] = al[lane];
  else
    load_bcol<T>(al, cb, lane, breg);
  double a3[2][4];
  zero_acc(a3);
  double d3 = 0.0;
  const int64_t cofs = u.pd.cbase - u.pd.vbase;  // vector row -> coefficient index
  // Rows of one chunk (clamped to the unit's last row; zeroed when staged).
  T qv[NODES_PER_WAVE], rv[NODES_PER_WAVE], pv[NODES_PER_WAVE], dv[NODES_PER_WAVE];
  T dinv_t = T(0);
  auto load_chunk = [&](int64_t base) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
      qv[i] = Q[v * S + lane];
      rv[i] = R[v * S + lane];
      if (WITH_D) {
        pv[i] = P[v * S + lane];
        dv[i] = D[v * S + lane];
      }
    }
    if (threadIdx.x < CH) dinv_t = c.dinv[min(base + threadIdx.x, u.end - 1) + cofs];
  };
  if (!DIAG) load_chunk(u.begin);
  for (int64_t base = u.begin; base < u.end; base += CH) {
    if (DIAG) {
      T qv[NODES_PER_WAVE], rv[NODES_PER_WAVE], pv[NODES_PER_WAVE], dv[NODES_PER_WAVE];
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
        qv[i] = Q[v * S + lane];
        rv[i] = R[v * S + lane];
        if (WITH_D) {
          pv[i] = P[v * S + lane];
          dv[i] = D[v * S + lane];
        }
      }
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < u.end) {
          const T r = rv[i] - breg[0] * qv[i];
          R[v * S + lane] = r;
          if (WITH_D) D[v * S + lane] = dv[i] + breg[0] * pv[i];
          d3 += (double)qv[i] * (double)(c.dinv[v + cofs] * r);
        }
      }
      continue;
    }
    // Stage this chunk (loaded one chunk ahead) and start loading the next.
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const bool ok = base + row < u.end;
      sQ[row][lane] = ok ? qv[i] : T(0);
      sR[row][lane] = ok ? rv[i] : T(0);
      if (WITH_D) {
        sP[row][lane] = ok ? pv[i] : T(0);
        sD[row][lane] = ok ? dv[i] : T(0);
      }
    }
    if (threadIdx.x < CH) sDinv[threadIdx.x] = base + threadIdx.x < u.end ? dinv_t : T(0);
    if (base + CH < u.end) load_chunk(base + CH);
    __syncthreads();
    typename Acc<T>::type qa, pa = {0, 0, 0, 0};
    if (WITH_D)
      prod_tile2<T>(sQ, sP, nb, breg, lane, qa, pa);
    else
      qa = prod_tile<T>(sQ, nb, breg, lane);
    T rn[4], zn[4], dn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      rn[r] = sR[row][col] - qa[r];
      zn[r] = sDinv[row] * rn[r];
      if (CHEB) zn[r] *= inv_theta;
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
    if (!CHEB) gram_chunk<T>(sQ, sP, w, lane, a3);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < u.end) {
        R[v * S + lane] = sR[row][lane];
        if (WITH_D) D[v * S + lane] = sD[row][lane];
        if (CHEB && Z1) Z1[v * S + lane] = sP[row][lane];
      }
    }
    __syncthreads();
  }
  if (DIAG)
    diag_store(part_of(part, uidx, 2), d3, w, lane);
  else if (!CHEB)
    gram_store<T>(part_of(part, uidx, 2), w, lane, a3);
}

// ---------------------------------------------------------------- K3
// Y = Dinv R - P B;  W4 = Y^T D Y (block variant).
// With ZBUF the argument R is the preconditioned residual Z (polynomial
// preconditioner) and Y = Z - P B.  With WITH_D (block variant with ZBUF
// only) the kernel also takes the solution update D += P A of this
// iteration from K2: it reads P anyway, so P is read once per iteration.
template <typename T, bool DIAG, bool ZBUF = false, bool WITH_D = false>
__global__ __launch_bounds__(WG, 4) void k_update_y(Coef<T> c, Work wk,
                                                    const T* __restrict__ delta,
                                                    const T* __restrict__ R,
                                                    const T* __restrict__ P, T* __restrict__ Y,
                                                    double* __restrict__ part,
                                                    const T* __restrict__ alpha = nullptr,
                                                    T* __restrict__ D = nullptr) {
  static_assert(!WITH_D || (ZBUF && !DIAG), "D update only in the polynomial block variant");
  __shared__ __align__(16) T sP[DIAG ? 1 : CH][LDW];  // P rows, then Y rows
  __shared__ __align__(16) T sR[DIAG ? 1 : CH][LDW];  // R rows, then D Y rows
  __shared__ __align__(16) T sD[WITH_D ? CH : 1][WITH_D ? LDW : 1];
  __shared__ __align__(16) T sDv[CH][2];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int nb = w >> 2, cb = w & 3;
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  const T* de = delta + (size_t)u.plan * S * S;
  T breg[DIAG ? 1 : S / 4], areg[WITH_D ? S / 4 : 1];
  if (DIAG)
    breg[0] = de[lane];
  else
    load_bcol<T>(de, cb, lane, breg);
  if (WITH_D) load_bcol<T>(alpha + (size_t)u.plan * S * S, cb, lane, areg);
  double a4[2][4];
  zero_acc(a4);
  const int64_t cofs = u.pd.cbase - u.pd.vbase;
  // Rows of one chunk (clamped to the unit's last row; zeroed when staged).
  T rv[NODES_PER_WAVE], pv[NODES_PER_WAVE], dv[WITH_D ? NODES_PER_WAVE : 1];
  T dinv_t = T(0), d_t = T(0);
  auto load_chunk = [&](int64_t base) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
      pv[i] = P[v * S + lane];
      rv[i] = R[v * S + lane];
      if (WITH_D) dv[i] = D[v * S + lane];
    }
    if (threadIdx.x < CH) {
      const int64_t v = min(base + threadIdx.x, u.end - 1) + cofs;
      dinv_t = c.dinv[v];
      d_t = c.d[v];
    }
  };
  if (!DIAG) load_chunk(u.begin);
  for (int64_t base = u.begin; base < u.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
        rv[i] = R[v * S + lane];
        pv[i] = P[v * S + lane];
      }
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < u.end) Y[v * S + lane] = c.dinv[v + cofs] * rv[i] - breg[0] * pv[i];
      }
      continue;
    }
    // Stage this chunk (loaded one chunk ahead) and start loading the next.
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const bool ok = base + row < u.end;
      sP[row][lane] = ok ? pv[i] : T(0);
      sR[row][lane] = ok ? rv[i] : T(0);
      if (WITH_D) sD[row][lane] = ok ? dv[i] : T(0);
    }
    if (threadIdx.x < CH) {
      const bool ok = base + threadIdx.x < u.end;
      sDv[threadIdx.x][0] = ok ? dinv_t : T(0);
      sDv[threadIdx.x][1] = ok ? d_t : T(0);
    }
    if (base + CH < u.end) load_chunk(base + CH);
    __syncthreads();
    const auto pd = prod_tile<T>(sP, nb, breg, lane);
    typename Acc<T>::type pa = {0, 0, 0, 0};
    if (WITH_D) pa = prod_tile<T>(sP, nb, areg, lane);
    T yn[4], dn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      yn[r] = (ZBUF ? sR[row][col] : sDv[row][0] * sR[row][col]) - pd[r];
      if (WITH_D) dn[r] = sD[row][col] + pa[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = nb * 16 + tile_row<T>(lane, r), col = cb * 16 + (lane & 15);
      sP[row][col] = yn[r];
      sR[row][col] = sDv[row][1] * yn[r];
      if (WITH_D) sD[row][col] = dn[r];
    }
    __syncthreads();
    gram_chunk<T>(sP, sR, w, lane, a4);
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < u.end) {
        Y[v * S + lane] = sP[row][lane];
        if (WITH_D) D[v * S + lane] = sD[row][lane];
      }
    }
    __syncthreads();
  }
  if (!DIAG) gram_store<T>(part_of(part, uidx, 3), w, lane, a4);
}

// Gram m of each unit: A^T B (DSCALE: A^T D B) over its rows.  Used for
// W4 = Y^T D Y when a solve starts from a new Y, and for W3 = Q^T Z when the
// preconditioner is a polynomial (Z then comes from its own kernels).
template <typename T, bool DSCALE>
__global__ __launch_bounds__(WG, 4) void k_gram_ab(Coef<T> c, Work wk, const T* __restrict__ A,
                                                   const T* __restrict__ B,
                                                   double* __restrict__ part, int m) {
  __shared__ __align__(16) T sA[CH][LDW];
  __shared__ __align__(16) T sB[CH][LDW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  const int64_t cofs = u.pd.cbase - u.pd.vbase;
  double acc[2][4];
  zero_acc(acc);
  // Rows of the chunk at base (clamped to the unit's last row; zeroed when
  // staged).  The next chunk's loads are issued before this chunk's Grams.
  T av[NODES_PER_WAVE], bv[NODES_PER_WAVE], dv[NODES_PER_WAVE];
  auto load = [&](int64_t base) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = min(base + w * NODES_PER_WAVE + i, u.end - 1);
      av[i] = A[v * S + lane];
      bv[i] = B[v * S + lane];
      if (DSCALE) dv[i] = ldc(c.d, v + cofs);
    }
  };
  load(u.begin);
  for (int64_t base = u.begin; base < u.end; base += CH) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const bool ok = base + row < u.end;
      sA[row][lane] = ok ? av[i] : T(0);
      sB[row][lane] = ok ? (DSCALE ? bv[i] * dv[i] : bv[i]) : T(0);
    }
    __syncthreads();
    load(min(base + CH, u.end - 1));  // the last chunk reads valid rows again
    gram_chunk<T>(sA, sB, w, lane, acc);
    __syncthreads();
  }
  gram_store<T>(part_of(part, uidx, m), w, lane, acc);
}

// One Chebyshev step at one node: u + a1 (u - up) + a2 Dinv (r - (G u)_v),
// (G u)_v = d u - cE ue - cW uw - cN un - cS us - t, where t = gU yu + gD yd
// is the TSV term (tsv_term).  Every kernel that forms a Chebyshev iterate
// goes through these two functions, with explicit fused multiply-adds, so a
// value recomputed by another workgroup (a strip halo, a TSV partner) is
// bitwise the value its owner writes.
template <typename T>
__device__ __forceinline__ T tsv_term(T gu, T yu, T gd, T yd) {
  return fma(gu, yu, gd * yd);
}

template <typename T>
__device__ __forceinline__ T cheb_node_t(T u, T ue, T uw, T un, T us, T t, T d, T ce, T cw, T cn,
                                         T cs, T up, T r, T dinv, T a1, T a2) {
  T g = d * u;
  g = fma(-ce, ue, g);
  g = fma(-cw, uw, g);
  g = fma(-cn, un, g);
  g = fma(-cs, us, g);
  g = g - t;
  return fma(a2 * dinv, r - g, fma(a1, u - up, u));
}

template <typename T>
__device__ __forceinline__ T cheb_node(T u, T ue, T uw, T un, T us, T yu, T yd, T d, T ce, T cw,
                                       T cn, T cs, T gu, T gd, T up, T r, T dinv, T a1, T a2) {
  return cheb_node_t(u, ue, uw, un, us, tsv_term(gu, yu, gd, yd), d, ce, cw, cn, cs, up, r, dinv,
                     a1, a2);
}

// z_1 = D^-1 R / theta at vector row v (coefficient index v + cofs), the
// start of the Chebyshev steps, in the one order every kernel that forms it
// uses.
template <typename T>
__device__ __forceinline__ T cheb_z1(const Coef<T>& c, const T* __restrict__ R, int64_t v,
                                     int64_t cofs, T ith) {
  return ldc(c.dinv, v + cofs) * R[v * S + (threadIdx.x & 63)] * ith;
}

// z_{j+1} at vector row p, node (xg, yy) of its tier, from global memory:
// cheb_node with the arguments a strip kernel passes from LDS (neighbours
// outside the tier are 0, with coupling 0 on the west and south side as
// there; a missing TSV partner reads the node itself, with coupling 0).
// With FIRST the z_j values are z_1, formed from R (zin unused).
template <typename T, bool HAS_PREV, bool FIRST = false>
__device__ __forceinline__ T cheb_point(const Coef<T>& c, const PlanDesc& pd,
                                        const T* __restrict__ zin, const T* __restrict__ zprev,
                                        const T* __restrict__ R, int64_t p, int xg, int yy, T a1,
                                        T a2, T ith = T(1)) {
  const int lane = threadIdx.x & 63;
  const int nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  const int64_t cofs = pd.cbase - pd.vbase;
  const int64_t pc = p + cofs;
  auto zj = [&](int64_t q) { return FIRST ? cheb_z1(c, R, q, cofs, ith) : zin[q * S + lane]; };
  const bool he = xg + 1 < nx, hw = xg > 0, hn = yy + 1 < ny, hs = yy > 0;
  const T u = zj(p);
  const T ue = zj(he ? p + 1 : p);
  const T uw = zj(hw ? p - 1 : p);
  const T un = zj(hn ? p + nx : p);
  const T us = zj(hs ? p - nx : p);
  const int sp = ldc(c.slot, pc);
  const int q = max(sp, 0);
  const T gu = sp >= 0 ? ldc(c.up, q) : T(0);
  const T gd = sp >= 0 ? ldc(c.dn, q) : T(0);
  const T yu = zj(gu != T(0) ? p + pd.plane : p);
  const T yd = zj(gd != T(0) ? p - pd.plane : p);
  const T up = HAS_PREV ? zprev[p * S + lane] : T(0);
  const T r = R[p * S + lane];
  const T cw = hw ? ldc(c.cE, hw ? pc - 1 : pc) : T(0);
  const T cs = hs ? ldc(c.cN, hs ? pc - nx : pc) : T(0);
  return cheb_node(u, he ? ue : T(0), hw ? uw : T(0), hn ? un : T(0), hs ? us : T(0), yu, yd,
                   ldc(c.d, pc), ldc(c.cE, pc), cw, ldc(c.cN, pc), cs, gu, gd, up, r,
                   ldc(c.dinv, pc), a1, a2);
}

// One step of the Chebyshev polynomial preconditioner Z = q(D^-1 G) D^-1 R
// (block variant, over strips like the stencil kernel):
//   zout = u + a1 (u - uprev) + a2 D^-1 (R - G u),   u = z_j, uprev = z_{j-1}
// (uprev = 0 without HAS_PREV).  zout may be the uprev array: each row of it
// is read in the iteration before the one that writes it, and those reads
// complete before the barrier that precedes the writes.
template <typename T, bool HAS_PREV>
__global__ __launch_bounds__(WG, 4) void k_cheb_strip(Coef<T> c, Work wk, const T* __restrict__ zin,
                                                      const T* zprev, const T* __restrict__ R,
                                                      T* zout, T a1, T a2) {
  constexpr int HWW = CH + 2;
  constexpr int NPW = NODES_PER_WAVE;
  __shared__ __align__(16) T win[3][HWW][LDW];
  __shared__ T cd[2][CH], ce[2][CH + 1], cn[2][CH], cdi[2][CH];
  __shared__ int cslot[2][CH];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int ls = active_item(wk, 1);
  if (ls < 0) return;
  const int sidx = wk.sid[ls];
  const Strip st = wk.strips[sidx];
  const PlanDesc pd = wk.plans[st.plan];
  const int64_t nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  const int wdt = st.wdt;
  const bool has_w = st.x0 > 0;
  const bool has_e = st.x0 + wdt < pd.nx;
  // Wave 0 reads the west halo column, wave 1 the east one (a strip
  // narrower than CH ends at the east edge of the plane).
  const int hoff = w == 0 ? (has_w ? -1 : 0) : (has_e ? wdt : 0);
  // Every global load of the loop reads a valid address (rows and columns
  // are clamped); values outside the plane or the strip are replaced by
  // zero only when they are written to LDS.  The next row's loads are then
  // never waited for before that point, and the loop body has no
  // data-dependent branch around a load or a store, so the compiler can
  // count outstanding loads exactly.
  auto load_row = [&](int yy, T (&v)[NPW], T& halo) {
    const bool in = yy >= 0 && yy < ny;
    const int64_t base = pd.vbase + st.lrow0 + (int64_t)((in ? yy : st.y0) - st.y0) * nx;
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = zin[(base + min(w * NPW + i, wdt - 1)) * S + lane];
    if (w < 2) halo = zin[(base + hoff) * S + lane];
  };
  auto store_row = [&](int slot, const T (&v)[NPW], T halo, int yy) {
    const bool in = yy >= 0 && yy < ny;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      win[slot][j + 1][lane] = (in && j < wdt) ? v[i] : T(0);
    }
    if (w == 0) win[slot][0][lane] = (in && has_w) ? halo : T(0);
    if (w == 1 && wdt == CH) win[slot][CH + 1][lane] = (in && has_e) ? halo : T(0);
  };
  // pointwise rows of strip row s: R and (HAS_PREV) uprev
  auto load_pt = [&](int s, T (&rv)[NPW], T (&pv)[NPW]) {
    const int64_t base = pd.vbase + st.lrow0 + (int64_t)min(s, st.nrows - 1) * nx;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int64_t v = base + min(w * NPW + i, wdt - 1);
      rv[i] = R[v * S + lane];
      pv[i] = HAS_PREV ? zprev[v * S + lane] : T(0);
    }
  };
  // Coefficients of strip row s, one value per thread t <= 5 CH of waves
  // 0 - 2: d (t < CH), cE from node x0 - 1 on (CH <= t <= 2 CH), cN, Dinv;
  // every such thread also reads one slot entry (used by 3 CH < t <= 4 CH).
  const int t = threadIdx.x;
  const int kc = t < CH ? t : t <= 2 * CH ? t - CH - 1 : t <= 3 * CH ? t - 2 * CH - 1 : t - 4 * CH - 1;
  const int klo = (t == CH && has_w) ? -1 : 0;
  const T* csrc = t < CH ? c.d : t <= 2 * CH ? c.cE : t <= 3 * CH ? c.cN : c.dinv;
  const int ks = t - 3 * CH - 1;
  auto load_coef = [&](int srow, T& val, int& sl) {
    if (w < 3) {
      const int64_t base = pd.cbase + st.lrow0 + (int64_t)min(srow, st.nrows - 1) * nx;
      val = csrc[base + min(max(kc, klo), wdt - 1)];
      sl = c.slot[base + min(max(ks, 0), wdt - 1)];
    }
  };
  auto store_coef = [&](int b, T val, int sl) {
    if (t < CH) {
      cd[b][t] = val;
    } else if (t <= 2 * CH) {
      const int e = t - CH;
      ce[b][e] = ((e > 0 || has_w) && e <= wdt) ? val : T(0);
    } else if (t <= 3 * CH) {
      cn[b][t - 2 * CH - 1] = val;
    } else if (t <= 4 * CH) {
      cslot[b][t - 3 * CH - 1] = sl;
    } else if (t <= 5 * CH) {
      cdi[b][t - 4 * CH - 1] = val;
    }
  };
  {
    T v[NPW], h = T(0), cv = T(0);
    int csl = -1;
    load_row(st.y0 - 1, v, h);
    store_row(0, v, h, st.y0 - 1);
    load_row(st.y0, v, h);
    store_row(1, v, h, st.y0);
    load_row(st.y0 + 1, v, h);
    store_row(2, v, h, st.y0 + 1);
    load_coef(0, cv, csl);
    store_coef(0, cv, csl);
    if (t > 2 * CH && t <= 3 * CH) {
      const int j = t - 2 * CH - 1;
      const int64_t ci = pd.cbase + st.lrow0 + min(j, wdt - 1) - nx;  // row y0 - 1
      cn[1][j] = st.y0 > 0 ? c.cN[st.y0 > 0 ? ci : ci + nx] : T(0);
    }
  }
  T rc[NPW], pc[NPW];
  load_pt(0, rc, pc);
  __syncthreads();
  // Iteration s: LDS holds window rows y - 1, y, y + 1 in slots s, s + 1,
  // s + 2 (mod 3) and the coefficients of row s in buffer s & 1 (cN of row
  // y - 1 in the other).  The loads of the next row are issued before the
  // row's arithmetic and written to LDS after it, in the same iteration, so
  // that their wait does not include this row's stores.
  for (int s = 0; s < st.nrows; ++s) {
    const int y = st.y0 + s;
    const int ss = s % 3, sc = (s + 1) % 3, sn = (s + 2) % 3;  // rows y-1, y, y+1
    const int b = s & 1;
    const int64_t obase = pd.vbase + st.lrow0 + (int64_t)s * nx;
    // TSV partners (tiers above / below) of this row's nodes
    int sl[NPW];
    bool any = false;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      sl[i] = __builtin_amdgcn_readfirstlane(cslot[b][min(w * NPW + i, wdt - 1)]);
      any |= sl[i] >= 0;
    }
    T gu[NPW], gd[NPW], yu[NPW], yd[NPW];
    if (any) {  // wave-uniform
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int64_t v = obase + min(w * NPW + i, wdt - 1);
        // slot 0 exists: some node of this wave has a TSV
        const int q = max(sl[i], 0);
        gu[i] = sl[i] >= 0 ? ldc(c.up, q) : T(0);
        gd[i] = sl[i] >= 0 ? ldc(c.dn, q) : T(0);
        yu[i] = zin[(gu[i] != T(0) ? v + pd.plane : v) * S + lane];
        yd[i] = zin[(gd[i] != T(0) ? v - pd.plane : v) * S + lane];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NPW; ++i) gu[i] = gd[i] = yu[i] = yd[i] = T(0);
    }
    // next row (the last iteration reads valid rows again and discards them)
    T ny_v[NPW], ny_h = T(0), r_v[NPW], p_v[NPW], c_v = T(0);
    int c_sl = -1;
    load_row(y + 2, ny_v, ny_h);
    load_pt(s + 1, r_v, p_v);
    load_coef(s + 1, c_v, c_sl);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      // nodes past the strip's width repeat the last node: same inputs, same
      // value, same address
      const int jc = min(w * NPW + i, wdt - 1);
      const T zn = cheb_node(win[sc][jc + 1][lane], win[sc][jc + 2][lane], win[sc][jc][lane],
                             win[sn][jc + 1][lane], win[ss][jc + 1][lane], yu[i], yd[i],
                             cd[b][jc], ce[b][jc + 1], ce[b][jc], cn[b][jc], cn[b ^ 1][jc], gu[i],
                             gd[i], pc[i], rc[i], cdi[b][jc], a1, a2);
      zout[(obase + jc) * S + lane] = zn;
    }
    __syncthreads();
    store_row(ss, ny_v, ny_h, y + 2);  // row y + 2 replaces row y - 1
    store_coef(b ^ 1, c_v, c_sl);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      rc[i] = r_v[i];
      pc[i] = p_v[i];
    }
    __syncthreads();
  }
}

// Two Chebyshev steps in one pass over a strip (block variant):
//   z_{j+1} = step(z_j, z_{j-1}; a1, a2),   z_{j+2} = step(z_{j+1}, z_j; b1, b2)
// (z_{j-1} = 0 without HAS_PREV).  The workgroup marches its strip in +y
// with two levels one row apart: level 1 forms z_{j+1} on row y + 1 over the
// strip and one halo column on each side (from z_j over two halo columns),
// level 2 forms z_{j+2} on row y from the z_{j+1} rows y - 1 .. y + 1 held in
// LDS.  z_{j+1} at the TSV partners of a row-y node (other tiers, other
// workgroups) is recomputed from z_j, z_{j-1} and R.  All values come from
// cheb_node, so each recomputed copy equals the owner's value bit for bit.
// z_{j+1} goes to out1 (the next pair's z_{j-1}), z_{j+2} to out2; neither
// may alias an input, since other workgroups read the inputs at halos and
// TSV partners.
template <typename T, bool HAS_PREV>
__global__ __launch_bounds__(WG, sizeof(T) == 4 ? 4 : 2) void k_cheb2_strip(Coef<T> c, Work wk,
                                                       const T* __restrict__ zin,
                                                       const T* __restrict__ zprev,
                                                       const T* __restrict__ R,
                                                       T* __restrict__ out1,
                                                       T* __restrict__ out2, T a1, T a2, T b1,
                                                       T b2) {
  constexpr int NPW = NODES_PER_WAVE;
  constexpr int NC = CH + 2;  // level-1 columns -1 .. CH, index c + 1
  // Ring of z_j rows (columns -2 .. CH + 1 at index c + 2): row y + k in
  // slot (s + 2 + k) % 4.  Ring of z_{j+1} rows: row y + k in slot
  // (s + 2 + k) % 3.  Coefficients of row y + k in slot (s + 2 + k) % 3,
  // cN of row y + k in slot (s + 2 + k) % 4.
  __shared__ __align__(16) T w1[4][CH + 4][LDW];
  __shared__ __align__(16) T w2[3][NC][LDW];
  __shared__ T cd[3][NC], cdi[3][NC], ce[3][NC + 1], cn[4][NC];  // ce: index c + 2
  __shared__ int cslot[3][NC];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int ls = active_item(wk, 1);
  if (ls < 0) return;
  const int sidx = wk.sid[ls];
  const Strip st = wk.strips[sidx];
  const PlanDesc pd = wk.plans[st.plan];
  const int nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  const int wdt = st.wdt;
  const int x0 = st.x0;
  const int64_t cofs = pd.cbase - pd.vbase;
  auto col_ok = [&](int cc) { return x0 + cc >= 0 && x0 + cc < nx; };
  auto row_ok = [&](int yy) { return yy >= 0 && yy < ny; };
  // Vector row of strip node (yy, cc), clamped into the tier: every load
  // reads a valid address; values of nodes outside the tier are replaced
  // by zero when they are written to LDS or registers used later.
  auto vidx = [&](int yy, int cc) -> int64_t {
    yy = min(max(yy, 0), ny - 1);
    cc = min(max(cc, -x0), nx - 1 - x0);
    return pd.vbase + st.lrow0 + (int64_t)(yy - st.y0) * nx + cc;
  };
  // z_j row: nodes j = 4w + i, halo columns -2, -1, wdt, wdt + 1 (waves 0-3)
  const int hc = w == 0 ? -2 : w == 1 ? -1 : wdt + (w - 2);
  auto load_w1 = [&](int yy, T (&v)[NPW], T& h) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = zin[vidx(yy, w * NPW + i) * S + lane];
    if (w < 4) h = zin[vidx(yy, hc) * S + lane];
  };
  auto store_w1 = [&](int slot, const T (&v)[NPW], T h, int yy) {
    const bool in = row_ok(yy);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      w1[slot][j + 2][lane] = (in && j < wdt) ? v[i] : T(0);
    }
    // east halo columns only for a full-width strip (a ragged strip ends at
    // the tier's east edge, and the columns past it are zero above)
    if (w < 2 || (w < 4 && wdt == CH)) w1[slot][hc + 2][lane] = (in && col_ok(hc)) ? h : T(0);
  };
  // pointwise rows on level-1 columns: nodes j, and -1 (wave 0), wdt (wave 1)
  const int lc = w == 0 ? -1 : wdt;
  auto load_pt = [&](const T* __restrict__ a, int yy, T (&v)[NPW], T& h) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = a[vidx(yy, w * NPW + i) * S + lane];
    if (w < 2) h = a[vidx(yy, lc) * S + lane];
  };
  // Coefficients of one row, one value per thread t < 5 NC + 1 (waves 0-2):
  // d, cE (columns -2 .. CH), cN, Dinv on level-1 columns, and the TSV slot.
  const int t = threadIdx.x;
  const int kind = t < NC ? 0 : t < 2 * NC + 1 ? 1 : t < 3 * NC + 1 ? 2 : t < 4 * NC + 1 ? 3 : 4;
  const int kcol = kind == 0   ? t - 1
                   : kind == 1 ? t - NC - 2
                   : kind == 2 ? t - (2 * NC + 1) - 1
                   : kind == 3 ? t - (3 * NC + 1) - 1
                               : t - (4 * NC + 1) - 1;
  const T* csrc = kind == 0 ? c.d : kind == 1 ? c.cE : kind == 2 ? c.cN : c.dinv;
  auto load_coef = [&](int yy, T& val, int& sl) {
    if (w < 3) {
      const int64_t ci = vidx(yy, kcol) + cofs;
      val = csrc[ci];
      sl = c.slot[ci];
    }
  };
  auto store_coef = [&](int k, int kn, T val, int sl) {
    const bool ok = col_ok(kcol);
    if (kind == 0)
      cd[k][kcol + 1] = ok ? val : T(0);
    else if (kind == 1)
      ce[k][kcol + 2] = ok ? val : T(0);
    else if (kind == 2)
      cn[kn][kcol + 1] = ok ? val : T(0);
    else if (kind == 3)
      cdi[k][kcol + 1] = ok ? val : T(0);
    else if (t < 5 * NC + 1)
      cslot[k][kcol + 1] = ok ? sl : -1;
  };
  // Prologue: z_j rows y0-2 .. y0 in slots 0 .. 2, coefficients of rows
  // y0-2 (slot 0) and y0-1 (slot 1), R and z_{j-1} of row y0-1.
  T rA[NPW], rAh = T(0), pA[NPW], pAh = T(0), rB[NPW];
  {
    T v[NPW], h = T(0), cv = T(0);
    int csl = -1;
    load_w1(st.y0 - 2, v, h);
    store_w1(0, v, h, st.y0 - 2);
    load_w1(st.y0 - 1, v, h);
    store_w1(1, v, h, st.y0 - 1);
    load_w1(st.y0, v, h);
    store_w1(2, v, h, st.y0);
    load_coef(st.y0 - 2, cv, csl);
    store_coef(0, 0, cv, csl);
    load_coef(st.y0 - 1, cv, csl);
    store_coef(1, 1, cv, csl);
    load_pt(R, st.y0 - 1, rA, rAh);
    if (HAS_PREV) {
      load_pt(zprev, st.y0 - 1, pA, pAh);
    } else {
#pragma unroll
      for (int i = 0; i < NPW; ++i) pA[i] = T(0);
    }
#pragma unroll
    for (int i = 0; i < NPW; ++i) rB[i] = T(0);
  }
  __syncthreads();

  // One row: level 1 on row y + 1, level 2 (L2) on row y.
  auto row = [&](int s, auto L2) {
    constexpr bool lvl2 = decltype(L2)::value;
    const int y = st.y0 + s;
    const int r0 = s + 2;
    const int sw0 = r0 % 4, sw1 = (r0 + 1) % 4, sw2 = (r0 + 2) % 4, sw3 = (r0 + 3) % 4;
    const int q0 = r0 % 3, q1 = (r0 + 1) % 3, qm = (r0 + 2) % 3;  // z_{j+1} rows y, y+1, y-1
    const int k0 = r0 % 3, k1 = (r0 + 1) % 3, k2 = (r0 + 2) % 3;  // coefficients of y, y+1, y+2
    const int n0 = r0 % 4, n1 = (r0 + 1) % 4, n2 = (r0 + 2) % 4, nm = (r0 + 3) % 4;  // cN
    // [A] TSV partners: z_j of level-1 nodes (row y + 1), and z_{j+1} of
    // level-2 nodes (row y), before the next row's loads.
    int sl1[NPW + 1];
    bool any1 = false;
#pragma unroll
    for (int i = 0; i <= NPW; ++i) {
      const int cc = i < NPW ? min(w * NPW + i, wdt - 1) : lc;
      sl1[i] = (i < NPW || w < 2) ? __builtin_amdgcn_readfirstlane(cslot[k1][cc + 1]) : -1;
      any1 |= sl1[i] >= 0;
    }
    T gu1[NPW + 1], gd1[NPW + 1], yu1[NPW + 1], yd1[NPW + 1];
    if (any1) {
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        const int cc = i < NPW ? min(w * NPW + i, wdt - 1) : lc;
        const int64_t v = vidx(y + 1, cc);
        const int q = max(sl1[i], 0);
        gu1[i] = sl1[i] >= 0 ? ldc(c.up, q) : T(0);
        gd1[i] = sl1[i] >= 0 ? ldc(c.dn, q) : T(0);
        yu1[i] = zin[(gu1[i] != T(0) ? v + pd.plane : v) * S + lane];
        yd1[i] = zin[(gd1[i] != T(0) ? v - pd.plane : v) * S + lane];
      }
    } else {
#pragma unroll
      for (int i = 0; i <= NPW; ++i) gu1[i] = gd1[i] = yu1[i] = yd1[i] = T(0);
    }
    T gu2[NPW], gd2[NPW], zu2[NPW], zd2[NPW];
#pragma unroll
    for (int i = 0; i < NPW; ++i) gu2[i] = gd2[i] = zu2[i] = zd2[i] = T(0);
    if constexpr (lvl2) {
      int sl2[NPW];
      bool any2 = false;
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        sl2[i] = __builtin_amdgcn_readfirstlane(cslot[k0][min(w * NPW + i, wdt - 1) + 1]);
        any2 |= sl2[i] >= 0;
      }
      if (any2) {
        // one partner at a time (wave-uniform branches), to bound the
        // registers of the loads in flight
#pragma unroll
        for (int i = 0; i < NPW; ++i) {
          if (sl2[i] < 0) continue;
          const int jc = min(w * NPW + i, wdt - 1);
          const int64_t v = vidx(y, jc);
          gu2[i] = ldc(c.up, sl2[i]);
          gd2[i] = ldc(c.dn, sl2[i]);
          if (gu2[i] != T(0))
            zu2[i] = cheb_point<T, HAS_PREV>(c, pd, zin, zprev, R, v + pd.plane, x0 + jc, y, a1, a2);
          if (gd2[i] != T(0))
            zd2[i] = cheb_point<T, HAS_PREV>(c, pd, zin, zprev, R, v - pd.plane, x0 + jc, y, a1, a2);
        }
      }
    }
    // [B] next row: z_j row y + 3, coefficients, R and z_{j-1} of row y + 2
    T v1n[NPW], h1n = T(0), rN[NPW], rNh = T(0), pN[NPW], pNh = T(0), cvN = T(0);
    int cslN = -1;
    load_w1(y + 3, v1n, h1n);
    load_coef(y + 2, cvN, cslN);
    load_pt(R, y + 2, rN, rNh);
    if (HAS_PREV) load_pt(zprev, y + 2, pN, pNh);
    // [C] level 1: z_{j+1} on row y + 1
    const bool in1 = row_ok(y + 1);
    T z1[NPW];
#pragma unroll
    for (int i = 0; i <= NPW; ++i) {
      if (i == NPW && w >= 2) break;
      const int j = i < NPW ? w * NPW + i : lc;
      const int cc = i < NPW ? min(j, wdt - 1) : lc;
      const T up = i < NPW ? pA[i] : pAh;
      const T r = i < NPW ? rA[i] : rAh;
      const T z = cheb_node(w1[sw1][cc + 2][lane], w1[sw1][cc + 3][lane], w1[sw1][cc + 1][lane],
                            w1[sw2][cc + 2][lane], w1[sw0][cc + 2][lane], yu1[i], yd1[i],
                            cd[k1][cc + 1], ce[k1][cc + 2], ce[k1][cc + 1], cn[n1][cc + 1],
                            cn[n0][cc + 1], gu1[i], gd1[i], up, r, cdi[k1][cc + 1], a1, a2);
      const bool ok = in1 && (i < NPW ? j < wdt : col_ok(lc));
      // the east halo column exists only for a full-width strip
      if (i < NPW || w == 0 || wdt == CH) w2[q1][(i < NPW ? j : lc) + 1][lane] = ok ? z : T(0);
      if (i < NPW) z1[i] = z;
    }
    __syncthreads();
    // [D] level 2: z_{j+2} on row y
    if constexpr (lvl2) {
      const int64_t obase = pd.vbase + st.lrow0 + (int64_t)s * nx;
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        // nodes past a ragged strip's width repeat the last node
        const int jc = min(w * NPW + i, wdt - 1);
        const T z = cheb_node(w2[q0][jc + 1][lane], w2[q0][jc + 2][lane], w2[q0][jc][lane],
                              w2[q1][jc + 1][lane], w2[qm][jc + 1][lane], zu2[i], zd2[i],
                              cd[k0][jc + 1], ce[k0][jc + 2], ce[k0][jc + 1], cn[n0][jc + 1],
                              cn[nm][jc + 1], gu2[i], gd2[i], w1[sw0][jc + 2][lane], rB[i],
                              cdi[k0][jc + 1], b1, b2);
        out2[(obase + jc) * S + lane] = z;
      }
    }
    // [E] the next row into the slots of rows y - 1 (z_j, coefficients) and
    // y - 2 (cN), which no step of this row reads
    store_w1(sw3, v1n, h1n, y + 3);
    store_coef(k2, n2, cvN, cslN);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      rB[i] = rA[i];
      rA[i] = rN[i];
      pA[i] = HAS_PREV ? pN[i] : T(0);
    }
    rAh = rNh;
    pAh = pNh;
    // z_{j+1} of row y + 1 if it is a row of this strip
    if (s + 1 >= 0 && s + 1 < st.nrows) {
      const int64_t b1row = pd.vbase + st.lrow0 + (int64_t)(s + 1) * nx;
#pragma unroll
      for (int i = 0; i < NPW; ++i) out1[(b1row + min(w * NPW + i, wdt - 1)) * S + lane] = z1[i];
    }
    __syncthreads();
  };
  row(-2, std::false_type{});
  row(-1, std::false_type{});
  for (int s = 0; s < st.nrows; ++s) row(s, std::true_type{});
}

// TSV side buffers of a three-step pass (z_{j+1}, z_{j+2}, z_{j+3} from z_j,
// z_{j-1}): the strip kernel's level 2 and level 3 need z_{j+1} and z_{j+2}
// at the TSV partners of their nodes, in tiers other workgroups own.  Slot q
// of block p has side row sbase + q - slot_begin.
//   TA[row][k][S]: z_{j+1} at every TSV node (k = 0) and its east, west,
//                  north and south neighbours (k = 1 .. 4; 0 where the
//                  neighbour does not exist);
//   TB[row][S]:    z_{j+2} at every TSV node, from TA.
// In the first pass of an application (no z_{j-1}) z_j is z_1, formed from R.
// Two launches, one wave per item (4 waves per workgroup, no synchronisation
// inside a launch): k_cheb_tsv_a forms TA item (slot, k), k_cheb_tsv_b then TB
// item (slot); a node's TSV partners are the next and previous slot (the
// slots of a TSV column are consecutive over its tiers).  Grid (x, active
// blocks): the waves of a block's row of workgroups stride over its items,
// and x is capped so that a batch of many plans, whose largest plan sets
// the item count, launches no more than about TSV_GRID_CAP workgroups.
constexpr int TSV_WAVES = 4;
constexpr int TSV_GRID_CAP = 65536;

template <typename T, bool HAS_PREV>
__global__ __launch_bounds__(64 * TSV_WAVES) void k_cheb_tsv_a(
    Coef<T> c, Work wk, const int32_t* __restrict__ act, const T* __restrict__ zin,
    const T* __restrict__ zprev, const T* __restrict__ R, T* __restrict__ TA, T a1, T a2,
    T ith) {
  constexpr bool FIRST = !HAS_PREV;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if ((int)blockIdx.y >= wk.cnt[2]) return;
  const PlanDesc pd = wk.plans[act[blockIdx.y]];
  const int nitems = 5 * (pd.slot_end - pd.slot_begin);
  const int nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  for (int item = blockIdx.x * TSV_WAVES + w; item < nitems;  // wave-uniform
       item += gridDim.x * TSV_WAVES) {
  const int qi = item / 5, k = item % 5;
  const int64_t loc = c.tnode[pd.slot_begin + qi] - pd.cbase;  // node within the stack
  const int64_t rem = loc % pd.plane;
  const int y = (int)(rem / nx), x = (int)(rem % nx);
  const int dx = k == 1 ? 1 : k == 2 ? -1 : 0, dy = k == 3 ? 1 : k == 4 ? -1 : 0;
  const int xn = x + dx, yn = y + dy;
  T z = T(0);
  if (xn >= 0 && xn < nx && yn >= 0 && yn < ny)
    z = cheb_point<T, HAS_PREV, FIRST>(c, pd, zin, zprev, R,
                                       pd.vbase + loc + dx + (int64_t)dy * nx, xn, yn, a1, a2,
                                       ith);
  TA[((pd.sbase + qi) * 5 + k) * S + lane] = z;
  }
}

template <typename T, bool HAS_PREV>
__global__ __launch_bounds__(64 * TSV_WAVES) void k_cheb_tsv_b(
    Coef<T> c, Work wk, const int32_t* __restrict__ act, const T* __restrict__ zin,
    const T* __restrict__ R, const T* __restrict__ TA, T* __restrict__ TB, T b1, T b2, T ith) {
  constexpr bool FIRST = !HAS_PREV;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if ((int)blockIdx.y >= wk.cnt[2]) return;
  const PlanDesc pd = wk.plans[act[blockIdx.y]];
  const int nslot = pd.slot_end - pd.slot_begin;
  const int nx = pd.nx;
  const int64_t cofs = pd.cbase - pd.vbase;
  for (int qi = blockIdx.x * TSV_WAVES + w; qi < nslot;  // wave-uniform
       qi += gridDim.x * TSV_WAVES) {
  const int q = pd.slot_begin + qi;
  const int64_t u = c.tnode[q];  // coefficient index
  const int64_t loc = u - pd.cbase;
  const int64_t v = pd.vbase + loc;
  const int64_t rem = loc % pd.plane;
  const int y = (int)(rem / nx), x = (int)(rem % nx);
  const int64_t a = (pd.sbase + qi) * 5;
  const T gu = ldc(c.up, q), gd = ldc(c.dn, q);
  const T yu = gu != T(0) ? TA[(a + 5) * S + lane] : T(0);
  const T yd = gd != T(0) ? TA[(a - 5) * S + lane] : T(0);
  const T cw = x > 0 ? ldc(c.cE, x > 0 ? u - 1 : u) : T(0);
  const T cs = y > 0 ? ldc(c.cN, y > 0 ? u - nx : u) : T(0);
  TB[(pd.sbase + qi) * S + lane] =
      cheb_node(TA[a * S + lane], TA[(a + 1) * S + lane], TA[(a + 2) * S + lane],
                TA[(a + 3) * S + lane], TA[(a + 4) * S + lane], yu, yd, ldc(c.d, u),
                ldc(c.cE, u), cw, ldc(c.cN, u), cs, gu, gd,
                FIRST ? cheb_z1(c, R, v, cofs, ith) : zin[v * S + lane], R[v * S + lane],
                ldc(c.dinv, u), b1, b2);
  }
}

// Three Chebyshev steps in one pass over a strip (float32, block variant):
//   z_{j+1} = step(z_j, z_{j-1}; a1, a2), z_{j+2} = step(z_{j+1}, z_j; b1, b2),
//   z_{j+3} = step(z_{j+2}, z_{j+1}; c1, c2)
// (z_{j-1} = 0 without HAS_PREV).  Three levels one row apart: level 1 forms
// z_{j+1} on row y + 2 over the strip and two halo columns each side (from
// z_j over three), level 2 forms z_{j+2} on row y + 1 over the strip and one
// halo column each side, level 3 forms z_{j+3} on row y.  A wave owns its
// columns at every level (nodes 4w .. 4w+3; waves 0-3 also one halo column,
// the same at levels 1 and 2), so the values above and below a node come
// from the wave's own registers; LDS holds one row per level for the east
// and west neighbours, double-buffered: each level reads the row written in
// the previous iteration, and one barrier per row suffices.  TSV partners:
// z_j from global memory, z_{j+1} and z_{j+2} from the side buffers of
// k_cheb_tsv_a / _b.  Without z_{j-1} (the first pass) z_j is z_1 = D^-1 R / theta,
// formed from R (ith = 1 / theta; zin unused), so that no kernel writes z_1.
// Writes z_{j+2} to outa (null for the last pass: nothing reads it) and
// z_{j+3} to outb (the next pass's z_{j-1} and z_j); neither may alias an
// input.
constexpr int WG3 = 512;
constexpr int NPW3 = CH / (WG3 / 64);  // 4

template <bool HAS_PREV>
__global__ __launch_bounds__(WG3, 4) void k_cheb3_strip(Coef<float> c, Work wk,
                                                        const float* __restrict__ zin,
                                                        const float* __restrict__ zprev,
                                                        const float* __restrict__ R,
                                                        const float* __restrict__ TA,
                                                        const float* __restrict__ TB,
                                                        float* __restrict__ outa,
                                                        float* __restrict__ outb, float a1,
                                                        float a2, float b1, float b2, float c1,
                                                        float c2, float ith) {
  using T = float;
  constexpr int NPW = NPW3;
  constexpr int N1 = CH + 4;  // coefficient columns -2 .. CH + 1, index c + 2
  // East / west neighbour rows, slot (s + 4) & 1 read in iteration s: z_j
  // row y + 2 (columns -3 .. CH + 2, index c + 3), z_{j+1} row y + 1 (index
  // c + 2), z_{j+2} row y (index c + 1); one lane per column, no padding.
  __shared__ T h1[2][CH + 6][S];
  __shared__ T h2[2][CH + 4][S];
  __shared__ T h3[2][CH + 2][S];
  // Everything a node's step reads besides the iterates, per row and column,
  // in two 16-byte entries: cfa = {d, Dinv, cE (east coupling), cN (north
  // coupling)}, cfb = {cW (west coupling, cE of column c - 1), cS (south
  // coupling, cN of the row below), TSV slot (int bits), 0}.  Row yy is in
  // ring slot (yy - y0 + 4) & 7 and again 8 slots on, so that the rows y - 1
  // .. y + 2 read in iteration s sit in the consecutive slots b .. b + 3,
  // b = (s + 3) & 7: one address per node column and row, the rest fixed
  // offsets.
  __shared__ f4v cfa[16][N1];
  __shared__ f4v cfb[16][N1];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int ls = active_item(wk, 1);
  if (ls < 0) return;
  const int sidx = wk.sid[ls];
  const Strip st = wk.strips[sidx];
  const PlanDesc pd = wk.plans[st.plan];
  const int nx = pd.nx;
  const int ny = (int)(pd.plane / pd.nx);
  const int wdt = st.wdt;
  const int x0 = st.x0;
  const int64_t cofs = pd.cbase - pd.vbase;
  auto col_ok = [&](int cc) { return x0 + cc >= 0 && x0 + cc < nx; };
  auto row_ok = [&](int yy) { return yy >= 0 && yy < ny; };
  auto vidx = [&](int yy, int cc) -> int64_t {
    yy = min(max(yy, 0), ny - 1);
    cc = min(max(cc, -x0), nx - 1 - x0);
    return pd.vbase + st.lrow0 + (int64_t)(yy - st.y0) * nx + cc;
  };
  // The strip's own rows are read and written through unsigned 32-bit byte
  // offsets from per-strip base pointers placed three rows and three columns
  // before its first node, so that every offset is non-negative (the host
  // keeps (nrows + 8) nx S sizeof(float) below 2^31); TSV partners, a tier
  // away, use 64-bit indices.
  const int64_t r0off = (pd.vbase + st.lrow0) * S;
  const int64_t bias = (3 * (int64_t)nx + 3) * S;
  const uint32_t lane4 = (uint32_t)lane * 4u;
  auto boff = [&](int yy, int cc) -> uint32_t {
    yy = min(max(yy, 0), ny - 1);
    cc = min(max(cc, -x0), nx - 1 - x0);
    return (uint32_t)((yy - st.y0 + 3) * nx + cc + 3) * (uint32_t)(S * sizeof(T)) + lane4;
  };
  auto at = [](const T* base, uint32_t off) -> T {
    return *(const T*)((const char*)base + off);
  };
  auto srow = [&](int q) -> int64_t { return pd.sbase + (q - pd.slot_begin); };
  // halo column of waves 0-3 (levels 1 and 2; level 2 uses waves 1, 2):
  // -2, -1, wdt, wdt + 1; outer z_j column of waves 4, 5: -3, wdt + 2.
  // Columns east of a ragged strip (which ends at the tier's east edge) are
  // outside the tier: only full-width strips write the east ones.
  const bool has_h = w < 4;
  const int hc = w < 2 ? w - 2 : wdt + (w - 2);
  const bool has_o = w == 4 || w == 5;
  const int oc = w == 4 ? -3 : wdt + 2;
  const bool east_ok = wdt == CH;
  // Node i of this wave at a level: column cc(i) (nodes past a ragged
  // strip's width repeat the last node: same inputs, same value).
  auto ccol = [&](int i) { return i < NPW ? min(w * NPW + i, wdt - 1) : hc; };
  // z_j row yy on this wave's columns (raw loads; rows outside the tier are
  // zeroed when the row enters the register history)
  // The first pass of an application (no z_{j-1}) forms z_j = z_1 from R:
  // a row is loaded raw with the nodes' Dinv (scalar loads) and scaled where
  // it enters the register history, so nothing waits for the load early.
  constexpr bool FIRST = !HAS_PREV;
  auto zj_at = [&](int64_t v) -> T {
    return FIRST ? cheb_z1(c, R, v, cofs, ith) : zin[v * S + lane];
  };
  const T* zsb = (FIRST ? R : zin) + (r0off - bias);
  const T* Rb = R + (r0off - bias);
  const T* pb = HAS_PREV ? zprev + (r0off - bias) : nullptr;
  auto load_zj = [&](int yy, T (&v)[NPW + 1], T& o, T (&dv)[NPW + 2]) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      v[i] = at(zsb, boff(yy, w * NPW + i));
      if (FIRST) dv[i] = ldc(c.dinv, vidx(yy, w * NPW + i) + cofs);
    }
    if (has_h) {
      v[NPW] = at(zsb, boff(yy, hc));
      if (FIRST) dv[NPW] = ldc(c.dinv, vidx(yy, hc) + cofs);
    }
    if (has_o) {
      o = at(zsb, boff(yy, oc));
      if (FIRST) dv[NPW + 1] = ldc(c.dinv, vidx(yy, oc) + cofs);
    }
  };
  // z_1 = Dinv R / theta in the order of cheb_z1
  auto scaled = [&](T raw, T d) -> T { return FIRST ? d * raw * ith : raw; };
  auto load_pt = [&](const T* __restrict__ ab, int yy, T (&v)[NPW + 1]) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) v[i] = at(ab, boff(yy, w * NPW + i));
    if (has_h) v[NPW] = at(ab, boff(yy, hc));
  };
  auto put_h1 = [&](int slot, const T (&v)[NPW + 1], T o, int yy) {
    const bool in = row_ok(yy);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int j = w * NPW + i;
      h1[slot][j + 3][lane] = (in && j < wdt) ? v[i] : T(0);
    }
    if (has_h && (w < 2 || east_ok)) h1[slot][hc + 3][lane] = (in && col_ok(hc)) ? v[NPW] : T(0);
    if (has_o && (w == 4 || east_ok)) h1[slot][oc + 3][lane] = (in && col_ok(oc)) ? o : T(0);
  };
  // The seven fields of a row's entries, one per thread t < 7 N1 (waves
  // 0-3): field f = t / N1 of column kcol = t % N1 - 2.  Values outside the
  // tier's columns are 0 (slot -1); rows are clamped as everywhere (a row
  // outside the tier multiplies zero iterates).
  const int t = threadIdx.x;
  const int kf = t / N1, kcol = t % N1 - 2;
  const bool has_c = t < 7 * N1;
  const T* csrc = kf == 0 ? c.d : kf == 1 ? c.dinv : (kf == 2 || kf == 4) ? c.cE : c.cN;
  const int kc_src = kf == 4 ? kcol - 1 : kcol;  // cW is cE of the column to the west
  const bool kc_ok = col_ok(kc_src);
  auto load_coef = [&](int yy, T& val) {
    if (has_c) {
      const int64_t ci = vidx(kf == 5 ? yy - 1 : yy, kc_src) + cofs;  // cS: the row below
      val = kf == 6 ? __int_as_float(c.slot[ci]) : csrc[ci];
    }
  };
  auto store_coef = [&](int k, T val) {
    if (has_c) {
      const T v = kf == 6 ? (kc_ok ? val : __int_as_float(-1)) : (kc_ok ? val : T(0));
      T* e = kf < 4 ? (T*)&cfa[k][kcol + 2] + kf : (T*)&cfb[k][kcol + 2] + (kf - 4);
      e[0] = v;
      e[8 * N1 * 4] = v;  // the copy 8 slots on
    }
  };

  // Register history: z_j rows y+1, y+2, y+3 (zA[0..2]), z_{j+1} rows y,
  // y+1 (z1h), z_{j+2} rows y-1, y (z2h), R rows y+2 (rA), y+1 (rB), y (rC),
  // z_{j-1} row y+2 (pA); outer z_j column: row y+3 (oA).
  T zA[3][NPW + 1], z1h[2][NPW + 1], z2h[2][NPW], rA[NPW + 1], rB[NPW + 1], rC[NPW],
      pA[NPW + 1], oA = T(0);
#pragma unroll
  for (int i = 0; i <= NPW; ++i) {
    z1h[0][i] = z1h[1][i] = rB[i] = pA[i] = T(0);
    if (i < NPW) z2h[0][i] = z2h[1][i] = rC[i] = T(0);
  }
  // Prologue (iteration s = -4 reads row y0 - 2 as its row y + 2): z_j rows
  // y0-3 .. y0-1, the east / west row y0-2, coefficients of rows y0-3 and
  // y0-2, R and z_{j-1} of row y0-2.
  {
    T o = T(0), cv = T(0), dv[NPW + 2];
#pragma unroll
    for (int i = 0; i < NPW + 2; ++i) dv[i] = T(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      load_zj(st.y0 - 3 + k, zA[k], o, dv);
      const bool in = row_ok(st.y0 - 3 + k);
#pragma unroll
      for (int i = 0; i <= NPW; ++i) zA[k][i] = in ? scaled(zA[k][i], dv[i]) : T(0);
      o = scaled(o, dv[NPW + 1]);
      if (k == 1) put_h1(0, zA[1], o, st.y0 - 2);
      if (k == 2) oA = o;
    }
    load_coef(st.y0 - 2, cv);
    store_coef(2, cv);
    load_pt(Rb, st.y0 - 2, rA);
    if (HAS_PREV) load_pt(pb, st.y0 - 2, pA);
  }
  __syncthreads();

  auto row = [&](int s, auto L2, auto L3) {
    constexpr bool lvl2 = decltype(L2)::value;
    constexpr bool lvl3 = decltype(L3)::value;
    const int y = st.y0 + s;
    const int r0 = s + 4;
    const int hs = r0 & 1;  // neighbour rows read now; hs ^ 1 written now
    // coefficient slots: rows y - 1 + m at b + m (m = 0 .. 3); row y + 3
    // is stored into k3 (and k3 + 8)
    const int b = (r0 + 7) & 7, k3 = (r0 + 3) & 7;
    // [A] TSV terms of the three levels (rows y+2, y+1, y), before the next
    // row's loads; a wave with a TSV node waits for its partners here.
    T t1[NPW + 1], t2[NPW + 1], t3[NPW];
    {
      int sl[NPW + 1];
      bool any = false;
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        sl[i] = (i < NPW || has_h)
                    ? __builtin_amdgcn_readfirstlane(__float_as_int(cfb[b + 3][ccol(i) + 2][2]))
                    : -1;
        any |= sl[i] >= 0;
        t1[i] = T(0);
      }
      if (any) {
#pragma unroll
        for (int i = 0; i <= NPW; ++i) {
          if (sl[i] < 0) continue;
          const int64_t v = vidx(y + 2, ccol(i));
          const T gu = ldc(c.up, sl[i]), gd = ldc(c.dn, sl[i]);
          const T yu = zj_at(gu != T(0) ? v + pd.plane : v);
          const T yd = zj_at(gd != T(0) ? v - pd.plane : v);
          t1[i] = tsv_term(gu, yu, gd, yd);
        }
      }
    }
#pragma unroll
    for (int i = 0; i <= NPW; ++i) t2[i] = T(0);
    if constexpr (lvl2) {
      int sl[NPW + 1];
      bool any = false;
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        sl[i] = (i < NPW || w == 1 || w == 2)
                    ? __builtin_amdgcn_readfirstlane(__float_as_int(cfb[b + 2][ccol(i) + 2][2]))
                    : -1;
        any |= sl[i] >= 0;
      }
      if (any) {
#pragma unroll
        for (int i = 0; i <= NPW; ++i) {
          if (sl[i] < 0) continue;
          const int64_t a = srow(sl[i]) * 5;
          const T gu = ldc(c.up, sl[i]), gd = ldc(c.dn, sl[i]);
          const T zu = gu != T(0) ? TA[(a + 5) * S + lane] : T(0);
          const T zd = gd != T(0) ? TA[(a - 5) * S + lane] : T(0);
          t2[i] = tsv_term(gu, zu, gd, zd);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NPW; ++i) t3[i] = T(0);
    if constexpr (lvl3) {
      int sl[NPW];
      bool any = false;
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        sl[i] = __builtin_amdgcn_readfirstlane(__float_as_int(cfb[b + 1][ccol(i) + 2][2]));
        any |= sl[i] >= 0;
      }
      if (any) {
#pragma unroll
        for (int i = 0; i < NPW; ++i) {
          if (sl[i] < 0) continue;
          const int64_t a = srow(sl[i]);
          const T gu = ldc(c.up, sl[i]), gd = ldc(c.dn, sl[i]);
          const T zu = gu != T(0) ? TB[(a + 1) * S + lane] : T(0);
          const T zd = gd != T(0) ? TB[(a - 1) * S + lane] : T(0);
          t3[i] = tsv_term(gu, zu, gd, zd);
        }
      }
    }
    // [B] next row: coefficients of row y + 3 first (written to LDS at the
    // end of this row), then z_j row y + 4, R and z_{j-1} of row y + 3
    T cvN = T(0), v1n[NPW + 1], o1n = T(0), rN[NPW + 1], pN[NPW + 1], dvn[NPW + 2];
#pragma unroll
    for (int i = 0; i < NPW + 2; ++i) dvn[i] = T(1);
    load_coef(y + 3, cvN);
    load_zj(y + 4, v1n, o1n, dvn);
    load_pt(Rb, y + 3, rN);
    if (HAS_PREV) load_pt(pb, y + 3, pN);
    // [C] level 1: z_{j+1} on row y + 2
    T z1n[NPW + 1];
    {
      const bool in = row_ok(y + 2);
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        if (i == NPW && !has_h) break;
        const int cc = ccol(i);
        const f4v A = cfa[b + 3][cc + 2], B = cfb[b + 3][cc + 2];
        const T z = cheb_node_t(zA[1][i], h1[hs][cc + 4][lane], h1[hs][cc + 2][lane], zA[2][i],
                                zA[0][i], t1[i], A[0], A[2], B[0], A[3], B[1], pA[i], rA[i],
                                A[1], a1, a2);
        if (i < NPW) {
          const int j = w * NPW + i;
          z1n[i] = in ? z : T(0);
          h2[hs ^ 1][j + 2][lane] = (in && j < wdt) ? z : T(0);
        } else {
          const bool ok = in && col_ok(hc);
          z1n[i] = ok ? z : T(0);
          if (w < 2 || east_ok) h2[hs ^ 1][hc + 2][lane] = ok ? z : T(0);
        }
      }
    }
    // [D] level 2: z_{j+2} on row y + 1
    T z2n[NPW + 1];
#pragma unroll
    for (int i = 0; i <= NPW; ++i) z2n[i] = T(0);
    if constexpr (lvl2) {
      const bool in = row_ok(y + 1);
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        if (i == NPW && w != 1 && w != 2) break;
        const int cc = ccol(i);
        const f4v A = cfa[b + 2][cc + 2], B = cfb[b + 2][cc + 2];
        const T z = cheb_node_t(z1h[1][i], h2[hs][cc + 3][lane], h2[hs][cc + 1][lane], z1n[i],
                                z1h[0][i], t2[i], A[0], A[2], B[0], A[3], B[1], zA[0][i], rB[i],
                                A[1], b1, b2);
        if (i < NPW) {
          const int j = w * NPW + i;
          z2n[i] = in ? z : T(0);
          h3[hs ^ 1][j + 1][lane] = (in && j < wdt) ? z : T(0);
        } else {
          const bool ok = in && col_ok(hc);
          z2n[i] = ok ? z : T(0);
          if (w == 1 || east_ok) h3[hs ^ 1][hc + 1][lane] = ok ? z : T(0);
        }
      }
    }
    // [E] level 3: z_{j+3} on row y
    if constexpr (lvl3) {
      char* ob = (char*)(outb + r0off);
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int jc = ccol(i);
        const f4v A = cfa[b + 1][jc + 2], B = cfb[b + 1][jc + 2];
        const T z = cheb_node_t(z2h[1][i], h3[hs][jc + 2][lane], h3[hs][jc][lane], z2n[i],
                                z2h[0][i], t3[i], A[0], A[2], B[0], A[3], B[1], z1h[0][i], rC[i],
                                A[1], c1, c2);
        // non-temporal: the iterates are streamed back by the next pass
        __builtin_nontemporal_store(
            z, (T*)(ob + ((uint32_t)(s * nx + jc) * (uint32_t)(S * sizeof(T)) + lane4)));
      }
    }
    // [F] the east / west z_j row y + 3 and the coefficients of row y + 3
    // for the next row; then the register histories move down one row.
    put_h1(hs ^ 1, zA[2], oA, y + 3);
    store_coef(k3, cvN);
    {
      const bool in4 = row_ok(y + 4);
#pragma unroll
      for (int i = 0; i <= NPW; ++i) {
        zA[0][i] = zA[1][i];
        zA[1][i] = zA[2][i];
        zA[2][i] = in4 ? scaled(v1n[i], dvn[i]) : T(0);
        z1h[0][i] = z1h[1][i];
        z1h[1][i] = z1n[i];
        if (i < NPW) {
          z2h[0][i] = z2h[1][i];
          z2h[1][i] = z2n[i];
          rC[i] = rB[i];
        }
        rB[i] = rA[i];
        rA[i] = rN[i];
        pA[i] = HAS_PREV ? pN[i] : T(0);
      }
      oA = scaled(o1n, dvn[NPW + 1]);
    }
    // z_{j+2} of row y + 1 if it is a row of this strip (and a later pass
    // needs it)
    if (lvl2 && outa && s + 1 >= 0 && s + 1 < st.nrows) {
      char* oa = (char*)(outa + r0off);
#pragma unroll
      for (int i = 0; i < NPW; ++i)
        __builtin_nontemporal_store(
            z2n[i],
            (T*)(oa + ((uint32_t)((s + 1) * nx + ccol(i)) * (uint32_t)(S * sizeof(T)) + lane4)));
    }
    __syncthreads();
  };
  row(-4, std::false_type{}, std::false_type{});
  row(-3, std::false_type{}, std::false_type{});
  row(-2, std::true_type{}, std::false_type{});
  row(-1, std::true_type{}, std::false_type{});
  for (int s = 0; s < st.nrows; ++s) row(s, std::true_type{}, std::true_type{});
}

// C = Xa^T (G Xb) over all nodes of a block (pair resistances: the
// bilinear cross terms x_u^T G x_v between two solved blocks of one stack).
template <typename T>
__global__ __launch_bounds__(WG, 4) void k_cross_gram(Coef<T> c, Work wk,
                                                      const T* __restrict__ Xa,
                                                      const T* __restrict__ Xb,
                                                      double* __restrict__ part) {
  __shared__ __align__(16) T sA[CH][LDW];
  __shared__ __align__(16) T sB[CH][LDW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  double acc[2][4];
  zero_acc(acc);
  for (int64_t base = u.begin; base < u.end; base += CH) {
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      const bool ok = v < u.end;
      sA[row][lane] = ok ? Xa[v * S + lane] : T(0);
      sB[row][lane] = ok ? stencil_row<T, T>(c, Xb, u.pd, v, lane) : T(0);
    }
    __syncthreads();
    gram_chunk<T>(sA, sB, w, lane, acc);
    __syncthreads();
  }
  gram_store<T>(part_of(part, uidx, 0), w, lane, acc);
}

// ---------------------------------------------------------------- Kr
// W[p][m][e] = sum over the units of block p of part[unit][m][e], for the
// active blocks p = act[blockIdx.y], m in [m0, m0+nmat), e < len, summed in
// a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part,
                                                double* __restrict__ W,
                                                const PlanDesc* __restrict__ plans,
                                                const int32_t* __restrict__ act, int m0,
                                                int nmat, int len, int strips,
                                                const int32_t* __restrict__ cnt) {
  __shared__ double red[4][64];
  if ((int)blockIdx.y >= cnt[2]) return;
  const int p = act[blockIdx.y];
  const int el = threadIdx.x & 63;
  const int grp = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  const int total = nmat * len;
  const int m = m0 + (e < total ? e / len : 0);
  const int off = e % len;
  const int ub = strips ? plans[p].strip_begin : plans[p].unit_begin;
  const int ue = strips ? plans[p].strip_end : plans[p].unit_end;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < total) {
    int g = ub + grp;
    for (; g + 12 < ue; g += 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += part[((size_t)(g + 4 * q) * NGRAM + m) * S * S + off];
    }
    for (; g < ue; g += 4) acc[0] += part[((size_t)g * NGRAM + m) * S * S + off];
  }
  red[grp][el] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (grp == 0 && e < total)
    W[((size_t)p * NGRAM + m) * S * S + off] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

// ---------------------------------------------------------------- small
// Dense S x S work, one workgroup per solve block, float64 throughout.
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
    if (itn >= HIST) {
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

// 1/x and 1/sqrt(x) for x > 0 from the hardware estimates plus two Newton
// steps each (full float64 accuracy, without the long IEEE division and
// square-root sequences, which dominate a latency-bound sweep step).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y * fma(-0.5 * x, y * y, 1.5);
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
  if (threadIdx.x < 64) {  // max over the diagonal: one wave, butterfly
    double m = fmax(dg[threadIdx.x], 0.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (threadIdx.x == 0) maxd = m;
  }
  __syncthreads();
  if (threadIdx.x < S) {
    const double d = dg[threadIdx.x];
    const bool live = isfinite(d) && d > 1e-300 && d > 1e-28 * maxd &&
                      (floor_ == nullptr || d > floor_[threadIdx.x]);
    sc[threadIdx.x] = live ? rsqrt64(d) : 0.0;
  }
  __syncthreads();
  const double sk = sc[lane];
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] *= sc[16 * w + r] * sk;
}

// Lane l's value of x (l wave-uniform), as a scalar.
__device__ __forceinline__ double readlane64(double x, int l) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
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
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ double rowb[2][S];
  // j = 16 jw + jr with jr unrolled, so that every register index is a
  // compile-time constant (a dynamic index would move a[] out of registers).
#pragma unroll 1
  for (int jw = 0; jw < 4; ++jw)
#pragma unroll
  for (int jr = 0; jr < 16; ++jr) {
    const int j = 16 * jw + jr;
    // The matrix stays symmetric under the sweep, so row j (one full-wave
    // store by the wave that holds it) also gives every wave column j.
    double* rj = rowb[jr & 1];
    if (w == jw) rj[lane] = a[jr];
    __syncthreads();
    const double piv = rj[j];
    const double ck = rj[lane];  // M[j][lane] = M[lane][j]
    const bool dj = !(piv > eps);
    if (threadIdx.x == 0) drop[j] = dj ? 1 : 0;
    if (Tl != nullptr && w == 0) {  // column j of T, one row per lane
      const double rs = dj ? 0.0 : rsqrt64(piv);
      double t = 0.0;
      if (!dj) t = lane < j ? (drop[lane] ? 0.0 : -ck * rs) : (lane == j ? rs : 0.0);
      (*Tl)[lane][j] = sc[lane] * t;
    }
    if (!dj) {
      const double inv = rcp64(piv);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 16 * w + r;
        const double ci = readlane64(a[r], j);  // M[i][j]
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
// from the target rows of P, convergence.  Block p = act[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small1(const double* __restrict__ Wall,
                                                       const T* __restrict__ P,
                                                       const PlanDesc* __restrict__ plans,
                                                       const int32_t* __restrict__ act,
                                                       const int64_t* __restrict__ tgt_all,
                                                       double* __restrict__ winv_all,
                                                       T* __restrict__ alpha_all,
                                                       BlockState* __restrict__ st_all,
                                                       double tol, double eps, int diag,
                                                       const int32_t* __restrict__ cnt) {
  __shared__ Mat Wi, B, PT;
  __shared__ double sc[S], dpsi[S];
  __shared__ int drop[S];
  if ((int)blockIdx.x >= cnt[2]) return;
  const int p = act[blockIdx.x];
  const int64_t vbase = plans[p].vbase;
  const double* W1 = Wall + (size_t)p * NGRAM * S * S;
  const double* W2 = W1 + S * S;
  const int64_t* tgt = tgt_all + (size_t)p * S;
  double* winv = winv_all + (size_t)p * S * S;
  T* alpha_out = alpha_all + (size_t)p * S * S;
  BlockState* st = st_all + p;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const bool frozen = st->frozen != 0;
  // outputs are written at the end so that no barrier waits on global stores
  if (diag) {
    if (tid < S) {
      const double w1 = W1[tid];
      const double a = (w1 > 0.0 && !frozen) ? W2[tid] / w1 : 0.0;
      winv[tid] = w1 > 0.0 ? 1.0 / w1 : 0.0;
      alpha_out[tid] = (T)a;
      const int64_t v = tgt[tid];
      dpsi[tid] = v >= 0 ? a * (double)P[(vbase + v) * S + tid] : 0.0;
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
    PT[i][lane] = v >= 0 ? (double)P[(vbase + v) * S + lane] : 0.0;
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
  double cc[16];
  mm_rows(Wi, B, cc);  // alpha = W1^+ W2
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) B[16 * w + r][lane] = frozen ? 0.0 : cc[r];
  __syncthreads();
  // psi_k increment: row tgt_k of P times column k of alpha.
  if (tid < S) {
    double acc = 0.0;
    for (int j = 0; j < S; ++j) acc += PT[tid][j] * B[j][tid];
    dpsi[tid] = acc;
  }
  if (tid < 64) {
    const uint64_t m = __ballot(drop[tid] != 0);
    if (tid == 0) st->n_drop = __popcll(m);
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
__global__ __launch_bounds__(SM_THREADS) void k_small2(const double* __restrict__ Wall,
                                                       const int32_t* __restrict__ act,
                                                       const double* __restrict__ winv_all,
                                                       T* __restrict__ delta_all,
                                                       const BlockState* __restrict__ st_all,
                                                       int diag, const int32_t* __restrict__ cnt) {
  __shared__ Mat A, B;
  if ((int)blockIdx.x >= cnt[2]) return;
  const int p = act[blockIdx.x];
  const double* W3 = Wall + ((size_t)p * NGRAM + 2) * S * S;
  const double* winv = winv_all + (size_t)p * S * S;
  T* delta_out = delta_all + (size_t)p * S * S;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const bool frozen = st_all[p].frozen != 0;
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
  double cc[16];
  mm_rows(A, B, cc);
#pragma unroll
  for (int r = 0; r < 16; ++r) delta_out[(16 * w + r) * S + lane] = frozen ? (T)0 : (T)cc[r];
}

// Ks3: T from the guarded sweep of W4 = Y^T D Y, so that the kept columns
// of Y T are D-orthonormal.  A column whose squared D-norm has fallen below
// tau times its value at the start of the solve carries only rounding noise
// (its residual has converged) and is dropped as well; the first call after
// a (re)start records those reference norms.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small3(const double* __restrict__ Wall,
                                                       const int32_t* __restrict__ act,
                                                       T* __restrict__ T_all,
                                                       BlockState* __restrict__ st_all,
                                                       double eps, double tau,
                                                       const int32_t* __restrict__ cnt) {
  __shared__ Mat tmp, Tl;
  __shared__ double sc[S], floor_[S];
  __shared__ int drop[S];
  if ((int)blockIdx.x >= cnt[2]) return;
  const int p = act[blockIdx.x];
  const double* W4 = Wall + ((size_t)p * NGRAM + 3) * S * S;
  T* Tg = T_all + (size_t)p * S * S;
  BlockState* st = st_all + p;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
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
// Zero the rows of the active units (grid-stride over each unit's range).
template <typename T>
__global__ void k_zero_units(Work wk, T* __restrict__ a) {
  const int uidx = wk.uid[blockIdx.x];
  const Unit u = wk.units[uidx];
  const int64_t cnt = (u.end - u.begin) * S;
  T* base = a + u.begin * S;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) base[i] = T(0);
}

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

// Per block p = act[blockIdx.x]: R = E (unit column k at node tgt[k]),
// Y = Dinv E, T = diag(sqrt(d_tgt)) (so that P = Y T is D-orthonormal; the
// identity for the independent variant), state cleared.  R, Y (and D) were
// zeroed before.
template <typename T>
__global__ void k_set_targets(Coef<T> c, const PlanDesc* __restrict__ plans,
                              const int32_t* __restrict__ act, const int64_t* __restrict__ tgt_all,
                              T* __restrict__ R, T* __restrict__ Y, T* __restrict__ T_all,
                              BlockState* __restrict__ st_all, int diag) {
  const int p = act[blockIdx.x];
  const int k = threadIdx.x;
  if (k < S) {
    const PlanDesc pd = plans[p];
    const int64_t v = tgt_all[(size_t)p * S + k];
    T* Tm = T_all + (size_t)p * S * S;
    BlockState* st = st_all + p;
    double dv = 1.0;
    if (v >= 0) {
      dv = (double)c.d[pd.cbase + v];
      R[(pd.vbase + v) * S + k] = T(1);
      Y[(pd.vbase + v) * S + k] = c.dinv[pd.cbase + v];
    }
    for (int j = 0; j < S; ++j)
      Tm[j * S + k] = (T)((j == k && v >= 0) ? (diag ? 1.0 : sqrt(dv)) : 0.0);
    reset_columns(st, k, true);
    st->scale0[k] = v >= 0 ? 1.0 / dv : 0.0;
  }
}

// ---------------------------------------------------------------- mixed path
// X += D over the active units (float64 accumulation of the float32
// correction).
__global__ void k_accum(Work wk, double* __restrict__ X, const float* __restrict__ D) {
  const Unit u = wk.units[wk.uid[blockIdx.x]];
  const int64_t cnt = (u.end - u.begin) * S;
  double* xb = X + u.begin * S;
  const float* db = D + u.begin * S;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) xb[i] += (double)db[i];
}

// r = E - G X in float64; partial sums of x_k . r_k per column.  r is also
// stored (as float) into R for a further refinement step, with Y = Dinv r
// and D = 0.
__global__ __launch_bounds__(WG) void k_resid(Coef<double> c, Coef<float> cf, Work wk,
                                              const double* __restrict__ X,
                                              const int64_t* __restrict__ tgt_all,
                                              float* __restrict__ Rf, float* __restrict__ Yf,
                                              float* __restrict__ Df,
                                              double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lu = active_item(wk, 0);
  if (lu < 0) return;
  const UnitCtx u = unit_ctx(wk, lu);
  const int uidx = wk.uid[lu];
  const int64_t tl = tgt_all[(size_t)u.plan * S + lane];
  const int64_t my_t = tl >= 0 ? u.pd.vbase + tl : -1;
  const int64_t cofs = u.pd.cbase - u.pd.vbase;
  double acc = 0.0;
  for (int64_t base = u.begin; base < u.end; base += CH) {
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int64_t v = base + w * NODES_PER_WAVE + i;
      if (v < u.end) {
        const double gx = stencil_row<double, double>(c, X, u.pd, v, lane);
        const double r = (v == my_t ? 1.0 : 0.0) - gx;
        acc += X[v * S + lane] * r;
        Rf[v * S + lane] = (float)r;
        Yf[v * S + lane] = cf.dinv[v + cofs] * (float)r;
        Df[v * S + lane] = 0.0f;
      }
    }
  }
  diag_store(part_of(part, uidx, 0), acc, w, lane);
}

// Variational estimate R_k = e^T x + x^T r = 2 e^T x - x^T G x (float64),
// whose error is the energy norm of the solution error (>= 0).
__global__ void k_finalize_mixed(const double* __restrict__ X, const PlanDesc* __restrict__ plans,
                                 const int32_t* __restrict__ act,
                                 const int64_t* __restrict__ tgt_all,
                                 const double* __restrict__ Wall, BlockState* st_all,
                                 double* __restrict__ out, const int64_t* __restrict__ pos_all) {
  const int p = act[blockIdx.x];
  const int k = threadIdx.x;
  if (k < S) {
    const int64_t v = tgt_all[(size_t)p * S + k];
    double val = 0.0;
    if (v >= 0) val = X[(plans[p].vbase + v) * S + k] + Wall[(size_t)p * NGRAM * S * S + k];
    st_all[p].ref[k] = val;
    const int64_t q = pos_all[(size_t)p * S + k];
    if (q >= 0) out[q] = val;
  }
}

__global__ void k_finalize_plain(const int32_t* __restrict__ act, const BlockState* st_all,
                                 double* __restrict__ out, const int64_t* __restrict__ pos_all) {
  const int p = act[blockIdx.x];
  const int k = threadIdx.x;
  const int64_t q = k < S ? pos_all[(size_t)p * S + k] : -1;
  if (q >= 0) out[q] = st_all[p].psi[k];
}

__global__ void k_reset_state(const int32_t* __restrict__ act, BlockState* st_all) {
  const int k = threadIdx.x;
  if (k < S) reset_columns(st_all + act[blockIdx.x], k, false);
}

__global__ void k_set_identity(const int32_t* __restrict__ act, float* __restrict__ T_all) {
  float* Tm = T_all + (size_t)act[blockIdx.x] * S * S;
  for (int e = threadIdx.x; e < S * S; e += blockDim.x) Tm[e] = (e / S == e % S) ? 1.0f : 0.0f;
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

__global__ void k_gather_rows(const double* __restrict__ X, const int64_t* __restrict__ nodes,
                              int64_t count, double* __restrict__ rows) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count * S;
       e += (int64_t)gridDim.x * blockDim.x)
    rows[e] = X[nodes[e / S] * S + (e % S)];
}

// z_1 = D^-1 R / theta over the active units (start of the Chebyshev steps
// when a solve starts from a new residual).
template <typename T>
__global__ void k_scale_units(Coef<T> c, Work wk, const T* __restrict__ R, T* __restrict__ Z,
                              T inv_theta) {
  const int uidx = wk.uid[blockIdx.x];
  const Unit u = wk.units[uidx];
  const PlanDesc pd = wk.plans[u.plan];
  const int64_t cofs = pd.cbase - pd.vbase;
  const int64_t cnt = (u.end - u.begin) * S;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t v = u.begin + i / S;
    Z[u.begin * S + i] = c.dinv[v + cofs] * R[u.begin * S + i] * inv_theta;
  }
}

// ---------------------------------------------------------------- compaction
// Active lists of a group from its blocks' convergence flags: blocks
// 0 .. nb-1 in order, a block staying active until every column met the
// tolerance (all_conv); its units and strips follow it.  One workgroup;
// 256 blocks per round, placed by block-wide exclusive scans of the active
// flag and of the unit and strip counts.
__global__ __launch_bounds__(256) void k_compact(const PlanDesc* __restrict__ plans, int nb,
                                                 const BlockState* __restrict__ st,
                                                 int32_t* __restrict__ act,
                                                 int32_t* __restrict__ uid,
                                                 int32_t* __restrict__ sid,
                                                 int32_t* __restrict__ cnt) {
  __shared__ int sa[256], su[256], ss[256];
  const int t = threadIdx.x;
  int ta = 0, tu = 0, ts = 0;  // totals of the rounds before
  for (int base = 0; base < nb; base += 256) {
    const int p = base + t;
    const bool on = p < nb && st[p].all_conv == 0;
    const int nu = on ? plans[p].unit_end - plans[p].unit_begin : 0;
    const int ns = on ? plans[p].strip_end - plans[p].strip_begin : 0;
    sa[t] = on ? 1 : 0;
    su[t] = nu;
    ss[t] = ns;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive scans
      const int a = t >= d ? sa[t - d] : 0, u = t >= d ? su[t - d] : 0,
                v = t >= d ? ss[t - d] : 0;
      __syncthreads();
      sa[t] += a;
      su[t] += u;
      ss[t] += v;
      __syncthreads();
    }
    if (on) {
      act[ta + sa[t] - 1] = p;
      const int u0 = tu + su[t] - nu, s0 = ts + ss[t] - ns;
      for (int i = 0; i < nu; ++i) uid[u0 + i] = plans[p].unit_begin + i;
      for (int i = 0; i < ns; ++i) sid[s0 + i] = plans[p].strip_begin + i;
    }
    ta += sa[255];
    tu += su[255];
    ts += ss[255];
    __syncthreads();
  }
  if (t == 0) {
    cnt[0] = tu;
    cnt[1] = ts;
    cnt[2] = ta;
  }
}

hipError_t launch_compact(const SolveBuffers& b, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, st, b.work.plans, nb, b.state, b.act_w,
                     b.uid_w, b.sid_w, b.cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
static void reduce(const SolveBuffers& b, int m0, int nmat, int len, hipStream_t st,
                   bool strips = false) {
  hipLaunchKernelGGL(k_reduce, dim3((nmat * len + 63) / 64, b.n_act), dim3(256), 0, st, b.part,
                     b.W, b.work.plans, b.act, m0, nmat, len, strips ? 1 : 0, b.work.cnt);
}

// True when the first Chebyshev pass of an application is a three-step pass
// that forms z_1 from R itself, so that no kernel writes z_1.
template <typename T>
static bool cheb_folds_z1(const SolveBuffers& b) {
  return sizeof(T) == 4 && b.cheb_k > 3 && b.TA != nullptr;
}

// Chebyshev steps j = 1 .. cheb_k - 1 from z_1: three per pass while three
// remain (float32), then two per pass while two remain, then one.  z_1 =
// D^-1 R / theta is in Za unless the first pass is a three-step pass, which
// forms it from R (cheb_folds_z1).  A pass reads z_j, z_{j-1} and
// writes its last two iterates (or one) to arrays that hold neither; the
// iterates rotate over Za .. Zd.  The last step writes to `last` if given.
// Returns the array that holds Z.
template <typename T>
static T* cheb_steps(const Coef<T>& c, const SolveBuffers& b, hipStream_t st, T* last) {
  const dim3 g(b.n_strips), blk(WG);
  T* buf[4] = {(T*)b.Za, (T*)b.Zb, (T*)b.Zc, (T*)b.Zd};
  const T* R = (const T*)b.R;
  int cur = 0, prev = -1;
  auto free_slot = [&](int skip) {
    for (int i = 0; i < 4; ++i)
      if (i != cur && i != prev && i != skip) return i;
    return -1;
  };
  auto coef = [&](int j, T& x1, T& x2) {
    x1 = (T)b.cheb_a1[j];
    x2 = (T)b.cheb_a2[j];
  };
  const T ith = (T)b.cheb_invtheta;
  int j = 1;
  if constexpr (sizeof(T) == 4) {
    while (j + 2 < b.cheb_k && b.TA) {
      const int f1 = free_slot(-1), f2 = free_slot(f1);
      T* o2 = (j + 3 == b.cheb_k && last) ? last : buf[f2];
      T a1, a2, b1, b2, c1, c2;
      coef(j, a1, a2);
      coef(j + 1, b1, b2);
      coef(j + 2, c1, c2);
      const T* zp = prev < 0 ? nullptr : buf[prev];
      if (b.max_tsv_slots > 0) {
        const int gcap = std::max(1, TSV_GRID_CAP / std::max(b.n_act, 1));
        const dim3 ga(std::min((5 * b.max_tsv_slots + TSV_WAVES - 1) / TSV_WAVES, gcap),
                      b.n_act);
        const dim3 gb(std::min((b.max_tsv_slots + TSV_WAVES - 1) / TSV_WAVES, gcap), b.n_act);
        const dim3 tb(64 * TSV_WAVES);
        const T* zc = (const T*)buf[cur];
        if (prev < 0) {
          hipLaunchKernelGGL((k_cheb_tsv_a<T, false>), ga, tb, 0, st, c, b.work, b.act, zc, zp, R,
                             (T*)b.TA, a1, a2, ith);
          hipLaunchKernelGGL((k_cheb_tsv_b<T, false>), gb, tb, 0, st, c, b.work, b.act, zc, R,
                             (const T*)b.TA, (T*)b.TB, b1, b2, ith);
        } else {
          hipLaunchKernelGGL((k_cheb_tsv_a<T, true>), ga, tb, 0, st, c, b.work, b.act, zc, zp, R,
                             (T*)b.TA, a1, a2, ith);
          hipLaunchKernelGGL((k_cheb_tsv_b<T, true>), gb, tb, 0, st, c, b.work, b.act, zc, R,
                             (const T*)b.TA, (T*)b.TB, b1, b2, ith);
        }
      }
      T* o1 = j + 3 == b.cheb_k ? nullptr : buf[f1];  // the last pass's z_{j+2} is not read
      if (prev < 0)
        hipLaunchKernelGGL((k_cheb3_strip<false>), g, dim3(WG3), 0, st, c, b.work,
                           (const T*)buf[cur], zp, R, (const T*)b.TA, (const T*)b.TB, o1, o2, a1,
                           a2, b1, b2, c1, c2, ith);
      else
        hipLaunchKernelGGL((k_cheb3_strip<true>), g, dim3(WG3), 0, st, c, b.work,
                           (const T*)buf[cur], zp, R, (const T*)b.TA, (const T*)b.TB, o1, o2, a1,
                           a2, b1, b2, c1, c2, ith);
      j += 3;
      if (o2 == last) return last;
      prev = f1;
      cur = f2;
    }
  }
  while (j + 1 < b.cheb_k) {  // two steps per pass (float64 throughout)
    const int f1 = free_slot(-1), f2 = free_slot(f1);
    T* o2 = (j + 2 == b.cheb_k && last) ? last : buf[f2];
    T a1, a2, b1, b2;
    coef(j, a1, a2);
    coef(j + 1, b1, b2);
    if (prev < 0)
      hipLaunchKernelGGL((k_cheb2_strip<T, false>), g, blk, 0, st, c, b.work, (const T*)buf[cur],
                         (const T*)nullptr, R, buf[f1], o2, a1, a2, b1, b2);
    else
      hipLaunchKernelGGL((k_cheb2_strip<T, true>), g, blk, 0, st, c, b.work, (const T*)buf[cur],
                         (const T*)buf[prev], R, buf[f1], o2, a1, a2, b1, b2);
    j += 2;
    if (o2 == last) return last;
    prev = f1;
    cur = f2;
  }
  if (j < b.cheb_k) {  // one step left
    T* o = last ? last : buf[free_slot(-1)];
    T a1, a2;
    coef(j, a1, a2);
    if (prev < 0)
      hipLaunchKernelGGL((k_cheb_strip<T, false>), g, blk, 0, st, c, b.work, (const T*)buf[cur],
                         (const T*)nullptr, R, o, a1, a2);
    else
      hipLaunchKernelGGL((k_cheb_strip<T, true>), g, blk, 0, st, c, b.work, (const T*)buf[cur],
                         (const T*)buf[prev], R, o, a1, a2);
    return o;
  }
  return buf[cur];
}

// Y = M^-1 R for a solve that starts from the residual in R, then T from
// the guarded sweep of Y^T D Y (block variant, polynomial preconditioner).
template <typename T>
static void precond_start(const Coef<T>& c, const SolveBuffers& b, hipStream_t st) {
  const double eps4 = sizeof(T) == 8 ? 1e-14 : 1e-6;
  const double tau = sizeof(T) == 8 ? 1e-26 : 1e-12;
  if (!cheb_folds_z1<T>(b))
    hipLaunchKernelGGL((k_scale_units<T>), dim3(b.n_units), dim3(256), 0, st, c, b.work,
                       (const T*)b.R, (T*)b.Za, (T)b.cheb_invtheta);
  cheb_steps<T>(c, b, st, (T*)b.Y);
  hipLaunchKernelGGL((k_gram_ab<T, true>), dim3(b.n_units), dim3(WG), 0, st, c, b.work,
                     (const T*)b.Y, (const T*)b.Y, b.part, 3);
  reduce(b, 3, 1, S * S, st);
  hipLaunchKernelGGL((k_small3<T>), dim3(b.n_act), dim3(SM_THREADS), 0, st, b.W, b.act,
                     (T*)b.Tm, b.state, eps4, tau, b.work.cnt);
}

template <typename T>
static hipError_t iteration_t(bool indep, bool with_d, const Coef<T>& c, const SolveBuffers& b,
                              double tol, hipStream_t st, hipEvent_t* ev) {
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
  const dim3 g(b.n_units), blk(WG), gs(b.n_act), bs(SM_THREADS);
  const Work wk = b.work;
  if (ev) hipEventRecord(ev[0], st);
  const bool strips = !indep && b.n_strips > 0 && sizeof(T) == 4;
  const bool cheb = !indep && b.cheb_k > 1;
  if (indep)
    hipLaunchKernelGGL((k_stencil_gram<T, true>), g, blk, 0, st, c, wk, Y, (const T*)b.Tm, R, P,
                       Q, b.part);
  else if (strips) {
    // float32 only (the float64 window would not fit two workgroups per CU)
    if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL((k_stencil_gram_strip<T>), dim3(b.n_strips), blk, 0, st, c, wk, Y,
                         (const T*)b.Tm, R, P, Q, b.part);
  } else
    hipLaunchKernelGGL((k_stencil_gram<T, false>), g, blk, 0, st, c, wk, Y, (const T*)b.Tm, R,
                       P, Q, b.part);
  if (ev) hipEventRecord(ev[1], st);
  reduce(b, 0, 2, len, st, strips);
  hipLaunchKernelGGL((k_small1<T>), gs, bs, 0, st, b.W, (const T*)P, wk.plans, b.act, b.tgt,
                     b.winv, (T*)b.alpha, b.state, tol, eps1, di, wk.cnt);
  if (ev) hipEventRecord(ev[2], st);
  const T* al = (const T*)b.alpha;
  if (indep) {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, true, true>), g, blk, 0, st, c, wk, al, Q, P, R, D,
                         b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, true, false>), g, blk, 0, st, c, wk, al, Q, P, R, D,
                         b.part);
  } else if (cheb) {
    const T it = (T)b.cheb_invtheta;
    T* z1 = cheb_folds_z1<T>(b) ? nullptr : (T*)b.Za;  // z_1 = D^-1 R / theta
    // D += P A moves to K3, which reads P anyway
    hipLaunchKernelGGL((k_update_r<T, false, false, true>), g, blk, 0, st, c, wk, al, Q, P, R, D,
                       b.part, z1, it);
  } else {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, false, true>), g, blk, 0, st, c, wk, al, Q, P, R, D,
                         b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, false, false>), g, blk, 0, st, c, wk, al, Q, P, R, D,
                         b.part);
  }
  if (ev) hipEventRecord(ev[3], st);
  // Z = M^-1 R and W3 = Q^T Z (polynomial preconditioner)
  if (ev) hipEventRecord(ev[6], st);
  const T* Z = R;
  if (cheb) Z = cheb_steps<T>(c, b, st, nullptr);
  if (ev) hipEventRecord(ev[7], st);
  if (ev) hipEventRecord(ev[8], st);
  if (cheb)
    hipLaunchKernelGGL((k_gram_ab<T, false>), g, blk, 0, st, c, wk, (const T*)Q, Z, b.part, 2);
  if (ev) hipEventRecord(ev[9], st);
  reduce(b, 2, 1, len, st);
  hipLaunchKernelGGL((k_small2<T>), gs, bs, 0, st, b.W, b.act, b.winv, (T*)b.delta, b.state, di,
                     wk.cnt);
  if (ev) hipEventRecord(ev[4], st);
  const T* de = (const T*)b.delta;
  if (indep) {
    hipLaunchKernelGGL((k_update_y<T, true>), g, blk, 0, st, c, wk, de, R, P, Y, b.part);
    if (ev) hipEventRecord(ev[5], st);
  } else {
    if (cheb && with_d)
      hipLaunchKernelGGL((k_update_y<T, false, true, true>), g, blk, 0, st, c, wk, de, Z, P, Y,
                         b.part, al, D);
    else if (cheb)
      hipLaunchKernelGGL((k_update_y<T, false, true>), g, blk, 0, st, c, wk, de, Z, P, Y, b.part);
    else
      hipLaunchKernelGGL((k_update_y<T, false>), g, blk, 0, st, c, wk, de, R, P, Y, b.part);
    if (ev) hipEventRecord(ev[5], st);
    reduce(b, 3, 1, len, st);
    hipLaunchKernelGGL((k_small3<T>), gs, bs, 0, st, b.W, b.act, (T*)b.Tm, b.state, eps4, tau,
                       wk.cnt);
  }
  // blocks that converged in this iteration leave the active lists
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, st, wk.plans, b.n_act, b.state, b.act_w,
                     b.uid_w, b.sid_w, b.cnt);
  return hipGetLastError();
}

hipError_t launch_iteration(bool fp32, bool indep, bool with_d, const void* coef,
                            const SolveBuffers& b, double tol, hipStream_t st, hipEvent_t* ev) {
  if (fp32) return iteration_t<float>(indep, with_d, *(const Coef<float>*)coef, b, tol, st, ev);
  return iteration_t<double>(indep, with_d, *(const Coef<double>*)coef, b, tol, st, ev);
}

template <typename T>
static hipError_t init_t(const Coef<T>& c, const SolveBuffers& b, bool indep, hipStream_t st) {
  const dim3 g(b.n_units), blk(256);
  hipLaunchKernelGGL((k_zero_units<T>), g, blk, 0, st, b.work, (T*)b.R);
  hipLaunchKernelGGL((k_zero_units<T>), g, blk, 0, st, b.work, (T*)b.Y);
  if (b.D) hipLaunchKernelGGL((k_zero_units<T>), g, blk, 0, st, b.work, (T*)b.D);
  hipLaunchKernelGGL((k_set_targets<T>), dim3(b.n_act), dim3(S), 0, st, c, b.work.plans, b.act,
                     b.tgt, (T*)b.R, (T*)b.Y, (T*)b.Tm, b.state, indep ? 1 : 0);
  if (!indep && b.cheb_k > 1) precond_start<T>(c, b, st);
  return hipGetLastError();
}

hipError_t launch_init_blocks(bool fp32, bool indep, const void* coef, const SolveBuffers& b,
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
                                 const SolveBuffers& b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_accum, dim3(b.n_units), dim3(256), 0, st, b.work, b.X,
                     (const float*)b.D);
  hipLaunchKernelGGL(k_resid, dim3(b.n_units), dim3(WG), 0, st, c, cf, b.work, b.X, b.tgt,
                     (float*)b.R, (float*)b.Y, (float*)b.D, b.part);
  reduce(b, 0, 1, S, st);
  hipLaunchKernelGGL(k_finalize_mixed, dim3(b.n_act), dim3(S), 0, st, b.X, b.work.plans, b.act,
                     b.tgt, b.W, b.state, out, b.pos);
  return hipGetLastError();
}

hipError_t launch_restart(const Coef<float>& cf, const SolveBuffers& b, bool indep,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_reset_state, dim3(b.n_act), dim3(S), 0, st, b.act, b.state);
  if (indep) {
    // T = I: the independent variant needs no orthonormalisation.
    hipLaunchKernelGGL(k_set_identity, dim3(b.n_act), dim3(256), 0, st, b.act, (float*)b.Tm);
  } else if (b.cheb_k > 1) {
    precond_start<float>(cf, b, st);  // Y = M^-1 r
  } else {
    hipLaunchKernelGGL((k_gram_ab<float, true>), dim3(b.n_units), dim3(WG), 0, st, cf, b.work,
                       (const float*)b.Y, (const float*)b.Y, b.part, 3);
    reduce(b, 3, 1, S * S, st);
    hipLaunchKernelGGL((k_small3<float>), dim3(b.n_act), dim3(SM_THREADS), 0, st, b.W, b.act,
                       (float*)b.Tm, b.state, 1e-6, 1e-12, b.work.cnt);
  }
  return hipGetLastError();
}

hipError_t launch_finalize_plain(const SolveBuffers& b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_plain, dim3(b.n_act), dim3(S), 0, st, b.act, b.state, out, b.pos);
  return hipGetLastError();
}

hipError_t launch_cross_gram(const Coef<double>& c, const double* Xa, const double* Xb,
                             const SolveBuffers& b, hipStream_t st) {
  hipLaunchKernelGGL((k_cross_gram<double>), dim3(b.n_units), dim3(WG), 0, st, c, b.work, Xa, Xb,
                     b.part);
  reduce(b, 0, 1, S * S, st);
  return hipGetLastError();
}

// Pair resistances from the solved endpoint blocks, on the device: with
// x_u the solution for endpoint u (block blk[u], column col[u]),
//   K(u, v) = x_u[v] + x_v[u] - x_u^T G x_v   (bilinear estimate),
//   R(a, b) = K(a, a) + K(b, b) - 2 K(a, b),  R = 0 when a and b coincide.
// rows[bb][w][k] = x of block bb, column k, at endpoint w's node;
// cg[b1][b2][i][j] = x_{b1,i}^T G x_{b2,j} for b1 <= b2 (the transpose
// serves b1 > b2).  ia / ib: endpoint index of a_i / b_j (-1: grounded).
__global__ void k_pairs_finish(int64_t m, int64_t n, const int64_t* __restrict__ ia,
                               const int64_t* __restrict__ ib, const int64_t* __restrict__ aid,
                               const int64_t* __restrict__ bid, const int32_t* __restrict__ blk,
                               const int32_t* __restrict__ col, const double* __restrict__ rows,
                               const double* __restrict__ cg, int64_t U, int64_t nblk,
                               int64_t grp, double* __restrict__ out) {
  // Blocks of one resident group (bu / grp == bv / grp) have their cross
  // Gram: bilinear estimate.  Across groups: the symmetric first-order one.
  auto K = [&](int64_t u, int64_t v) -> double {
    if (u < 0 || v < 0) return 0.0;
    const int64_t bu = blk[u], cu = col[u], bv = blk[v], cv = col[v];
    const double xuv = rows[(bu * U + v) * S + cu];
    const double xvu = rows[(bv * U + u) * S + cv];
    if (bu / grp != bv / grp) return 0.5 * (xuv + xvu);
    const double g = bu <= bv ? cg[((bu * nblk + bv) * S + cu) * S + cv]
                              : cg[((bv * nblk + bu) * S + cv) * S + cu];
    return xuv + xvu - g;
  };
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < m * n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / n, j = q % n;
    double r = 0.0;
    if (aid[i] != bid[j]) r = K(ia[i], ia[i]) + K(ib[j], ib[j]) - 2.0 * K(ia[i], ib[j]);
    out[q] = r;
  }
}

hipError_t launch_pairs_finish(int64_t m, int64_t n, const int64_t* ia, const int64_t* ib,
                               const int64_t* aid, const int64_t* bid, const int32_t* blk,
                               const int32_t* col, const double* rows, const double* cg, int64_t U,
                               int64_t nblk, int64_t grp, double* out, hipStream_t st) {
  if (m * n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((m * n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pairs_finish, dim3((unsigned)blocks), dim3(256), 0, st, m, n, ia, ib, aid,
                     bid, blk, col, rows, cg, U, nblk, std::max<int64_t>(grp, 1), out);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double* X, const int64_t* nodes, int64_t count,
                              double* rows, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((count * S + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(256), 0, st, X, nodes, count, rows);
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
