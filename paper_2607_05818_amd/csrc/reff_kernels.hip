// gfx950 kernels of the block-PCG effective-resistance solver.
//
// Vectors are n x S blocks stored node-major with the S = 64 right-hand
// sides contiguous (V[v*S + k]).  One wavefront owns one node at a time and
// lane k owns column k, so every vector access of a wave is one coalesced
// 64-element row and a node's stencil coefficients are wave-uniform (scalar
// loads).
//
// Block PCG with rank-revealing orthonormalised search directions.  The
// search block is kept as Y (any basis) plus an S x S map T such that
// P = Y T has D-orthonormal kept columns (D = diag G) and zero dropped ones.
// One iteration for all S columns:
//   K1  Qt = G Y (stencil); P = Y T; Q = Qt T;  W1 = P^T Q, W2 = P^T R
//   Ks1 W1^+ by guarded Cholesky;  A = W1^+ W2;
//       psi_k += sum_j P[tgt_k, j] A[j, k]   (= change of x_k at node tgt_k)
//   K2  R -= Q A;  (D += P A);  Z = Dinv R;  W3 = Q^T Z
//   Ks2 B = W1^+ W3
//   K3  Y = Z - P B;  W4 = Y^T D Y
//   Ks3 T = Sc L^-T from the guarded Cholesky of W4 (directions whose pivot
//       falls below eps are numerically dependent and are dropped)
// (each Grams' per-workgroup partials are reduced by Kr first).  With x0 = 0
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

__device__ __forceinline__ double* part_of(double* part, int m) {
  return part + ((size_t)blockIdx.x * NGRAM + m) * S * S;
}

// ---------------------------------------------------------------- K1
template <typename T, bool DIAG>
__global__ __launch_bounds__(WG) void k_spmv_gram(Coef<T> c, const T* __restrict__ Y,
                                                  const T* __restrict__ Tm,
                                                  const T* __restrict__ R, T* __restrict__ P,
                                                  T* __restrict__ Q, double* __restrict__ part) {
  __shared__ T sA[CH][S];  // Y rows, then P rows
  __shared__ T sB[CH][S];  // G Y rows, then Q rows
  __shared__ T sR[DIAG ? 1 : CH][S];
  __shared__ T sT[DIAG ? 1 : S][S + 1];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  const int j0 = w * 8;
  if (!DIAG) {
    for (int e = threadIdx.x; e < S * S; e += WG) sT[e / S][e % S] = Tm[e];
    __syncthreads();
  }
  double a1[8], a2[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a1[i] = a2[i] = 0.0;

  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) {
          const T p = Y[v * S + lane];
          const T q = stencil_row<T, T>(c, Y, v, lane);
          const T r = R[v * S + lane];
          P[v * S + lane] = p;
          Q[v * S + lane] = q;
          a1[0] += (double)p * (double)q;
          a2[0] += (double)p * (double)r;
        }
      }
      continue;
    }
    // Phase A: stencil on the wave's own nodes, stage Y, G Y and R rows.
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      T y = 0, qt = 0, r = 0;
      if (v < rg.end) {
        y = Y[v * S + lane];
        r = R[v * S + lane];
        qt = stencil_row<T, T>(c, Y, v, lane);
      }
      sA[row][lane] = y;
      sB[row][lane] = qt;
      sR[row][lane] = r;
    }
    __syncthreads();
    // Phase B: P = Y T, Q = (G Y) T on the wave's own rows.
    T pv[NODES_PER_WAVE], qv[NODES_PER_WAVE];
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      T ap = 0, aq = 0;
#pragma unroll 8
      for (int j = 0; j < S; ++j) {
        const T t = sT[j][lane];
        ap += sA[row][j] * t;
        aq += sB[row][j] * t;
      }
      pv[i] = ap;
      qv[i] = aq;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      if (v < rg.end) {
        P[v * S + lane] = pv[i];
        Q[v * S + lane] = qv[i];
      }
      sA[row][lane] = v < rg.end ? pv[i] : T(0);
      sB[row][lane] = v < rg.end ? qv[i] : T(0);
    }
    __syncthreads();
    // Phase C: W1 += P^T Q, W2 += P^T R over the chunk.
    for (int row = 0; row < CH; ++row) {
      const double q = (double)sB[row][lane];
      const double r = (double)sR[row][lane];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double pj = (double)sA[row][j0 + i];
        a1[i] += pj * q;
        a2[i] += pj * r;
      }
    }
    __syncthreads();
  }
  if (DIAG) {
    __shared__ double red[2][WG / 64][S];
    red[0][w][lane] = a1[0];
    red[1][w][lane] = a2[0];
    __syncthreads();
    if (w == 0) {
      double s1 = 0, s2 = 0;
      for (int u = 0; u < WG / 64; ++u) {
        s1 += red[0][u][lane];
        s2 += red[1][u][lane];
      }
      part_of(part, 0)[lane] = s1;
      part_of(part, 1)[lane] = s2;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      part_of(part, 0)[(j0 + i) * S + lane] = a1[i];
      part_of(part, 1)[(j0 + i) * S + lane] = a2[i];
    }
  }
}

// ---------------------------------------------------------------- Kr
// W[m][e] = sum_g part[g][m][e] for m in [m0, m0+nmat), e < len, summed in
// a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part,
                                                double* __restrict__ W, int G, int m0,
                                                int nmat, int len) {
  __shared__ double red[4][64];
  const int el = threadIdx.x & 63;
  const int grp = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  const int total = nmat * len;
  const int m = m0 + (e / len);
  const int off = e % len;
  double acc = 0.0;
  if (e < total) {
    for (int g = grp; g < G; g += 4) acc += part[((size_t)g * NGRAM + m) * S * S + off];
  }
  red[grp][el] = acc;
  __syncthreads();
  if (grp == 0 && e < total)
    W[(size_t)m * S * S + off] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

// ---------------------------------------------------------------- small
// Dense S x S work in one workgroup, float64 throughout.
constexpr int SM_THREADS = 256;

// Guarded Cholesky of the Jacobi-scaled symmetric part of M (global,
// row-major).  On return (all in LDS): Li = L^-1 on the kept indices (zero
// rows/columns for dropped ones), sc = scaling (1/sqrt(diag), 0 for empty
// columns), drop flags.  A direction is dropped when its scaled pivot is
// not above eps (numerically in the span of the earlier ones).
__device__ void guarded_cholesky_inverse(const double* __restrict__ M, double (*A)[S + 1],
                                         double (*Li)[S + 1], double* sc, int* drop,
                                         double eps, const double* absfloor) {
  const int tid = threadIdx.x;
  for (int e = tid; e < S * S; e += SM_THREADS) {
    const int i = e / S, j = e % S;
    A[i][j] = 0.5 * (M[i * S + j] + M[j * S + i]);
  }
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < S; ++j) maxd = fmax(maxd, A[j][j]);
  if (tid < S) {
    const double dj = A[tid][tid];
    const bool live = isfinite(dj) && dj > 1e-300 && dj > 1e-28 * maxd &&
                      (absfloor == nullptr || dj > absfloor[tid]);
    sc[tid] = live ? 1.0 / sqrt(dj) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < S * S; e += SM_THREADS) {
    const int i = e / S, j = e % S;
    A[i][j] *= sc[i] * sc[j];
  }
  __syncthreads();
  for (int j = 0; j < S; ++j) {
    if (tid == 0) {
      const double piv = A[j][j];
      const bool dj = !(piv > eps) || sc[j] == 0.0;
      drop[j] = dj;
      A[j][j] = dj ? 0.0 : sqrt(piv);
    }
    __syncthreads();
    const double ljj = A[j][j];
    const bool dj = drop[j] != 0;
    for (int i = j + 1 + tid; i < S; i += SM_THREADS) A[i][j] = dj ? 0.0 : A[i][j] / ljj;
    __syncthreads();
    const int m = S - j - 1;
    for (int e = tid; e < m * m; e += SM_THREADS) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) A[i][l] -= A[i][j] * A[l][j];
    }
    __syncthreads();
  }
  // Li = L^-1 by forward substitution on the identity; thread c owns column c.
  if (tid < S) {
    const int c = tid;
    for (int i = 0; i < S; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= A[i][k] * Li[k][c];
      Li[i][c] = (drop[i] || drop[c]) ? 0.0 : v / A[i][i];
    }
  }
  __syncthreads();
}

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

// Ks1: W1^+ (kept in `winv`), A = W1^+ W2, psi update from the target rows
// of P, convergence.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small1(const double* __restrict__ W,
                                                       const T* __restrict__ P,
                                                       const int64_t* __restrict__ tgt,
                                                       double* __restrict__ winv,
                                                       T* __restrict__ alpha_out,
                                                       BlockState* __restrict__ st, double tol,
                                                       double eps, int diag) {
  __shared__ double A[S][S + 1];
  __shared__ double Li[S][S + 1];
  __shared__ double Wi[S][S + 1];
  __shared__ double sc[S];
  __shared__ int drop[S];
  __shared__ double dpsi[S];
  const int tid = threadIdx.x;
  const bool frozen = st->frozen != 0;
  const double* W1 = W;
  const double* W2 = W + S * S;

  if (diag) {
    if (tid < S) {
      const double w1 = W1[tid];
      const double w2 = W2[tid];
      const double a = (w1 > 0.0 && !frozen) ? w2 / w1 : 0.0;
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

  guarded_cholesky_inverse(W1, A, Li, sc, drop, eps, nullptr);
  // W1^+ = Sc Li^T Li Sc
  for (int e = tid; e < S * S; e += SM_THREADS) {
    const int i = e / S, j = e % S;
    double acc = 0.0;
    const int k0 = i > j ? i : j;
    for (int k = k0; k < S; ++k) acc += Li[k][i] * Li[k][j];
    const double wij = sc[i] * acc * sc[j];
    Wi[i][j] = wij;
    winv[e] = wij;
  }
  __syncthreads();
  // alpha = W1^+ W2 (into A)
  for (int e = tid; e < S * S; e += SM_THREADS) {
    const int i = e / S, j = e % S;
    double acc = 0.0;
    for (int k = 0; k < S; ++k) acc += Wi[i][k] * W2[k * S + j];
    A[i][j] = frozen ? 0.0 : acc;
  }
  __syncthreads();
  for (int e = tid; e < S * S; e += SM_THREADS) alpha_out[e] = (T)A[e / S][e % S];
  // psi_k increment: row tgt_k of P times column k of alpha.
  if (tid < S) {
    const int64_t v = tgt[tid];
    double acc = 0.0;
    if (v >= 0)
      for (int j = 0; j < S; ++j) acc += (double)P[v * S + j] * A[j][tid];
    dpsi[tid] = acc;
  }
  if (tid == 0) {
    int nd = 0;
    for (int j = 0; j < S; ++j) nd += drop[j];
    st->n_drop = nd;
  }
  __syncthreads();
  if (!frozen) convergence_update(st, dpsi, tol);
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
  const int tid = threadIdx.x;
  const double* W3 = W + 2 * S * S;
  const bool frozen = st->frozen != 0;
  if (diag) {
    if (tid < S) delta_out[tid] = frozen ? (T)0 : (T)(W3[tid] * winv[tid]);
    return;
  }
  for (int e = tid; e < S * S; e += SM_THREADS) {
    const int i = e / S, j = e % S;
    double acc = 0.0;
    for (int k = 0; k < S; ++k) acc += winv[i * S + k] * W3[k * S + j];
    delta_out[e] = frozen ? (T)0 : (T)acc;
  }
}

// Ks3: T = Sc L^-T from the guarded Cholesky of W4 = Y^T D Y, so that the
// kept columns of Y T are D-orthonormal.  A column whose squared D-norm has
// fallen below tau times its value at the start of the solve carries only
// rounding noise (its residual has converged) and is dropped as well; the
// first call after a (re)start records those reference norms.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_small3(const double* __restrict__ W,
                                                       T* __restrict__ t_out,
                                                       BlockState* __restrict__ st, double eps,
                                                       double tau) {
  __shared__ double A[S][S + 1];
  __shared__ double Li[S][S + 1];
  __shared__ double sc[S];
  __shared__ int drop[S];
  __shared__ double floor_[S];
  const double* W4 = W + 3 * S * S;
  const bool first = st->it == 0;
  if (threadIdx.x < S) {
    const double djj = W4[threadIdx.x * S + threadIdx.x];
    if (first) st->scale0[threadIdx.x] = djj;
    floor_[threadIdx.x] = first ? 0.0 : tau * st->scale0[threadIdx.x];
  }
  __syncthreads();
  guarded_cholesky_inverse(W4, A, Li, sc, drop, eps, floor_);
  for (int e = threadIdx.x; e < S * S; e += SM_THREADS) {
    const int j = e / S, k = e % S;
    t_out[e] = (T)(sc[j] * Li[k][j]);
  }
}

// ---------------------------------------------------------------- K2
template <typename T, bool DIAG, bool WITH_D>
__global__ __launch_bounds__(WG) void k_update_r(Coef<T> c, const T* __restrict__ alpha,
                                                 const T* __restrict__ Q,
                                                 const T* __restrict__ P, T* __restrict__ R,
                                                 T* __restrict__ D, double* __restrict__ part) {
  __shared__ T sQ[DIAG ? 1 : CH][S];
  __shared__ T sZ[DIAG ? 1 : CH][S];
  __shared__ T sP[(WITH_D && !DIAG) ? CH : 1][S];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  const int j0 = w * 8;
  T a[DIAG ? 1 : S];
  if (DIAG) {
    a[0] = alpha[lane];
  } else {
#pragma unroll
    for (int j = 0; j < S; ++j) a[j] = alpha[j * S + lane];
  }
  double g[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) g[i] = 0.0;

  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) {
          const T q = Q[v * S + lane];
          const T r = R[v * S + lane] - a[0] * q;
          R[v * S + lane] = r;
          if (WITH_D) D[v * S + lane] += a[0] * P[v * S + lane];
          g[0] += (double)q * (double)(c.dinv[v] * r);
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
      if (WITH_D) sP[row][lane] = ok ? P[v * S + lane] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      T z = 0;
      if (v < rg.end) {
        T acc = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) acc += sQ[row][j] * a[j];
        const T r = R[v * S + lane] - acc;
        R[v * S + lane] = r;
        z = c.dinv[v] * r;
        if (WITH_D) {
          T accd = 0;
#pragma unroll
          for (int j = 0; j < S; ++j) accd += sP[row][j] * a[j];
          D[v * S + lane] += accd;
        }
      }
      sZ[row][lane] = z;
    }
    __syncthreads();
    for (int row = 0; row < CH; ++row) {
      const double z = (double)sZ[row][lane];
#pragma unroll
      for (int i = 0; i < 8; ++i) g[i] += (double)sQ[row][j0 + i] * z;
    }
    __syncthreads();
  }
  double* p0 = part_of(part, 2);
  if (DIAG) {
    __shared__ double red[WG / 64][S];
    red[w][lane] = g[0];
    __syncthreads();
    if (w == 0) {
      double s = 0;
      for (int u = 0; u < WG / 64; ++u) s += red[u][lane];
      p0[lane] = s;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) p0[(j0 + i) * S + lane] = g[i];
  }
}

// ---------------------------------------------------------------- K3
// Y = Dinv R - P B;  W4 = Y^T D Y (block variant only).
template <typename T, bool DIAG>
__global__ __launch_bounds__(WG) void k_update_y(Coef<T> c, const T* __restrict__ delta,
                                                 const T* __restrict__ R,
                                                 const T* __restrict__ P, T* __restrict__ Y,
                                                 double* __restrict__ part) {
  __shared__ T sP[DIAG ? 1 : CH][S];
  __shared__ T sY[DIAG ? 1 : CH][S];
  __shared__ T sDY[DIAG ? 1 : CH][S];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  const int j0 = w * 8;
  T dl[DIAG ? 1 : S];
  if (DIAG) {
    dl[0] = delta[lane];
  } else {
#pragma unroll
    for (int j = 0; j < S; ++j) dl[j] = delta[j * S + lane];
  }
  double g[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) g[i] = 0.0;
  for (int64_t base = rg.begin; base < rg.end; base += CH) {
    if (DIAG) {
#pragma unroll
      for (int i = 0; i < NODES_PER_WAVE; ++i) {
        const int64_t v = base + w * NODES_PER_WAVE + i;
        if (v < rg.end) Y[v * S + lane] = c.dinv[v] * R[v * S + lane] - dl[0] * P[v * S + lane];
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      sP[row][lane] = v < rg.end ? P[v * S + lane] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NODES_PER_WAVE; ++i) {
      const int row = w * NODES_PER_WAVE + i;
      const int64_t v = base + row;
      T y = 0, dy = 0;
      if (v < rg.end) {
        T acc = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) acc += sP[row][j] * dl[j];
        y = c.dinv[v] * R[v * S + lane] - acc;
        Y[v * S + lane] = y;
        dy = c.d[v] * y;
      }
      sY[row][lane] = y;
      sDY[row][lane] = dy;
    }
    __syncthreads();
    for (int row = 0; row < CH; ++row) {
      const double dy = (double)sDY[row][lane];
#pragma unroll
      for (int i = 0; i < 8; ++i) g[i] += (double)sY[row][j0 + i] * dy;
    }
    __syncthreads();
  }
  if (!DIAG) {
#pragma unroll
    for (int i = 0; i < 8; ++i) part_of(part, 3)[(j0 + i) * S + lane] = g[i];
  }
}

// W4 = Y^T D Y alone (used when a refinement step restarts from a new Y).
template <typename T>
__global__ __launch_bounds__(WG) void k_gram_dy(Coef<T> c, const T* __restrict__ Y,
                                                double* __restrict__ part) {
  __shared__ T sY[CH][S];
  __shared__ T sDY[CH][S];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const Range rg = block_range(c.n, gridDim.x);
  const int j0 = w * 8;
  double g[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) g[i] = 0.0;
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
    for (int row = 0; row < CH; ++row) {
      const double dy = (double)sDY[row][lane];
#pragma unroll
      for (int i = 0; i < 8; ++i) g[i] += (double)sY[row][j0 + i] * dy;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) part_of(part, 3)[(j0 + i) * S + lane] = g[i];
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
                              T* __restrict__ Y, T* __restrict__ Tm, BlockState* st, int diag) {
  const int k = threadIdx.x;
  if (k < S) {
    const int64_t v = tgt[k];
    if (v >= 0) {
      R[v * S + k] = T(1);
      Y[v * S + k] = dinv[v];
    }
    for (int j = 0; j < S; ++j)
      Tm[j * S + k] = (j == k && v >= 0) ? (diag ? T(1) : (T)sqrt((double)d[v])) : T(0);
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
  const dim3 g(G), blk(WG);
  if (ev) hipEventRecord(ev[0], st);
  if (indep)
    hipLaunchKernelGGL((k_spmv_gram<T, true>), g, blk, 0, st, c, Y, (const T*)b.Tm, R, P, Q,
                       b.part);
  else
    hipLaunchKernelGGL((k_spmv_gram<T, false>), g, blk, 0, st, c, Y, (const T*)b.Tm, R, P, Q,
                       b.part);
  if (ev) hipEventRecord(ev[1], st);
  hipLaunchKernelGGL(k_reduce, dim3((2 * len + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 0,
                     2, len);
  hipLaunchKernelGGL((k_small1<T>), dim3(1), dim3(SM_THREADS), 0, st, b.W, (const T*)P, b.tgt,
                     b.winv, (T*)b.alpha, b.state, tol, eps1, indep ? 1 : 0);
  if (ev) hipEventRecord(ev[2], st);
  if (indep) {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, true, true>), g, blk, 0, st, c, (const T*)b.alpha, Q,
                         P, R, D, b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, true, false>), g, blk, 0, st, c, (const T*)b.alpha, Q,
                         P, R, D, b.part);
  } else {
    if (with_d)
      hipLaunchKernelGGL((k_update_r<T, false, true>), g, blk, 0, st, c, (const T*)b.alpha, Q,
                         P, R, D, b.part);
    else
      hipLaunchKernelGGL((k_update_r<T, false, false>), g, blk, 0, st, c, (const T*)b.alpha, Q,
                         P, R, D, b.part);
  }
  if (ev) hipEventRecord(ev[3], st);
  hipLaunchKernelGGL(k_reduce, dim3((len + 63) / 64), dim3(256), 0, st, b.part, b.W, G, 2, 1,
                     len);
  hipLaunchKernelGGL((k_small2<T>), dim3(1), dim3(SM_THREADS), 0, st, b.W, b.winv,
                     (T*)b.delta, b.state, indep ? 1 : 0);
  if (ev) hipEventRecord(ev[4], st);
  if (indep) {
    hipLaunchKernelGGL((k_update_y<T, true>), g, blk, 0, st, c, (const T*)b.delta, R, P, Y,
                       b.part);
    if (ev) hipEventRecord(ev[5], st);
  } else {
    hipLaunchKernelGGL((k_update_y<T, false>), g, blk, 0, st, c, (const T*)b.delta, R, P, Y,
                       b.part);
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

__global__ void k_set_diag_one(float* __restrict__ Tm) {
  if (threadIdx.x < S) Tm[threadIdx.x * S + threadIdx.x] = 1.0f;
}

hipError_t launch_restart(const Coef<float>& cf, const SolveBuffers& b, bool indep,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(S), 0, st, b.state);
  const int G = grid_for(cf.n);
  if (indep) {
    // T = I: the independent variant needs no orthonormalisation.
    hipLaunchKernelGGL((k_zero<float>), dim3(16), dim3(256), 0, st, (float*)b.Tm, S * S);
    hipLaunchKernelGGL(k_set_diag_one, dim3(1), dim3(S), 0, st, (float*)b.Tm);
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
