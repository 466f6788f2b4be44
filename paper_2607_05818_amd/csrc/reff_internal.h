// Internal declarations shared by the host runtime (reff_api.cpp) and the
// gfx950 kernels (reff_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/reff.h"

namespace reff {

constexpr int S = 64;        // right-hand sides per block (one per lane)
constexpr int CH = 32;       // nodes per LDS chunk in the block kernels
constexpr int WG = 512;      // threads per workgroup of the block kernels
constexpr int NODES_PER_WAVE = CH / (WG / 64);  // 4
constexpr int HIST = 16;     // convergence window (iterations)
constexpr int MAX_GRID = 512;
// A column is converged once its estimated remaining relative error is
// below CONV_SAFETY * rel_tol.
constexpr double CONV_SAFETY = 0.25;

// Per-node stencil coefficients of the grounded conductance matrix G, one
// structure-of-arrays copy per precision.  For a node v (pads are identity
// rows with all couplings zero):
//   (G p)_v = d_v p_v - cE_v p_{v+1} - cE_{v-1} p_{v-1}
//             - cN_v p_{v+nx} - cN_{v-nx} p_{v-nx}
//             - up_v p_{v+plane} - dn_v p_{v-plane}
// where up/dn come from the TSV side list (slot_v >= 0 only on nodes that
// carry a TSV segment).
template <typename T>
struct Coef {
  const T* d;
  const T* dinv;
  const T* cE;
  const T* cN;
  const int32_t* slot;   // [n] index into up/dn, -1 if the node has no TSV
  const T* up;           // [n_slots] coupling to v + plane
  const T* dn;           // [n_slots] coupling to v - plane
  int64_t n;
  int32_t nx;
  int64_t plane;
};

// Device-resident convergence state of one block solve.
struct BlockState {
  double psi[S];          // accumulated R estimate per column
  double hist[HIST][S];   // last HIST increments per column
  double est_rel[S];      // estimated remaining relative error per column
  double ref[S];          // reference R for relative tests (0: use psi)
  double scale0[S];       // squared D-norm of each search column at (re)start
  int32_t it;             // iterations done
  int32_t all_conv;       // 1 once every column met the tolerance
  int32_t frozen;         // 1: later iterations make no update
  int32_t n_drop;         // directions dropped by the rank guard (last it)
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace reff

struct reff_pdn_t {
  int device = 0;
  int32_t nt = 0, nx = 0, ny = 0;
  int64_t n = 0, plane = 0;
  int64_t n_slots = 0;
  int64_t n_free = 0;
  std::vector<uint8_t> is_pad;       // host copy
  // device coefficient storage
  double *d64 = nullptr, *dinv64 = nullptr, *cE64 = nullptr, *cN64 = nullptr,
         *up64 = nullptr, *dn64 = nullptr;
  float *d32 = nullptr, *dinv32 = nullptr, *cE32 = nullptr, *cN32 = nullptr,
        *up32 = nullptr, *dn32 = nullptr;
  int32_t* slot = nullptr;
  // workspace (grown on demand)
  reff::DevBuf ws_Y, ws_P, ws_Q, ws_R, ws_D, ws_X, ws_part, ws_W, ws_small, ws_state,
      ws_tgt, ws_out;
  std::vector<void*> extra;  // misc allocations freed with the handle
};

namespace reff {

// Kernel launchers (reff_kernels.hip).  All launch on `st` and return the
// HIP error of the launch.
struct SolveBuffers {
  void* Y;       // n x S, T: search block before orthonormalisation
  void* P;       // n x S, T: P = Y T
  void* Q;       // n x S, T: Q = G P
  void* R;       // n x S, T: residual block
  void* D;       // n x S, T: accumulated solution (mixed path), may be null
  double* X;     // n x S, float64 (mixed path accumulated solution), may be null
  double* part;  // grid x 4 x S*S partial Grams
  double* W;     // 4 x S*S reduced Grams
  double* winv;  // S*S: W1^+
  void* alpha;   // S*S in T
  void* delta;   // S*S in T
  void* Tm;      // S*S in T: orthonormalising map T
  BlockState* state;
  int64_t* tgt;  // S target node ids (-1 = empty column)
};

int grid_for(int64_t n);

hipError_t launch_init_block(bool fp32, bool indep, const void* coef, const SolveBuffers& b,
                             hipStream_t st);
// ev (nullable): 6 events recorded around the three block kernels
// (before/after K1, K2, K3).
hipError_t launch_iteration(bool fp32, bool indep, bool with_d, const void* coef,
                            const SolveBuffers& b, int64_t n, double tol, hipStream_t st,
                            hipEvent_t* ev);
hipError_t launch_zero_x(double* X, int64_t cnt, hipStream_t st);
hipError_t launch_mixed_residual(const Coef<double>& c, const Coef<float>& cf,
                                 const SolveBuffers& b, double* out, const int64_t* pos,
                                 hipStream_t st);
hipError_t launch_restart(const Coef<float>& cf, const SolveBuffers& b, bool indep,
                          hipStream_t st);
hipError_t launch_finalize_plain(const SolveBuffers& b, double* out, const int64_t* pos,
                                 hipStream_t st);
hipError_t launch_gather_out(const double* res, const int64_t* map, double* out,
                             int64_t count, hipStream_t st);

}  // namespace reff
