// Internal declarations shared by the host runtime (reff_api.cpp) and the
// gfx950 kernels (reff_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/reff.h"

namespace reff {

struct SelinvPlan;    // selinv_plan.h
struct SelinvDevice;  // selinv.hip

// Set the calling thread's reff_last_error() text and return s.
reff_status host_fail(reff_status s, const std::string& msg);
// The stack validation every entry point performs before device work.
reff_status host_validate_desc(const reff_pdn_desc* d);
// Eq. 3 resistances of every pair of P points (device xy) on a uniform
// M x N tier into device out[P * P] (grid_pairs.hip); returns once the
// stream has run the kernels.
hipError_t grid_pairs_device(int M, int N, double r, double s, const int32_t* dxy, int64_t P,
                             double* dout, hipStream_t st);

constexpr int S = 64;        // right-hand sides per block (one per lane)
constexpr int CH = 32;       // nodes per LDS chunk in the block kernels
constexpr int WG = 512;      // threads per workgroup of the block kernels
constexpr int NODES_PER_WAVE = CH / (WG / 64);  // 4
constexpr int HIST = 8;      // convergence window (iterations)
constexpr int MAX_GRID = 512;
constexpr int NGRAM = 4;     // Gram partials per work unit
constexpr int MAX_CHEB = 32;  // largest Chebyshev preconditioner degree
constexpr int NEV = 10;       // timing events per block iteration (5 spans)
// A column is converged once its estimated remaining relative error is
// below CONV_SAFETY * rel_tol.
constexpr double CONV_SAFETY = 0.25;

// Per-node stencil coefficients of the grounded conductance matrix G, one
// structure-of-arrays copy per precision.  For a node v of a stack with row
// length nx and tier size plane (pads and the other grounded nodes are
// identity rows with all couplings zero):
//   (G p)_v = d_v p_v - cE_v p_{v+1} - cE_{v-1} p_{v-1}
//             - cN_v p_{v+nx} - cN_{v-nx} p_{v-nx}
//             - up_v p_{v+plane} - dn_v p_{v-plane}
// where up/dn come from the TSV side list (slot_v >= 0 only on nodes that
// carry a TSV segment).  Several stacks may be concatenated (a batch).
template <typename T>
struct Coef {
  const T* d;
  const T* dinv;
  const T* cE;
  const T* cN;
  const int32_t* slot;   // index into up/dn, -1 if the node has no TSV
  const T* up;           // coupling to v + plane
  const T* dn;           // coupling to v - plane
  const int64_t* tnode;  // slot -> coefficient index of its node
};

// One solve block: a stack (coefficients from node cbase on, n nodes, row
// length nx, tier size plane) with its own S right-hand sides, whose vectors
// occupy rows vbase .. vbase+n-1 of the n x S work arrays.  Its work units
// are unit_begin .. unit_end-1.
struct PlanDesc {
  int64_t cbase;
  int64_t vbase;
  int64_t n;
  int64_t plane;
  int32_t nx;
  int32_t unit_begin, unit_end;
  int32_t strip_begin, strip_end;  // its strips (stencil kernel), if any
  int32_t slot_begin, slot_end;    // its stack's TSV slots (coefficient set indices)
  int64_t sbase;                   // first row of its slots in the TSV side buffers
};

// A contiguous range of vector rows [begin, end) of one solve block,
// processed by one workgroup of the vector kernels.
struct Unit {
  int64_t begin, end;
  int32_t plan;
  int32_t pad_;
};

// A strip of one tier of a solve block for the stencil kernel: nodes
// x0 .. x0+wdt-1 (wdt <= CH) of rows y0 .. y0+nrows-1; lrow0 is the
// block-local id of node (x0, y0).  The kernel marches in +y keeping the
// rows y-1, y, y+1 on chip, so each Y row is fetched once.
struct Strip {
  int64_t lrow0;
  int32_t plan;
  int32_t nrows;
  int32_t wdt;
  int32_t y0;
  int32_t x0;
  int32_t pad_;
};

// Argument bundle of the vector kernels.  The active work lives on the
// device: cnt[0] units uid[0 .. cnt[0]), cnt[1] strips sid[0 .. cnt[1]) and
// cnt[2] solve blocks (act[]), rewritten by k_compact at the end of every
// iteration as blocks converge.  Launch grids cover the whole group; a
// workgroup whose logical item is not active returns at once, so a captured
// sequence of launches stays valid while the active set shrinks.
struct Work {
  const PlanDesc* plans;
  const Unit* units;
  const int32_t* uid;
  const Strip* strips;
  const int32_t* sid;
  const int32_t* cnt;
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

// Device work arrays of the block solver (grown on demand, reused).
struct Workspace {
  DevBuf Y, P, Q, R, D, X, part, W, small, state, tgt, pos, plans, units, uid, act, out, xs,
      rows, map, flags, strips, sid, Za, Zb, Zc, Zd, TA, TB, cnt;
  void release();
};

}  // namespace reff

namespace reff {

// Stencil coefficients of one grounded system on the device, both
// precisions.  `grounded` marks the Dirichlet nodes of this system (the pads
// for node-to-supply resistance; one reference node for the floating
// network of the whole stack).
struct CoefSet {
  bool ready = false;
  double *d64 = nullptr, *dinv64 = nullptr, *cE64 = nullptr, *cN64 = nullptr,
         *up64 = nullptr, *dn64 = nullptr;
  float *d32 = nullptr, *dinv32 = nullptr, *cE32 = nullptr, *cN32 = nullptr,
        *up32 = nullptr, *dn32 = nullptr;
  int32_t* slot = nullptr;
  int64_t* tnode = nullptr;  // slot -> coefficient index of its node
  std::vector<uint8_t> grounded;
  int64_t n_free = 0;
  int64_t n_slots = 0;
};

}  // namespace reff

struct reff_pdn_t {
  int device = 0;
  int32_t nt = 0, nx = 0, ny = 0;
  int64_t n = 0, plane = 0;
  // host copy of the description (to build further coefficient sets)
  std::vector<double> gx, gy, tsv_g;
  std::vector<int32_t> tsv_xy, pad_xy;
  reff::CoefSet gnd;   // pads grounded (node-to-supply resistance)
  reff::CoefSet flt;   // one reference node grounded (floating pairs)
  int64_t flt_ref = -1;
  reff::Workspace ws;         // solver work arrays (grown on demand)
  std::vector<void*> extra;  // coefficient allocations freed with the handle
  std::shared_ptr<reff::SelinvPlan> sel_plan;  // sparse-direct plan, built on first use
  std::shared_ptr<reff::SelinvDevice> sel_dev;  // its device tables and work buffers
};

namespace reff {

// Kernel launchers (reff_kernels.hip).  All launch on `st` and return the
// HIP error of the launch.
// Work arrays of one solve (nb solve blocks at once).  Vectors are
// rows x S; the S x S matrices and states are per solve block.
struct SolveBuffers {
  void* Y;       // rows x S, T: search block before orthonormalisation
  void* P;       // rows x S, T: P = Y T
  void* Q;       // rows x S, T: Q = G P
  void* R;       // rows x S, T: residual block
  void* D;       // rows x S, T: accumulated solution (mixed path / pairs), may be null
  double* X;     // rows x S, float64 (mixed path accumulated solution), may be null
  double* part;  // max(units, strips) x NGRAM x S*S partial Grams
  double* W;     // nb x NGRAM x S*S reduced Grams
  double* winv;  // nb x S*S: W1^+
  void* alpha;   // nb x S*S in T
  void* delta;   // nb x S*S in T
  void* Tm;      // nb x S*S in T: orthonormalising map T
  BlockState* state;  // nb
  int64_t* tgt;  // nb x S target node ids, local to the stack (-1 = empty)
  int64_t* pos;  // nb x S output positions (-1 = none)
  Work work;     // device plan / unit tables
  const int32_t* act;  // active solve blocks (small kernels, reductions)
  int32_t* act_w;      // the same lists, writable (k_compact)
  int32_t* uid_w;
  int32_t* sid_w;
  int32_t* cnt;        // device active counts (= work.cnt)
  int n_act;     // solve blocks of the group (grid of the small kernels)
  int n_units;   // units of the group (grid of the vector kernels)
  int n_strips;  // strips of the group (grid of the strip kernels; 0 = not used)
  int64_t rows;  // vector rows covered by the active units' blocks
  // Chebyshev polynomial preconditioner of degree cheb_k (block variant;
  // 1 = Jacobi): Z = q(D^-1 G) D^-1 R by cheb_k - 1 strip steps from
  // z_1 = D^-1 R / theta, step j using cheb_a1[j], cheb_a2[j].
  int cheb_k = 1;
  double cheb_invtheta = 1.0;
  double cheb_a1[MAX_CHEB] = {};
  double cheb_a2[MAX_CHEB] = {};
  void* Za = nullptr;  // rows x S, T: Chebyshev iterates (z_1 in Za, then
  void* Zb = nullptr;  // rotating over the four arrays)
  void* Zc = nullptr;
  void* Zd = nullptr;
  // TSV side buffers of the three-step passes: z_{j+1} at every TSV node and
  // its four in-plane neighbours ([slot row][5][S]) and z_{j+2} at every TSV
  // node ([slot row][S]); max_tsv_slots = most TSV slots of one block.
  void* TA = nullptr;
  void* TB = nullptr;
  int max_tsv_slots = 0;
};

int grid_for(int64_t n);

hipError_t launch_init_blocks(bool fp32, bool indep, const void* coef, const SolveBuffers& b,
                              hipStream_t st);
// ev (nullable): NEV events, before/after K1, K2, K3, the Chebyshev passes
// and the Q^T Z Gram (ev[0..1], [2..3], [4..5], [6..7], [8..9]).
hipError_t launch_iteration(bool fp32, bool indep, bool with_d, const void* coef,
                            const SolveBuffers& b, double tol, hipStream_t st, hipEvent_t* ev);
hipError_t launch_zero_x(double* X, int64_t cnt, hipStream_t st);
// Rebuild the active lists and counts of a group from its blocks'
// convergence flags (blocks 0 .. nb-1, all of them, in order).
hipError_t launch_compact(const SolveBuffers& b, int nb, hipStream_t st);
hipError_t launch_mixed_residual(const Coef<double>& c, const Coef<float>& cf,
                                 const SolveBuffers& b, double* out, hipStream_t st);
hipError_t launch_restart(const Coef<float>& cf, const SolveBuffers& b, bool indep,
                          hipStream_t st);
hipError_t launch_finalize_plain(const SolveBuffers& b, double* out, hipStream_t st);
hipError_t launch_gather_out(const double* res, const int64_t* map, double* out,
                             int64_t count, hipStream_t st);
// C = Xa^T (G Xb) for two solved blocks of the same stack (plan 0 of b.work;
// partials + reduction; result in b.W[0 .. S*S)).
// out[c * ld + r] += sum_k (sum_{e in row r} w_e X[node_e][k]) amps[k][c] for the
// weighted node rows r < nrows (CSR rptr / rnode / rw, device) of a solved
// float64 block X (n x S) and its S x n_scen load matrix (ir_drop.hip).
hipError_t launch_rows_times_loads(const double* X, const int32_t* rptr, const int64_t* rnode,
                                   const double* rw, int64_t nrows, const double* amps,
                                   int n_scen, double* out, int64_t ld, hipStream_t st);
// R(a_i, b_j) on the device from gathered endpoint rows and block cross Grams
// (see k_pairs_finish in reff_kernels.hip); blocks bu, bv with bu / grp !=
// bv / grp were not resident together and have no cross Gram.
hipError_t launch_pairs_finish(int64_t m, int64_t n, const int64_t* ia, const int64_t* ib,
                               const int64_t* aid, const int64_t* bid, const int32_t* blk,
                               const int32_t* col, const double* rows, const double* cg, int64_t U,
                               int64_t nblk, int64_t grp, double* out, hipStream_t st);
hipError_t launch_cross_gram(const Coef<double>& c, const double* Xa, const double* Xb,
                             const SolveBuffers& b, hipStream_t st);
// rows[i*S + k] = X[nodes[i]*S + k] for i < count.
hipError_t launch_gather_rows(const double* X, const int64_t* nodes, int64_t count,
                              double* rows, hipStream_t st);

}  // namespace reff
