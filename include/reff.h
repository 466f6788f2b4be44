/*
 * reff.h -- C ABI of libreff: effective resistance of stacked 3D-IC power
 * delivery networks on AMD Instinct MI355X (gfx950).
 *
 * Problem (arxiv 2607.05818):
 *   The early-stage PDN is a stack of 2D resistive tier meshes joined by
 *   TSV segments; supply bumps are ideal voltage sources (Sec. III-B).  Its
 *   DC model is G V = I with G sparse, symmetric, positive definite
 *   (Sec. II-A, Eq. 1).  The effective resistance between nodes a and b is
 *   R(a,b) = (e_a - e_b)^T L^+ (e_a - e_b) (Sec. II-B, Eq. 2).  With every
 *   bump merged into one grounded supply node, a node's resistance to the
 *   supply is R_i = (G^-1)_ii, G being the Laplacian restricted to the
 *   non-pad nodes.
 *
 * Conventions shared by every entry point:
 *   - Node id = t*nx*ny + y*nx + x; tier 0 carries the pads (bumps).
 *   - Every call returns reff_status; nothing throws or aborts across the ABI.
 *   - All argument validation happens on the host before any device work;
 *     on error the outputs are left untouched (one documented exception:
 *     REFF_ERR_NO_CONVERGENCE).
 *   - Pointers documented as "host" must be host memory; "device" pointers
 *     must be device memory of the handle's device.
 *   - A handle must be used by one thread at a time; distinct handles may be
 *     used concurrently.  reff_last_error() is thread-local.
 */
#ifndef REFF_H
#define REFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  REFF_OK = 0,
  REFF_ERR_INVALID_ARG = -1,    /* NULL pointer, dims < 1, conductance <= 0 or
                                   non-finite, (x,y) out of range, duplicate
                                   TSV column, node id out of range        */
  REFF_ERR_DISCONNECTED = -2,   /* some node has no path to a pad: G singular */
  REFF_ERR_NO_CONVERGENCE = -3, /* max_iters reached; R_out holds the solver's
                                   lower bounds, stats->n_unconverged > 0    */
  REFF_ERR_OUT_OF_MEMORY = -4,
  REFF_ERR_DEVICE = -5,         /* HIP runtime error; see reff_last_error();
                                   the handle stays valid for reff_free_pdn */
  REFF_ERR_UNSUPPORTED = -6
} reff_status;

/* Opaque handle to a PDN resident on one GPU (library-owned). */
typedef struct reff_pdn_t* reff_pdn;

/*
 * Stack description (Sec. III-B: 2D tier meshes joined by TSVs, bumps on one
 * tier).  All arrays are host memory, borrowed for the duration of the call
 * and deep-copied by reff_build_pdn.
 */
typedef struct {
  int32_t n_tiers, nx, ny;  /* each >= 1                                     */
  const double* gx;         /* [n_tiers][ny][nx-1] S, edge (t,x,y)-(t,x+1,y)  */
  const double* gy;         /* [n_tiers][ny-1][nx] S, edge (t,x,y)-(t,x,y+1)  */
  int32_t n_tsv;            /* >= 0                                          */
  const int32_t* tsv_xy;    /* [n_tsv][2] (x,y); the column joins (t,x,y) and
                               (t+1,x,y) for every t < n_tiers-1; distinct   */
  const double* tsv_g;      /* [n_tsv][n_tiers-1] segment conductance, S     */
  int32_t n_pads;           /* >= 1                                          */
  const int32_t* pad_xy;    /* [n_pads][2] (x,y) on tier 0: ideal supply bumps,
                               grounded (Dirichlet); duplicates allowed      */
} reff_pdn_desc;

typedef enum {
  REFF_PREC_FP64 = 0,   /* block-PCG entirely in float64                    */
  REFF_PREC_MIXED = 1   /* float32 block-PCG inside float64 iterative
                           refinement; final R_i accumulated in float64     */
} reff_precision;

typedef enum {
  REFF_KRYLOV_BLOCK = 0,       /* block-PCG: columns share one block Krylov
                                  space, s x s Gram products              */
  REFF_KRYLOV_INDEPENDENT = 1  /* s independent PCGs run side by side       */
} reff_krylov;

typedef struct {
  reff_precision precision;
  double rel_tol;        /* target relative error per R_i; 0 => 1e-8 (FP64)
                            or 1e-5 (MIXED)                                 */
  int32_t max_iters;     /* per block-PCG solve; 0 => 20000                 */
  int32_t block_rhs;     /* right-hand sides dealt to one block: 32 or 64;
                            0 => 64.  The kernels give every right-hand
                            side one lane of a 64-wide wave, so a block
                            streams 64 columns either way: 32 halves the
                            columns per block (twice the bytes per node
                            solved) and is never faster                  */
  void* stream;          /* hipStream_t to run on; NULL => default stream    */
  int32_t out_on_device; /* 1: R_out is a device pointer; 0: host pointer   */
  reff_krylov krylov;    /* 0 => block                                       */
  int32_t max_ir_steps;  /* MIXED only: outer refinement steps; 0 => 3       */
  int32_t timing;        /* 1: time the three block kernels with HIP events on
                            `stream` (fills the kernel_* fields of stats)    */
  int32_t graphs;        /* 0 (automatic) or 1: replay chunks of four
                            iterations as HIP graphs unless timing is on or
                            `stream` is itself being captured; on the NULL
                            stream the solve then runs on a stream of its
                            own (drained before the call returns).  Blocks
                            that converge leave device-resident work lists,
                            so a captured chunk stays valid.  Same results
                            bitwise as plain launches.  2: plain launches  */
  int32_t progress;      /* 1: write a progress line (iterations, active
                            blocks) to stderr at most every 10 s of a solve */
  int32_t precond_degree;/* block Krylov variant: 1 = Jacobi (D^-1); 2..32 =
                            Chebyshev polynomial preconditioner
                            q(D^-1 G) D^-1 of that degree (SPD and fixed,
                            so the results are those of PCG with a stronger
                            preconditioner; fewer, costlier iterations);
                            0 => by the larger side of the stack's tiers
                            (of a batch's largest plan): 19 up to 640
                            nodes, 31 above.  The independent variant uses
                            Jacobi. */
  int32_t pairs_resident_blocks;
                         /* reff_query_pairs: solution blocks (64 endpoints
                            each, n_nodes x 64 float64) kept on the device
                            at once; 0 => as many as half the free device
                            memory holds.  When the request needs more, the
                            endpoints are solved in groups of that many
                            blocks and memory stays bounded by the group
                            (see reff_query_pairs). */
} reff_solve_opts;

typedef struct {
  int64_t n_solved;       /* distinct free nodes solved                      */
  int64_t n_unconverged;  /* columns that hit max_iters                      */
  int32_t iters_max;      /* largest inner iteration count of any block      */
  int32_t ir_steps;       /* largest number of refinement steps (MIXED)      */
  double seconds;         /* wall time of the call                           */
  double est_max_rel_err; /* solver's own estimate of the worst relative
                             error (not a bound)                             */
  int64_t iters_total;    /* sum of block iterations over all blocks         */
  /* With opts->timing, per block iteration: summed device time (ms) and
     count of the stencil+Gram kernel [0], the residual-update kernel [1],
     the search-block kernel [2], the polynomial preconditioner's Chebyshev
     passes [3] (one entry covers all passes of an iteration) and its Q^T Z
     Gram [4], and the node rows those launches streamed (one row = one
     node of one 64-column block; a launch covers every unconverged block
     of its group). */
  double kernel_ms[5];
  int64_t kernel_launches[5];
  int64_t kernel_rows[5];
  /* reff_batch_plans with a surrogate: 1 if the plan's results are the
     model's predictions (solved values at the checked nodes), 0 if it fell
     back to the solver; the largest relative error of the prediction over
     the checked nodes. */
  int32_t screened;
  double spot_max_rel_err;
} reff_solve_stats;

/*
 * Validate a stack, check that every node reaches a pad (breadth-first
 * search), build the per-node stencil coefficients of G and upload them to
 * `device`.  *out receives a new handle; free it with reff_free_pdn.
 * Errors: INVALID_ARG, DISCONNECTED, OUT_OF_MEMORY, DEVICE.
 */
reff_status reff_build_pdn(const reff_pdn_desc* d, int32_t device, reff_pdn* out);

/* Release a handle and its device memory.  NULL is ignored. */
void reff_free_pdn(reff_pdn p);

/* Number of nodes of a handle (n_tiers*nx*ny), or -1 for NULL. */
int64_t reff_pdn_num_nodes(reff_pdn p);

/*
 * Node-to-supply effective resistance R_i = (G^-1)_ii (Eq. 2 with all bumps
 * merged into the grounded supply, Sec. II-B / III-B).
 *   nodes    host int64[n_nodes] node ids, or NULL for all nodes in id order;
 *            duplicates allowed; pads give 0.0.
 *   R_out    float64[n_nodes] (host, or device if opts->out_on_device).
 *   opts     NULL => defaults.  st nullable.
 * Errors: INVALID_ARG (bad id, bad option), NO_CONVERGENCE (R_out holds the
 * block-PCG lower bounds), OUT_OF_MEMORY, DEVICE.
 */
reff_status reff_solve_diag(reff_pdn p, const int64_t* nodes, int64_t n_nodes,
                            double* R_out, const reff_solve_opts* opts,
                            reff_solve_stats* st);

/*
 * Statistics of a sparse-direct selected inversion (reff_selinv_diag), or of
 * its plan alone (reff_selinv_info: the timing fields stay 0).
 */
typedef struct {
  int64_t n_fronts;       /* supernodes of the nested-dissection tree         */
  int32_t n_levels;       /* depth of the tree + 1                            */
  int32_t reserved;
  int64_t max_front;      /* rows of the largest dense front                  */
  int64_t device_bytes;   /* device memory one call allocates                 */
  double flops_factor;    /* float64 flops of the factorisation               */
  double flops_selinv;    /* float64 flops of the selected inversion          */
  double seconds;         /* wall time of the call                            */
  double seconds_plan;    /* symbolic analysis (on a handle's first use only) */
  double seconds_factor;  /* factorisation (device set-up included)          */
  double seconds_selinv;  /* selected inversion and output                    */
  double seconds_setup;   /* of seconds_factor: device allocation and upload of
                             the plan's tables (0 when a handle reuses them) */
} reff_selinv_stats;

/*
 * R_i = (G^-1)_ii (Eq. 2 with all bumps merged into the grounded supply,
 * Sec. II-B / III-B) by sparse-direct selected inversion: nested dissection
 * of the stacked grid (walls of columns through every tier), a multifrontal
 * float64 Cholesky factorisation G = L L^T and the Takahashi recurrence for
 * the entries of G^-1 on the structure of L, all numeric work on the GPU.
 * The definition itself, to float64 rounding: there is no tolerance and no
 * iteration.  The cost does not depend on how many nodes are asked for, so
 * it is the method for full maps; block PCG (reff_solve_diag) is the method
 * for samples.  The plan (ordering and front structure), its device tables
 * and the work buffers (reff_selinv_info().device_bytes) are set up on the
 * handle's first call and kept with it until reff_free_pdn; calls on one
 * handle must not overlap.
 *   nodes, n_nodes, R_out   as reff_solve_diag (pads give 0.0).
 *   opts     NULL => defaults; only stream and out_on_device are read.
 *   st       nullable.
 * Errors: INVALID_ARG (bad id or option), OUT_OF_MEMORY (the fronts need
 * reff_selinv_info().device_bytes of device memory), DEVICE (HIP error, or
 * a Cholesky pivot that is not positive).
 */
reff_status reff_selinv_diag(reff_pdn p, const int64_t* nodes, int64_t n_nodes,
                             double* R_out, const reff_solve_opts* opts,
                             reff_selinv_stats* st);

/*
 * reff_selinv_diag for many stacks (candidate TSV plans, Sec. I and IV-B) in
 * one call, with no handle: the plans' dissection trees are analysed on
 * host threads and merged by depth, so every plan's fronts of one tree
 * level share the same launches.  Batches above 4M nodes run as up to four
 * chunks of consecutive plans, the host analysis of a chunk overlapping the
 * device work of the one before.  Device memory (about the sum of a chunk's
 * plans' reff_selinv_info().device_bytes) comes from a workspace the library
 * keeps between calls (reff_release_cached_memory frees it).  With node
 * lists, only the fronts holding the requested nodes and their ancestors go
 * through the selected inversion (same values bit for bit).  In `st`,
 * seconds_plan is the host analysis the device work did not hide.  Inputs
 * as reff_batch_plans:
 *   plans    host array of n_plans stack descriptions (validated as
 *            reff_build_pdn does, and checked for connectivity).
 *   nodes    NULL, or host array of n_plans node-id arrays (an entry NULL =
 *            all nodes of that plan); n_nodes their lengths.
 *   R_out    n_plans output arrays (host, or device if opts->out_on_device).
 *   opts     NULL => defaults; only stream and out_on_device are read.  Runs
 *            on the current device.
 * Errors: INVALID_ARG (naming the plan), DISCONNECTED, OUT_OF_MEMORY, DEVICE.
 * Descriptors and node ids are validated before any device work, and so is
 * the analysis of the first chunk (of every plan, below 4M nodes); R_out is
 * written only when the call succeeds.
 */
reff_status reff_selinv_batch(const reff_pdn_desc* plans, int32_t n_plans,
                              const int64_t* const* nodes, const int64_t* n_nodes,
                              double* const* R_out, const reff_solve_opts* opts,
                              reff_selinv_stats* st);

/*
 * reff_selinv_batch carves its device buffers from one workspace per device
 * that the library keeps between calls (grown when a call needs more), so
 * that repeated batches do not map their fronts afresh.  This frees the
 * workspace of `device` (a no-op while a batch is using it).
 * Errors: INVALID_ARG, DEVICE.
 */
reff_status reff_release_cached_memory(int32_t device);

/* The plan reff_selinv_diag would use for a stack (host only, no device
 * needed): fronts, levels, largest front, device bytes and flop counts.
 * Errors: INVALID_ARG (as reff_build_pdn's validation), DISCONNECTED. */
reff_status reff_selinv_info(const reff_pdn_desc* d, reff_selinv_stats* info);

/*
 * HBM bandwidth probe (a measurement helper; no part of any result): one
 * launch of a plain streaming kernel with 16-byte accesses, `blocks`
 * workgroups of 256 threads walking the data grid-stride, on `stream`.
 *   kind 0  copy src -> dst (bytes each)
 *        1  read src; dst receives blocks x 256 floats (partial sums)
 *        2  write dst
 *        3  read three arrays, write two (the Chebyshev pass's mix): src
 *           holds 3 x bytes, dst 2 x bytes, element-wise sums
 *        4  copy with non-temporal loads and stores
 * src, dst: device pointers.  bytes: per array, a positive multiple of 16.
 * Errors: INVALID_ARG, DEVICE (launch error).  Asynchronous: time it with
 * events on `stream`.
 */
reff_status reff_stream_probe(int32_t kind, const void* src, void* dst, int64_t bytes,
                              int32_t blocks, void* stream);

typedef enum {
  REFF_PAIRS_GROUNDED = 0, /* pads merged into the grounded supply:
                              R(a,b) = K_aa + K_bb - 2 K_ab with K = G^-1   */
  REFF_PAIRS_FLOATING = 1  /* Eq. 2 on the whole un-grounded stack: pads are
                              ordinary nodes (the paper's bump-to-load
                              resistance, Sec. III-C/D)                    */
} reff_pair_mode;

/*
 * m x n pair resistances R(a_i, b_j), from m + n solves by linearity
 * (Sec. III-D: m x n bump-load pairs from m + n solves).
 *   a, b     host int64 node ids; R_out float64[m*n] row-major (host, or
 *            device if opts->out_on_device).  R(x,x) = 0.
 * The distinct endpoints are solved in blocks of 64 columns.  When every
 * solution block fits on the device at once (opts->pairs_resident_blocks),
 * K_uv = (G^-1)_uv comes from the bilinear estimate x_u[v] + x_v[u] -
 * x_u^T G x_v, whose error is second order in the solve error.  Otherwise
 * the blocks are solved in groups that fit and dropped after each group:
 * device memory is bounded by the group, K_uv within a group as above and
 * across groups the first-order estimate (x_u[v] + x_v[u]) / 2; the solves
 * then run to min(rel_tol, max(rel_tol^2, 1e-14)) so that the first-order
 * terms stay near the requested accuracy.
 * Errors as reff_solve_diag.
 */
reff_status reff_query_pairs(reff_pdn p, const int64_t* a, int64_t m,
                             const int64_t* b, int64_t n, reff_pair_mode mode,
                             double* R_out, const reff_solve_opts* opts,
                             reff_solve_stats* st);

/*
 * IR drop and through-bump currents of load scenarios (Sec. II-B, Eq. 4;
 * Sec. IV-B).  Bumps (pads) are ideal sources at the supply voltage, loads
 * are ideal current sources (Sec. III-B).  Scenario c draws
 * load_amps[c * n_loads + k] amperes at node load_nodes[k].  By Eq. 4 with
 * every bump merged into the supply node, the drop below the supply at node
 * j is sum_k I_k (R_j + R_{l_k} - R(j, l_k)) / 2 = sum_k I_k (G^-1 e_{l_k})_j:
 * each distinct free load node is solved once with a unit current (block
 * PCG, 64 loads per block) and the responses are superposed on the device,
 * a bounded group of solved blocks at a time.
 *   load_nodes  host int64[n_loads]; duplicates add; a load on a pad draws
 *               straight from that pad (no drop).
 *   load_amps   host double[n_scen][n_loads].
 *   nodes       host int64[n_nodes] node ids to report, NULL = all nodes.
 *   drop_out    double[n_scen][n_nodes] (host, or device if
 *               opts->out_on_device): supply voltage minus node voltage, in
 *               volts per ampere of load current; 0 on pads.
 *   pad_amps_out  host double[n_scen][n_pads] (nullable): the current each
 *               pad entry of the descriptor delivers; a position listed twice
 *               reports its current at its first entry and 0 at the others.
 *               The pad currents of a scenario sum to its total load current.
 *   opts        rel_tol applies to the unit-load responses' R values; point
 *               values are accurate to about its square root, so the default
 *               (rel_tol 0) is 1e-12 in float64 and 1e-7 in mixed precision.
 * Errors: INVALID_ARG (ids out of range, negative counts, non-finite
 * currents, NULL pointers), NO_CONVERGENCE, OUT_OF_MEMORY, DEVICE.
 */
reff_status reff_ir_drop(reff_pdn p, const int64_t* load_nodes, int64_t n_loads,
                         const double* load_amps, int32_t n_scen, const int64_t* nodes,
                         int64_t n_nodes, double* drop_out, double* pad_amps_out,
                         const reff_solve_opts* opts, reff_solve_stats* st);

typedef struct {
  reff_solve_opts solve;   /* precision, tolerance, stream, out_on_device   */
  const void* surrogate;   /* NULL: solve every node.  A reff_surrogate
                              (reff_surrogate.h) whose geometry every plan
                              matches: screen the batch with it            */
  double spot_frac;        /* screened: fraction of each plan's requested
                              free nodes checked by the solver (seeded
                              choice, at least one); 0 => 0.01             */
  double fallback_rel_err; /* screened: a plan whose checked relative error
                              exceeds this is solved in full; 0 => 1e-2    */
  const char* tune_db;     /* NULL, or a tuning database file (created if
                              absent): per size class of a launch group
                              (precision, variant, rows, blocks) the work
                              units per launch of the row-range kernels and
                              the strips per launch of the stencil passes
                              (which sets the strip height, i.e. the tile
                              shape); a class not yet in it is timed on 12
                              candidate pairs first and added             */
  int32_t calibrate;       /* screened: 0 = every checked node checks the
                              prediction; 1 = the checked nodes at even
                              positions of the seeded order fit one log
                              offset per tier (mean of log(solved /
                              predicted)), every prediction of the plan is
                              scaled by it, and the odd positions check it */
} reff_batch_opts;

/*
 * Many candidate TSV plans in one call (design-option exploration, Sec. I
 * and Sec. IV-B).  plans[i] is validated and solved like reff_build_pdn +
 * reff_solve_diag; nodes[i] (host, NULL => all) and n_nodes[i] select the
 * nodes of plan i and R_out[i] receives them.  per_plan (nullable) gets one
 * stats record per plan.  The solve blocks of all plans advance together in
 * the same kernel launches.  With opts->surrogate the batch is screened
 * (see reff_batch_opts); results of screened plans carry the model's error,
 * not the solver tolerance.
 */
reff_status reff_batch_plans(const reff_pdn_desc* plans, int32_t n_plans,
                             const int64_t* const* nodes, const int64_t* n_nodes,
                             double* const* R_out, const reff_batch_opts* opts,
                             reff_solve_stats* per_plan);

/*
 * Two-point resistances of every pair of P points on one uniform M x N
 * resistor grid by the closed form of Eq. 3 (Sec. II-B): x in [0, M) along
 * the edges of resistance r, y in [0, N) along those of resistance s.  It is
 * the intra-die building block of the paper's divide-and-conquer pair method
 * for uniformly meshed tiers (Sec. III-C/D, TSV-TSV and bump/load-TSV
 * resistances of one die); each pair (i < j) is evaluated once and mirrored,
 * the double sum with cosines of multiple angles from the multiple-angle
 * recurrence (the GPU evaluation of Sec. III-D).
 *   xy       host int32[2 P]: point k at (xy[2k], xy[2k+1]).
 *   R_out    float64[P*P] row-major (host, or device if out_on_device);
 *            R(k,k) = 0, R(i,j) = R(j,i).
 *   stream   hipStream_t to run on; NULL => default stream.  The call
 *            returns after R_out is written.
 * The call allocates and frees its own device work memory: the weight table
 * ((M-1)(N-1) doubles), a cosine table (P (N-1) doubles), partial sums of
 * at most about 16.8M + P^2 doubles (134 MB + 8 P^2 bytes), and a P^2
 * staging array when R_out is a host pointer.
 * Errors: INVALID_ARG (M, N < 1, r or s not finite and positive, P < 0 or
 * P > 65535, a point off the grid, NULL pointers with P > 0),
 * OUT_OF_MEMORY, DEVICE.
 */
reff_status reff_grid_pairs(int32_t M, int32_t N, double r, double s, const int32_t* xy,
                            int64_t P, double* R_out, int32_t out_on_device, void* stream);

/*
 * Bump-to-load pair resistances of a stack of uniformly meshed tiers by the
 * paper's divide-and-conquer method (Sec. III-C and III-D): intra-die
 * resistances from Eq. 3 (TSV-TSV on every tier, bump-TSV on tier 0,
 * load-TSV on the last tier), the reduced system C x = b of size
 * (p+1)(d-1) over the TSV currents of the d-1 tier interfaces and the
 * supply-voltage differences, factorised once, m + n solves (one per bump
 * and per load, the linearity of Sec. III-D), and
 * R(i, j) = -(x^1_i + x^d_j)^T (b^1_i + b^d_j) with the m x n cross term as
 * one matrix product.  The network is the floating stack (Eq. 2 with no
 * other grounding), the same as reff_query_pairs in REFF_PAIRS_FLOATING mode
 * on the equivalent reff_pdn_desc (gx = 1 / r_t, gy = 1 / s_t, tsv_g =
 * 1 / tsv_r).
 *   n_tiers  d >= 2 uniform tiers of nx x ny nodes; tier 0 carries the
 *            bumps, tier d-1 the loads.
 *   r_t,s_t  host double[d]: edge resistance along x and along y on tier t.
 *   tsv_xy   host int32[2 p]: TSV columns (distinct), p >= 1.
 *   tsv_r    host double[p][d-1]: segment resistance of TSV k between
 *            tiers t and t+1.
 *   bump_xy  host int32[2 m] on tier 0; load_xy host int32[2 n] on tier d-1.
 *   R_out    double[m*n] row-major (host, or device if out_on_device):
 *            R(bump i, load j).
 *   stream   hipStream_t to run on; NULL => default stream.  The call
 *            returns after R_out is written.
 * The call allocates and frees its own device work memory (about
 * 8 ((p-1)(d-1))^2 x 2 bytes for the reduced matrix and its factor, plus
 * the intra-die tables).  Errors: INVALID_ARG (d < 2, p < 1, counts < 0,
 * non-positive or non-finite resistances, a point off the grid, duplicate
 * TSV columns, more than 65535 TSVs + bumps or TSVs + loads, NULL
 * pointers), OUT_OF_MEMORY, DEVICE (also when the reduced matrix is not
 * positive definite on the constrained currents, which a connected stack
 * does not produce).
 */
reff_status reff_reduced_pairs(int32_t n_tiers, int32_t nx, int32_t ny, const double* r_t,
                               const double* s_t, int32_t p, const int32_t* tsv_xy,
                               const double* tsv_r, int64_t m, const int32_t* bump_xy, int64_t n,
                               const int32_t* load_xy, double* R_out, int32_t out_on_device,
                               void* stream);

/*
 * reff_grid_pairs without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * reff_grid_pairs, which it shares its kernels with; its work memory (points,
 * weights, cosine table, partial Gram blocks, and the staging of R_out when
 * it is a host pointer) lives in one 64 MiB array per GPU that the library
 * holds from the first call on that device until the process ends.  Inputs
 * whose work memory does not fit (one m segment of P^2 doubles plus 8 (M-1)
 * (N-1) + 8 P (N-1) + 8 P + (host output) 8 P^2 bytes, each part rounded up
 * to 256 bytes, above 64 MiB; for example P above about 2,800 points) are
 * rejected with REFF_ERR_INVALID_ARG before any device work.  When fewer m
 * segments fit than the allocating call uses, the partial sums are grouped
 * differently (results agree to rounding).  Calls on one GPU share the
 * array: calls that overlap in time on the same GPU (two host threads, or
 * two streams) race and must be serialised by the caller.  The call
 * returns after R_out is written; it makes no hipMalloc or hipFree call.
 */
reff_status reff_grid_pairs_noalloc(int32_t M, int32_t N, double r, double s, const int32_t* xy,
                                    int64_t P, double* R_out, int32_t out_on_device,
                                    void* stream);

/* Static description of a status code. */
const char* reff_status_string(reff_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char* reff_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REFF_H */
