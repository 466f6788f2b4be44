// Symbolic analysis for the sparse-direct full map diag(G^-1): nested
// dissection of the stacked grid and the multifrontal structure the device
// kernels of selinv.hip run over.  Plain C++ (no HIP types).
//
// Ordering.  Boxes of the (x, y) plane are bisected across their longer
// side; the separator is the whole line of columns through every tier (the
// TSVs are vertical, so a wall of columns cuts the stack in two), and a box
// with at most `leaf_area` columns is eliminated as one leaf.  Every tree
// node (a separator, or a leaf box) is a supernode whose pivots are its free
// nodes; supernodes are numbered in postorder, which is the elimination
// order.
//
// Fronts.  The update set Q of a supernode is the set of free nodes just
// outside its box (the lines x0-1, x1, y0-1, y1 within the box's extent, all
// tiers): these lie on ancestor separators, and the eliminated interior of
// the box couples them all, so the front of the supernode is dense over
// [pivots, Q] (Q in elimination order).  Q of a child lies inside its
// parent's index set, and `rel` maps it there (monotone, so the lower
// triangle maps to the lower triangle).  A front is one F x F column-major
// float64 block of the device arena; fronts of one tree depth are
// contiguous and are processed together.
#pragma once

#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace reff {

struct SnFront {
  int64_t off = 0;       // arena offset (doubles) of the F x F block
  int32_t F = 0, k = 0;  // front size, pivots
  int32_t parent = -1;   // front index of the parent, -1 at a root
  int32_t depth = 0;
  int32_t rank = 0;      // 0 / 1: which child of the parent
  int64_t rel = 0;       // offset into SelinvPlan::rel of its F - k entries
  int64_t piv = 0;       // offset into SelinvPlan::piv_node of its k node ids
  int32_t x0 = 0, x1 = 0, y0 = 0, y1 = 0;  // box
};

struct SelinvLevel {
  std::vector<int32_t> fronts;  // front indices at this depth
  int64_t arena_begin = 0, arena_end = 0;
  int32_t max_panels = 0;       // ceil(max k / 64)
  int64_t max_F = 0;
  // original entries of G assembled into this level's fronts:
  // arena index (lower triangle of the owning front) and value
  std::vector<int64_t> ent_idx;
  std::vector<double> ent_val;
};

struct SelinvPlan {
  int32_t nt = 0, nx = 0, ny = 0;
  int64_t n = 0, n_free = 0;
  std::vector<SnFront> fronts;     // postorder
  std::vector<SelinvLevel> levels; // by depth, 0 = roots
  std::vector<int32_t> rel;        // child Q -> parent front positions
  std::vector<int64_t> piv_node;   // pivots' node ids, front by front
  std::vector<int32_t> node_front; // front whose pivot a node is, -1 for pads
  int64_t arena = 0;               // doubles
  double flops_factor = 0.0, flops_selinv = 0.0;
};

// Several plans as one (a forest): fronts, maps and node ids offset plan by
// plan (plan i's node v becomes base[i] + v), levels merged by depth, the
// arena laid out again level by level.  base receives each plan's first
// node id.
SelinvPlan merge_selinv_plans(const std::vector<SelinvPlan>& plans, std::vector<int64_t>& base);

// The fronts a selected inversion must visit to produce R for the given
// node ids: each node's own front and all of that front's ancestors (the
// recurrence for a front reads only its parent's finished block).  Returns
// one flag per front (1 = needed) and their share of flops_selinv in
// *flops.  Node ids must lie in [0, n).
std::vector<uint8_t> needed_fronts(const SelinvPlan& P, const std::vector<int64_t>& ids,
                                   double* flops);

// Run body(i) for i < count on up to 16 host threads.
void selinv_parallel_for(size_t count, const std::function<void(size_t)>& body);

// Build the plan from the stack description (arrays as in reff_pdn_desc:
// gx [nt][ny][nx-1], gy [nt][ny-1][nx], tsv_xy [n_tsv][2], tsv_g
// [n_tsv][nt-1], pads on tier 0).  Returns false with `err` set on
// inconsistent input, or when some node has no resistive path to a pad
// (G singular; breadth-first search from the pads).
bool build_selinv_plan(int32_t nt, int32_t nx, int32_t ny, const double* gx, const double* gy,
                       int32_t n_tsv, const int32_t* tsv_xy, const double* tsv_g, int32_t n_pads,
                       const int32_t* pad_xy, int32_t leaf_area, SelinvPlan& plan,
                       std::string& err, bool* disconnected = nullptr);

}  // namespace reff
