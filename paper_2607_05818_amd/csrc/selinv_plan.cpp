// Symbolic analysis of the sparse-direct full map (see selinv_plan.h).
#include "selinv_plan.h"

#include <algorithm>
#include <atomic>
#include <functional>
#include <thread>

namespace reff {

// Selected-inversion flops of one front: per 64-column panel of width w
// with m rows below it, Lhat (m w^2), Y = -Z_RR Lhat (2 m^2 w), the
// -Lhat^T Y product (2 m w^2), and the tile's L^-T L^-1 (w^3).
static double selinv_front_flops(const SnFront& f) {
  double fl = 0.0;
  for (int32_t j0 = 0; j0 < f.k; j0 += 64) {
    const double w = std::min(64, f.k - j0), m = f.F - j0 - w;
    fl += 2.0 * m * w * w + 2.0 * m * m * w + 2.0 * m * w * w + w * w * w;
  }
  return fl;
}

std::vector<uint8_t> needed_fronts(const SelinvPlan& P, const std::vector<int64_t>& ids,
                                   double* flops) {
  std::vector<uint8_t> need(P.fronts.size(), 0);
  for (int64_t v : ids)
    for (int32_t f = P.node_front[(size_t)v]; f >= 0 && !need[(size_t)f];
         f = P.fronts[(size_t)f].parent)
      need[(size_t)f] = 1;
  double fl = 0.0;
  for (size_t i = 0; i < P.fronts.size(); ++i)
    if (need[i]) fl += selinv_front_flops(P.fronts[i]);
  if (flops) *flops = fl;
  return need;
}

namespace {

struct Builder {
  int32_t nt, nx, ny;
  int64_t plane;
  const double *gx, *gy, *tsv_g;
  std::vector<int32_t> tsv_of;  // column -> TSV index, -1 if none
  std::vector<uint8_t> pad;     // tier-0 column is a pad
  int32_t leaf;
  SelinvPlan& P;
  std::vector<int64_t> ord;     // elimination position of a node, -1 = pad
  std::vector<std::vector<int32_t>> kids;
  int64_t next_ord = 0;

  bool is_free(int64_t v) const { return !(v < plane && pad[(size_t)v]); }

  void add_pivot(int64_t v) {
    if (!is_free(v)) return;
    ord[(size_t)v] = next_ord++;
    P.piv_node.push_back(v);
  }

  // Build the subtree of the box; returns its front index, -1 if empty.
  int32_t rec(int32_t x0, int32_t x1, int32_t y0, int32_t y1, int32_t depth) {
    const int32_t w = x1 - x0, h = y1 - y0;
    if (w <= 0 || h <= 0) return -1;
    std::vector<int32_t> ch;
    SnFront f;
    f.x0 = x0, f.x1 = x1, f.y0 = y0, f.y1 = y1, f.depth = depth;
    if ((int64_t)w * h <= leaf) {
      f.piv = (int64_t)P.piv_node.size();
      for (int32_t t = 0; t < nt; ++t)
        for (int32_t y = y0; y < y1; ++y)
          for (int32_t x = x0; x < x1; ++x) add_pivot(t * plane + (int64_t)y * nx + x);
    } else if (w >= h) {
      const int32_t m = x0 + w / 2;
      for (int32_t c : {rec(x0, m, y0, y1, depth + 1), rec(m + 1, x1, y0, y1, depth + 1)})
        if (c >= 0) ch.push_back(c);
      f.piv = (int64_t)P.piv_node.size();
      for (int32_t t = 0; t < nt; ++t)
        for (int32_t y = y0; y < y1; ++y) add_pivot(t * plane + (int64_t)y * nx + m);
    } else {
      const int32_t m = y0 + h / 2;
      for (int32_t c : {rec(x0, x1, y0, m, depth + 1), rec(x0, x1, m + 1, y1, depth + 1)})
        if (c >= 0) ch.push_back(c);
      f.piv = (int64_t)P.piv_node.size();
      for (int32_t t = 0; t < nt; ++t)
        for (int32_t x = x0; x < x1; ++x) add_pivot(t * plane + (int64_t)m * nx + x);
    }
    f.k = (int32_t)((int64_t)P.piv_node.size() - f.piv);
    const int32_t id = (int32_t)P.fronts.size();
    for (size_t r = 0; r < ch.size(); ++r) {
      P.fronts[(size_t)ch[r]].parent = id;
      P.fronts[(size_t)ch[r]].rank = (int32_t)r;
    }
    P.fronts.push_back(f);
    kids.push_back(ch);
    return id;
  }

  // Free nodes just outside the box, all tiers, in elimination order.  Each
  // side of the box lies on one ancestor separator, whose pivots run tier by
  // tier along the line, so a side taken tier by tier is one increasing run
  // of that separator's order; the runs of different sides do not
  // interleave, so ordering them by their first node orders the set.
  void boundary(const SnFront& f, std::vector<int64_t>& q) const {
    q.clear();
    int64_t run[4][2];  // [first ord, start in q] per side
    int nrun = 0;
    std::vector<int64_t> tmp;
    auto side = [&](int64_t x0, int64_t dx, int64_t y0, int64_t dy, int32_t len) {
      const size_t start = q.size();
      for (int32_t t = 0; t < nt; ++t)
        for (int32_t i = 0; i < len; ++i) {
          const int64_t v = t * plane + (y0 + dy * i) * nx + x0 + dx * i;
          if (is_free(v)) q.push_back(v);
        }
      if (q.size() > start) {
        run[nrun][0] = ord[(size_t)q[start]];
        run[nrun][1] = (int64_t)start;
        ++nrun;
      }
    };
    if (f.x0 > 0) side(f.x0 - 1, 0, f.y0, 1, f.y1 - f.y0);
    if (f.x1 < nx) side(f.x1, 0, f.y0, 1, f.y1 - f.y0);
    if (f.y0 > 0) side(f.x0, 1, f.y0 - 1, 0, f.x1 - f.x0);
    if (f.y1 < ny) side(f.x0, 1, f.y1, 0, f.x1 - f.x0);
    if (nrun <= 1) return;
    int idx[4] = {0, 1, 2, 3};
    std::sort(idx, idx + nrun, [&](int a, int b) { return run[a][0] < run[b][0]; });
    tmp.reserve(q.size());
    for (int r = 0; r < nrun; ++r) {
      const int k = idx[r];
      int64_t end = (int64_t)q.size();
      for (int j = 0; j < nrun; ++j)
        if (run[j][1] > run[k][1]) end = std::min(end, run[j][1]);
      tmp.insert(tmp.end(), q.begin() + run[k][1], q.begin() + end);
    }
    q.swap(tmp);
  }

  // Conductances of the edges at node v: calls fn(u, g) for every neighbour
  // u (pads included) and returns the sum.
  template <typename Fn>
  double edges(int64_t v, Fn fn) const {
    const int32_t vi = (int32_t)v, pl = (int32_t)plane;
    const int32_t t = vi / pl, rem = vi - t * pl, y = rem / nx, x = rem - y * nx;
    double s = 0.0;
    auto e = [&](int64_t u, double g) {
      s += g;
      fn(u, g);
    };
    const double* gxt = gx + (int64_t)t * ny * (nx - 1);
    const double* gyt = gy + (int64_t)t * (ny - 1) * nx;
    if (x > 0) e(v - 1, gxt[(int64_t)y * (nx - 1) + x - 1]);
    if (x + 1 < nx) e(v + 1, gxt[(int64_t)y * (nx - 1) + x]);
    if (y > 0) e(v - nx, gyt[(int64_t)(y - 1) * nx + x]);
    if (y + 1 < ny) e(v + nx, gyt[(int64_t)y * nx + x]);
    const int32_t j = tsv_of[(size_t)rem];
    if (j >= 0) {
      if (t > 0) e(v - plane, tsv_g[(int64_t)j * (nt - 1) + t - 1]);
      if (t + 1 < nt) e(v + plane, tsv_g[(int64_t)j * (nt - 1) + t]);
    }
    return s;
  }
};

}  // namespace

bool build_selinv_plan(int32_t nt, int32_t nx, int32_t ny, const double* gx, const double* gy,
                       int32_t n_tsv, const int32_t* tsv_xy, const double* tsv_g, int32_t n_pads,
                       const int32_t* pad_xy, int32_t leaf_area, SelinvPlan& plan,
                       std::string& err, bool* disconnected) {
  plan = SelinvPlan();
  if (disconnected) *disconnected = false;
  plan.nt = nt, plan.nx = nx, plan.ny = ny;
  Builder b{nt, nx, ny, (int64_t)nx * ny, gx, gy, tsv_g, {}, {}, std::max(1, leaf_area), plan,
            {}, {}, 0};
  const int64_t n = b.plane * nt;
  plan.n = n;
  if (n >= ((int64_t)1 << 31)) {
    err = "more than 2^31 - 1 nodes";
    return false;
  }
  b.tsv_of.assign((size_t)b.plane, -1);
  for (int32_t j = 0; j < n_tsv; ++j)
    b.tsv_of[(size_t)((int64_t)tsv_xy[2 * j + 1] * nx + tsv_xy[2 * j])] = j;
  b.pad.assign((size_t)b.plane, 0);
  for (int32_t j = 0; j < n_pads; ++j) b.pad[(size_t)((int64_t)pad_xy[2 * j + 1] * nx + pad_xy[2 * j])] = 1;
  b.ord.assign((size_t)n, -1);
  b.rec(0, nx, 0, ny, 0);
  plan.n_free = b.next_ord;
  {
    // every free node must reach a pad (breadth-first search over the edges)
    std::vector<uint8_t> seen((size_t)n, 0);
    std::vector<int64_t> q;
    q.reserve((size_t)n);
    for (int64_t v = 0; v < b.plane; ++v)
      if (b.pad[(size_t)v]) {
        seen[(size_t)v] = 1;
        q.push_back(v);
      }
    for (size_t h = 0; h < q.size(); ++h)
      b.edges(q[h], [&](int64_t u, double) {
        if (!seen[(size_t)u]) {
          seen[(size_t)u] = 1;
          q.push_back(u);
        }
      });
    if ((int64_t)q.size() != n) {
      err = std::to_string(n - (int64_t)q.size()) + " node(s) have no resistive path to a pad";
      if (disconnected) *disconnected = true;
      return false;
    }
  }

  plan.node_front.assign((size_t)n, -1);
  for (size_t i = 0; i < plan.fronts.size(); ++i)
    for (int32_t a = 0; a < plan.fronts[i].k; ++a)
      plan.node_front[(size_t)plan.piv_node[(size_t)(plan.fronts[i].piv + a)]] = (int32_t)i;
  // update sets, sizes, levels
  std::vector<std::vector<int64_t>> Q(plan.fronts.size());
  int32_t max_depth = 0;
  for (size_t i = 0; i < plan.fronts.size(); ++i) {
    b.boundary(plan.fronts[i], Q[i]);
    SnFront& f = plan.fronts[i];
    const int64_t F = (int64_t)f.k + (int64_t)Q[i].size();
    if (F > (int64_t)1 << 30) {
      err = "front too large";
      return false;
    }
    f.F = (int32_t)F;
    max_depth = std::max(max_depth, f.depth);
  }
  plan.levels.assign((size_t)max_depth + 1, SelinvLevel());
  for (size_t i = 0; i < plan.fronts.size(); ++i)
    plan.levels[(size_t)plan.fronts[i].depth].fronts.push_back((int32_t)i);
  int64_t off = 0;
  for (SelinvLevel& L : plan.levels) {
    L.arena_begin = off;
    for (int32_t i : L.fronts) {
      SnFront& f = plan.fronts[(size_t)i];
      f.off = off;
      off += (int64_t)f.F * f.F;
      L.max_panels = std::max<int32_t>(L.max_panels, (f.k + 63) / 64);
      L.max_F = std::max<int64_t>(L.max_F, f.F);
      const double k = f.k, q = f.F - f.k;
      plan.flops_factor += k * k * k / 3.0 + k * k * q + k * q * q;
      plan.flops_selinv += selinv_front_flops(f);
    }
    L.arena_end = off;
  }
  plan.arena = off;

  // positions inside a front's index set; child maps and original entries
  std::vector<int32_t> pos((size_t)n, -1);
  {
    std::vector<int64_t> piv_per_level(plan.levels.size(), 0);
    for (const SnFront& f : plan.fronts) piv_per_level[(size_t)f.depth] += f.k;
    for (size_t d = 0; d < plan.levels.size(); ++d) {
      plan.levels[d].ent_idx.reserve((size_t)(piv_per_level[d] * 4));
      plan.levels[d].ent_val.reserve((size_t)(piv_per_level[d] * 4));
    }
    int64_t nrel = 0;
    for (const SnFront& f : plan.fronts)
      if (f.parent >= 0) nrel += f.F - f.k;
    plan.rel.reserve((size_t)nrel);
  }
  for (size_t s = 0; s < plan.fronts.size(); ++s) {
    const SnFront& f = plan.fronts[s];
    for (int32_t a = 0; a < f.k; ++a) pos[(size_t)plan.piv_node[(size_t)(f.piv + a)]] = a;
    for (size_t a = 0; a < Q[s].size(); ++a) pos[(size_t)Q[s][a]] = f.k + (int32_t)a;
    for (int32_t c : b.kids[s]) {
      SnFront& cf = plan.fronts[(size_t)c];
      cf.rel = (int64_t)plan.rel.size();
      int32_t prev = -1;
      for (int64_t u : Q[(size_t)c]) {
        const int32_t p = pos[(size_t)u];
        if (p < 0 || p <= prev) {
          err = "update set of a child outside its parent's front";
          return false;
        }
        prev = p;
        plan.rel.push_back(p);
      }
    }
    SelinvLevel& L = plan.levels[(size_t)f.depth];
    for (int32_t a = 0; a < f.k; ++a) {
      const int64_t v = plan.piv_node[(size_t)(f.piv + a)];
      bool bad = false;
      const double dv = b.edges(v, [&](int64_t u, double g) {
        if (!b.is_free(u) || b.ord[(size_t)u] < b.ord[(size_t)v]) return;
        const int32_t p = pos[(size_t)u];
        if (p < 0) {
          bad = true;
          return;
        }
        L.ent_idx.push_back(f.off + (int64_t)a * f.F + p);
        L.ent_val.push_back(-g);
      });
      if (bad) {
        err = "neighbour outside the front of its pivot";
        return false;
      }
      L.ent_idx.push_back(f.off + (int64_t)a * f.F + a);
      L.ent_val.push_back(dv);
    }
    for (int32_t a = 0; a < f.k; ++a) pos[(size_t)plan.piv_node[(size_t)(f.piv + a)]] = -1;
    for (int64_t u : Q[s]) pos[(size_t)u] = -1;
  }
  return true;
}

SelinvPlan merge_selinv_plans(const std::vector<SelinvPlan>& plans, std::vector<int64_t>& base) {
  SelinvPlan M;
  const size_t np = plans.size();
  base.assign(np, 0);
  size_t nlev = 0;
  for (const SelinvPlan& P : plans) nlev = std::max(nlev, P.levels.size());
  M.levels.assign(nlev, SelinvLevel());
  // offsets of every plan's fronts, maps, pivots and node ids
  std::vector<int32_t> f0(np);
  std::vector<int64_t> r0(np), p0(np);
  int64_t nf = 0, nr = 0, npv = 0;
  for (size_t i = 0; i < np; ++i) {
    base[i] = M.n;
    f0[i] = (int32_t)nf;
    r0[i] = nr;
    p0[i] = npv;
    nf += (int64_t)plans[i].fronts.size();
    nr += (int64_t)plans[i].rel.size();
    npv += (int64_t)plans[i].piv_node.size();
    M.n += plans[i].n;
    M.n_free += plans[i].n_free;
    M.flops_factor += plans[i].flops_factor;
    M.flops_selinv += plans[i].flops_selinv;
  }
  // per level, plan-major: where each plan's fronts, entries and arena start
  std::vector<std::vector<int64_t>> lf(nlev, std::vector<int64_t>(np + 1, 0)),
      le(nlev, std::vector<int64_t>(np + 1, 0)), la(nlev, std::vector<int64_t>(np + 1, 0));
  int64_t off = 0;
  for (size_t d = 0; d < nlev; ++d) {
    SelinvLevel& L = M.levels[d];
    L.arena_begin = off;
    la[d][0] = off;
    for (size_t i = 0; i < np; ++i) {
      int64_t cf = 0, ce = 0, ca = 0;
      if (d < plans[i].levels.size()) {
        const SelinvLevel& PL = plans[i].levels[d];
        cf = (int64_t)PL.fronts.size();
        ce = (int64_t)PL.ent_idx.size();
        ca = PL.arena_end - PL.arena_begin;
        L.max_panels = std::max(L.max_panels, PL.max_panels);
        L.max_F = std::max(L.max_F, PL.max_F);
      }
      lf[d][i + 1] = lf[d][i] + cf;
      le[d][i + 1] = le[d][i] + ce;
      la[d][i + 1] = la[d][i] + ca;
    }
    off = la[d][np];
    L.arena_end = off;
    L.fronts.resize((size_t)lf[d][np]);
    L.ent_idx.resize((size_t)le[d][np]);
    L.ent_val.resize((size_t)le[d][np]);
  }
  M.arena = off;
  M.fronts.resize((size_t)nf);
  M.rel.resize((size_t)nr);
  M.piv_node.resize((size_t)npv);
  M.node_front.resize((size_t)M.n);
  // every plan fills its own slices
  selinv_parallel_for(np, [&](size_t i) {
    const SelinvPlan& P = plans[i];
    for (size_t j = 0; j < P.fronts.size(); ++j) {
      SnFront f = P.fronts[j];
      if (f.parent >= 0) f.parent += f0[i];
      f.rel += r0[i];
      f.piv += p0[i];
      M.fronts[(size_t)f0[i] + j] = f;
    }
    std::copy(P.rel.begin(), P.rel.end(), M.rel.begin() + r0[i]);
    for (size_t j = 0; j < P.piv_node.size(); ++j)
      M.piv_node[(size_t)p0[i] + j] = P.piv_node[j] + base[i];
    for (size_t v = 0; v < P.node_front.size(); ++v)
      M.node_front[(size_t)base[i] + v] = P.node_front[v] < 0 ? -1 : P.node_front[v] + f0[i];
    for (size_t d = 0; d < P.levels.size(); ++d) {
      const SelinvLevel& PL = P.levels[d];
      SelinvLevel& L = M.levels[d];
      // the level's arena moves from PL.arena_begin to la[d][i]; fronts keep
      // their order, so every front and entry shifts by the same amount
      const int64_t shift = la[d][i] - PL.arena_begin;
      for (size_t j = 0; j < PL.fronts.size(); ++j) {
        const int32_t fi = f0[i] + PL.fronts[j];
        L.fronts[(size_t)lf[d][i] + j] = fi;
        M.fronts[(size_t)fi].off = P.fronts[(size_t)PL.fronts[j]].off + shift;
      }
      const size_t e0 = (size_t)le[d][i];
      for (size_t e = 0; e < PL.ent_idx.size(); ++e) {
        L.ent_idx[e0 + e] = PL.ent_idx[e] + shift;
        L.ent_val[e0 + e] = PL.ent_val[e];
      }
    }
  });
  return M;
}

void selinv_parallel_for(size_t count, const std::function<void(size_t)>& body) {
  const size_t hw = std::max<unsigned>(1, std::thread::hardware_concurrency());
  const size_t nthr = std::min<size_t>({hw, (size_t)16, count});
  if (nthr <= 1) {
    for (size_t i = 0; i < count; ++i) body(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> pool;
  for (size_t t = 0; t < nthr; ++t)
    pool.emplace_back([&]() {
      for (size_t i = next++; i < count; i = next++) body(i);
    });
  for (auto& th : pool) th.join();
}

}  // namespace reff
