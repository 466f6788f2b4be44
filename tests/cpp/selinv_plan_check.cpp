// Host check of the sparse-direct plan (selinv_plan.cpp): the symbolic
// structure (nested-dissection fronts, update sets, child-to-parent maps,
// original entries) driven through the same panel factorisation and block
// Takahashi recurrence the device kernels run, written as plain loops, and
// compared with a dense Gauss-Jordan inverse of G.  Every front access is
// bounds-checked.  Exit status 0 when every stack matches to 1e-10.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>
#include <cassert>

#include "../../paper_2607_05818_amd/csrc/selinv_plan.h"

using namespace reff;

static void chk(bool c, const char* m) {
  if (!c) {
    fprintf(stderr, "FAIL %s\n", m);
    exit(1);
  }
}

struct Stack {
  int nt, nx, ny, ntsv, npad;
  std::vector<double> gx, gy, tg;
  std::vector<int32_t> txy, pxy;
};

static Stack make_stack(int seed, int nt, int nx, int ny, int ntsv, int npad) {
  Stack S{nt, nx, ny, ntsv, npad, {}, {}, {}, {}, {}};
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.5, 2.0);
  S.gx.resize((size_t)nt * ny * std::max(nx - 1, 0));
  S.gy.resize((size_t)nt * std::max(ny - 1, 0) * nx);
  for (auto& v : S.gx) v = U(rng);
  for (auto& v : S.gy) v = U(rng);
  std::vector<char> used((size_t)nx * ny, 0);
  for (int j = 0; j < ntsv; ++j) {
    int x, y;
    do { x = rng() % nx; y = rng() % ny; } while (used[(size_t)y * nx + x]);
    used[(size_t)y * nx + x] = 1;
    S.txy.push_back(x); S.txy.push_back(y);
  }
  if (nt > 1 && ntsv == 0) { S.txy = {0, 0}; S.ntsv = 1; }
  S.tg.resize((size_t)S.ntsv * std::max(nt - 1, 0));
  for (auto& v : S.tg) v = U(rng) * 3;
  for (int j = 0; j < npad; ++j) { S.pxy.push_back(rng() % nx); S.pxy.push_back(rng() % ny); }
  return S;
}

static bool plan_of(const Stack& S, int leaf, SelinvPlan& P) {
  std::string err;
  if (!build_selinv_plan(S.nt, S.nx, S.ny, S.gx.data(), S.gy.data(), S.ntsv, S.txy.data(),
                         S.tg.data(), S.npad, S.pxy.data(), leaf, P, err)) {
    fprintf(stderr, "plan error %s\n", err.c_str());
    return false;
  }
  return true;
}

// diag(G^-1) by Gauss-Jordan on the dense grounded matrix; 0 on pads.
static std::vector<double> dense_diag(const Stack& S) {
  const int nt = S.nt, nx = S.nx, ny = S.ny;
  const int64_t plane = (int64_t)nx * ny, n = plane * nt;
  std::vector<char> pad((size_t)n, 0);
  for (int j = 0; j < S.npad; ++j) pad[(size_t)(S.pxy[2 * j + 1] * nx + S.pxy[2 * j])] = 1;
  std::vector<int64_t> fid((size_t)n, -1);
  int64_t nf = 0;
  for (int64_t v = 0; v < n; ++v) if (!pad[v]) fid[v] = nf++;
  std::vector<double> G((size_t)(nf * nf), 0.0);
  auto add = [&](int64_t a, int64_t b, double g) {
    if (fid[a] >= 0) G[fid[a] * nf + fid[a]] += g;
    if (fid[b] >= 0) G[fid[b] * nf + fid[b]] += g;
    if (fid[a] >= 0 && fid[b] >= 0) { G[fid[a] * nf + fid[b]] -= g; G[fid[b] * nf + fid[a]] -= g; }
  };
  for (int t = 0; t < nt; ++t)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t v = t * plane + (int64_t)y * nx + x;
        if (x + 1 < nx) add(v, v + 1, S.gx[(size_t)(t * ny + y) * (nx - 1) + x]);
        if (y + 1 < ny) add(v, v + nx, S.gy[(size_t)(t * (ny - 1) + y) * nx + x]);
      }
  for (int j = 0; j < S.ntsv; ++j)
    for (int t = 0; t + 1 < nt; ++t) {
      int64_t v = t * plane + (int64_t)S.txy[2 * j + 1] * nx + S.txy[2 * j];
      add(v, v + plane, S.tg[(size_t)j * (nt - 1) + t]);
    }
  std::vector<double> A = G, Inv((size_t)(nf * nf), 0.0);
  for (int64_t i = 0; i < nf; ++i) Inv[i * nf + i] = 1;
  for (int64_t c = 0; c < nf; ++c) {
    double p = A[c * nf + c];
    chk(p > 0, "dense pivot");
    for (int64_t j = 0; j < nf; ++j) { A[c * nf + j] /= p; Inv[c * nf + j] /= p; }
    for (int64_t r = 0; r < nf; ++r) if (r != c) {
      double f = A[r * nf + c];
      if (f == 0) continue;
      for (int64_t j = 0; j < nf; ++j) { A[r * nf + j] -= f * A[c * nf + j]; Inv[r * nf + j] -= f * Inv[c * nf + j]; }
    }
  }
  std::vector<double> R((size_t)n, 0.0);
  for (int64_t v = 0; v < n; ++v) if (fid[v] >= 0) R[v] = Inv[fid[v] * nf + fid[v]];
  return R;
}

// The panel factorisation and block Takahashi recurrence of the device
// kernels, as plain loops over a plan (any forest); R per node id.
// need: with a flag per front, the selected inversion visits only the
// flagged fronts (R stays 0 elsewhere).
static std::vector<double> numeric(const SelinvPlan& P,
                                   const std::vector<uint8_t>* need = nullptr) {
  std::vector<double> ar((size_t)P.arena, 0.0);
  auto at = [&](const SnFront& f, int64_t r, int64_t c) -> double& {
    chk(r >= 0 && r < f.F && c >= 0 && c < f.F, "front index");
    chk(f.off + c * f.F + r < P.arena, "arena index");
    return ar[(size_t)(f.off + c * f.F + r)];
  };
  for (int d = (int)P.levels.size() - 1; d >= 0; --d) {
    const SelinvLevel& L = P.levels[(size_t)d];
    for (size_t e = 0; e < L.ent_idx.size(); ++e) {
      chk(L.ent_idx[e] >= L.arena_begin && L.ent_idx[e] < L.arena_end, "entry range");
      ar[(size_t)L.ent_idx[e]] += L.ent_val[e];
    }
    if (d + 1 < (int)P.levels.size())
      for (int32_t ci : P.levels[(size_t)d + 1].fronts) {
        const SnFront& c = P.fronts[(size_t)ci];
        if (c.parent < 0) continue;
        const SnFront& p = P.fronts[(size_t)c.parent];
        chk(p.depth == d, "parent depth");
        const int32_t q = c.F - c.k;
        for (int b = 0; b < q; ++b)
          for (int a = b; a < q; ++a) {
            int ra = P.rel[(size_t)(c.rel + a)], rb = P.rel[(size_t)(c.rel + b)];
            chk(ra >= rb, "monotone");
            at(p, ra, rb) += at(c, c.k + a, c.k + b);
          }
      }
    for (int32_t fi : L.fronts) {
      const SnFront& f = P.fronts[(size_t)fi];
      for (int j0 = 0; j0 < f.k; j0 += 64) {
        int w = std::min(64, f.k - j0);
        for (int c = j0; c < j0 + w; ++c) {
          double piv = at(f, c, c);
          chk(piv > 0, "front pivot");
          double sq = std::sqrt(piv);
          at(f, c, c) = sq;
          for (int r = c + 1; r < j0 + w; ++r) at(f, r, c) /= sq;
          for (int cc = c + 1; cc < j0 + w; ++cc)
            for (int r = cc; r < j0 + w; ++r) at(f, r, cc) -= at(f, r, c) * at(f, cc, c);
        }
        for (int r = j0 + w; r < f.F; ++r)
          for (int c = j0; c < j0 + w; ++c) {
            double v = at(f, r, c);
            for (int t = j0; t < c; ++t) v -= at(f, r, t) * at(f, c, t);
            at(f, r, c) = v / at(f, c, c);
          }
        for (int c = j0 + w; c < f.F; ++c)
          for (int r = c; r < f.F; ++r) {
            double v = 0;
            for (int t = j0; t < j0 + w; ++t) v += at(f, r, t) * at(f, c, t);
            at(f, r, c) -= v;
          }
      }
    }
  }
  std::vector<double> R((size_t)P.n, 0.0);
  for (size_t d = 0; d < P.levels.size(); ++d) {
    for (int32_t fi : P.levels[d].fronts) {
      if (need && !(*need)[(size_t)fi]) continue;
      const SnFront& f = P.fronts[(size_t)fi];
      const int32_t q = f.F - f.k;
      if (f.parent >= 0) {
        const SnFront& p = P.fronts[(size_t)f.parent];
        for (int b = 0; b < q; ++b)
          for (int a = 0; a < q; ++a)
            at(f, f.k + a, f.k + b) = at(p, P.rel[(size_t)(f.rel + a)], P.rel[(size_t)(f.rel + b)]);
      } else chk(q == 0, "root with update set");
      for (int jp = (f.k + 63) / 64 - 1; jp >= 0; --jp) {
        int j0 = 64 * jp, w = std::min(64, f.k - j0), r0 = j0 + w, m = f.F - r0;
        std::vector<double> Li(64 * 64, 0.0), Z0(64 * 64, 0.0);
        for (int c = 0; c < w; ++c)
          for (int i = 0; i < w; ++i) {
            double v = (i == c);
            for (int t = c; t < i; ++t) v -= at(f, j0 + i, j0 + t) * Li[t * 64 + c];
            Li[i * 64 + c] = i < c ? 0 : v / at(f, j0 + i, j0 + i);
          }
        for (int a = 0; a < w; ++a)
          for (int bb = 0; bb < w; ++bb) {
            double v = 0;
            for (int c = std::max(a, bb); c < w; ++c) v += Li[c * 64 + a] * Li[c * 64 + bb];
            Z0[a * 64 + bb] = v;
          }
        std::vector<double> Lh((size_t)m * w), Y((size_t)m * w, 0.0);
        for (int r = 0; r < m; ++r)
          for (int c = 0; c < w; ++c) {
            double v = 0;
            for (int t = c; t < w; ++t) v += at(f, r0 + r, j0 + t) * Li[t * 64 + c];
            Lh[(size_t)r * w + c] = v;
          }
        for (int r = 0; r < m; ++r)
          for (int c = 0; c < w; ++c) {
            double v = 0;
            for (int t = 0; t < m; ++t) v -= at(f, r0 + r, r0 + t) * Lh[(size_t)t * w + c];
            Y[(size_t)r * w + c] = v;
          }
        for (int a = 0; a < w; ++a)
          for (int bb = 0; bb < w; ++bb) {
            double v = Z0[a * 64 + bb];
            for (int r = 0; r < m; ++r) v -= Lh[(size_t)r * w + a] * Y[(size_t)r * w + bb];
            at(f, j0 + a, j0 + bb) = v;
          }
        for (int r = 0; r < m; ++r)
          for (int c = 0; c < w; ++c) {
            at(f, r0 + r, j0 + c) = Y[(size_t)r * w + c];
            at(f, j0 + c, r0 + r) = Y[(size_t)r * w + c];
          }
        for (int a = 0; a < w; ++a) R[(size_t)P.piv_node[(size_t)(f.piv + j0 + a)]] = at(f, j0 + a, j0 + a);
      }
    }
  }
  return R;
}

static double worst_rel(const std::vector<double>& got, const double* want, int64_t n) {
  double worst = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (want[v] == 0) { chk(got[v] == 0, "pad zero"); continue; }
    worst = std::max(worst, std::fabs(got[v] - want[v]) / want[v]);
  }
  return worst;
}

// node_front: every pivot maps to its own front, nothing else maps.
static void check_node_front(const SelinvPlan& P) {
  chk((int64_t)P.node_front.size() == P.n, "node_front size");
  int64_t mapped = 0;
  for (int32_t f : P.node_front) mapped += f >= 0;
  chk(mapped == P.n_free, "node_front covers the free nodes");
  for (size_t i = 0; i < P.fronts.size(); ++i)
    for (int32_t a = 0; a < P.fronts[i].k; ++a)
      chk(P.node_front[(size_t)P.piv_node[(size_t)(P.fronts[i].piv + a)]] == (int32_t)i,
          "pivot maps to its front");
}

// A request of a few node ids: the flagged fronts are closed under
// parents, contain every requested free node, the partial recurrence
// gives the requested values bit for bit, and all ids flag every front
// that has pivots.
static int partial(const SelinvPlan& P, const std::vector<double>& full, int seed, int count) {
  std::mt19937_64 rng(seed);
  std::vector<int64_t> ids((size_t)count);
  for (auto& v : ids) v = (int64_t)(rng() % (uint64_t)P.n);
  double fl = -1;
  const std::vector<uint8_t> need = needed_fronts(P, ids, &fl);
  size_t nn = 0;
  for (size_t i = 0; i < P.fronts.size(); ++i) {
    if (!need[i]) continue;
    ++nn;
    if (P.fronts[i].parent >= 0) chk(need[(size_t)P.fronts[i].parent], "closed under parents");
  }
  for (int64_t v : ids)
    if (P.node_front[(size_t)v] >= 0) chk(need[(size_t)P.node_front[(size_t)v]], "own front");
  const std::vector<double> R = numeric(P, &need);
  for (int64_t v : ids) chk(R[(size_t)v] == full[(size_t)v], "partial value");
  std::vector<int64_t> all((size_t)P.n);
  for (int64_t v = 0; v < P.n; ++v) all[(size_t)v] = v;
  double fa = -1;
  const std::vector<uint8_t> every = needed_fronts(P, all, &fa);
  for (size_t i = 0; i < P.fronts.size(); ++i)  // fronts without pivots may go unflagged
    chk(every[i] == 1 || P.fronts[i].k == 0, "all ids need every front with pivots");
  chk(std::fabs(fa - P.flops_selinv) <= 1e-9 * P.flops_selinv + 1e-9, "flops of all fronts");
  chk(fl <= fa, "partial flops");
  printf("  partial request of %d ids: %zu of %zu fronts, %.1f%% of the inversion flops\n",
         count, nn, P.fronts.size(), fa > 0 ? 100.0 * fl / fa : 0.0);
  return 0;
}

int run(int seed, int nt, int nx, int ny, int ntsv, int npad, int leaf) {
  const Stack S = make_stack(seed, nt, nx, ny, ntsv, npad);
  SelinvPlan P;
  if (!plan_of(S, leaf, P)) return 1;
  const std::vector<double> want = dense_diag(S);
  check_node_front(P);
  const std::vector<double> R = numeric(P);
  const double worst = worst_rel(R, want.data(), P.n);
  printf("seed %d %dx%dx%d tsv %d pads %d leaf %d: fronts %zu levels %zu arena %lld worst %.3e\n",
         seed, nt, nx, ny, ntsv, npad, leaf, P.fronts.size(), P.levels.size(),
         (long long)P.arena, worst);
  partial(P, R, seed + 1000, 3);
  return worst < 1e-10 ? 0 : 1;
}

// Several stacks merged into one forest (the batched path): each plan's
// segment of the merged result against its own dense inverse.
int run_merged() {
  const Stack S[3] = {make_stack(21, 2, 17, 9, 6, 2), make_stack(22, 3, 6, 13, 4, 1),
                      make_stack(23, 1, 30, 20, 0, 3)};
  std::vector<SelinvPlan> plans(3);
  for (int i = 0; i < 3; ++i)
    if (!plan_of(S[i], 16, plans[i])) return 1;
  std::vector<int64_t> base;
  const SelinvPlan M = merge_selinv_plans(plans, base);
  check_node_front(M);
  const std::vector<double> R = numeric(M);
  partial(M, R, 99, 5);
  double worst = 0;
  for (int i = 0; i < 3; ++i) {
    const std::vector<double> want = dense_diag(S[i]);
    std::vector<double> seg(R.begin() + base[i], R.begin() + base[i] + plans[i].n);
    worst = std::max(worst, worst_rel(seg, want.data(), plans[i].n));
  }
  printf("merged forest of 3 stacks: fronts %zu levels %zu worst %.3e\n", M.fronts.size(),
         M.levels.size(), worst);
  return worst < 1e-10 ? 0 : 1;
}

int main() {
  int bad = 0;
  bad |= run(1, 1, 7, 5, 0, 1, 4);
  bad |= run(2, 3, 9, 11, 6, 3, 4);
  bad |= run(3, 2, 33, 3, 4, 2, 16);
  bad |= run(4, 4, 10, 10, 6, 3, 1);
  bad |= run(5, 1, 1, 1, 0, 1, 16);
  bad |= run(6, 2, 17, 19, 9, 5, 16);
  bad |= run(7, 5, 6, 4, 3, 1, 2);
  bad |= run(8, 2, 40, 30, 30, 6, 16);
  bad |= run(9, 3, 20, 20, 40, 1, 9);
  bad |= run(10, 1, 1, 30, 0, 2, 4);
  bad |= run(11, 3, 30, 1, 5, 1, 4);
  bad |= run(12, 2, 70, 20, 30, 4, 16);
  bad |= run(14, 8, 16, 14, 12, 2, 16);
  bad |= run_merged();
  printf(bad ? "FAILED\n" : "all ok\n");
  return bad;
}
