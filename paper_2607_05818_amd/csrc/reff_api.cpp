// Host runtime behind the C ABI of include/reff.h: argument validation,
// connectivity check, stencil-coefficient build and upload, workspace
// management, and the block-PCG driver that sequences the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <new>
#include <thread>
#include <numeric>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "reff_internal.h"
#include "surrogate_internal.h"

using namespace reff;

namespace {

thread_local std::string g_err;

reff_status fail(reff_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)            \
        return fail(REFF_ERR_OUT_OF_MEMORY, std::string(#call) + ": " +           \
                                                hipGetErrorString(e_));           \
      return fail(REFF_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                             \
  } while (0)

bool finite_pos(double g) { return std::isfinite(g) && g > 0.0; }

// Validation of a stack description (everything the ABI promises to check
// before any device work).
reff_status validate_desc(const reff_pdn_desc* d) {
  if (!d) return fail(REFF_ERR_INVALID_ARG, "descriptor is NULL");
  if (d->n_tiers < 1 || d->nx < 1 || d->ny < 1)
    return fail(REFF_ERR_INVALID_ARG, "n_tiers, nx and ny must be >= 1");
  const int64_t nt = d->n_tiers, nx = d->nx, ny = d->ny;
  const int64_t n = nt * nx * ny;
  if (n > (int64_t(1) << 40)) return fail(REFF_ERR_INVALID_ARG, "stack too large");
  const int64_t ngx = nt * ny * (nx - 1), ngy = nt * (ny - 1) * nx;
  if (ngx > 0 && !d->gx) return fail(REFF_ERR_INVALID_ARG, "gx is NULL");
  if (ngy > 0 && !d->gy) return fail(REFF_ERR_INVALID_ARG, "gy is NULL");
  for (int64_t i = 0; i < ngx; ++i)
    if (!finite_pos(d->gx[i]))
      return fail(REFF_ERR_INVALID_ARG, "gx[" + std::to_string(i) + "] not finite and > 0");
  for (int64_t i = 0; i < ngy; ++i)
    if (!finite_pos(d->gy[i]))
      return fail(REFF_ERR_INVALID_ARG, "gy[" + std::to_string(i) + "] not finite and > 0");
  if (d->n_tsv < 0) return fail(REFF_ERR_INVALID_ARG, "n_tsv < 0");
  if (d->n_tsv > 0) {
    if (!d->tsv_xy) return fail(REFF_ERR_INVALID_ARG, "tsv_xy is NULL");
    if (nt > 1 && !d->tsv_g) return fail(REFF_ERR_INVALID_ARG, "tsv_g is NULL");
    std::vector<uint8_t> seen((size_t)(nx * ny), 0);
    for (int32_t j = 0; j < d->n_tsv; ++j) {
      const int32_t x = d->tsv_xy[2 * j], y = d->tsv_xy[2 * j + 1];
      if (x < 0 || x >= nx || y < 0 || y >= ny)
        return fail(REFF_ERR_INVALID_ARG, "tsv " + std::to_string(j) + " out of range");
      if (seen[(size_t)(y * nx + x)])
        return fail(REFF_ERR_INVALID_ARG, "duplicate TSV column " + std::to_string(j));
      seen[(size_t)(y * nx + x)] = 1;
      for (int64_t t = 0; t + 1 < nt; ++t)
        if (!finite_pos(d->tsv_g[j * (nt - 1) + t]))
          return fail(REFF_ERR_INVALID_ARG, "tsv_g of TSV " + std::to_string(j) +
                                                " not finite and > 0");
    }
  }
  if (d->n_pads < 1) return fail(REFF_ERR_INVALID_ARG, "n_pads must be >= 1");
  if (!d->pad_xy) return fail(REFF_ERR_INVALID_ARG, "pad_xy is NULL");
  for (int32_t j = 0; j < d->n_pads; ++j) {
    const int32_t x = d->pad_xy[2 * j], y = d->pad_xy[2 * j + 1];
    if (x < 0 || x >= nx || y < 0 || y >= ny)
      return fail(REFF_ERR_INVALID_ARG, "pad " + std::to_string(j) + " out of range");
  }
  return REFF_OK;
}

}  // namespace

namespace reff {
reff_status host_fail(reff_status s, const std::string& msg) { return fail(s, msg); }
reff_status host_validate_desc(const reff_pdn_desc* d) { return validate_desc(d); }
// D^-1 and the float32 coefficient copies from the float64 arrays
// (coef_prep.hip)
hipError_t launch_coef_derived(const double* d, const double* cE, const double* cN, int64_t n,
                               double* dinv64, float* d32, float* dinv32, float* cE32,
                               float* cN32, hipStream_t st);
}  // namespace reff

namespace {

// Host-side stencil coefficients in float64 (see Coef in reff_internal.h).
struct HostCoef {
  std::vector<double> d, cE, cN, up, dn;
  std::vector<int32_t> slot;
  std::vector<uint8_t> is_pad;
};

// Destination of one stack's coefficients inside (possibly concatenated)
// arrays: node v of the stack is entry off + v, its TSV slots are entries
// soff .. soff + n_tsv * n_tiers - 1 (global slot ids), and tnode maps a
// global slot back to its global node entry.
struct CoefOut {
  double *d, *cE, *cN, *up, *dn;
  int32_t* slot;
  uint8_t* is_pad;
  int64_t* tnode;  // may be null
  int64_t off, soff;
};

// Coefficients of G = L[F, F] for the grounded (Dirichlet) node set `gnd`
// and a breadth-first connectivity check from those nodes.  Thread-safe:
// touches only its own entries of `o`; on failure `msg` says why.
reff_status build_into(const reff_pdn_desc* ds, const std::vector<int64_t>& gnd, const CoefOut& o,
                       std::string& msg) {
  const int64_t nt = ds->n_tiers, nx = ds->nx, ny = ds->ny;
  const int64_t plane = nx * ny, n = nt * plane;
  double* d = o.d + o.off;
  double* cE = o.cE + o.off;
  double* cN = o.cN + o.off;
  int32_t* slot = o.slot + o.off;
  uint8_t* is_pad = o.is_pad + o.off;
  std::fill(d, d + n, 0.0);
  std::fill(cE, cE + n, 0.0);
  std::fill(cN, cN + n, 0.0);
  std::fill(slot, slot + n, -1);
  std::fill(is_pad, is_pad + n, (uint8_t)0);
  for (int64_t v : gnd) is_pad[v] = 1;
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t y = 0; y < ny; ++y) {
      const double* gx = ds->gx + (t * ny + y) * (nx - 1);
      const double* gy = y + 1 < ny ? ds->gy + (t * (ny - 1) + y) * nx : nullptr;
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t v = t * plane + y * nx + x;
        const bool fv = !is_pad[v];
        if (x + 1 < nx) {
          const double g = gx[x];
          const bool fu = !is_pad[v + 1];
          if (fv) d[v] += g;
          if (fu) d[v + 1] += g;
          if (fu && fv) cE[v] = g;
        }
        if (gy) {
          const double g = gy[x];
          const bool fu = !is_pad[v + nx];
          if (fv) d[v] += g;
          if (fu) d[v + nx] += g;
          if (fu && fv) cN[v] = g;
        }
      }
    }
  // TSV side list: one slot per (column, tier) node.
  int64_t k = 0;
  for (int32_t j = 0; j < ds->n_tsv; ++j) {
    const int64_t x = ds->tsv_xy[2 * j], y = ds->tsv_xy[2 * j + 1];
    for (int64_t t = 0; t < nt; ++t, ++k) {
      const int64_t v = t * plane + y * nx + x;
      double gu = 0.0, gd = 0.0;
      if (t + 1 < nt) {
        const double g = ds->tsv_g[j * (nt - 1) + t];
        const bool fu = !is_pad[v], fv = !is_pad[v + plane];
        if (fu) d[v] += g;
        if (fu && fv) gu = g;
      }
      if (t > 0) {
        const double g = ds->tsv_g[j * (nt - 1) + t - 1];
        const bool fu = !is_pad[v], fv = !is_pad[v - plane];
        if (fu) d[v] += g;
        if (fu && fv) gd = g;
      }
      slot[v] = (int32_t)(o.soff + k);
      o.up[o.soff + k] = gu;
      o.dn[o.soff + k] = gd;
      if (o.tnode) o.tnode[o.soff + k] = o.off + v;
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (is_pad[v]) d[v] = 1.0;
  // Connectivity: breadth-first search from the pads over all resistors
  // (the queue is a plain array: every node enters it at most once).
  std::vector<uint8_t> seen((size_t)n, 0);
  std::vector<uint8_t> has_tsv((size_t)plane, 0);
  for (int32_t j = 0; j < ds->n_tsv; ++j)
    has_tsv[(size_t)(ds->tsv_xy[2 * j + 1] * nx + ds->tsv_xy[2 * j])] = 1;
  std::vector<int64_t> q;
  q.reserve((size_t)n);
  for (int64_t v : gnd)
    if (!seen[(size_t)v]) {
      seen[(size_t)v] = 1;
      q.push_back(v);
    }
  for (size_t h = 0; h < q.size(); ++h) {
    const int64_t v = q[h];
    const int64_t t = v / plane, rem = v % plane, y = rem / nx, x = rem % nx;
    int64_t nb[6];
    int c = 0;
    if (x > 0) nb[c++] = v - 1;
    if (x + 1 < nx) nb[c++] = v + 1;
    if (y > 0) nb[c++] = v - nx;
    if (y + 1 < ny) nb[c++] = v + nx;
    if (has_tsv[(size_t)rem]) {
      if (t > 0) nb[c++] = v - plane;
      if (t + 1 < nt) nb[c++] = v + plane;
    }
    for (int i = 0; i < c; ++i)
      if (!seen[(size_t)nb[i]]) {
        seen[(size_t)nb[i]] = 1;
        q.push_back(nb[i]);
      }
  }
  if ((int64_t)q.size() != n) {
    msg = std::to_string(n - (int64_t)q.size()) + " node(s) have no resistive path to a pad";
    return REFF_ERR_DISCONNECTED;
  }
  return REFF_OK;
}

reff_status build_host(const reff_pdn_desc* ds, const std::vector<int64_t>& gnd, HostCoef& h) {
  const int64_t n = (int64_t)ds->n_tiers * ds->nx * ds->ny;
  const int64_t ns = (int64_t)ds->n_tsv * ds->n_tiers;
  h.d.resize((size_t)n);
  h.cE.resize((size_t)n);
  h.cN.resize((size_t)n);
  h.slot.resize((size_t)n);
  h.is_pad.resize((size_t)n);
  h.up.resize((size_t)ns);
  h.dn.resize((size_t)ns);
  const CoefOut o{h.d.data(), h.cE.data(), h.cN.data(), h.up.data(), h.dn.data(),
                  h.slot.data(), h.is_pad.data(), nullptr, 0, 0};
  std::string msg;
  const reff_status s = build_into(ds, gnd, o, msg);
  return s == REFF_OK ? s : fail(s, msg);
}

// Run body(i) for i < count on up to 16 host threads (dynamic assignment).
template <typename F>
void parallel_for(size_t count, F body) {
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

// Apply body(lo, hi) to [0, n) in chunks spread over parallel_for.
template <typename F>
void parallel_chunks(size_t n, F body) {
  constexpr size_t CH = size_t(1) << 20;
  parallel_for((n + CH - 1) / CH, [&](size_t c) { body(c * CH, std::min(n, (c + 1) * CH)); });
}

template <typename T>
reff_status upload(const std::vector<double>& src, T** dst, std::vector<void*>& owned) {
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  HIPCHK(hipMalloc((void**)dst, bytes));
  owned.push_back(*dst);
  if (src.empty()) return REFF_OK;
  if (sizeof(T) == sizeof(double)) {
    HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return REFF_OK;
  }
  std::vector<T> tmp(src.size());
  parallel_chunks(src.size(), [&](size_t lo, size_t hi) {
    for (size_t i = lo; i < hi; ++i) tmp[i] = (T)src[i];
  });
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return REFF_OK;
}

reff_status ensure(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return REFF_OK;
  if (b.p) {
    HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  HIPCHK(hipMalloc(&b.p, std::max<size_t>(bytes, 256)));
  b.bytes = std::max<size_t>(bytes, 256);
  return REFF_OK;
}

Coef<double> coef64(const CoefSet& cs) {
  return Coef<double>{cs.d64, cs.dinv64, cs.cE64, cs.cN64, cs.slot, cs.up64, cs.dn64, cs.tnode};
}
Coef<float> coef32(const CoefSet& cs) {
  return Coef<float>{cs.d32, cs.dinv32, cs.cE32, cs.cN32, cs.slot, cs.up32, cs.dn32, cs.tnode};
}

// The handle's copy of its description, as a reff_pdn_desc view.
reff_pdn_desc desc_view(const reff_pdn_t* p) {
  reff_pdn_desc d;
  d.n_tiers = p->nt;
  d.nx = p->nx;
  d.ny = p->ny;
  d.gx = p->gx.data();
  d.gy = p->gy.data();
  d.n_tsv = (int32_t)(p->tsv_xy.size() / 2);
  d.tsv_xy = p->tsv_xy.data();
  d.tsv_g = p->tsv_g.data();
  d.n_pads = (int32_t)(p->pad_xy.size() / 2);
  d.pad_xy = p->pad_xy.data();
  return d;
}

// Build and upload one coefficient set for several stacks (a batch), each
// with its own grounded node list, concatenated in order; cbase[i] receives
// the first coefficient index of stack i.
reff_status make_coefset_multi(const std::vector<const reff_pdn_desc*>& ds,
                               const std::vector<std::vector<int64_t>>& gnds, CoefSet& cs,
                               std::vector<int64_t>& cbase, std::vector<void*>& extra,
                               std::vector<int32_t>* slot0s = nullptr) {
  // Every stack's entries go straight into the concatenated arrays; the
  // stacks are built on parallel host threads.
  const size_t np = ds.size();
  std::vector<int64_t> off(np + 1, 0), soff(np + 1, 0);
  for (size_t i = 0; i < np; ++i) {
    off[i + 1] = off[i] + (int64_t)ds[i]->n_tiers * ds[i]->nx * ds[i]->ny;
    soff[i + 1] = soff[i] + (int64_t)ds[i]->n_tsv * ds[i]->n_tiers;
  }
  HostCoef h;
  std::vector<int64_t> tnode((size_t)soff[np]);
  h.d.resize((size_t)off[np]);
  h.cE.resize((size_t)off[np]);
  h.cN.resize((size_t)off[np]);
  h.slot.resize((size_t)off[np]);
  h.is_pad.resize((size_t)off[np]);
  h.up.resize((size_t)soff[np]);
  h.dn.resize((size_t)soff[np]);
  cbase.assign(off.begin(), off.end() - 1);
  if (slot0s) {
    slot0s->clear();
    for (size_t i = 0; i < np; ++i) slot0s->push_back((int32_t)soff[i]);
  }
  std::vector<reff_status> st(np, REFF_OK);
  std::vector<std::string> msg(np);
  parallel_for(np, [&](size_t i) {
    const CoefOut o{h.d.data(), h.cE.data(), h.cN.data(), h.up.data(), h.dn.data(),
                    h.slot.data(), h.is_pad.data(), tnode.data(), off[i], soff[i]};
    st[i] = build_into(ds[i], gnds[i], o, msg[i]);
  });
  for (size_t i = 0; i < np; ++i)
    if (st[i] != REFF_OK) return fail(st[i], "plan " + std::to_string(i) + ": " + msg[i]);
  reff_status rs = REFF_OK;
  auto& owned = extra;
  auto upload_owned = [&](const std::vector<double>& src, double** d64, float** d32) {
    if (rs != REFF_OK) return;
    rs = upload<double>(src, d64, owned);
    if (rs == REFF_OK) rs = upload<float>(src, d32, owned);
  };
  // d, cE and cN go up in float64; D^-1 and the float32 copies of the four
  // per-node arrays are formed on the device (coef_prep.hip)
  const size_t nn = h.d.size();
  auto alloc = [&](auto** out) {
    if (rs != REFF_OK) return;
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*out)>>;
    if (hipMalloc((void**)out, std::max<size_t>(1, nn) * sizeof(T)) != hipSuccess) {
      rs = fail(REFF_ERR_OUT_OF_MEMORY, "coefficient arrays");
      return;
    }
    owned.push_back(*out);
  };
  if (rs == REFF_OK) rs = upload<double>(h.d, &cs.d64, owned);
  if (rs == REFF_OK) rs = upload<double>(h.cE, &cs.cE64, owned);
  if (rs == REFF_OK) rs = upload<double>(h.cN, &cs.cN64, owned);
  alloc(&cs.dinv64);
  alloc(&cs.d32);
  alloc(&cs.dinv32);
  alloc(&cs.cE32);
  alloc(&cs.cN32);
  if (rs != REFF_OK) return rs;
  HIPCHK(reff::launch_coef_derived(cs.d64, cs.cE64, cs.cN64, (int64_t)nn, cs.dinv64, cs.d32, cs.dinv32,
                             cs.cE32, cs.cN32, nullptr));
  HIPCHK(hipStreamSynchronize(nullptr));
  upload_owned(h.up, &cs.up64, &cs.up32);
  upload_owned(h.dn, &cs.dn64, &cs.dn32);
  if (rs != REFF_OK) return rs;
  HIPCHK(hipMalloc((void**)&cs.slot, std::max<size_t>(1, h.slot.size()) * sizeof(int32_t)));
  owned.push_back(cs.slot);
  HIPCHK(hipMemcpy(cs.slot, h.slot.data(), h.slot.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc((void**)&cs.tnode, std::max<size_t>(1, tnode.size()) * sizeof(int64_t)));
  owned.push_back(cs.tnode);
  if (!tnode.empty())
    HIPCHK(hipMemcpy(cs.tnode, tnode.data(), tnode.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice));
  cs.grounded = h.is_pad;
  cs.n_free = 0;
  for (uint8_t f : h.is_pad) cs.n_free += f ? 0 : 1;
  cs.n_slots = (int64_t)h.up.size();
  cs.ready = true;
  return REFF_OK;
}

// One stack of a handle.
reff_status make_coefset(reff_pdn_t* p, const std::vector<int64_t>& gnd, CoefSet& cs) {
  const reff_pdn_desc d = desc_view(p);
  std::vector<int64_t> cbase;
  return make_coefset_multi({&d}, {gnd}, cs, cbase, p->extra);
}

struct Opts {
  bool mixed;
  bool indep;  // independent columns (requested, or forced for tiny stacks)
  double tol;
  int32_t max_iters;
  int32_t max_ir;
  hipStream_t stream;
  bool out_dev;
  bool timing;
  bool graphs;  // replay iteration chunks as HIP graphs where possible
  const char* tune_db = nullptr;  // tuning database path (batched solves)
  bool progress = false;          // progress lines on stderr
  int cheb = 19;                  // Chebyshev preconditioner degree (1 = Jacobi)
  bool cheb_auto = false;         // degree chosen by the stack's size (precond_degree 0)
  int brhs = S;                   // right-hand sides dealt to one block (32 or 64)
  int32_t resident = 0;           // reff_query_pairs: solution blocks on the device (0 = auto)
};

// Default Chebyshev degree by the larger side of the stack's tiers: the
// spectrum of D^-1 G widens with the grid, so larger grids take a higher
// degree (fewer, costlier iterations).  Measured (mixed precision, 64 to 512
// sampled nodes): 4 x 512 x 512, degrees 13 / 16 / 19 / 22 / 25 give 820 /
// 852 / 872 / 861 / 863 nodes/s; 8 x 1024 x 1024, 19 / 25 / 31 give 55.4 /
// 58.3 / 59.7; 8 x 2048 x 2048, 2.25 / 2.39 / 2.47.
int auto_cheb_degree(int64_t side) { return side <= 640 ? 19 : 31; }

reff_status parse_opts(const reff_solve_opts* o, Opts& out) {
  reff_solve_opts z;
  std::memset(&z, 0, sizeof(z));
  if (!o) o = &z;
  if (o->precision != REFF_PREC_FP64 && o->precision != REFF_PREC_MIXED)
    return fail(REFF_ERR_INVALID_ARG, "unknown precision");
  if (o->krylov != REFF_KRYLOV_BLOCK && o->krylov != REFF_KRYLOV_INDEPENDENT)
    return fail(REFF_ERR_INVALID_ARG, "unknown krylov variant");
  if (!(o->rel_tol >= 0.0) || !std::isfinite(o->rel_tol) || o->rel_tol >= 1.0)
    return fail(REFF_ERR_INVALID_ARG, "rel_tol must be in [0, 1)");
  if (o->max_iters < 0) return fail(REFF_ERR_INVALID_ARG, "max_iters < 0");
  if (o->max_ir_steps < 0) return fail(REFF_ERR_INVALID_ARG, "max_ir_steps < 0");
  if (o->block_rhs != 0 && o->block_rhs != 32 && o->block_rhs != S)
    return fail(REFF_ERR_INVALID_ARG, "block_rhs must be 0, 32 or 64");
  if (o->out_on_device != 0 && o->out_on_device != 1)
    return fail(REFF_ERR_INVALID_ARG, "out_on_device must be 0 or 1");
  out.mixed = o->precision == REFF_PREC_MIXED;
  out.indep = o->krylov == REFF_KRYLOV_INDEPENDENT;
  out.tol = o->rel_tol > 0.0 ? o->rel_tol : (out.mixed ? 1e-5 : 1e-8);
  out.max_iters = o->max_iters > 0 ? o->max_iters : 20000;
  out.max_ir = o->max_ir_steps > 0 ? o->max_ir_steps : 3;
  out.stream = (hipStream_t)o->stream;
  out.out_dev = o->out_on_device == 1;
  if (o->timing != 0 && o->timing != 1) return fail(REFF_ERR_INVALID_ARG, "timing must be 0 or 1");
  if (o->graphs < 0 || o->graphs > 2)
    return fail(REFF_ERR_INVALID_ARG, "graphs must be 0 (automatic), 1 (replay) or 2 (plain)");
  out.graphs = o->graphs != 2;
  if (o->progress != 0 && o->progress != 1) return fail(REFF_ERR_INVALID_ARG, "progress must be 0 or 1");
  out.progress = o->progress == 1;
  if (o->precond_degree < 0 || o->precond_degree > MAX_CHEB)
    return fail(REFF_ERR_INVALID_ARG, "precond_degree must be in [0, 32]");
  out.cheb = o->precond_degree == 0 ? 19 : o->precond_degree;
  out.cheb_auto = o->precond_degree == 0;
  // The kernels map one right-hand side to one lane of a 64-wide wave, so a
  // block always streams 64 columns: 32 leaves half of them empty (no saving)
  // and the automatic choice (0) is 64.
  out.brhs = o->block_rhs == 32 ? 32 : S;
  out.timing = o->timing == 1;
  if (o->pairs_resident_blocks < 0) return fail(REFF_ERR_INVALID_ARG, "pairs_resident_blocks < 0");
  out.resident = o->pairs_resident_blocks;
  return REFF_OK;
}

// ---------------------------------------------------------------- solver core
// A stack as seen by the block solver.
struct StackInfo {
  int64_t cbase, n, plane;
  int32_t nx;
  int32_t slot_begin = 0, slot_end = 0;  // its TSV slots in the coefficient set
};

// One block of up to S unit-current columns on one stack: local target node
// ids and the output positions of their results.
struct BlockJob {
  int32_t stack = 0;
  int ncol = 0;
  int64_t tgt[S];
  int64_t pos[S];
};

struct BlockResult {
  int32_t iters = 0;
  int32_t ir = 0;
  bool conv = false;
  double est_max = 0.0;
  int64_t n_unconv = 0;
};

}  // namespace

void reff::Workspace::release() {
  for (DevBuf* b : {&Y, &P, &Q, &R, &D, &X, &part, &W, &small, &state, &tgt, &pos, &plans, &units,
                    &uid, &act, &out, &xs, &rows, &map, &flags, &strips, &sid, &Za, &Zb, &Zc, &Zd,
                    &TA, &TB, &cnt})
    if (b->p) {
      (void)hipFree(b->p);
      b->p = nullptr;
      b->bytes = 0;
    }
}

namespace {

// Pinned host staging (freed on scope exit).
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  reff_status ensure(size_t b) {
    if (bytes >= b && p) return REFF_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    HIPCHK(hipHostMalloc(&p, std::max<size_t>(b, 64)));
    bytes = std::max<size_t>(b, 64);
    return REFF_OK;
  }
};

constexpr int TARGET_UNITS = 1024;  // 4 workgroups of 512 threads per CU

// Split the solve blocks of a group into work units: each block's row range
// is cut into chunk-aligned pieces, about TARGET_UNITS in total, in
// proportion to the block sizes, and at least `floor` per block where the
// block has 64 chunks per unit to give: blocks converge at different times
// and leave the active lists, so a block that runs on alone still spreads
// over the whole device.
// Most work pieces a floor may bring a launch to: every piece has its S x S
// partial Grams reduced each iteration, so a batch of thousands of small
// plans keeps the proportional split instead.
constexpr int64_t MAX_FLOOR_PIECES = 16384;

void make_units(const std::vector<PlanDesc>& in, std::vector<PlanDesc>& plans,
                std::vector<Unit>& units, int target = TARGET_UNITS, int floor = 0) {
  int64_t rows = 0;
  for (const PlanDesc& p : in) rows += p.n;
  if (floor > 0) {
    int64_t total = 0;
    for (const PlanDesc& p : in) {
      const int64_t nch = (p.n + CH - 1) / CH;
      total += std::max<int64_t>((target * p.n + rows - 1) / std::max<int64_t>(rows, 1),
                                 std::min<int64_t>(floor, nch / 64));
    }
    if (total > MAX_FLOOR_PIECES) floor = 0;
  }
  plans = in;
  units.clear();
  for (size_t i = 0; i < plans.size(); ++i) {
    PlanDesc& p = plans[i];
    const int64_t nch = (p.n + CH - 1) / CH;
    int64_t k = (target * p.n + rows - 1) / std::max<int64_t>(rows, 1);
    k = std::max<int64_t>(k, std::min<int64_t>(floor, nch / 64));
    k = std::max<int64_t>(1, std::min<int64_t>(k, nch));
    const int64_t cpu = (nch + k - 1) / k;  // chunks per unit
    p.unit_begin = (int32_t)units.size();
    for (int64_t c0 = 0; c0 < nch; c0 += cpu) {
      Unit u;
      u.begin = p.vbase + c0 * CH;
      u.end = p.vbase + std::min<int64_t>(p.n, (c0 + cpu) * CH);
      u.plan = (int32_t)i;
      u.pad_ = 0;
      units.push_back(u);
    }
    p.unit_end = (int32_t)units.size();
  }
}

// Most rows of one strip for the three-step Chebyshev pass, which addresses
// a strip's rows through unsigned 32-bit byte offsets from a base three rows
// before it: (rows + 8) x nx x S floats stay below 2^31 bytes.  0 when even
// one row does not fit (the pass is then not used).
int64_t max_strip_rows(int64_t nx) {
  return std::max<int64_t>(0, (int64_t(1) << 31) / (nx * S * (int64_t)sizeof(float)) - 8);
}

// Strips for the stencil kernel of a group (float32 block variant): every
// block's tiers are cut into CH-wide x strips and, when that gives too few
// workgroups, into y segments, about TARGET_UNITS strips in total (and no
// more than max_strip_rows rows each); at least `floor` per block while the
// segments keep 64 rows or more (as for work units).
void make_strips(std::vector<PlanDesc>& plans, std::vector<Strip>& strips,
                 int target = TARGET_UNITS, int floor = 0) {
  int64_t rows = 0;
  for (const PlanDesc& p : plans) rows += p.n;
  if (floor > 0) {
    int64_t total = 0;
    for (const PlanDesc& p : plans) {
      const int64_t nx = p.nx, ny = p.plane / p.nx, nt = p.n / p.plane;
      const int64_t nsx = (nx + CH - 1) / CH;
      total += std::max<int64_t>((target * p.n + rows - 1) / std::max<int64_t>(rows, 1),
                                 std::min<int64_t>(floor, nt * nsx * std::max<int64_t>(1, ny / 64)));
    }
    if (total > MAX_FLOOR_PIECES) floor = 0;
  }
  strips.clear();
  for (size_t i = 0; i < plans.size(); ++i) {
    PlanDesc& p = plans[i];
    const int64_t nx = p.nx, ny = p.plane / p.nx, nt = p.n / p.plane;
    const int64_t nsx = (nx + CH - 1) / CH;
    int64_t want = std::max<int64_t>(1, (target * p.n + rows - 1) / std::max<int64_t>(rows, 1));
    want = std::max<int64_t>(want, std::min<int64_t>(floor, nt * nsx * std::max<int64_t>(1, ny / 64)));
    const int64_t ysegs = std::min<int64_t>(ny, std::max<int64_t>(1, (want + nt * nsx - 1) / (nt * nsx)));
    const int64_t hcap = max_strip_rows(nx);
    const int64_t H = std::min<int64_t>((ny + ysegs - 1) / ysegs, std::max<int64_t>(hcap, 1));
    p.strip_begin = (int32_t)strips.size();
    for (int64_t t = 0; t < nt; ++t)
      for (int64_t y0 = 0; y0 < ny; y0 += H)
        for (int64_t x0 = 0; x0 < nx; x0 += CH) {
          Strip s{};
          s.lrow0 = t * p.plane + y0 * nx + x0;
          s.plan = (int32_t)i;
          s.nrows = (int32_t)std::min<int64_t>(H, ny - y0);
          s.wdt = (int32_t)std::min<int64_t>(CH, nx - x0);
          s.y0 = (int32_t)y0;
          s.x0 = (int32_t)x0;
          strips.push_back(s);
        }
    p.strip_end = (int32_t)strips.size();
  }
}

__global__ void k_gather_flags(const BlockState* __restrict__ st, int nb, int32_t* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
    out[2 * i] = st[i].it;
    out[2 * i + 1] = st[i].all_conv;
  }
}

// Tuning database: one line "<size class> <work units> <strips>" per entry:
// the work units per launch of the row-range kernels and the strips per
// launch of the stencil passes (which fixes the strips' height, the tile
// shape of those passes: CH nodes wide, H rows tall).  The size class is the
// precision, the Krylov variant, log2 of the rows of a launch group and the
// number of its blocks.
struct TuneChoice {
  int units = 0, strips = 0;
};
struct TuneDb {
  std::vector<std::pair<std::string, TuneChoice>> e;
  static bool ok(int v) { return v >= 64 && v <= (1 << 16); }
  void load(const char* path) {
    e.clear();
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[128];
    TuneChoice c;
    while (std::fscanf(f, "%127s %d %d", key, &c.units, &c.strips) == 3)
      if (ok(c.units) && ok(c.strips)) e.emplace_back(key, c);
    std::fclose(f);
  }
  TuneChoice get(const std::string& k) const {
    for (const auto& kv : e)
      if (kv.first == k) return kv.second;
    return TuneChoice{};
  }
  bool save(const char* path, const std::string& k, TuneChoice v) {
    load(path);
    bool found = false;
    for (auto& kv : e)
      if (kv.first == k) kv.second = v, found = true;
    if (!found) e.emplace_back(k, v);
    FILE* f = std::fopen(path, "w");
    if (!f) return false;
    for (const auto& kv : e)
      std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.units, kv.second.strips);
    return std::fclose(f) == 0;
  }
};

std::string tune_key(bool fp32, bool indep, int64_t rows, int nb) {
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= rows) ++lg;
  int bb = 1;
  while (bb < nb && bb < 256) bb <<= 1;
  return std::string(fp32 ? "f32" : "f64") + (indep ? "-indep" : "-block") + "-r" +
         std::to_string(lg) + "-b" + std::to_string(bb);
}

// Solve every job (block of unit-current columns) with the block PCG,
// several blocks per launch (as many as fit the row budget), writing result
// j of block b to res_dev[b.pos[j]].  With xstore, the float64 solution of
// job i is copied to xstore + xoff[i] (stack n x S).
reff_status run_blocks(Workspace& ws, const CoefSet& cs, const std::vector<StackInfo>& stacks,
                       const std::vector<BlockJob>& jobs, double* res_dev, const Opts& o_in,
                       std::vector<BlockResult>& br, reff_solve_stats* st,
                       double* xstore = nullptr, const std::vector<int64_t>* xoff = nullptr) {
  br.assign(jobs.size(), BlockResult());
  if (jobs.empty()) return REFF_OK;
  // Iteration chunks are replayed as HIP graphs unless plain launches were
  // asked for or the kernels are being timed.  On the legacy default stream
  // (NULL) the solve runs on a stream of its own, which orders itself with
  // the default stream both ways and is drained before returning.
  Opts o = o_in;
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    }
  } own;
  if (o.graphs && !o.timing && o.stream == nullptr) {
    HIPCHK(hipStreamCreate(&own.s));
    o.stream = own.s;
  }
  const bool fp32 = o.mixed;
  const bool with_d = o.mixed || xstore != nullptr;
  const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
  const int ncheb = (!o.indep && o.cheb > 1) ? (o.cheb > 2 ? 4 : 2) : 0;  // iterate arrays
  const size_t row_bytes =
      S * (tsz * (5 + (with_d ? 1 : 0) + ncheb) + (o.mixed ? sizeof(double) : 0));
  const int64_t budget_rows = std::max<int64_t>(1, (int64_t)(96e9 / (double)row_bytes));
  const Coef<double> c64 = coef64(cs);
  const Coef<float> c32 = coef32(cs);
  const void* coef = fp32 ? (const void*)&c32 : (const void*)&c64;
  // Iterations between convergence checks (each costs a host round trip):
  // every iteration once the polynomial preconditioner makes iterations
  // costly, every fourth with Jacobi.
  int poll = (!o.indep && o.cheb > 1) ? 1 : 4;

  struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } evp;
  if (o.timing) {
    evp.ev.resize(NEV * poll);
    for (auto& e : evp.ev) HIPCHK(hipEventCreate(&e));
  }
  PinnedBuf pin_tab, pin_flags;
  bool any_unconv = false;
  auto last_report = std::chrono::steady_clock::now();
  // Chunks of `poll` iterations are captured once and replayed as a HIP
  // graph (the launch sequence of a chunk only changes with the active set),
  // on a created stream that is not itself being captured, without timing.
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int k = -1;
    void reset() {
      if (exec) (void)hipGraphExecDestroy(exec);
      exec = nullptr;
      k = -1;
    }
    ~GraphCache() { reset(); }
  } gc;
  bool use_graph = o.graphs && !o.timing && o.stream != nullptr;
  if (use_graph) {
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(o.stream, &cst) != hipSuccess || cst != hipStreamCaptureStatusNone)
      use_graph = false;
  }
  // A replayed chunk stays valid while blocks converge (they leave the
  // device-resident active lists), so chunks can span several iterations
  // with one host round trip each.
  if (use_graph) poll = 4;
  // rows of the jobs from j on, so that groups come out balanced: a group
  // closes once it holds its share of the remaining rows (16 equal blocks
  // under a budget of 15 make two groups of 8, not 15 + 1)
  std::vector<int64_t> rows_from(jobs.size() + 1, 0);
  for (size_t j = jobs.size(); j-- > 0;)
    rows_from[j] = rows_from[j + 1] + stacks[(size_t)jobs[j].stack].n;
  size_t j0 = 0;
  while (j0 < jobs.size()) {
    // ---- group of jobs within the row budget
    const int64_t ngr = (rows_from[j0] + budget_rows - 1) / budget_rows;
    const int64_t cap = std::min(budget_rows, (rows_from[j0] + ngr - 1) / std::max<int64_t>(ngr, 1));
    size_t j1 = j0;
    int64_t rows = 0, slot_rows = 0;
    int max_slots = 0;  // most TSV slots of one block
    std::vector<PlanDesc> pin;
    while (j1 < jobs.size()) {
      const StackInfo& sk = stacks[(size_t)jobs[j1].stack];
      if (j1 > j0 && (rows >= cap || rows + sk.n > budget_rows)) break;
      PlanDesc pd{};
      pd.cbase = sk.cbase;
      pd.vbase = rows;
      pd.n = sk.n;
      pd.plane = sk.plane;
      pd.nx = sk.nx;
      pd.slot_begin = sk.slot_begin;
      pd.slot_end = sk.slot_end;
      pd.sbase = slot_rows;
      slot_rows += sk.slot_end - sk.slot_begin;
      max_slots = std::max(max_slots, (int)(sk.slot_end - sk.slot_begin));
      pin.push_back(pd);
      rows += sk.n;
      ++j1;
    }
    const int nb = (int)(j1 - j0);
    gc.reset();  // work arrays may be reallocated for this group
    // Work units per launch: the tuning database's entry for this size
    // class, or (new class) the fastest of a few candidates, each timed over
    // one chunk of iterations from a fresh start.
    TuneChoice target{TARGET_UNITS, TARGET_UNITS};
    std::vector<TuneChoice> trials;
    std::string tkey;
    TuneDb tdb;
    if (o.tune_db) {
      tkey = tune_key(fp32, o.indep, rows, nb);
      tdb.load(o.tune_db);
      const TuneChoice v = tdb.get(tkey);
      if (v.units > 0) {
        target = v;
      } else {
        for (int u : {512, 1024, 2048})
          for (int sp : {256, 512, 1024, 2048}) trials.push_back(TuneChoice{u, sp});
      }
    }
    std::vector<float> trial_ms;
    std::vector<PlanDesc> plans;
    std::vector<Unit> units;
    std::vector<Strip> strips;
    int nu = 0, ns = 0;
    PlanDesc* h_plans = nullptr;
    Unit* h_units = nullptr;
    int64_t *h_tgt = nullptr, *h_pos = nullptr;
    int32_t *h_uid = nullptr, *h_act = nullptr, *h_sid = nullptr, *h_cnt = nullptr;
    Strip* h_strips = nullptr;
    SolveBuffers b;
    for (size_t attempt = 0; attempt <= trials.size(); ++attempt) {
    const bool trial = attempt < trials.size();
    const TuneChoice tc = trial ? trials[attempt] : target;
    // a floor of work per block (where the block is large enough), so that
    // the last unconverged blocks of a group still fill the device
    const int floor = TARGET_UNITS / 2;
    make_units(pin, plans, units, tc.units, floor);
    nu = (int)units.size();
    strips.clear();
    const bool cheb = !o.indep && o.cheb > 1;
    if ((fp32 || cheb) && !o.indep) make_strips(plans, strips, tc.strips, floor);
    ns = (int)strips.size();
    // ---- buffers
    reff_status rs;
    const size_t vec = (size_t)rows * S * tsz;
    if ((rs = ensure(ws.Y, vec)) != REFF_OK) return rs;
    if ((rs = ensure(ws.P, vec)) != REFF_OK) return rs;
    if ((rs = ensure(ws.Q, vec)) != REFF_OK) return rs;
    if ((rs = ensure(ws.R, vec)) != REFF_OK) return rs;
    if (with_d && (rs = ensure(ws.D, vec)) != REFF_OK) return rs;
    if (o.mixed && (rs = ensure(ws.X, (size_t)rows * S * sizeof(double))) != REFF_OK) return rs;
    if (cheb && (rs = ensure(ws.Za, vec)) != REFF_OK) return rs;
    if (cheb && (rs = ensure(ws.Zb, vec)) != REFF_OK) return rs;
    if (cheb && o.cheb > 2 && (rs = ensure(ws.Zc, vec)) != REFF_OK) return rs;
    if (cheb && o.cheb > 2 && (rs = ensure(ws.Zd, vec)) != REFF_OK) return rs;
    bool triples = cheb && o.cheb > 3;
    for (const PlanDesc& p : plans) triples = triples && max_strip_rows(p.nx) >= 1;
    if (triples && (rs = ensure(ws.TA, (size_t)slot_rows * 5 * S * tsz)) != REFF_OK) return rs;
    if (triples && (rs = ensure(ws.TB, (size_t)slot_rows * S * tsz)) != REFF_OK) return rs;
    if ((rs = ensure(ws.part, (size_t)std::max(nu, ns) * NGRAM * S * S * sizeof(double))) != REFF_OK)
      return rs;
    if ((rs = ensure(ws.W, (size_t)nb * NGRAM * S * S * sizeof(double))) != REFF_OK) return rs;
    if ((rs = ensure(ws.small, (size_t)nb * 4 * S * S * sizeof(double))) != REFF_OK) return rs;
    if ((rs = ensure(ws.strips, (size_t)std::max(ns, 1) * sizeof(Strip))) != REFF_OK) return rs;
    if ((rs = ensure(ws.sid, (size_t)std::max(ns, 1) * sizeof(int32_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.state, (size_t)nb * sizeof(BlockState))) != REFF_OK) return rs;
    if ((rs = ensure(ws.tgt, (size_t)nb * S * sizeof(int64_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.pos, (size_t)nb * S * sizeof(int64_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.plans, (size_t)nb * sizeof(PlanDesc))) != REFF_OK) return rs;
    if ((rs = ensure(ws.units, (size_t)nu * sizeof(Unit))) != REFF_OK) return rs;
    if ((rs = ensure(ws.uid, (size_t)nu * sizeof(int32_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.act, (size_t)nb * sizeof(int32_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.flags, (size_t)nb * 2 * sizeof(int32_t))) != REFF_OK) return rs;
    if ((rs = ensure(ws.cnt, 4 * sizeof(int32_t))) != REFF_OK) return rs;
    // ---- tables (one pinned staging area, uploaded asynchronously)
    const size_t tab_bytes = nb * sizeof(PlanDesc) + nu * sizeof(Unit) + nb * S * 16 +
                             (nu + nb) * sizeof(int32_t) * 2 + ns * sizeof(Strip) +
                             ns * sizeof(int32_t) + 256 + 64;
    if ((rs = pin_tab.ensure(tab_bytes)) != REFF_OK) return rs;
    if ((rs = pin_flags.ensure((size_t)nb * 2 * sizeof(int32_t))) != REFF_OK) return rs;
    char* hp = (char*)pin_tab.p;
    h_plans = (PlanDesc*)hp;
    h_units = (Unit*)(h_plans + nb);
    h_tgt = (int64_t*)(h_units + nu);
    h_pos = h_tgt + (size_t)nb * S;
    h_uid = (int32_t*)(h_pos + (size_t)nb * S);
    h_act = h_uid + nu;
    h_strips = (Strip*)(((uintptr_t)(h_act + nb) + 15) & ~(uintptr_t)15);
    h_sid = (int32_t*)(h_strips + ns);
    h_cnt = (int32_t*)(((uintptr_t)(h_sid + ns) + 15) & ~(uintptr_t)15);
    h_cnt[0] = nu;
    h_cnt[1] = ns;
    h_cnt[2] = nb;
    h_cnt[3] = 0;
    std::memcpy(h_plans, plans.data(), nb * sizeof(PlanDesc));
    std::memcpy(h_units, units.data(), nu * sizeof(Unit));
    for (int i = 0; i < nb; ++i) {
      const BlockJob& jb = jobs[j0 + (size_t)i];
      for (int k = 0; k < S; ++k) {
        h_tgt[(size_t)i * S + k] = k < jb.ncol ? jb.tgt[k] : -1;
        h_pos[(size_t)i * S + k] = k < jb.ncol ? jb.pos[k] : -1;
      }
      h_act[i] = i;
    }
    for (int u = 0; u < nu; ++u) h_uid[u] = u;
    if (ns > 0) std::memcpy(h_strips, strips.data(), ns * sizeof(Strip));
    for (int u = 0; u < ns; ++u) h_sid[u] = u;
    if (ns > 0) {
      HIPCHK(hipMemcpyAsync(ws.strips.p, h_strips, ns * sizeof(Strip), hipMemcpyHostToDevice, o.stream));
      HIPCHK(hipMemcpyAsync(ws.sid.p, h_sid, ns * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
    }
    HIPCHK(hipMemcpyAsync(ws.plans.p, h_plans, nb * sizeof(PlanDesc), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.units.p, h_units, nu * sizeof(Unit), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.tgt.p, h_tgt, (size_t)nb * S * sizeof(int64_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.pos.p, h_pos, (size_t)nb * S * sizeof(int64_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.uid.p, h_uid, nu * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.act.p, h_act, nb * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(ws.cnt.p, h_cnt, 4 * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));

    b = SolveBuffers{};
    b.Y = ws.Y.p;
    b.P = ws.P.p;
    b.Q = ws.Q.p;
    b.R = ws.R.p;
    b.D = with_d ? ws.D.p : nullptr;
    b.X = o.mixed ? (double*)ws.X.p : nullptr;
    b.part = (double*)ws.part.p;
    b.W = (double*)ws.W.p;
    b.winv = (double*)ws.small.p;
    b.alpha = (double*)ws.small.p + (size_t)nb * S * S;
    b.delta = (double*)ws.small.p + (size_t)2 * nb * S * S;
    b.Tm = (double*)ws.small.p + (size_t)3 * nb * S * S;
    b.state = (BlockState*)ws.state.p;
    b.tgt = (int64_t*)ws.tgt.p;
    b.pos = (int64_t*)ws.pos.p;
    b.work.plans = (const PlanDesc*)ws.plans.p;
    b.work.units = (const Unit*)ws.units.p;
    b.work.uid = (const int32_t*)ws.uid.p;
    b.work.strips = (const Strip*)ws.strips.p;
    b.work.sid = (const int32_t*)ws.sid.p;
    b.act = (const int32_t*)ws.act.p;
    b.act_w = (int32_t*)ws.act.p;
    b.uid_w = (int32_t*)ws.uid.p;
    b.sid_w = (int32_t*)ws.sid.p;
    b.cnt = (int32_t*)ws.cnt.p;
    b.work.cnt = b.cnt;
    b.n_act = nb;
    b.n_units = nu;
    b.n_strips = ns;
    b.rows = rows;
    if (cheb) {
      // Chebyshev semi-iteration for D^-1 G on [lmax / (6 k^2), lmax], lmax = 2
      // (the spectrum of D^-1 G lies in (0, 2]): q > 0 on (0, 2], so
      // M^-1 = q(D^-1 G) D^-1 is SPD.
      const double lmax = 2.0, lmin = lmax / (6.0 * o.cheb * o.cheb);
      const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
      const double sigma = theta / delta;
      double rho = 1.0 / sigma;
      b.cheb_k = o.cheb;
      b.cheb_invtheta = 1.0 / theta;
      for (int j = 1; j < o.cheb; ++j) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        b.cheb_a1[j] = rn * rho;
        b.cheb_a2[j] = 2.0 * rn / delta;
        rho = rn;
      }
      b.Za = ws.Za.p;
      b.Zb = ws.Zb.p;
      b.Zc = ws.Zc.p;
      b.Zd = ws.Zd.p;
      b.TA = triples ? ws.TA.p : nullptr;  // no three-step passes without them
      b.TB = triples ? ws.TB.p : nullptr;
      b.max_tsv_slots = max_slots;
    }

    HIPCHK(launch_init_blocks(fp32, o.indep, coef, b, o.stream));
    if (with_d && !fp32) HIPCHK(launch_zero_x((double*)b.D, rows * S, o.stream));
    if (o.mixed) HIPCHK(launch_zero_x(b.X, rows * S, o.stream));
    if (trial) {
      struct Ev {
        hipEvent_t a = nullptr, z = nullptr;
        ~Ev() {
          if (a) (void)hipEventDestroy(a);
          if (z) (void)hipEventDestroy(z);
        }
      } ev;
      HIPCHK(hipEventCreate(&ev.a));
      HIPCHK(hipEventCreate(&ev.z));
      HIPCHK(hipEventRecord(ev.a, o.stream));
      for (int i = 0; i < poll; ++i)
        HIPCHK(launch_iteration(fp32, o.indep, with_d, coef, b, o.tol, o.stream, nullptr));
      HIPCHK(hipEventRecord(ev.z, o.stream));
      HIPCHK(hipEventSynchronize(ev.z));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.z));
      trial_ms.push_back(ms);
      if (attempt + 1 == trials.size()) {
        const size_t best = (size_t)(std::min_element(trial_ms.begin(), trial_ms.end()) -
                                     trial_ms.begin());
        target = trials[best];
        (void)tdb.save(o.tune_db, tkey, target);
      }
    }
    }  // attempts

    std::vector<char> done((size_t)nb, 0);     // converged in the current step
    std::vector<int32_t> iters((size_t)nb, 0);   // block iterations over all inner solves
    std::vector<int32_t> cur_it((size_t)nb, 0);  // of the current inner solve (device count)
    std::vector<int32_t> irs((size_t)nb, 0);
    std::vector<int> active(nb);
    for (int i = 0; i < nb; ++i) active[(size_t)i] = i;
    auto rows_of = [&](const std::vector<int>& a) {
      int64_t r = 0;
      for (int bi : a) r += plans[(size_t)bi].n;
      return r;
    };
    int ir = 0;
    while (true) {
      // ---- inner block-PCG iterations over the active blocks
      int it = 0;
      while (it < o.max_iters && !active.empty()) {
        const int k = std::min(poll, o.max_iters - it);
        const int64_t act_rows = rows_of(active);
        if (use_graph) {
          if (!gc.exec || gc.k != k) {
            gc.reset();
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(o.stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (int i = 0; i < k; ++i) {
              const hipError_t e = launch_iteration(fp32, o.indep, with_d, coef, b, o.tol,
                                                    o.stream, nullptr);
              if (le == hipSuccess) le = e;
            }
            const hipError_t ee = hipStreamEndCapture(o.stream, &graph);
            if (le != hipSuccess || ee != hipSuccess) {
              if (graph) (void)hipGraphDestroy(graph);
              HIPCHK(le);
              HIPCHK(ee);
            }
            const hipError_t ie = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) gc.exec = nullptr;
            HIPCHK(ie);
            gc.k = k;
          }
          HIPCHK(hipGraphLaunch(gc.exec, o.stream));
        } else {
          for (int i = 0; i < k; ++i)
            HIPCHK(launch_iteration(fp32, o.indep, with_d, coef, b, o.tol, o.stream,
                                    o.timing ? &evp.ev[NEV * i] : nullptr));
        }
        it += k;
        if (o.progress) {
          const auto now = std::chrono::steady_clock::now();
          if (std::chrono::duration<double>(now - last_report).count() >= 10.0) {
            std::fprintf(stderr, "[reff] group of %d blocks: iteration %d, %zu blocks active\n", nb,
                         it, active.size());
            std::fflush(stderr);
            last_report = now;
          }
        }
        hipLaunchKernelGGL(k_gather_flags, dim3(1), dim3(256), 0, o.stream, b.state, nb,
                           (int32_t*)ws.flags.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(pin_flags.p, ws.flags.p, (size_t)nb * 2 * sizeof(int32_t),
                              hipMemcpyDeviceToHost, o.stream));
        HIPCHK(hipStreamSynchronize(o.stream));
        if (o.timing && st) {
          for (int i = 0; i < k; ++i)
            for (int kk = 0; kk < NEV / 2; ++kk) {
              float ms = 0.f;
              HIPCHK(hipEventElapsedTime(&ms, evp.ev[NEV * i + 2 * kk],
                                         evp.ev[NEV * i + 2 * kk + 1]));
              st->kernel_ms[kk] += ms;
              st->kernel_launches[kk] += 1;
              st->kernel_rows[kk] += act_rows;
            }
        }
        // flags of every block (gathered into a small device array); the
        // device has already dropped converged blocks from its active lists
        // (k_compact at the end of every iteration), this is bookkeeping
        const int32_t* fl = (const int32_t*)pin_flags.p;
        std::vector<int> still;
        for (int bi : active) {
          cur_it[(size_t)bi] = fl[(size_t)bi * 2];
          if (fl[(size_t)bi * 2 + 1]) {
            done[(size_t)bi] = 1;
          } else {
            still.push_back(bi);
          }
        }
        active = still;
      }
      for (int i = 0; i < nb; ++i) {
        iters[(size_t)i] += cur_it[(size_t)i];
        cur_it[(size_t)i] = 0;
      }
      ++ir;
      for (int i = 0; i < nb; ++i) irs[(size_t)i] = ir;
      // ---- all blocks of the group again for the float64 step / results
      for (int i = 0; i < nb; ++i) h_act[i] = i;
      for (int u = 0; u < nu; ++u) h_uid[u] = u;
      for (int u = 0; u < ns; ++u) h_sid[u] = u;
      HIPCHK(hipMemcpyAsync(ws.uid.p, h_uid, nu * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
      HIPCHK(hipMemcpyAsync(ws.act.p, h_act, nb * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
      if (ns > 0)
        HIPCHK(hipMemcpyAsync(ws.sid.p, h_sid, ns * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
      HIPCHK(hipMemcpyAsync(ws.cnt.p, h_cnt, 4 * sizeof(int32_t), hipMemcpyHostToDevice, o.stream));
      if (!o.mixed) break;
      HIPCHK(launch_mixed_residual(c64, c32, b, res_dev, o.stream));
      // One float32 solve carried to the tolerance plus the float64
      // variational correction suffices unless the inner solve stalled or
      // the tolerance is below what float32 iterates resolve.
      bool need_more = o.tol < 2e-6;
      for (int i = 0; i < nb; ++i) need_more = need_more || !done[(size_t)i];
      if (!need_more || ir >= o.max_ir) break;
      HIPCHK(launch_restart(c32, b, o.indep, o.stream));
      std::fill(done.begin(), done.end(), 0);
      active.resize(nb);
      for (int i = 0; i < nb; ++i) active[(size_t)i] = i;
    }
    if (!o.mixed) HIPCHK(launch_finalize_plain(b, res_dev, o.stream));
    if (xstore)
      for (int i = 0; i < nb; ++i)
        HIPCHK(hipMemcpyAsync(xstore + (*xoff)[j0 + (size_t)i],
                              o.mixed ? (const void*)(b.X + plans[(size_t)i].vbase * S)
                                      : (const void*)((double*)b.D + plans[(size_t)i].vbase * S),
                              (size_t)plans[(size_t)i].n * S * sizeof(double),
                              hipMemcpyDeviceToDevice, o.stream));
    std::vector<BlockState> hs((size_t)nb);
    HIPCHK(hipMemcpyAsync(hs.data(), b.state, (size_t)nb * sizeof(BlockState),
                          hipMemcpyDeviceToHost, o.stream));
    HIPCHK(hipStreamSynchronize(o.stream));
    for (int i = 0; i < nb; ++i) {
      BlockResult& r = br[j0 + (size_t)i];
      const BlockJob& jb = jobs[j0 + (size_t)i];
      r.iters = iters[(size_t)i];
      r.ir = irs[(size_t)i];
      r.conv = done[(size_t)i] != 0;
      for (int k = 0; k < jb.ncol; ++k) {
        const double e = hs[(size_t)i].est_rel[k];
        if (std::isfinite(e)) r.est_max = std::max(r.est_max, e);
        if (!r.conv && !(e <= CONV_SAFETY * o.tol)) r.n_unconv++;
      }
      if (!r.conv) any_unconv = true;
    }
    j0 = j1;
  }
  return any_unconv ? fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached before the tolerance")
                    : REFF_OK;
}

void add_stats(reff_solve_stats* st, const std::vector<BlockResult>& br, size_t b0, size_t b1) {
  if (!st) return;
  for (size_t i = b0; i < b1; ++i) {
    st->iters_max = std::max(st->iters_max, br[i].iters);
    st->iters_total += br[i].iters;
    st->ir_steps = std::max(st->ir_steps, br[i].ir);
    st->est_max_rel_err = std::max(st->est_max_rel_err, br[i].est_max);
    st->n_unconverged += br[i].n_unconv;
  }
}

// Deal the free columns `cols` (distinct ids local to stack `stack`) to
// blocks of S in a fixed pseudo-random order: right-hand sides that sit next
// to each other span nearly the same block Krylov space, while spread-out
// ones give every block independent directions.  Column i's result goes to
// position pos0 + i.
void deal_blocks(const std::vector<int64_t>& cols, int32_t stack, int64_t pos0,
                 std::vector<BlockJob>& jobs, int per = S) {
  std::vector<int64_t> order(cols.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
  std::mt19937_64 rng(0x9e3779b97f4a7c15ull);
  std::shuffle(order.begin(), order.end(), rng);
  for (size_t j = 0; j < order.size(); j += (size_t)per) {
    BlockJob jb;
    jb.stack = stack;
    jb.ncol = (int)std::min<size_t>((size_t)per, order.size() - j);
    for (int k = 0; k < jb.ncol; ++k) {
      const int64_t i = order[j + (size_t)k];
      jb.tgt[k] = cols[(size_t)i];
      jb.pos[k] = pos0 + i;
    }
    jobs.push_back(jb);
  }
}

// Device work tables for a single plan covering a whole stack (used by the
// pair cross terms): returns buffers with part/W/act/work filled.
reff_status single_work(Workspace& ws, const StackInfo& sk, SolveBuffers& b, hipStream_t stream,
                        PinnedBuf& pin) {
  std::vector<PlanDesc> in(1), plans;
  in[0] = PlanDesc{};
  in[0].cbase = sk.cbase;
  in[0].vbase = 0;
  in[0].n = sk.n;
  in[0].plane = sk.plane;
  in[0].nx = sk.nx;
  std::vector<Unit> units;
  make_units(in, plans, units);
  const int nu = (int)units.size();
  reff_status rs;
  if ((rs = ensure(ws.part, (size_t)nu * NGRAM * S * S * sizeof(double))) != REFF_OK) return rs;
  if ((rs = ensure(ws.W, (size_t)NGRAM * S * S * sizeof(double))) != REFF_OK) return rs;
  if ((rs = ensure(ws.plans, sizeof(PlanDesc))) != REFF_OK) return rs;
  if ((rs = ensure(ws.units, (size_t)nu * sizeof(Unit))) != REFF_OK) return rs;
  if ((rs = ensure(ws.uid, (size_t)nu * sizeof(int32_t))) != REFF_OK) return rs;
  if ((rs = ensure(ws.act, 2 * sizeof(int32_t))) != REFF_OK) return rs;
  if ((rs = ensure(ws.cnt, 4 * sizeof(int32_t))) != REFF_OK) return rs;
  if ((rs = pin.ensure(sizeof(PlanDesc) + nu * (sizeof(Unit) + sizeof(int32_t)) + 64)) != REFF_OK)
    return rs;
  char* hp = (char*)pin.p;
  std::memcpy(hp, plans.data(), sizeof(PlanDesc));
  std::memcpy(hp + sizeof(PlanDesc), units.data(), nu * sizeof(Unit));
  int32_t* uid = (int32_t*)(hp + sizeof(PlanDesc) + nu * sizeof(Unit));
  for (int u = 0; u < nu; ++u) uid[u] = u;
  uid[nu] = 0;
  HIPCHK(hipMemcpyAsync(ws.plans.p, hp, sizeof(PlanDesc), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(ws.units.p, hp + sizeof(PlanDesc), nu * sizeof(Unit), hipMemcpyHostToDevice,
                        stream));
  HIPCHK(hipMemcpyAsync(ws.uid.p, uid, nu * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(ws.act.p, uid + nu, sizeof(int32_t), hipMemcpyHostToDevice, stream));
  int32_t* cnt = (int32_t*)(((uintptr_t)(uid + nu + 1) + 15) & ~(uintptr_t)15);
  cnt[0] = nu;
  cnt[1] = 0;
  cnt[2] = 1;
  cnt[3] = 0;
  HIPCHK(hipMemcpyAsync(ws.cnt.p, cnt, 4 * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  b = SolveBuffers{};
  b.part = (double*)ws.part.p;
  b.W = (double*)ws.W.p;
  b.work.plans = (const PlanDesc*)ws.plans.p;
  b.work.units = (const Unit*)ws.units.p;
  b.work.uid = (const int32_t*)ws.uid.p;
  b.act = (const int32_t*)ws.act.p;
  b.cnt = (int32_t*)ws.cnt.p;
  b.work.cnt = b.cnt;
  b.n_act = 1;
  b.n_units = nu;
  b.rows = sk.n;
  return REFF_OK;
}

}  // namespace

extern "C" {

const char* reff_status_string(reff_status s) {
  switch (s) {
    case REFF_OK: return "ok";
    case REFF_ERR_INVALID_ARG: return "invalid argument";
    case REFF_ERR_DISCONNECTED: return "disconnected network (singular G)";
    case REFF_ERR_NO_CONVERGENCE: return "no convergence within max_iters";
    case REFF_ERR_OUT_OF_MEMORY: return "out of memory";
    case REFF_ERR_DEVICE: return "device error";
    case REFF_ERR_UNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

const char* reff_last_error(void) { return g_err.c_str(); }

int64_t reff_pdn_num_nodes(reff_pdn p) { return p ? p->n : -1; }

reff_status reff_build_pdn(const reff_pdn_desc* d, int32_t device, reff_pdn* out) {
  g_err.clear();
  if (!out) return fail(REFF_ERR_INVALID_ARG, "out is NULL");
  reff_status s = validate_desc(d);
  if (s != REFF_OK) return s;
  if (device < 0) return fail(REFF_ERR_INVALID_ARG, "device < 0");
  std::vector<int64_t> pads;
  for (int32_t j = 0; j < d->n_pads; ++j)
    pads.push_back((int64_t)d->pad_xy[2 * j + 1] * d->nx + d->pad_xy[2 * j]);
  {
    // Connectivity check on the host, before any device work.
    HostCoef h;
    s = build_host(d, pads, h);
    if (s != REFF_OK) return s;
  }
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device >= ndev) return fail(REFF_ERR_INVALID_ARG, "no such device");
  HIPCHK(hipSetDevice(device));
  reff_pdn_t* p = new (std::nothrow) reff_pdn_t();
  if (!p) return fail(REFF_ERR_OUT_OF_MEMORY, "host allocation");
  p->device = device;
  p->nt = d->n_tiers;
  p->nx = d->nx;
  p->ny = d->ny;
  p->plane = (int64_t)d->nx * d->ny;
  p->n = p->plane * d->n_tiers;
  const int64_t ngx = (int64_t)d->n_tiers * d->ny * (d->nx - 1);
  const int64_t ngy = (int64_t)d->n_tiers * (d->ny - 1) * d->nx;
  if (ngx > 0) p->gx.assign(d->gx, d->gx + ngx);
  if (ngy > 0) p->gy.assign(d->gy, d->gy + ngy);
  if (d->n_tsv > 0) p->tsv_xy.assign(d->tsv_xy, d->tsv_xy + 2 * (int64_t)d->n_tsv);
  if (d->n_tiers > 1 && d->n_tsv > 0)
    p->tsv_g.assign(d->tsv_g, d->tsv_g + (int64_t)d->n_tsv * (d->n_tiers - 1));
  p->pad_xy.assign(d->pad_xy, d->pad_xy + 2 * (int64_t)d->n_pads);
  s = make_coefset(p, pads, p->gnd);
  if (s != REFF_OK) {
    const std::string msg = g_err;
    reff_free_pdn(p);
    return fail(s, msg);
  }
  *out = p;
  return REFF_OK;
}

void reff_free_pdn(reff_pdn p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  for (void* q : p->extra) (void)hipFree(q);
  p->ws.release();
  delete p;
}

// Results of the distinct free nodes `cols` -> caller order (map[i] = index
// into cols, -1 for grounded nodes), host or device output.
static reff_status write_out(Workspace& ws, const double* res_dev, int64_t ncols,
                             const std::vector<int64_t>& map, double* R_out, bool out_dev,
                             hipStream_t stream) {
  const int64_t count = (int64_t)map.size();
  if (count == 0) return REFF_OK;
  if (out_dev) {
    reff_status rs = ensure(ws.map, (size_t)count * sizeof(int64_t));
    if (rs != REFF_OK) return rs;
    HIPCHK(hipMemcpyAsync(ws.map.p, map.data(), (size_t)count * sizeof(int64_t),
                          hipMemcpyHostToDevice, stream));
    HIPCHK(launch_gather_out(res_dev, (const int64_t*)ws.map.p, R_out, count, stream));
    HIPCHK(hipStreamSynchronize(stream));
  } else {
    std::vector<double> res((size_t)ncols);
    if (ncols > 0)
      HIPCHK(hipMemcpyAsync(res.data(), res_dev, (size_t)ncols * sizeof(double),
                            hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int64_t i = 0; i < count; ++i)
      R_out[i] = map[(size_t)i] >= 0 ? res[(size_t)map[(size_t)i]] : 0.0;
  }
  return REFF_OK;
}

// Distinct free ids of a request (sorted) and the caller-order map.
static reff_status columns_of(const int64_t* nodes, int64_t count, int64_t n,
                              const std::vector<uint8_t>& grounded, std::vector<int64_t>& cols,
                              std::vector<int64_t>& map) {
  cols.resize((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t v = nodes ? nodes[i] : i;
    if (v < 0 || v >= n)
      return fail(REFF_ERR_INVALID_ARG, "node id " + std::to_string(v) + " out of range");
    cols[(size_t)i] = v;
  }
  std::vector<int64_t> ids = cols;
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  cols.erase(std::remove_if(cols.begin(), cols.end(),
                            [&](int64_t v) { return grounded[(size_t)v] != 0; }),
             cols.end());
  map.resize((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t v = ids[(size_t)i];
    map[(size_t)i] = grounded[(size_t)v]
                         ? -1
                         : (int64_t)(std::lower_bound(cols.begin(), cols.end(), v) - cols.begin());
  }
  return REFF_OK;
}

reff_status reff_solve_diag(reff_pdn p, const int64_t* nodes, int64_t n_nodes, double* R_out,
                            const reff_solve_opts* opts, reff_solve_stats* st) {
  g_err.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  Opts o;
  reff_status s = parse_opts(opts, o);
  if (s != REFF_OK) return s;
  if (o.cheb_auto) o.cheb = auto_cheb_degree(std::max<int64_t>(p->nx, p->ny));
  if (nodes && n_nodes < 0) return fail(REFF_ERR_INVALID_ARG, "n_nodes < 0");
  const int64_t count = nodes ? n_nodes : p->n;
  if (count > 0 && !R_out) return fail(REFF_ERR_INVALID_ARG, "R_out is NULL");
  std::vector<int64_t> cols, map;
  s = columns_of(nodes, count, p->n, p->gnd.grounded, cols, map);
  if (s != REFF_OK) return s;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->n_solved = (int64_t)cols.size();
  }
  HIPCHK(hipSetDevice(p->device));
  // A block Krylov space of S columns exhausts a stack of only a few S free
  // nodes within a handful of iterations, where the block residual loses
  // column rank; such stacks use S independent PCGs instead.
  if (p->gnd.n_free < 16 * (int64_t)S) o.indep = true;
  reff_status rs = ensure(p->ws.out, (cols.size() + 1) * sizeof(double));
  if (rs != REFF_OK) return rs;
  double* res_dev = (double*)p->ws.out.p;
  std::vector<StackInfo> stacks{
      StackInfo{0, p->n, p->plane, p->nx, 0, (int32_t)p->gnd.n_slots}};
  std::vector<BlockJob> jobs;
  deal_blocks(cols, 0, 0, jobs, o.brhs);
  std::vector<BlockResult> br;
  reff_status solve_rs = run_blocks(p->ws, p->gnd, stacks, jobs, res_dev, o, br, st);
  if (solve_rs != REFF_OK && solve_rs != REFF_ERR_NO_CONVERGENCE) return solve_rs;
  add_stats(st, br, 0, br.size());
  rs = write_out(p->ws, res_dev, (int64_t)cols.size(), map, R_out, o.out_dev, o.stream);
  if (rs != REFF_OK) return rs;
  if (st)
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (solve_rs == REFF_ERR_NO_CONVERGENCE)
    return fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached; R_out holds lower bounds");
  return REFF_OK;
}

reff_status reff_query_pairs(reff_pdn p, const int64_t* a, int64_t m, const int64_t* b,
                             int64_t n, reff_pair_mode mode, double* R_out,
                             const reff_solve_opts* opts, reff_solve_stats* st) {
  g_err.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  if (m < 0 || n < 0) return fail(REFF_ERR_INVALID_ARG, "m, n must be >= 0");
  if ((m > 0 && !a) || (n > 0 && !b)) return fail(REFF_ERR_INVALID_ARG, "NULL node list");
  if (m * n > 0 && !R_out) return fail(REFF_ERR_INVALID_ARG, "R_out is NULL");
  if (mode != REFF_PAIRS_GROUNDED && mode != REFF_PAIRS_FLOATING)
    return fail(REFF_ERR_INVALID_ARG, "unknown pair mode");
  Opts o;
  reff_status s = parse_opts(opts, o);
  if (s != REFF_OK) return s;
  if (o.cheb_auto) o.cheb = auto_cheb_degree(std::max<int64_t>(p->nx, p->ny));
  for (int64_t i = 0; i < m; ++i)
    if (a[i] < 0 || a[i] >= p->n) return fail(REFF_ERR_INVALID_ARG, "node id out of range in a");
  for (int64_t j = 0; j < n; ++j)
    if (b[j] < 0 || b[j] >= p->n) return fail(REFF_ERR_INVALID_ARG, "node id out of range in b");
  if (st) std::memset(st, 0, sizeof(*st));
  HIPCHK(hipSetDevice(p->device));
  // FLOATING: Eq. 2 on the whole stack; ground one reference node (the first
  // pad) instead of every pad -- R(a,b) does not depend on that choice.
  CoefSet* cs = &p->gnd;
  if (mode == REFF_PAIRS_FLOATING) {
    if (!p->flt.ready) {
      p->flt_ref = (int64_t)p->pad_xy[1] * p->nx + p->pad_xy[0];
      s = make_coefset(p, std::vector<int64_t>{p->flt_ref}, p->flt);
      if (s != REFF_OK) return s;
    }
    cs = &p->flt;
  }
  if (cs->n_free < 16 * (int64_t)S) o.indep = true;
  // Distinct non-grounded endpoints, each solved once (m + n solves).
  std::vector<int64_t> cols(a, a + m);
  cols.insert(cols.end(), b, b + n);
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  cols.erase(std::remove_if(cols.begin(), cols.end(),
                            [&](int64_t v) { return cs->grounded[(size_t)v] != 0; }),
             cols.end());
  const int64_t U = (int64_t)cols.size();
  reff_status solve_rs = REFF_OK;
  // Endpoint index of every a_i / b_j (-1: grounded, K row and column 0).
  auto idx = [&](int64_t v) -> int64_t {
    auto it = std::lower_bound(cols.begin(), cols.end(), v);
    return (it != cols.end() && *it == v) ? (int64_t)(it - cols.begin()) : -1;
  };
  std::vector<int64_t> ia((size_t)m), ib((size_t)n);
  for (int64_t i = 0; i < m; ++i) ia[(size_t)i] = idx(a[i]);
  for (int64_t j = 0; j < n; ++j) ib[(size_t)j] = idx(b[j]);
  const int64_t nn = p->n;
  std::vector<StackInfo> stacks{StackInfo{0, nn, p->plane, p->nx, 0, (int32_t)cs->n_slots}};
  std::vector<BlockJob> jobs;
  if (U > 0) deal_blocks(cols, 0, 0, jobs, o.brhs);
  const int64_t nblk = (int64_t)jobs.size();
  std::vector<int32_t> blk_of((size_t)std::max<int64_t>(U, 1)), col_of((size_t)std::max<int64_t>(U, 1));
  for (int64_t bb = 0; bb < nblk; ++bb)
    for (int k = 0; k < jobs[(size_t)bb].ncol; ++k) {
      blk_of[(size_t)jobs[(size_t)bb].pos[k]] = (int32_t)bb;
      col_of[(size_t)jobs[(size_t)bb].pos[k]] = k;
    }
  // device tables: endpoint nodes, maps, gathered rows, cross Grams, output
  struct Local {
    std::vector<void*> ptrs;
    ~Local() {
      for (void* q : ptrs) (void)hipFree(q);
    }
    hipError_t get(void** out, size_t bytes) {
      hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 8));
      if (e == hipSuccess) ptrs.push_back(*out);
      return e;
    }
  } loc;
  void *d_nodes, *d_ia, *d_ib, *d_aid, *d_bid, *d_blk, *d_col, *d_rows, *d_cg, *d_out;
  HIPCHK(loc.get(&d_nodes, (size_t)U * sizeof(int64_t)));
  HIPCHK(loc.get(&d_ia, (size_t)m * sizeof(int64_t)));
  HIPCHK(loc.get(&d_ib, (size_t)n * sizeof(int64_t)));
  HIPCHK(loc.get(&d_aid, (size_t)m * sizeof(int64_t)));
  HIPCHK(loc.get(&d_bid, (size_t)n * sizeof(int64_t)));
  HIPCHK(loc.get(&d_blk, (size_t)U * sizeof(int32_t)));
  HIPCHK(loc.get(&d_col, (size_t)U * sizeof(int32_t)));
  HIPCHK(loc.get(&d_rows, (size_t)nblk * U * S * sizeof(double)));
  HIPCHK(loc.get(&d_cg, (size_t)nblk * nblk * S * S * sizeof(double)));
  HIPCHK(loc.get(&d_out, o.out_dev ? 8 : (size_t)(m * n) * sizeof(double)));
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, o.stream) : hipSuccess;
  };
  HIPCHK(up(d_nodes, cols.data(), (size_t)U * sizeof(int64_t)));
  HIPCHK(up(d_ia, ia.data(), (size_t)m * sizeof(int64_t)));
  HIPCHK(up(d_ib, ib.data(), (size_t)n * sizeof(int64_t)));
  HIPCHK(up(d_aid, a, (size_t)m * sizeof(int64_t)));
  HIPCHK(up(d_bid, b, (size_t)n * sizeof(int64_t)));
  HIPCHK(up(d_blk, blk_of.data(), (size_t)U * sizeof(int32_t)));
  HIPCHK(up(d_col, col_of.data(), (size_t)U * sizeof(int32_t)));
  // Solution blocks kept on the device at once: all of them when they fit
  // (every cross term exact to second order), else groups of `grp` blocks,
  // each dropped once its endpoint rows and in-group cross terms are taken.
  const size_t blk_bytes = (size_t)nn * S * sizeof(double);
  int64_t grp = std::max<int64_t>(nblk, 1);
  if (o.resident > 0) {
    grp = std::min<int64_t>(grp, o.resident);
  } else if (nblk > 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const size_t avail = fr + p->ws.xs.bytes;  // the held solution buffer is reusable
    grp = std::min<int64_t>(grp, std::max<int64_t>(1, (int64_t)(avail / 2 / blk_bytes)));
  }
  Opts og = o;
  if (grp < nblk) og.tol = std::min(o.tol, std::max(o.tol * o.tol, 1e-14));
  if (U > 0) {
    reff_status rs;
    if ((rs = ensure(p->ws.xs, (size_t)grp * blk_bytes)) != REFF_OK) return rs;
    if ((rs = ensure(p->ws.out, (size_t)(U + 1) * sizeof(double))) != REFF_OK) return rs;
    double* xs = (double*)p->ws.xs.p;
    const Coef<double> c64 = coef64(*cs);
    for (int64_t g0 = 0; g0 < nblk; g0 += grp) {
      const int64_t g1 = std::min(nblk, g0 + grp);
      std::vector<BlockJob> gj(jobs.begin() + g0, jobs.begin() + g1);
      std::vector<int64_t> xoff((size_t)(g1 - g0));
      for (int64_t bb = g0; bb < g1; ++bb) xoff[(size_t)(bb - g0)] = (bb - g0) * nn * S;
      std::vector<BlockResult> br;
      const reff_status gs =
          run_blocks(p->ws, *cs, stacks, gj, (double*)p->ws.out.p, og, br, st, xs, &xoff);
      if (gs != REFF_OK && gs != REFF_ERR_NO_CONVERGENCE) return gs;
      if (gs != REFF_OK) solve_rs = gs;
      add_stats(st, br, 0, br.size());
      // x_u[v] for every endpoint pair: the endpoint rows of each block
      for (int64_t bb = g0; bb < g1; ++bb)
        HIPCHK(launch_gather_rows(xs + (bb - g0) * nn * S, (const int64_t*)d_nodes, U,
                                  (double*)d_rows + bb * U * S, o.stream));
      // Cross terms x_u^T G x_v between (and within) the group's blocks: the
      // bilinear estimate K_uv = x_u[v] + x_v[u] - x_u^T G x_v has an error
      // that is a product of the two solution errors (second order).  The
      // group's pairs are queued on the stream; the host waits once per
      // group, before the next group's solves overwrite the blocks.
      SolveBuffers sb;
      PinnedBuf pin;
      if ((rs = single_work(p->ws, stacks[0], sb, o.stream, pin)) != REFF_OK) return rs;
      for (int64_t b1 = g0; b1 < g1; ++b1)
        for (int64_t b2 = b1; b2 < g1; ++b2) {
          HIPCHK(launch_cross_gram(c64, xs + (b1 - g0) * nn * S, xs + (b2 - g0) * nn * S, sb,
                                   o.stream));
          HIPCHK(hipMemcpyAsync((double*)d_cg + (b1 * nblk + b2) * S * S, sb.W,
                                S * S * sizeof(double), hipMemcpyDeviceToDevice, o.stream));
        }
      HIPCHK(hipStreamSynchronize(o.stream));  // the pinned tables of single_work
    }
  }
  if (m * n > 0) {
    double* dst = o.out_dev ? R_out : (double*)d_out;
    HIPCHK(launch_pairs_finish(m, n, (const int64_t*)d_ia, (const int64_t*)d_ib,
                               (const int64_t*)d_aid, (const int64_t*)d_bid,
                               (const int32_t*)d_blk, (const int32_t*)d_col,
                               (const double*)d_rows, (const double*)d_cg, U, nblk, grp,
                               dst, o.stream));
    if (!o.out_dev)
      HIPCHK(hipMemcpyAsync(R_out, d_out, (size_t)(m * n) * sizeof(double),
                            hipMemcpyDeviceToHost, o.stream));
    HIPCHK(hipStreamSynchronize(o.stream));
  }
  if (st) {
    st->n_solved = U;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (solve_rs == REFF_ERR_NO_CONVERGENCE)
    return fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached before the tolerance");
  return REFF_OK;
}

// IR drop and through-bump currents by superposition of unit-load responses
// (Eq. 4 with every bump merged into the supply node: 1/2 (R_j + R_l -
// R(j, l)) = (G^-1 e_l)_j).  The distinct free load nodes are solved 64 at a
// time; each group of solved blocks is folded into the drop and pad-current
// accumulators on the device and then dropped, so memory stays bounded by
// the group size, not by the number of loads.
reff_status reff_ir_drop(reff_pdn p, const int64_t* load_nodes, int64_t n_loads,
                         const double* load_amps, int32_t n_scen, const int64_t* nodes,
                         int64_t n_nodes, double* drop_out, double* pad_amps_out,
                         const reff_solve_opts* opts, reff_solve_stats* st) {
  g_err.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  if (n_loads < 0 || n_scen < 0) return fail(REFF_ERR_INVALID_ARG, "n_loads, n_scen must be >= 0");
  if (n_loads > 0 && n_scen > 0 && (!load_nodes || !load_amps))
    return fail(REFF_ERR_INVALID_ARG, "NULL load nodes or currents");
  if (nodes && n_nodes < 0) return fail(REFF_ERR_INVALID_ARG, "n_nodes < 0");
  const int64_t count = nodes ? n_nodes : p->n;
  if (count * (int64_t)n_scen > 0 && !drop_out) return fail(REFF_ERR_INVALID_ARG, "drop_out is NULL");
  for (int64_t i = 0; i < n_loads; ++i)
    if (load_nodes[i] < 0 || load_nodes[i] >= p->n)
      return fail(REFF_ERR_INVALID_ARG, "load node id out of range");
  for (int64_t i = 0; i < n_loads * (int64_t)n_scen; ++i)
    if (!std::isfinite(load_amps[i])) return fail(REFF_ERR_INVALID_ARG, "non-finite load current");
  if (nodes)
    for (int64_t i = 0; i < count; ++i)
      if (nodes[i] < 0 || nodes[i] >= p->n) return fail(REFF_ERR_INVALID_ARG, "node id out of range");
  Opts o;
  reff_status s = parse_opts(opts, o);
  if (s != REFF_OK) return s;
  if (o.cheb_auto) o.cheb = auto_cheb_degree(std::max<int64_t>(p->nx, p->ny));
  // Point values of a response are accurate to about the square root of the
  // energy-norm error the solver controls; the defaults are tighter than
  // those of reff_solve_diag accordingly.
  if (!opts || opts->rel_tol == 0.0) o.tol = o.mixed ? 1e-7 : 1e-12;
  if (st) std::memset(st, 0, sizeof(*st));
  HIPCHK(hipSetDevice(p->device));
  const CoefSet& cs = p->gnd;
  if (cs.n_free < 16 * (int64_t)S) o.indep = true;
  const int64_t nn = p->n;
  // distinct free load columns; per column the summed currents per scenario
  std::vector<int64_t> cols;
  for (int64_t i = 0; i < n_loads; ++i)
    if (!cs.grounded[(size_t)load_nodes[i]]) cols.push_back(load_nodes[i]);
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  const int64_t U = (int64_t)cols.size();
  std::vector<double> colamp((size_t)(U * n_scen), 0.0);
  // pad entries (descriptor order, first entry of a position only)
  const int npad = (int)(p->pad_xy.size() / 2);
  std::vector<int32_t> pad_first(npad, -1);
  std::vector<double> pad_direct((size_t)npad * n_scen, 0.0);  // loads placed on pads
  {
    std::vector<int32_t> first_at((size_t)p->plane, -1);
    for (int k = 0; k < npad; ++k) {
      const int64_t v = (int64_t)p->pad_xy[2 * k + 1] * p->nx + p->pad_xy[2 * k];
      if (first_at[(size_t)v] < 0) first_at[(size_t)v] = k;
      pad_first[k] = first_at[(size_t)v];
    }
    for (int64_t i = 0; i < n_loads; ++i) {
      const int64_t v = load_nodes[i];
      if (cs.grounded[(size_t)v]) {
        const int k = first_at[(size_t)v];
        for (int c = 0; c < n_scen; ++c)
          pad_direct[(size_t)c * npad + k] += load_amps[(size_t)c * n_loads + i];
      } else {
        const int64_t u = std::lower_bound(cols.begin(), cols.end(), v) - cols.begin();
        for (int c = 0; c < n_scen; ++c)
          colamp[(size_t)(u * n_scen + c)] += load_amps[(size_t)c * n_loads + i];
      }
    }
  }
  // weighted node rows: requested nodes (weight 1), then the pads' edges
  std::vector<int32_t> rptr(1, 0);
  std::vector<int64_t> rnode;
  std::vector<double> rwt;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t v = nodes ? nodes[i] : i;
    if (!cs.grounded[(size_t)v]) rnode.push_back(v), rwt.push_back(1.0);
    rptr.push_back((int32_t)rnode.size());
  }
  {
    std::vector<int32_t> tsv_at((size_t)p->plane, -1);
    for (size_t j = 0; j < p->tsv_xy.size() / 2; ++j)
      tsv_at[(size_t)p->tsv_xy[2 * j + 1] * p->nx + p->tsv_xy[2 * j]] = (int32_t)j;
    const int nx = p->nx, ny = p->ny;
    for (int k = 0; k < npad; ++k) {
      if (pad_first[k] == k) {
        const int x = p->pad_xy[2 * k], y = p->pad_xy[2 * k + 1];
        const int64_t v = (int64_t)y * nx + x;
        auto edge = [&](int64_t u, double g) {
          if (!cs.grounded[(size_t)u]) rnode.push_back(u), rwt.push_back(g);
        };
        if (x + 1 < nx) edge(v + 1, p->gx[(size_t)y * (nx - 1) + x]);
        if (x > 0) edge(v - 1, p->gx[(size_t)y * (nx - 1) + x - 1]);
        if (y + 1 < ny) edge(v + nx, p->gy[(size_t)y * nx + x]);
        if (y > 0) edge(v - nx, p->gy[(size_t)(y - 1) * nx + x]);
        const int32_t j = tsv_at[(size_t)v];
        if (j >= 0 && p->nt > 1) edge(v + p->plane, p->tsv_g[(size_t)j * (p->nt - 1)]);
      }
      rptr.push_back((int32_t)rnode.size());
    }
  }
  const int64_t nrows = count + npad;
  // device buffers of this call
  struct Local {
    std::vector<void*> ptrs;
    ~Local() {
      for (void* q : ptrs) (void)hipFree(q);
    }
    hipError_t get(void** out, size_t bytes) {
      hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 8));
      if (e == hipSuccess) ptrs.push_back(*out);
      return e;
    }
  } loc;
  void *d_rptr = nullptr, *d_rnode = nullptr, *d_rw = nullptr, *d_acc = nullptr, *d_amp = nullptr;
  HIPCHK(loc.get(&d_rptr, rptr.size() * sizeof(int32_t)));
  HIPCHK(loc.get(&d_rnode, rnode.size() * sizeof(int64_t)));
  HIPCHK(loc.get(&d_rw, rwt.size() * sizeof(double)));
  HIPCHK(loc.get(&d_acc, (size_t)nrows * n_scen * sizeof(double)));
  HIPCHK(hipMemcpyAsync(d_rptr, rptr.data(), rptr.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                        o.stream));
  if (!rnode.empty()) {
    HIPCHK(hipMemcpyAsync(d_rnode, rnode.data(), rnode.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(d_rw, rwt.data(), rwt.size() * sizeof(double), hipMemcpyHostToDevice,
                          o.stream));
  }
  HIPCHK(launch_zero_x((double*)d_acc, nrows * n_scen, o.stream));
  reff_status solve_rs = REFF_OK;
  if (U > 0 && n_scen > 0) {
    std::vector<StackInfo> stacks{StackInfo{0, nn, p->plane, p->nx, 0, (int32_t)cs.n_slots}};
    std::vector<BlockJob> jobs;
    deal_blocks(cols, 0, 0, jobs, o.brhs);
    const int64_t nblk = (int64_t)jobs.size();
    // blocks per group: solution vectors of a group within 8 GB
    const int64_t per = std::max<int64_t>(
        1, std::min<int64_t>(nblk, (int64_t)(8e9 / ((double)nn * S * sizeof(double)))));
    reff_status rs;
    if ((rs = ensure(p->ws.xs, (size_t)per * nn * S * sizeof(double))) != REFF_OK) return rs;
    if ((rs = ensure(p->ws.out, (size_t)(U + 1) * sizeof(double))) != REFF_OK) return rs;
    HIPCHK(loc.get(&d_amp, (size_t)per * S * n_scen * sizeof(double)));
    double* xs = (double*)p->ws.xs.p;
    std::vector<double> hamp((size_t)per * S * n_scen);
    for (int64_t g0 = 0; g0 < nblk; g0 += per) {
      const int64_t g1 = std::min(nblk, g0 + per);
      std::vector<BlockJob> gj(jobs.begin() + g0, jobs.begin() + g1);
      std::vector<int64_t> xoff((size_t)(g1 - g0));
      for (int64_t bb = 0; bb < g1 - g0; ++bb) xoff[(size_t)bb] = bb * nn * S;
      std::vector<BlockResult> br;
      rs = run_blocks(p->ws, cs, stacks, gj, (double*)p->ws.out.p, o, br, st, xs, &xoff);
      if (rs != REFF_OK && rs != REFF_ERR_NO_CONVERGENCE) return rs;
      if (rs == REFF_ERR_NO_CONVERGENCE) solve_rs = rs;
      add_stats(st, br, 0, br.size());
      std::fill(hamp.begin(), hamp.end(), 0.0);
      for (int64_t bb = 0; bb < g1 - g0; ++bb) {
        const BlockJob& jb = gj[(size_t)bb];
        for (int k = 0; k < jb.ncol; ++k)
          for (int c = 0; c < n_scen; ++c)
            hamp[(size_t)((bb * S + k) * n_scen + c)] = colamp[(size_t)(jb.pos[k] * n_scen + c)];
      }
      HIPCHK(hipMemcpyAsync(d_amp, hamp.data(), (size_t)(g1 - g0) * S * n_scen * sizeof(double),
                            hipMemcpyHostToDevice, o.stream));
      for (int64_t bb = 0; bb < g1 - g0; ++bb)
        HIPCHK(launch_rows_times_loads(xs + bb * nn * S, (const int32_t*)d_rptr,
                                       (const int64_t*)d_rnode, (const double*)d_rw, nrows,
                                       (const double*)d_amp + bb * S * n_scen, n_scen,
                                       (double*)d_acc, nrows, o.stream));
      HIPCHK(hipStreamSynchronize(o.stream));  // hamp is refilled by the next group
    }
  }
  // drop: rows 0 .. count-1 of each scenario's accumulator row
  if (count > 0 && n_scen > 0) {
    if (o.out_dev) {
      HIPCHK(hipMemcpy2DAsync(drop_out, count * sizeof(double), d_acc, nrows * sizeof(double),
                              count * sizeof(double), n_scen, hipMemcpyDeviceToDevice, o.stream));
    } else {
      HIPCHK(hipMemcpy2DAsync(drop_out, count * sizeof(double), d_acc, nrows * sizeof(double),
                              count * sizeof(double), n_scen, hipMemcpyDeviceToHost, o.stream));
    }
  }
  if (pad_amps_out && npad > 0 && n_scen > 0) {
    std::vector<double> pa((size_t)npad * n_scen);
    HIPCHK(hipMemcpy2DAsync(pa.data(), npad * sizeof(double), (double*)d_acc + count,
                            nrows * sizeof(double), npad * sizeof(double), n_scen,
                            hipMemcpyDeviceToHost, o.stream));
    HIPCHK(hipStreamSynchronize(o.stream));
    for (int c = 0; c < n_scen; ++c)
      for (int k = 0; k < npad; ++k)
        pad_amps_out[(size_t)c * npad + k] =
            pad_first[k] == k ? pa[(size_t)c * npad + k] + pad_direct[(size_t)c * npad + k] : 0.0;
  }
  HIPCHK(hipStreamSynchronize(o.stream));
  if (st) {
    st->n_solved = U;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (solve_rs == REFF_ERR_NO_CONVERGENCE)
    return fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached before the tolerance");
  return REFF_OK;
}

// Screening of a batch with the learned model: predict every plan's map,
// solve a seeded fraction of each plan's requested free nodes, and fall back
// to solving all requested nodes of a plan whose checked relative error
// exceeds fb_err.  Solved values replace predictions wherever they exist.
static reff_status screen_plans(reff_surrogate sg, const reff_pdn_desc* plans, int32_t n_plans,
                                Workspace& ws, const CoefSet& cs,
                                const std::vector<StackInfo>& stacks,
                                const std::vector<std::vector<int64_t>>& cols,
                                const std::vector<std::vector<int64_t>>& maps,
                                double* const* R_out, const Opts& o, double spot_frac,
                                double fb_err, int calibrate, reff_solve_stats* per_plan,
                                std::chrono::steady_clock::time_point t0) {
  const int64_t per = stacks[0].n;  // every plan has the model's geometry
  const int64_t plane = stacks[0].plane;
  reff_status rs = ensure(ws.xs, (size_t)n_plans * per * sizeof(double));
  if (rs != REFF_OK) return rs;
  rs = reffsg::predict_device(sg, plans, n_plans, (double*)ws.xs.p, o.stream);
  if (rs != REFF_OK) return rs;
  std::vector<double> pred((size_t)(n_plans * per));
  HIPCHK(hipMemcpyAsync(pred.data(), ws.xs.p, pred.size() * sizeof(double), hipMemcpyDeviceToHost,
                        o.stream));
  HIPCHK(hipStreamSynchronize(o.stream));
  // values[i][j] = result for cols[i][j]
  std::vector<std::vector<double>> values((size_t)n_plans);
  std::vector<std::vector<int64_t>> spot_idx((size_t)n_plans);  // indices into cols[i]
  std::vector<BlockJob> sjobs;
  std::vector<size_t> sjob0((size_t)n_plans + 1);
  std::vector<int64_t> spos0((size_t)n_plans);
  int64_t spos = 0;
  for (int32_t i = 0; i < n_plans; ++i) {
    const auto& c = cols[(size_t)i];
    values[(size_t)i].resize(c.size());
    for (size_t j = 0; j < c.size(); ++j)
      values[(size_t)i][j] = pred[(size_t)(i * per + c[j])];
    sjob0[(size_t)i] = sjobs.size();
    spos0[(size_t)i] = spos;
    if (c.empty()) continue;
    const size_t k = std::max<size_t>(
        1, std::min(c.size(), (size_t)std::ceil(spot_frac * (double)c.size() - 1e-9)));
    std::vector<int64_t> order(c.size());
    std::iota(order.begin(), order.end(), 0);
    std::mt19937_64 rng(0x5eedull * 1000003ull + (uint64_t)i);
    std::shuffle(order.begin(), order.end(), rng);
    order.resize(k);
    spot_idx[(size_t)i] = order;
    std::vector<int64_t> ids(k);
    for (size_t j = 0; j < k; ++j) ids[j] = c[(size_t)order[j]];
    deal_blocks(ids, i, spos, sjobs, o.brhs);
    spos += (int64_t)k;
  }
  sjob0[(size_t)n_plans] = sjobs.size();
  std::vector<BlockResult> sbr, fbr;
  reff_solve_stats agg;
  std::memset(&agg, 0, sizeof(agg));
  if ((rs = ensure(ws.out, (size_t)(spos + 1) * sizeof(double))) != REFF_OK) return rs;
  reff_status solve_rs = run_blocks(ws, cs, stacks, sjobs, (double*)ws.out.p, o, sbr, &agg);
  if (solve_rs != REFF_OK && solve_rs != REFF_ERR_NO_CONVERGENCE) return solve_rs;
  std::vector<double> spot((size_t)spos);
  if (spos > 0)
    HIPCHK(hipMemcpyAsync(spot.data(), ws.out.p, (size_t)spos * sizeof(double),
                          hipMemcpyDeviceToHost, o.stream));
  HIPCHK(hipStreamSynchronize(o.stream));
  std::vector<double> err((size_t)n_plans, 0.0);
  std::vector<char> fallback((size_t)n_plans, 0);
  std::vector<BlockJob> fjobs;
  std::vector<size_t> fjob0((size_t)n_plans + 1);
  std::vector<int64_t> fpos0((size_t)n_plans, -1);
  int64_t fpos = 0;
  const int nt = (int)(per / plane);
  for (int32_t i = 0; i < n_plans; ++i) {
    const auto& si = spot_idx[(size_t)i];
    const auto& c = cols[(size_t)i];
    // With calibration, the checked nodes at even positions of the seeded
    // order fit one log-offset per tier (the mean of log(solved / predicted)
    // there; the overall mean on a tier with none), the prediction of every
    // requested node is scaled by it, and the odd positions check the
    // scaled prediction.  Without, every checked node checks.
    const bool cal = calibrate && si.size() >= 2;
    if (cal) {
      std::vector<double> sum((size_t)nt, 0.0);
      std::vector<int> num((size_t)nt, 0);
      double all = 0.0;
      int nall = 0;
      for (size_t j = 0; j < si.size(); j += 2) {
        const double r = spot[(size_t)(spos0[(size_t)i] + (int64_t)j)];
        const double v = values[(size_t)i][(size_t)si[j]];
        if (!(r > 0.0) || !(v > 0.0)) continue;
        const int t = (int)(c[(size_t)si[j]] / plane);
        const double d = std::log(r / v);
        sum[(size_t)t] += d, num[(size_t)t] += 1;
        all += d, nall += 1;
      }
      std::vector<double> scale((size_t)nt, 1.0);
      for (int t = 0; t < nt; ++t)
        scale[(size_t)t] = std::exp(num[(size_t)t] ? sum[(size_t)t] / num[(size_t)t]
                                                   : (nall ? all / nall : 0.0));
      for (size_t j = 0; j < c.size(); ++j) values[(size_t)i][j] *= scale[(size_t)(c[j] / plane)];
    }
    for (size_t j = 0; j < si.size(); ++j) {
      const double r = spot[(size_t)(spos0[(size_t)i] + (int64_t)j)];
      double& v = values[(size_t)i][(size_t)si[j]];
      if (!cal || (j & 1)) err[(size_t)i] = std::max(err[(size_t)i], std::fabs(v - r) / r);
      v = r;
    }
    fallback[(size_t)i] = !(err[(size_t)i] <= fb_err);
    fjob0[(size_t)i] = fjobs.size();
    if (fallback[(size_t)i] && !cols[(size_t)i].empty()) {
      fpos0[(size_t)i] = fpos;
      deal_blocks(cols[(size_t)i], i, fpos, fjobs, o.brhs);
      fpos += (int64_t)cols[(size_t)i].size();
    }
  }
  fjob0[(size_t)n_plans] = fjobs.size();
  if (!fjobs.empty()) {
    if ((rs = ensure(ws.out, (size_t)(fpos + 1) * sizeof(double))) != REFF_OK) return rs;
    reff_status frs = run_blocks(ws, cs, stacks, fjobs, (double*)ws.out.p, o, fbr, &agg);
    if (frs != REFF_OK && frs != REFF_ERR_NO_CONVERGENCE) return frs;
    if (frs == REFF_ERR_NO_CONVERGENCE) solve_rs = frs;
    std::vector<double> fres((size_t)fpos);
    HIPCHK(hipMemcpyAsync(fres.data(), ws.out.p, (size_t)fpos * sizeof(double),
                          hipMemcpyDeviceToHost, o.stream));
    HIPCHK(hipStreamSynchronize(o.stream));
    for (int32_t i = 0; i < n_plans; ++i)
      if (fpos0[(size_t)i] >= 0)
        for (size_t j = 0; j < cols[(size_t)i].size(); ++j)
          values[(size_t)i][j] = fres[(size_t)(fpos0[(size_t)i] + (int64_t)j)];
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int32_t i = 0; i < n_plans; ++i) {
    const auto& mp = maps[(size_t)i];
    std::vector<double> outv(mp.size());
    for (size_t j = 0; j < mp.size(); ++j)
      outv[j] = mp[j] >= 0 ? values[(size_t)i][(size_t)mp[j]] : 0.0;
    if (!outv.empty()) {
      if (o.out_dev) {
        HIPCHK(hipMemcpyAsync(R_out[i], outv.data(), outv.size() * sizeof(double),
                              hipMemcpyHostToDevice, o.stream));
        HIPCHK(hipStreamSynchronize(o.stream));
      } else {
        std::memcpy(R_out[i], outv.data(), outv.size() * sizeof(double));
      }
    }
    if (per_plan) {
      reff_solve_stats& ps = per_plan[i];
      std::memset(&ps, 0, sizeof(ps));
      ps.n_solved = (int64_t)spot_idx[(size_t)i].size() +
                    (fallback[(size_t)i] ? (int64_t)cols[(size_t)i].size() : 0);
      add_stats(&ps, sbr, sjob0[(size_t)i], sjob0[(size_t)i + 1]);
      add_stats(&ps, fbr, fjob0[(size_t)i], fjob0[(size_t)i + 1]);
      ps.seconds = secs;
      ps.screened = fallback[(size_t)i] ? 0 : 1;
      ps.spot_max_rel_err = err[(size_t)i];
    }
  }
  if (solve_rs == REFF_ERR_NO_CONVERGENCE)
    return fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached; R_out holds lower bounds");
  return REFF_OK;
}

reff_status reff_batch_plans(const reff_pdn_desc* plans, int32_t n_plans,
                             const int64_t* const* nodes, const int64_t* n_nodes,
                             double* const* R_out, const reff_batch_opts* opts,
                             reff_solve_stats* per_plan) {
  g_err.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (n_plans < 0) return fail(REFF_ERR_INVALID_ARG, "n_plans < 0");
  if (n_plans == 0) return REFF_OK;
  if (!plans || !R_out) return fail(REFF_ERR_INVALID_ARG, "NULL plans or R_out");
  Opts o;
  reff_status s = parse_opts(opts ? &opts->solve : nullptr, o);
  if (s != REFF_OK) return s;
  if (o.cheb_auto && plans) {
    int64_t side = 0;
    for (int32_t i = 0; i < n_plans; ++i)
      side = std::max<int64_t>(side, std::max(plans[i].nx, plans[i].ny));
    o.cheb = auto_cheb_degree(side);
  }
  o.tune_db = opts ? opts->tune_db : nullptr;
  reff_surrogate sg = opts ? (reff_surrogate)opts->surrogate : nullptr;
  double spot_frac = 0.01, fb_err = 1e-2;
  int calibrate = 0;
  if (sg) {
    if (opts->calibrate != 0 && opts->calibrate != 1)
      return fail(REFF_ERR_INVALID_ARG, "calibrate must be 0 or 1");
    calibrate = opts->calibrate;
    if (opts->spot_frac != 0.0) spot_frac = opts->spot_frac;
    if (opts->fallback_rel_err != 0.0) fb_err = opts->fallback_rel_err;
    if (!(spot_frac > 0.0 && spot_frac <= 1.0))
      return fail(REFF_ERR_INVALID_ARG, "spot_frac must be in (0, 1]");
    if (!(fb_err > 0.0) || !std::isfinite(fb_err))
      return fail(REFF_ERR_INVALID_ARG, "fallback_rel_err must be finite and > 0");
  }
  // Validate every plan (and its node list) before any device work.
  std::vector<const reff_pdn_desc*> ds((size_t)n_plans);
  std::vector<std::vector<int64_t>> gnds((size_t)n_plans);
  std::vector<StackInfo> stacks((size_t)n_plans);
  {
    // descriptors checked on host threads; the first bad plan is reported
    std::vector<reff_status> vs((size_t)n_plans, REFF_OK);
    std::vector<std::string> vm((size_t)n_plans);
    parallel_for((size_t)n_plans, [&](size_t i) {
      vs[i] = validate_desc(&plans[i]);
      if (vs[i] != REFF_OK) vm[i] = g_err;  // this thread's message
    });
    for (int32_t i = 0; i < n_plans; ++i)
      if (vs[(size_t)i] != REFF_OK)
        return fail(vs[(size_t)i], "plan " + std::to_string(i) + ": " + vm[(size_t)i]);
  }
  for (int32_t i = 0; i < n_plans; ++i) {
    ds[(size_t)i] = &plans[i];
    for (int32_t j = 0; j < plans[i].n_pads; ++j)
      gnds[(size_t)i].push_back((int64_t)plans[i].pad_xy[2 * j + 1] * plans[i].nx +
                                plans[i].pad_xy[2 * j]);
    const int64_t pl = (int64_t)plans[i].nx * plans[i].ny;
    stacks[(size_t)i] = StackInfo{0, pl * plans[i].n_tiers, pl, plans[i].nx};
    const bool given = nodes && nodes[i];
    if (given && (!n_nodes || n_nodes[i] < 0))
      return fail(REFF_ERR_INVALID_ARG, "plan " + std::to_string(i) + ": bad n_nodes");
    const int64_t cnt = given ? n_nodes[i] : stacks[(size_t)i].n;
    if (cnt > 0 && !R_out[i]) return fail(REFF_ERR_INVALID_ARG, "plan " + std::to_string(i) + ": R_out NULL");
    if (sg && !reffsg::geometry_matches(sg, &plans[i]))
      return fail(REFF_ERR_INVALID_ARG,
                  "plan " + std::to_string(i) + " does not match the surrogate's geometry");
    if (given)
      for (int64_t k = 0; k < cnt; ++k)
        if (nodes[i][k] < 0 || nodes[i][k] >= stacks[(size_t)i].n)
          return fail(REFF_ERR_INVALID_ARG, "plan " + std::to_string(i) + ": node id " +
                                                std::to_string(nodes[i][k]) + " out of range");
  }
  // Connectivity of every plan is checked (host breadth-first search) before
  // the first upload.
  // All plans' coefficients in one concatenated set (one upload).
  CoefSet cs;
  std::vector<void*> owned;
  struct Free {
    std::vector<void*>& v;
    ~Free() {
      for (void* q : v) (void)hipFree(q);
    }
  } free_owned{owned};
  std::vector<int64_t> cbase;
  std::vector<int32_t> slot0;
  s = make_coefset_multi(ds, gnds, cs, cbase, owned, &slot0);
  if (s != REFF_OK) return s;
  std::vector<std::vector<int64_t>> cols((size_t)n_plans), maps((size_t)n_plans);
  std::vector<BlockJob> jobs;
  std::vector<size_t> job0((size_t)n_plans + 1);
  int64_t pos0 = 0;
  std::vector<int64_t> res0((size_t)n_plans);
  bool any_small = false;
  for (int32_t i = 0; i < n_plans; ++i) {
    stacks[(size_t)i].cbase = cbase[(size_t)i];
    stacks[(size_t)i].slot_begin = slot0[(size_t)i];
    stacks[(size_t)i].slot_end =
        i + 1 < n_plans ? slot0[(size_t)i + 1] : (int32_t)cs.n_slots;
    const bool given = nodes && nodes[i];
    const int64_t cnt = given ? n_nodes[i] : stacks[(size_t)i].n;
    std::vector<uint8_t> g(cs.grounded.begin() + cbase[(size_t)i],
                           cs.grounded.begin() + cbase[(size_t)i] + stacks[(size_t)i].n);
    s = columns_of(given ? nodes[i] : nullptr, cnt, stacks[(size_t)i].n, g, cols[(size_t)i],
                   maps[(size_t)i]);
    if (s != REFF_OK) return fail(s, "plan " + std::to_string(i) + ": " + g_err);
    int64_t nfree = 0;
    for (uint8_t f : g) nfree += f ? 0 : 1;
    if (nfree < 16 * (int64_t)S) any_small = true;
    job0[(size_t)i] = jobs.size();
    res0[(size_t)i] = pos0;
    deal_blocks(cols[(size_t)i], i, pos0, jobs, o.brhs);
    pos0 += (int64_t)cols[(size_t)i].size();
  }
  job0[(size_t)n_plans] = jobs.size();
  if (any_small) o.indep = true;
  Workspace ws;
  struct Rel {
    Workspace& w;
    ~Rel() { w.release(); }
  } rel{ws};
  if (sg)
    return screen_plans(sg, plans, n_plans, ws, cs, stacks, cols, maps, R_out, o, spot_frac,
                        fb_err, calibrate, per_plan, t0);
  reff_status rs = ensure(ws.out, (size_t)(pos0 + 1) * sizeof(double));
  if (rs != REFF_OK) return rs;
  std::vector<BlockResult> br;
  reff_solve_stats agg;
  std::memset(&agg, 0, sizeof(agg));
  reff_status solve_rs = run_blocks(ws, cs, stacks, jobs, (double*)ws.out.p, o, br, &agg);
  if (solve_rs != REFF_OK && solve_rs != REFF_ERR_NO_CONVERGENCE) return solve_rs;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int32_t i = 0; i < n_plans; ++i) {
    rs = write_out(ws, (double*)ws.out.p + res0[(size_t)i], (int64_t)cols[(size_t)i].size(),
                   maps[(size_t)i], R_out[i], o.out_dev, o.stream);
    if (rs != REFF_OK) return rs;
    if (per_plan) {
      reff_solve_stats& ps = per_plan[i];
      std::memset(&ps, 0, sizeof(ps));
      ps.n_solved = (int64_t)cols[(size_t)i].size();
      add_stats(&ps, br, job0[(size_t)i], job0[(size_t)i + 1]);
      ps.seconds = secs;
      if (i == 0)
        for (int k = 0; k < NEV / 2; ++k) {
          ps.kernel_ms[k] = agg.kernel_ms[k];
          ps.kernel_launches[k] = agg.kernel_launches[k];
          ps.kernel_rows[k] = agg.kernel_rows[k];
        }
    }
  }
  if (solve_rs == REFF_ERR_NO_CONVERGENCE)
    return fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached; R_out holds lower bounds");
  return REFF_OK;
}

}  // extern "C"
