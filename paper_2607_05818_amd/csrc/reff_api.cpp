// Host runtime behind the C ABI of include/reff.h: argument validation,
// connectivity check, stencil-coefficient build and upload, workspace
// management, and the block-PCG driver that sequences the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <deque>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "reff_internal.h"

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

// Host-side stencil coefficients in float64 (see Coef in reff_internal.h).
struct HostCoef {
  std::vector<double> d, cE, cN, up, dn;
  std::vector<int32_t> slot;
  std::vector<uint8_t> is_pad;
};

reff_status build_host(const reff_pdn_desc* ds, HostCoef& h) {
  const int64_t nt = ds->n_tiers, nx = ds->nx, ny = ds->ny;
  const int64_t plane = nx * ny, n = nt * plane;
  h.d.assign((size_t)n, 0.0);
  h.cE.assign((size_t)n, 0.0);
  h.cN.assign((size_t)n, 0.0);
  h.slot.assign((size_t)n, -1);
  h.is_pad.assign((size_t)n, 0);
  for (int32_t j = 0; j < ds->n_pads; ++j)
    h.is_pad[(size_t)(ds->pad_xy[2 * j + 1] * nx + ds->pad_xy[2 * j])] = 1;
  auto edge = [&](int64_t u, int64_t v, double g, double* cu) {
    const bool fu = !h.is_pad[(size_t)u], fv = !h.is_pad[(size_t)v];
    if (fu) h.d[(size_t)u] += g;
    if (fv) h.d[(size_t)v] += g;
    if (fu && fv && cu) *cu = g;
  };
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t v = t * plane + y * nx + x;
        if (x + 1 < nx) edge(v, v + 1, ds->gx[(t * ny + y) * (nx - 1) + x], &h.cE[(size_t)v]);
        if (y + 1 < ny) edge(v, v + nx, ds->gy[(t * (ny - 1) + y) * nx + x], &h.cN[(size_t)v]);
      }
  // TSV side list: one slot per (column, tier) node.
  h.up.clear();
  h.dn.clear();
  for (int32_t j = 0; j < ds->n_tsv; ++j) {
    const int64_t x = ds->tsv_xy[2 * j], y = ds->tsv_xy[2 * j + 1];
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t v = t * plane + y * nx + x;
      double gu = 0.0, gd = 0.0;
      if (t + 1 < nt) {
        const double g = ds->tsv_g[j * (nt - 1) + t];
        const bool fu = !h.is_pad[(size_t)v], fv = !h.is_pad[(size_t)(v + plane)];
        if (fu) h.d[(size_t)v] += g;
        if (fu && fv) gu = g;
      }
      if (t > 0) {
        const double g = ds->tsv_g[j * (nt - 1) + t - 1];
        const bool fu = !h.is_pad[(size_t)v], fv = !h.is_pad[(size_t)(v - plane)];
        if (fu) h.d[(size_t)v] += g;
        if (fu && fv) gd = g;
      }
      h.slot[(size_t)v] = (int32_t)h.up.size();
      h.up.push_back(gu);
      h.dn.push_back(gd);
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (h.is_pad[(size_t)v]) h.d[(size_t)v] = 1.0;
  // Connectivity: breadth-first search from the pads over all resistors.
  std::vector<uint8_t> seen((size_t)n, 0);
  std::vector<int32_t> col((size_t)plane, -1);
  for (int32_t j = 0; j < ds->n_tsv; ++j) col[(size_t)(ds->tsv_xy[2 * j + 1] * nx + ds->tsv_xy[2 * j])] = j;
  std::deque<int64_t> q;
  for (int64_t v = 0; v < plane; ++v)
    if (h.is_pad[(size_t)v]) {
      seen[(size_t)v] = 1;
      q.push_back(v);
    }
  int64_t reached = (int64_t)q.size();
  while (!q.empty()) {
    const int64_t v = q.front();
    q.pop_front();
    const int64_t t = v / plane, rem = v % plane, y = rem / nx, x = rem % nx;
    int64_t nb[6];
    int k = 0;
    if (x > 0) nb[k++] = v - 1;
    if (x + 1 < nx) nb[k++] = v + 1;
    if (y > 0) nb[k++] = v - nx;
    if (y + 1 < ny) nb[k++] = v + nx;
    if (col[(size_t)rem] >= 0) {
      if (t > 0) nb[k++] = v - plane;
      if (t + 1 < nt) nb[k++] = v + plane;
    }
    for (int i = 0; i < k; ++i)
      if (!seen[(size_t)nb[i]]) {
        seen[(size_t)nb[i]] = 1;
        ++reached;
        q.push_back(nb[i]);
      }
  }
  if (reached != n)
    return fail(REFF_ERR_DISCONNECTED, std::to_string(n - reached) +
                                           " node(s) have no resistive path to a pad");
  return REFF_OK;
}

template <typename T>
reff_status upload(const std::vector<double>& src, T** dst, std::vector<void*>& owned) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  const size_t bytes = std::max<size_t>(1, tmp.size()) * sizeof(T);
  HIPCHK(hipMalloc((void**)dst, bytes));
  owned.push_back(*dst);
  if (!tmp.empty()) HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
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

template <typename T>
Coef<T> coef_of(const reff_pdn_t* p);

template <>
Coef<double> coef_of<double>(const reff_pdn_t* p) {
  Coef<double> c{p->d64, p->dinv64, p->cE64, p->cN64, p->slot, p->up64, p->dn64,
                 p->n,   p->nx,     p->plane};
  return c;
}
template <>
Coef<float> coef_of<float>(const reff_pdn_t* p) {
  Coef<float> c{p->d32, p->dinv32, p->cE32, p->cN32, p->slot, p->up32, p->dn32,
                p->n,   p->nx,     p->plane};
  return c;
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
};

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
  if (o->block_rhs != 0 && o->block_rhs != S)
    return fail(REFF_ERR_UNSUPPORTED, "block_rhs must be 0 or 64");
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
  out.timing = o->timing == 1;
  return REFF_OK;
}

// Pinned host staging for the per-block small transfers.
struct Pinned {
  int64_t* tgt = nullptr;
  int64_t* pos = nullptr;
  int32_t* flags = nullptr;
  double* est = nullptr;
  ~Pinned() {
    if (tgt) (void)hipHostFree(tgt);
    if (pos) (void)hipHostFree(pos);
    if (flags) (void)hipHostFree(flags);
    if (est) (void)hipHostFree(est);
  }
};

// Solve the unit-current columns for the free nodes `cols` (distinct, all
// free), writing R estimates of column i into res_dev[i].
reff_status solve_columns(reff_pdn_t* p, const std::vector<int64_t>& cols, double* res_dev,
                          const Opts& o, reff_solve_stats* st) {
  const int64_t n = p->n;
  const bool fp32 = o.mixed;
  const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
  const size_t vec = (size_t)n * S * tsz;
  const int G = grid_for(n);
  reff_status rs;
  if ((rs = ensure(p->ws_Y, vec)) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_P, vec)) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_Q, vec)) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_R, vec)) != REFF_OK) return rs;
  if (o.mixed) {
    if ((rs = ensure(p->ws_D, vec)) != REFF_OK) return rs;
    if ((rs = ensure(p->ws_X, (size_t)n * S * sizeof(double))) != REFF_OK) return rs;
  }
  if ((rs = ensure(p->ws_part, (size_t)G * 4 * S * S * sizeof(double))) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_W, 4 * S * S * sizeof(double))) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_small, 4 * S * S * sizeof(double))) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_state, sizeof(BlockState))) != REFF_OK) return rs;
  if ((rs = ensure(p->ws_tgt, 2 * S * sizeof(int64_t))) != REFF_OK) return rs;

  SolveBuffers b;
  b.Y = p->ws_Y.p;
  b.P = p->ws_P.p;
  b.Q = p->ws_Q.p;
  b.R = p->ws_R.p;
  b.D = o.mixed ? p->ws_D.p : nullptr;
  b.X = o.mixed ? (double*)p->ws_X.p : nullptr;
  b.part = (double*)p->ws_part.p;
  b.W = (double*)p->ws_W.p;
  b.winv = (double*)p->ws_small.p;
  b.alpha = (double*)p->ws_small.p + S * S;
  b.delta = (double*)p->ws_small.p + 2 * S * S;
  b.Tm = (double*)p->ws_small.p + 3 * S * S;
  b.state = (BlockState*)p->ws_state.p;
  b.tgt = (int64_t*)p->ws_tgt.p;
  int64_t* pos_dev = (int64_t*)p->ws_tgt.p + S;

  Coef<double> c64 = coef_of<double>(p);
  Coef<float> c32 = coef_of<float>(p);
  const void* coef = fp32 ? (const void*)&c32 : (const void*)&c64;

  Pinned pin;
  HIPCHK(hipHostMalloc((void**)&pin.tgt, S * sizeof(int64_t)));
  HIPCHK(hipHostMalloc((void**)&pin.pos, S * sizeof(int64_t)));
  HIPCHK(hipHostMalloc((void**)&pin.flags, 4 * sizeof(int32_t)));
  HIPCHK(hipHostMalloc((void**)&pin.est, S * sizeof(double)));

  const int poll = 8;
  // Optional per-kernel timing: one set of 6 events per iteration of a poll
  // chunk, read back after the chunk's synchronisation.
  struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } evp;
  if (o.timing) {
    evp.ev.resize(6 * poll);
    for (auto& e : evp.ev) HIPCHK(hipEventCreate(&e));
  }
  const int64_t nblk = ((int64_t)cols.size() + S - 1) / S;
  // Columns are dealt to blocks in a fixed pseudo-random order: right-hand
  // sides that sit next to each other span nearly the same block Krylov
  // space, while spread-out ones give every block independent directions.
  std::vector<int64_t> order(cols.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
  std::mt19937_64 rng(0x9e3779b97f4a7c15ull);
  std::shuffle(order.begin(), order.end(), rng);
  bool any_unconv = false;
  for (int64_t blk = 0; blk < nblk; ++blk) {
    int ncol = 0;
    for (int k = 0; k < S; ++k) {
      const int64_t j = blk * S + k;
      if (j < (int64_t)cols.size()) {
        const int64_t i = order[(size_t)j];
        pin.tgt[k] = cols[(size_t)i];
        pin.pos[k] = i;
        ++ncol;
      } else {
        pin.tgt[k] = -1;
        pin.pos[k] = -1;
      }
    }
    HIPCHK(hipMemcpyAsync(b.tgt, pin.tgt, S * sizeof(int64_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(hipMemcpyAsync(pos_dev, pin.pos, S * sizeof(int64_t), hipMemcpyHostToDevice, o.stream));
    HIPCHK(launch_init_block(fp32, o.indep, coef, b, o.stream));
    if (o.mixed) HIPCHK(launch_zero_x(b.X, n * S, o.stream));
    int ir = 0;
    int it_block = 0;
    bool conv = false;
    while (true) {
      int it = 0;
      conv = false;
      while (it < o.max_iters) {
        const int k = std::min(poll, o.max_iters - it);
        for (int i = 0; i < k; ++i)
          HIPCHK(launch_iteration(fp32, o.indep, o.mixed, coef, b, n, o.tol, o.stream,
                                  o.timing ? &evp.ev[6 * i] : nullptr));
        it += k;
        HIPCHK(hipMemcpyAsync(pin.flags, &b.state->it, 2 * sizeof(int32_t),
                              hipMemcpyDeviceToHost, o.stream));
        HIPCHK(hipStreamSynchronize(o.stream));
        if (o.timing && st) {
          for (int i = 0; i < k; ++i)
            for (int kk = 0; kk < 3; ++kk) {
              float ms = 0.f;
              HIPCHK(hipEventElapsedTime(&ms, evp.ev[6 * i + 2 * kk], evp.ev[6 * i + 2 * kk + 1]));
              st->kernel_ms[kk] += ms;
              st->kernel_launches[kk] += 1;
            }
        }
        if (pin.flags[1]) {
          conv = true;
          it = pin.flags[0];
          break;
        }
      }
      it_block += it;
      ++ir;
      if (!o.mixed) break;
      HIPCHK(launch_mixed_residual(c64, c32, b, res_dev, pos_dev, o.stream));
      // One float32 solve carried to the tolerance plus the float64
      // variational correction is enough unless the inner solve stalled or
      // the tolerance is below what float32 iterates can resolve.
      const bool need_more = !conv || o.tol < 2e-6;
      if (!need_more || ir >= o.max_ir) break;
      HIPCHK(launch_restart(c32, b, o.indep, o.stream));
    }
    if (!o.mixed) HIPCHK(launch_finalize_plain(b, res_dev, pos_dev, o.stream));
    HIPCHK(hipMemcpyAsync(pin.est, b.state->est_rel, S * sizeof(double), hipMemcpyDeviceToHost,
                          o.stream));
    HIPCHK(hipStreamSynchronize(o.stream));
    if (st) {
      st->iters_max = std::max(st->iters_max, (int32_t)it_block);
      st->iters_total += it_block;
      st->ir_steps = std::max(st->ir_steps, (int32_t)ir);
      for (int k = 0; k < ncol; ++k) {
        if (std::isfinite(pin.est[k])) st->est_max_rel_err = std::max(st->est_max_rel_err, pin.est[k]);
      }
      if (!conv) {
        for (int k = 0; k < ncol; ++k)
          if (!(pin.est[k] <= CONV_SAFETY * o.tol)) st->n_unconverged++;
      }
    }
    if (!conv) any_unconv = true;
  }
  return any_unconv ? fail(REFF_ERR_NO_CONVERGENCE, "max_iters reached before the tolerance")
                    : REFF_OK;
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
  HostCoef h;
  s = build_host(d, h);
  if (s != REFF_OK) return s;
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
  p->n_slots = (int64_t)h.up.size();
  p->is_pad = h.is_pad;
  p->n_free = 0;
  for (uint8_t f : h.is_pad) p->n_free += f ? 0 : 1;
  std::vector<double> dinv(h.d.size());
  for (size_t i = 0; i < h.d.size(); ++i) dinv[i] = 1.0 / h.d[i];
  reff_status rs = REFF_OK;
  auto up = [&](const std::vector<double>& src, double** d64, float** d32) {
    if (rs != REFF_OK) return;
    rs = upload<double>(src, d64, p->extra);
    if (rs == REFF_OK) rs = upload<float>(src, d32, p->extra);
  };
  up(h.d, &p->d64, &p->d32);
  up(dinv, &p->dinv64, &p->dinv32);
  up(h.cE, &p->cE64, &p->cE32);
  up(h.cN, &p->cN64, &p->cN32);
  up(h.up, &p->up64, &p->up32);
  up(h.dn, &p->dn64, &p->dn32);
  if (rs == REFF_OK) {
    hipError_t e = hipMalloc((void**)&p->slot, h.slot.size() * sizeof(int32_t));
    if (e == hipSuccess) {
      p->extra.push_back(p->slot);
      e = hipMemcpy(p->slot, h.slot.data(), h.slot.size() * sizeof(int32_t),
                    hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) rs = fail(REFF_ERR_DEVICE, std::string("slot upload: ") + hipGetErrorString(e));
  }
  if (rs != REFF_OK) {
    reff_free_pdn(p);
    return rs;
  }
  *out = p;
  return REFF_OK;
}

void reff_free_pdn(reff_pdn p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  for (void* q : p->extra) (void)hipFree(q);
  for (DevBuf* b : {&p->ws_Y, &p->ws_P, &p->ws_Q, &p->ws_R, &p->ws_D, &p->ws_X, &p->ws_part, &p->ws_W,
                    &p->ws_small, &p->ws_state, &p->ws_tgt, &p->ws_out})
    if (b->p) (void)hipFree(b->p);
  delete p;
}

reff_status reff_solve_diag(reff_pdn p, const int64_t* nodes, int64_t n_nodes, double* R_out,
                            const reff_solve_opts* opts, reff_solve_stats* st) {
  g_err.clear();
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  Opts o;
  reff_status s = parse_opts(opts, o);
  if (s != REFF_OK) return s;
  const int64_t count = nodes ? n_nodes : p->n;
  if (nodes && n_nodes < 0) return fail(REFF_ERR_INVALID_ARG, "n_nodes < 0");
  if (count > 0 && !R_out) return fail(REFF_ERR_INVALID_ARG, "R_out is NULL");
  // Distinct free nodes in id order; map[i] = index of node i's result.
  std::vector<int64_t> map((size_t)count);
  std::vector<int64_t> cols;
  {
    std::vector<int64_t> ids((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
      const int64_t v = nodes ? nodes[i] : i;
      if (v < 0 || v >= p->n)
        return fail(REFF_ERR_INVALID_ARG, "node id " + std::to_string(v) + " out of range");
      ids[(size_t)i] = v;
    }
    cols = ids;
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    cols.erase(std::remove_if(cols.begin(), cols.end(),
                              [&](int64_t v) { return p->is_pad[(size_t)v] != 0; }),
               cols.end());
    for (int64_t i = 0; i < count; ++i) {
      const int64_t v = ids[(size_t)i];
      if (p->is_pad[(size_t)v]) {
        map[(size_t)i] = -1;
      } else {
        map[(size_t)i] = std::lower_bound(cols.begin(), cols.end(), v) - cols.begin();
      }
    }
  }
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->n_solved = (int64_t)cols.size();
  }
  HIPCHK(hipSetDevice(p->device));
  reff_status rs;
  if ((rs = ensure(p->ws_out, (cols.size() + count + 1) * sizeof(double) +
                                  (count + 1) * sizeof(int64_t))) != REFF_OK)
    return rs;
  double* res_dev = (double*)p->ws_out.p;
  int64_t* map_dev = (int64_t*)(res_dev + cols.size() + count + 1);
  // A block Krylov space of S columns exhausts a stack of only a few S free
  // nodes within a handful of iterations, where the block residual loses
  // column rank; such stacks use S independent PCGs instead.
  if (p->n_free < 16 * (int64_t)S) o.indep = true;
  reff_status solve_rs = REFF_OK;
  if (!cols.empty()) {
    solve_rs = solve_columns(p, cols, res_dev, o, st);
    if (solve_rs != REFF_OK && solve_rs != REFF_ERR_NO_CONVERGENCE) return solve_rs;
  }
  if (count > 0) {
    if (o.out_dev) {
      HIPCHK(hipMemcpyAsync(map_dev, map.data(), count * sizeof(int64_t), hipMemcpyHostToDevice,
                            o.stream));
      HIPCHK(launch_gather_out(res_dev, map_dev, R_out, count, o.stream));
      HIPCHK(hipStreamSynchronize(o.stream));
    } else {
      std::vector<double> res(cols.size());
      if (!cols.empty())
        HIPCHK(hipMemcpyAsync(res.data(), res_dev, cols.size() * sizeof(double),
                              hipMemcpyDeviceToHost, o.stream));
      HIPCHK(hipStreamSynchronize(o.stream));
      for (int64_t i = 0; i < count; ++i)
        R_out[i] = map[(size_t)i] >= 0 ? res[(size_t)map[(size_t)i]] : 0.0;
    }
  }
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
  (void)a; (void)m; (void)b; (void)n; (void)mode; (void)R_out; (void)opts; (void)st;
  if (!p) return fail(REFF_ERR_INVALID_ARG, "handle is NULL");
  return fail(REFF_ERR_UNSUPPORTED, "reff_query_pairs: not available in this build");
}

reff_status reff_batch_plans(const reff_pdn_desc* plans, int32_t n_plans,
                             const int64_t* const* nodes, const int64_t* n_nodes,
                             double* const* R_out, const reff_batch_opts* opts,
                             reff_solve_stats* per_plan) {
  g_err.clear();
  if (n_plans < 0) return fail(REFF_ERR_INVALID_ARG, "n_plans < 0");
  if (n_plans > 0 && (!plans || !R_out)) return fail(REFF_ERR_INVALID_ARG, "NULL plans/R_out");
  if (opts && opts->surrogate) return fail(REFF_ERR_UNSUPPORTED, "surrogate screening not available");
  for (int32_t i = 0; i < n_plans; ++i) {
    reff_status s = validate_desc(&plans[i]);
    if (s != REFF_OK) return fail(s, "plan " + std::to_string(i) + ": " + g_err);
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  for (int32_t i = 0; i < n_plans; ++i) {
    reff_pdn h = nullptr;
    reff_status s = reff_build_pdn(&plans[i], dev, &h);
    if (s != REFF_OK) return fail(s, "plan " + std::to_string(i) + ": " + g_err);
    s = reff_solve_diag(h, nodes ? nodes[i] : nullptr, nodes ? n_nodes[i] : 0, R_out[i],
                        opts ? &opts->solve : nullptr, per_plan ? &per_plan[i] : nullptr);
    reff_free_pdn(h);
    if (s != REFF_OK) return fail(s, "plan " + std::to_string(i) + ": " + g_err);
  }
  return REFF_OK;
}

}  // extern "C"
