// Host runtime of the screening model (include/reff_surrogate.h): layer
// table, parameter and activation buffers, the forward / backward sequence
// over the BF16 GEMM kernels, Adam training, prediction and file I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "reff_internal.h"
#include "surrogate_internal.h"

using namespace reffsg;
using reff::host_fail;

namespace {

#define SGCHK(call)                                                                   \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)                \
        return host_fail(REFF_ERR_OUT_OF_MEMORY, std::string(#call) + ": " +          \
                                                     hipGetErrorString(e_));          \
      return host_fail(REFF_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                                 \
  } while (0)

#define SGRET(expr)                  \
  do {                               \
    reff_status s_ = (expr);         \
    if (s_ != REFF_OK) return s_;    \
  } while (0)

constexpr int MAX_BATCH = 64;

uint16_t host_f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// One layer: a K x K convolution (K = 3 or 1) or a 2x2 stride-2 transposed
// convolution (UP: a 1x1 GEMM to 4 Cout channels in space-to-depth order).
struct Layer {
  bool up;
  int cin, cout, k;
  bool relu;
  int64_t w_off, b_off;  // into the parameter vector
  uint16_t* wb = nullptr;  // bf16 W [k*k*cin][gcout]
  uint16_t* wt = nullptr;  // bf16 flipped transpose [k*k*gcout][cin]
  int gcout() const { return up ? 4 * cout : cout; }
  int64_t nw() const { return (int64_t)k * k * cin * gcout(); }
};

// Activation (and gradient) buffers of one batch capacity.
struct Acts {
  int cap = 0;
  uint16_t *x0, *e1a, *cat1, *p1, *e2a, *cat2, *p2, *e3a, *cat3, *p3, *b1, *b2, *s3, *d3a, *d3b,
      *s2, *d2a, *d2b, *s1, *d1a, *d1b;
  float* out;
  uint16_t *ge1a, *gcat1, *gp1, *ge2a, *gcat2, *gp2, *ge3a, *gcat3, *gp3, *gb1, *gb2, *gs3, *gd3a,
      *gd3b, *gs2, *gd2a, *gd2b, *gs1, *gd1a, *gd1b, *gout;
  uint16_t* col;
  uint8_t* padm;
  double* R;
  std::vector<void*> owned;
};

}  // namespace

struct reff_surrogate_t {
  int device = 0;
  int nt = 0, nx = 0, ny = 0, C = 32, cin0 = 0;
  uint64_t seed = 0;
  std::vector<Layer> L;
  int64_t n_params = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int64_t adam_t = 0;
  uint16_t* wbuf = nullptr;
  float* part = nullptr;  // split-K / column-sum partials
  size_t part_floats = 0;
  double* lpart = nullptr;  // loss partials
  LabelRec* lab = nullptr;
  size_t lab_cap = 0;
  Acts a;
};

namespace {

constexpr size_t PART_FLOATS = (size_t)32 << 20;  // 128 MB of partials
constexpr int LOSS_BLOCKS = 128;

reff_status dmalloc(void** p, size_t bytes, std::vector<void*>& owned) {
  SGCHK(hipMalloc(p, std::max<size_t>(bytes, 256)));
  owned.push_back(*p);
  return REFF_OK;
}

void free_acts(Acts& a) {
  for (void* q : a.owned) (void)hipFree(q);
  a.owned.clear();
  a.cap = 0;
}

reff_status ensure_acts(reff_surrogate_t* s, int B) {
  Acts& a = s->a;
  if (a.cap >= B) return REFF_OK;
  free_acts(a);
  const int64_t P1 = (int64_t)B * s->nx * s->ny, P2 = P1 / 4, P3 = P1 / 16, P4 = P1 / 64;
  const int C = s->C;
  struct Req {
    uint16_t** p;
    int64_t n;
  };
  const Req reqs[] = {
      {&a.x0, P1 * s->cin0}, {&a.e1a, P1 * C},     {&a.cat1, P1 * 2 * C}, {&a.p1, P2 * C},
      {&a.e2a, P2 * 2 * C},  {&a.cat2, P2 * 4 * C}, {&a.p2, P3 * 2 * C},  {&a.e3a, P3 * 4 * C},
      {&a.cat3, P3 * 8 * C}, {&a.p3, P4 * 4 * C},   {&a.b1, P4 * 8 * C},  {&a.b2, P4 * 8 * C},
      {&a.s3, P4 * 16 * C},  {&a.d3a, P3 * 4 * C},  {&a.d3b, P3 * 4 * C}, {&a.s2, P3 * 8 * C},
      {&a.d2a, P2 * 2 * C},  {&a.d2b, P2 * 2 * C},  {&a.s1, P2 * 4 * C},  {&a.d1a, P1 * C},
      {&a.d1b, P1 * C},
      {&a.ge1a, P1 * C},     {&a.gcat1, P1 * 2 * C}, {&a.gp1, P2 * C},     {&a.ge2a, P2 * 2 * C},
      {&a.gcat2, P2 * 4 * C}, {&a.gp2, P3 * 2 * C}, {&a.ge3a, P3 * 4 * C}, {&a.gcat3, P3 * 8 * C},
      {&a.gp3, P4 * 4 * C},  {&a.gb1, P4 * 8 * C},  {&a.gb2, P4 * 8 * C}, {&a.gs3, P4 * 16 * C},
      {&a.gd3a, P3 * 4 * C}, {&a.gd3b, P3 * 4 * C}, {&a.gs2, P3 * 8 * C}, {&a.gd2a, P2 * 2 * C},
      {&a.gd2b, P2 * 2 * C}, {&a.gs1, P2 * 4 * C},  {&a.gd1a, P1 * C},    {&a.gd1b, P1 * C},
      {&a.gout, P1 * s->nt},
      // im2col: at most 9 x (2C input channels) per pixel at full resolution
      // (every level has 9 x 16 C / 4^l <= 18 C per full-resolution pixel).
      {&a.col, P1 * 18 * C},
  };
  for (const Req& r : reqs) SGRET(dmalloc((void**)r.p, (size_t)r.n * 2, a.owned));
  SGRET(dmalloc((void**)&a.out, (size_t)P1 * s->nt * 4, a.owned));
  SGRET(dmalloc((void**)&a.padm, (size_t)P1, a.owned));
  SGRET(dmalloc((void**)&a.R, (size_t)P1 * s->nt * 8, a.owned));
  a.cap = B;
  return REFF_OK;
}

void build_layers(reff_surrogate_t* s) {
  const int C = s->C;
  struct Spec {
    bool up;
    int cin, cout, k;
    bool relu;
  };
  const Spec spec[] = {
      {false, s->cin0, C, 3, true}, {false, C, C, 3, true},             // e1a, e1b
      {false, C, 2 * C, 3, true},   {false, 2 * C, 2 * C, 3, true},     // e2a, e2b
      {false, 2 * C, 4 * C, 3, true}, {false, 4 * C, 4 * C, 3, true},   // e3a, e3b
      {false, 4 * C, 8 * C, 3, true}, {false, 8 * C, 8 * C, 3, true},   // b1, b2
      {true, 8 * C, 4 * C, 1, false},                                   // u3
      {false, 8 * C, 4 * C, 3, true}, {false, 4 * C, 4 * C, 3, true},   // d3a, d3b
      {true, 4 * C, 2 * C, 1, false},                                   // u2
      {false, 4 * C, 2 * C, 3, true}, {false, 2 * C, 2 * C, 3, true},   // d2a, d2b
      {true, 2 * C, C, 1, false},                                       // u1
      {false, 2 * C, C, 3, true},   {false, C, C, 3, true},             // d1a, d1b
      {false, C, s->nt, 1, false},                                      // head
  };
  s->L.clear();
  int64_t off = 0;
  for (const Spec& sp : spec) {
    Layer l;
    l.up = sp.up;
    l.cin = sp.cin;
    l.cout = sp.cout;
    l.k = sp.k;
    l.relu = sp.relu;
    l.w_off = off;
    off += l.nw();
    l.b_off = off;
    off += l.gcout();
    s->L.push_back(l);
  }
  s->n_params = off;
}

reff_status refresh_weights(reff_surrogate_t* s, hipStream_t st) {
  for (Layer& l : s->L)
    SGCHK(weight_copies(s->p + l.w_off, l.cin, l.gcout(), l.k, l.wb, l.wt, st));
  return REFF_OK;
}

reff_status alloc_model(reff_surrogate_t* s) {
  std::vector<void*> owned;  // model buffers are freed individually
  const size_t np = (size_t)s->n_params;
  SGCHK(hipMalloc((void**)&s->p, np * 4));
  SGCHK(hipMalloc((void**)&s->g, np * 4));
  SGCHK(hipMalloc((void**)&s->m, np * 4));
  SGCHK(hipMalloc((void**)&s->v, np * 4));
  SGCHK(hipMemset(s->m, 0, np * 4));
  SGCHK(hipMemset(s->v, 0, np * 4));
  int64_t nw = 0;
  for (const Layer& l : s->L) nw += 2 * l.nw();
  SGCHK(hipMalloc((void**)&s->wbuf, (size_t)nw * 2));
  int64_t o = 0;
  for (Layer& l : s->L) {
    l.wb = s->wbuf + o;
    o += l.nw();
    l.wt = s->wbuf + o;
    o += l.nw();
  }
  s->part_floats = PART_FLOATS;
  SGCHK(hipMalloc((void**)&s->part, s->part_floats * 4));
  SGCHK(hipMalloc((void**)&s->lpart, LOSS_BLOCKS * sizeof(double)));
  return REFF_OK;
}

void free_model(reff_surrogate_t* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  for (void* q : {(void*)s->p, (void*)s->g, (void*)s->m, (void*)s->v, (void*)s->wbuf,
                  (void*)s->part, (void*)s->lpart, (void*)s->lab})
    if (q) (void)hipFree(q);
  free_acts(s->a);
  delete s;
}

// Input channels of one plan (see the header), bf16, [ny][nx][cin0], and its
// tier-0 pad mask [ny][nx].
void plan_features(const reff_surrogate_t* s, const reff_pdn_desc* d, uint16_t* f, uint8_t* pad) {
  const int nt = s->nt, nx = s->nx, ny = s->ny, ci = s->cin0;
  std::vector<float> x((size_t)nx * ny * ci, 0.f);
  for (int t = 0; t < nt; ++t)
    for (int y = 0; y < ny; ++y)
      for (int xx = 0; xx < nx; ++xx) {
        float* px = &x[((size_t)y * nx + xx) * ci];
        if (xx + 1 < nx) px[t] = (float)std::log(d->gx[((size_t)t * ny + y) * (nx - 1) + xx]);
        if (y + 1 < ny) px[nt + t] = (float)std::log(d->gy[((size_t)t * (ny - 1) + y) * nx + xx]);
      }
  for (int j = 0; j < d->n_tsv; ++j) {
    const int xx = d->tsv_xy[2 * j], y = d->tsv_xy[2 * j + 1];
    double mean = 0.0;
    for (int t = 0; t + 1 < nt; ++t) mean += d->tsv_g[(size_t)j * (nt - 1) + t];
    mean = nt > 1 ? mean / (nt - 1) : 0.0;
    x[((size_t)y * nx + xx) * ci + 2 * nt] = (float)std::log1p(mean);
  }
  std::memset(pad, 0, (size_t)nx * ny);
  for (int j = 0; j < d->n_pads; ++j) {
    const int xx = d->pad_xy[2 * j], y = d->pad_xy[2 * j + 1];
    x[((size_t)y * nx + xx) * ci + 2 * nt + 1] = 1.f;
    pad[(size_t)y * nx + xx] = 1;
  }
  for (size_t i = 0; i < x.size(); ++i) f[i] = host_f2bf(x[i]);
}

reff_status check_plans(const reff_surrogate_t* s, const reff_pdn_desc* plans, int32_t n) {
  if (n < 0) return host_fail(REFF_ERR_INVALID_ARG, "n_plans < 0");
  if (n > 0 && !plans) return host_fail(REFF_ERR_INVALID_ARG, "plans is NULL");
  for (int32_t i = 0; i < n; ++i) {
    SGRET(reff::host_validate_desc(&plans[i]));
    if (plans[i].n_tiers != s->nt || plans[i].nx != s->nx || plans[i].ny != s->ny)
      return host_fail(REFF_ERR_INVALID_ARG,
                       "plan " + std::to_string(i) + " does not match the model geometry");
  }
  return REFF_OK;
}

// Upload the features and pad masks of plans idx[0..B) into the batch input.
reff_status load_inputs(reff_surrogate_t* s, const reff_pdn_desc* plans, const int32_t* idx,
                        int B, hipStream_t st) {
  const size_t hw = (size_t)s->nx * s->ny;
  std::vector<uint16_t> f(hw * s->cin0 * B);
  std::vector<uint8_t> pad(hw * B);
  for (int b = 0; b < B; ++b)
    plan_features(s, &plans[idx[b]], f.data() + hw * s->cin0 * b, pad.data() + hw * b);
  SGCHK(hipMemcpyAsync(s->a.x0, f.data(), f.size() * 2, hipMemcpyHostToDevice, st));
  SGCHK(hipMemcpyAsync(s->a.padm, pad.data(), pad.size(), hipMemcpyHostToDevice, st));
  SGCHK(hipStreamSynchronize(st));
  return REFF_OK;
}

// ---- layer sequencing

reff_status conv_fwd(reff_surrogate_t* s, const Layer& l, const uint16_t* X, int64_t ldx, int B,
                     int H, int W, void* Y, int64_t ldy, bool y_fp32, hipStream_t st) {
  const int64_t P = (int64_t)B * H * W;
  GemmArgs g{};
  if (l.k == 1) {
    g.A = X;
    g.sAm = ldx;
    g.K = l.cin;
  } else {
    SGCHK(im2col(X, ldx, l.cin, B, H, W, l.k, s->a.col, st));
    g.A = s->a.col;
    g.sAm = (int64_t)l.k * l.k * l.cin;
    g.K = l.k * l.k * l.cin;
  }
  g.sAk = 1;
  g.B = l.wb;
  g.sBk = l.gcout();
  g.M = (int)P;
  g.N = l.gcout();
  g.bias = s->p + l.b_off;
  g.relu = l.relu ? 1 : 0;
  g.C = Y;
  g.ldc = ldy;
  g.c_fp32 = y_fp32 ? 1 : 0;
  g.kchunk = (g.K + 31) / 32 * 32;
  SGCHK(gemm(g, 1, st));
  return REFF_OK;
}

// Gradients of one layer: dY (row stride lddy) is the gradient of its
// output Y (post-activation); writes dW, db into the gradient vector and,
// when dX != nullptr, overwrites dX (row stride lddx).
reff_status conv_bwd(reff_surrogate_t* s, const Layer& l, const uint16_t* X, int64_t ldx, int B,
                     int H, int W, const uint16_t* Y, int64_t ldy, uint16_t* dY, int64_t lddy,
                     uint16_t* dX, int64_t lddx, hipStream_t st) {
  const int64_t P = (int64_t)B * H * W;
  const int co = l.gcout();
  if (l.relu) SGCHK(relu_bwd(dY, lddy, Y, ldy, co, P, st));
  // bias gradient
  const int nblk = (int)std::min<int64_t>(256, std::max<int64_t>(1, P / 256));
  SGCHK(colsum(dY, lddy, co, P, s->part, nblk, s->g + l.b_off, st));
  // weight gradient: dW = im2col(X)^T dY, K dimension = pixels, split
  GemmArgs g{};
  const int kdim = l.k * l.k * l.cin;
  if (l.k == 1) {
    g.A = X;
    g.sAm = 1;
    g.sAk = ldx;
  } else {
    SGCHK(im2col(X, ldx, l.cin, B, H, W, l.k, s->a.col, st));
    g.A = s->a.col;
    g.sAm = 1;
    g.sAk = kdim;
  }
  g.B = dY;
  g.sBk = lddy;
  g.M = kdim;
  g.N = co;
  g.K = (int)P;
  g.relu = 0;
  g.bias = nullptr;
  g.ldc = co;
  g.c_fp32 = 1;
  const int64_t mn = (int64_t)kdim * co;
  int64_t nsplit = std::min<int64_t>({(P + 4095) / 4096, 64, (int64_t)s->part_floats / mn});
  nsplit = std::max<int64_t>(1, nsplit);
  g.kchunk = (int)(((P + nsplit - 1) / nsplit + 31) / 32 * 32);
  nsplit = (P + g.kchunk - 1) / g.kchunk;
  if (nsplit > 1) {
    g.C = s->part;
    SGCHK(gemm(g, (int)nsplit, st));
    SGCHK(splitk_reduce(s->part, (int)nsplit, mn, s->g + l.w_off, 0, st));
  } else {
    g.C = s->g + l.w_off;
    SGCHK(gemm(g, 1, st));
  }
  if (!dX) return REFF_OK;
  // input gradient: dX = im2col(dY) Wt
  GemmArgs h{};
  if (l.k == 1) {
    h.A = dY;
    h.sAm = lddy;
    h.K = co;
  } else {
    SGCHK(im2col(dY, lddy, co, B, H, W, l.k, s->a.col, st));
    h.A = s->a.col;
    h.sAm = (int64_t)l.k * l.k * co;
    h.K = l.k * l.k * co;
  }
  h.sAk = 1;
  h.B = l.wt;
  h.sBk = l.cin;
  h.M = (int)P;
  h.N = l.cin;
  h.bias = nullptr;
  h.relu = 0;
  h.C = dX;
  h.ldc = lddx;
  h.c_fp32 = 0;
  h.kchunk = (h.K + 31) / 32 * 32;
  SGCHK(gemm(h, 1, st));
  return REFF_OK;
}

reff_status forward(reff_surrogate_t* s, int B, hipStream_t st) {
  Acts& a = s->a;
  const int C = s->C, H = s->ny, W = s->nx;
  const std::vector<Layer>& L = s->L;
  SGRET(conv_fwd(s, L[0], a.x0, s->cin0, B, H, W, a.e1a, C, false, st));
  SGRET(conv_fwd(s, L[1], a.e1a, C, B, H, W, a.cat1 + C, 2 * C, false, st));
  SGCHK(pool_fwd(a.cat1 + C, 2 * C, C, B, H, W, a.p1, st));
  SGRET(conv_fwd(s, L[2], a.p1, C, B, H / 2, W / 2, a.e2a, 2 * C, false, st));
  SGRET(conv_fwd(s, L[3], a.e2a, 2 * C, B, H / 2, W / 2, a.cat2 + 2 * C, 4 * C, false, st));
  SGCHK(pool_fwd(a.cat2 + 2 * C, 4 * C, 2 * C, B, H / 2, W / 2, a.p2, st));
  SGRET(conv_fwd(s, L[4], a.p2, 2 * C, B, H / 4, W / 4, a.e3a, 4 * C, false, st));
  SGRET(conv_fwd(s, L[5], a.e3a, 4 * C, B, H / 4, W / 4, a.cat3 + 4 * C, 8 * C, false, st));
  SGCHK(pool_fwd(a.cat3 + 4 * C, 8 * C, 4 * C, B, H / 4, W / 4, a.p3, st));
  SGRET(conv_fwd(s, L[6], a.p3, 4 * C, B, H / 8, W / 8, a.b1, 8 * C, false, st));
  SGRET(conv_fwd(s, L[7], a.b1, 8 * C, B, H / 8, W / 8, a.b2, 8 * C, false, st));
  SGRET(conv_fwd(s, L[8], a.b2, 8 * C, B, H / 8, W / 8, a.s3, 16 * C, false, st));
  SGCHK(d2s(a.s3, 4 * C, B, H / 8, W / 8, a.cat3, 8 * C, st));
  SGRET(conv_fwd(s, L[9], a.cat3, 8 * C, B, H / 4, W / 4, a.d3a, 4 * C, false, st));
  SGRET(conv_fwd(s, L[10], a.d3a, 4 * C, B, H / 4, W / 4, a.d3b, 4 * C, false, st));
  SGRET(conv_fwd(s, L[11], a.d3b, 4 * C, B, H / 4, W / 4, a.s2, 8 * C, false, st));
  SGCHK(d2s(a.s2, 2 * C, B, H / 4, W / 4, a.cat2, 4 * C, st));
  SGRET(conv_fwd(s, L[12], a.cat2, 4 * C, B, H / 2, W / 2, a.d2a, 2 * C, false, st));
  SGRET(conv_fwd(s, L[13], a.d2a, 2 * C, B, H / 2, W / 2, a.d2b, 2 * C, false, st));
  SGRET(conv_fwd(s, L[14], a.d2b, 2 * C, B, H / 2, W / 2, a.s1, 4 * C, false, st));
  SGCHK(d2s(a.s1, C, B, H / 2, W / 2, a.cat1, 2 * C, st));
  SGRET(conv_fwd(s, L[15], a.cat1, 2 * C, B, H, W, a.d1a, C, false, st));
  SGRET(conv_fwd(s, L[16], a.d1a, C, B, H, W, a.d1b, C, false, st));
  SGRET(conv_fwd(s, L[17], a.d1b, C, B, H, W, a.out, s->nt, true, st));
  return REFF_OK;
}

// Gradients of every parameter from a.gout (the loss gradient w.r.t. out).
reff_status backward(reff_surrogate_t* s, int B, hipStream_t st) {
  Acts& a = s->a;
  const int C = s->C, H = s->ny, W = s->nx;
  const std::vector<Layer>& L = s->L;
  SGRET(conv_bwd(s, L[17], a.d1b, C, B, H, W, nullptr, 0, a.gout, s->nt, a.gd1b, C, st));
  SGRET(conv_bwd(s, L[16], a.d1a, C, B, H, W, a.d1b, C, a.gd1b, C, a.gd1a, C, st));
  SGRET(conv_bwd(s, L[15], a.cat1, 2 * C, B, H, W, a.d1a, C, a.gd1a, C, a.gcat1, 2 * C, st));
  SGCHK(s2d(a.gcat1, 2 * C, C, B, H / 2, W / 2, a.gs1, st));
  SGRET(conv_bwd(s, L[14], a.d2b, 2 * C, B, H / 2, W / 2, nullptr, 0, a.gs1, 4 * C, a.gd2b,
                 2 * C, st));
  SGRET(conv_bwd(s, L[13], a.d2a, 2 * C, B, H / 2, W / 2, a.d2b, 2 * C, a.gd2b, 2 * C, a.gd2a,
                 2 * C, st));
  SGRET(conv_bwd(s, L[12], a.cat2, 4 * C, B, H / 2, W / 2, a.d2a, 2 * C, a.gd2a, 2 * C, a.gcat2,
                 4 * C, st));
  SGCHK(s2d(a.gcat2, 4 * C, 2 * C, B, H / 4, W / 4, a.gs2, st));
  SGRET(conv_bwd(s, L[11], a.d3b, 4 * C, B, H / 4, W / 4, nullptr, 0, a.gs2, 8 * C, a.gd3b,
                 4 * C, st));
  SGRET(conv_bwd(s, L[10], a.d3a, 4 * C, B, H / 4, W / 4, a.d3b, 4 * C, a.gd3b, 4 * C, a.gd3a,
                 4 * C, st));
  SGRET(conv_bwd(s, L[9], a.cat3, 8 * C, B, H / 4, W / 4, a.d3a, 4 * C, a.gd3a, 4 * C, a.gcat3,
                 8 * C, st));
  SGCHK(s2d(a.gcat3, 8 * C, 4 * C, B, H / 8, W / 8, a.gs3, st));
  SGRET(conv_bwd(s, L[8], a.b2, 8 * C, B, H / 8, W / 8, nullptr, 0, a.gs3, 16 * C, a.gb2, 8 * C,
                 st));
  SGRET(conv_bwd(s, L[7], a.b1, 8 * C, B, H / 8, W / 8, a.b2, 8 * C, a.gb2, 8 * C, a.gb1, 8 * C,
                 st));
  SGRET(conv_bwd(s, L[6], a.p3, 4 * C, B, H / 8, W / 8, a.b1, 8 * C, a.gb1, 8 * C, a.gp3, 4 * C,
                 st));
  SGCHK(pool_bwd(a.cat3 + 4 * C, 8 * C, a.gp3, 4 * C, B, H / 4, W / 4, a.gcat3 + 4 * C, st));
  SGRET(conv_bwd(s, L[5], a.e3a, 4 * C, B, H / 4, W / 4, a.cat3 + 4 * C, 8 * C, a.gcat3 + 4 * C,
                 8 * C, a.ge3a, 4 * C, st));
  SGRET(conv_bwd(s, L[4], a.p2, 2 * C, B, H / 4, W / 4, a.e3a, 4 * C, a.ge3a, 4 * C, a.gp2,
                 2 * C, st));
  SGCHK(pool_bwd(a.cat2 + 2 * C, 4 * C, a.gp2, 2 * C, B, H / 2, W / 2, a.gcat2 + 2 * C, st));
  SGRET(conv_bwd(s, L[3], a.e2a, 2 * C, B, H / 2, W / 2, a.cat2 + 2 * C, 4 * C, a.gcat2 + 2 * C,
                 4 * C, a.ge2a, 2 * C, st));
  SGRET(conv_bwd(s, L[2], a.p1, C, B, H / 2, W / 2, a.e2a, 2 * C, a.ge2a, 2 * C, a.gp1, C, st));
  SGCHK(pool_bwd(a.cat1 + C, 2 * C, a.gp1, C, B, H, W, a.gcat1 + C, st));
  SGRET(conv_bwd(s, L[1], a.e1a, C, B, H, W, a.cat1 + C, 2 * C, a.gcat1 + C, 2 * C, a.ge1a, C,
                 st));
  SGRET(conv_bwd(s, L[0], a.x0, s->cin0, B, H, W, a.e1a, C, a.ge1a, C, nullptr, 0, st));
  return REFF_OK;
}

// Labels of plans idx[0..B) -> device records; returns their count.
reff_status load_labels(reff_surrogate_t* s, const reff_pdn_desc* plans,
                        const reff_labels* labels, const int32_t* idx, int B, int64_t* count,
                        hipStream_t st) {
  std::vector<LabelRec> recs;
  const int64_t hw = (int64_t)s->nx * s->ny, n = hw * s->nt;
  for (int b = 0; b < B; ++b) {
    const reff_labels& lb = labels[idx[b]];
    const reff_pdn_desc& d = plans[idx[b]];
    std::vector<uint8_t> pad((size_t)hw, 0);
    for (int j = 0; j < d.n_pads; ++j) pad[(size_t)d.pad_xy[2 * j + 1] * s->nx + d.pad_xy[2 * j]] = 1;
    std::vector<uint8_t> seen((size_t)n, 0);  // a node labelled twice counts once (first value)
    for (int64_t i = 0; i < lb.n_nodes; ++i) {
      const int64_t v = lb.nodes[i];
      const int64_t t = v / hw, pix = v % hw;
      if (t == 0 && pad[(size_t)pix]) continue;
      if (seen[(size_t)v]) continue;
      seen[(size_t)v] = 1;
      LabelRec r;
      r.pix = (int32_t)(b * hw + pix);
      r.t = (int32_t)t;
      r.logR = (float)std::log(lb.R[i]);
      r.pad_ = 0.f;
      recs.push_back(r);
    }
  }
  *count = (int64_t)recs.size();
  if (recs.empty()) return REFF_OK;
  if (recs.size() > s->lab_cap) {
    if (s->lab) (void)hipFree(s->lab);
    s->lab = nullptr;
    s->lab_cap = 0;
    SGCHK(hipMalloc((void**)&s->lab, recs.size() * sizeof(LabelRec)));
    s->lab_cap = recs.size();
  }
  SGCHK(hipMemcpyAsync(s->lab, recs.data(), recs.size() * sizeof(LabelRec), hipMemcpyHostToDevice,
                       st));
  SGCHK(hipStreamSynchronize(st));
  return REFF_OK;
}

reff_status check_labels(const reff_surrogate_t* s, const reff_labels* labels, int32_t n) {
  if (n > 0 && !labels) return host_fail(REFF_ERR_INVALID_ARG, "labels is NULL");
  const int64_t nn = (int64_t)s->nt * s->nx * s->ny;
  for (int32_t i = 0; i < n; ++i) {
    const reff_labels& l = labels[i];
    if (l.n_nodes < 0 || (l.n_nodes > 0 && (!l.nodes || !l.R)))
      return host_fail(REFF_ERR_INVALID_ARG, "bad labels of plan " + std::to_string(i));
    for (int64_t k = 0; k < l.n_nodes; ++k) {
      if (l.nodes[k] < 0 || l.nodes[k] >= nn)
        return host_fail(REFF_ERR_INVALID_ARG, "label node out of range in plan " + std::to_string(i));
      if (!(std::isfinite(l.R[k]) && l.R[k] > 0.0))
        return host_fail(REFF_ERR_INVALID_ARG, "label R must be finite and > 0");
    }
  }
  return REFF_OK;
}

// One forward + loss + backward over plans idx[0..B); loss in *loss.
reff_status step_grad(reff_surrogate_t* s, const reff_pdn_desc* plans, const reff_labels* labels,
                      const int32_t* idx, int B, double* loss, hipStream_t st) {
  SGRET(ensure_acts(s, B));
  SGRET(load_inputs(s, plans, idx, B, st));
  int64_t nl = 0;
  SGRET(load_labels(s, plans, labels, idx, B, &nl, st));
  SGRET(forward(s, B, st));
  const int64_t P1 = (int64_t)B * s->nx * s->ny;
  SGCHK(fill16(s->a.gout, P1 * s->nt, 0, st));
  double l = 0.0;
  if (nl > 0) {
    SGCHK(masked_loss(s->a.out, s->nt, s->lab, (int)nl, 1.f / (float)nl, s->a.gout, s->lpart,
                      LOSS_BLOCKS, st));
    std::vector<double> hp(LOSS_BLOCKS);
    SGCHK(hipMemcpyAsync(hp.data(), s->lpart, LOSS_BLOCKS * sizeof(double), hipMemcpyDeviceToHost,
                         st));
    SGCHK(hipStreamSynchronize(st));
    for (double x : hp) l += x;
    l /= (double)nl;
  }
  SGRET(backward(s, B, st));
  *loss = l;
  return REFF_OK;
}

reff_status new_model(const reff_surrogate_config* cfg, int32_t device, reff_surrogate_t** out) {
  if (!cfg || !out) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  if (cfg->n_tiers < 1 || cfg->nx < 8 || cfg->ny < 8 || cfg->nx % 8 || cfg->ny % 8)
    return host_fail(REFF_ERR_INVALID_ARG, "n_tiers >= 1 and nx, ny multiples of 8 required");
  if ((int64_t)cfg->nx * cfg->ny > (1 << 22))
    return host_fail(REFF_ERR_INVALID_ARG, "plane larger than 2048 x 2048");
  const int C = cfg->base_channels ? cfg->base_channels : 32;
  if (C < 4 || C > 128 || C % 4)
    return host_fail(REFF_ERR_INVALID_ARG, "base_channels must be a multiple of 4 in [4, 128]");
  if (2 * cfg->n_tiers + 2 > 2 * C)
    return host_fail(REFF_ERR_INVALID_ARG, "n_tiers must be below base_channels");
  if (device < 0) return host_fail(REFF_ERR_INVALID_ARG, "device < 0");
  int ndev = 0;
  SGCHK(hipGetDeviceCount(&ndev));
  if (device >= ndev) return host_fail(REFF_ERR_INVALID_ARG, "no such device");
  SGCHK(hipSetDevice(device));
  reff_surrogate_t* s = new (std::nothrow) reff_surrogate_t();
  if (!s) return host_fail(REFF_ERR_OUT_OF_MEMORY, "host allocation");
  s->device = device;
  s->nt = cfg->n_tiers;
  s->nx = cfg->nx;
  s->ny = cfg->ny;
  s->C = C;
  s->cin0 = 2 * cfg->n_tiers + 2;
  s->seed = cfg->seed;
  build_layers(s);
  reff_status rs = alloc_model(s);
  if (rs != REFF_OK) {
    const std::string msg = reff_last_error();
    free_model(s);
    return host_fail(rs, msg);
  }
  *out = s;
  return REFF_OK;
}

reff_status upload_params(reff_surrogate_t* s, const float* host) {
  const size_t np = (size_t)s->n_params;
  SGCHK(hipMemcpy(s->p, host, np * 4, hipMemcpyHostToDevice));
  SGCHK(hipMemset(s->m, 0, np * 4));
  SGCHK(hipMemset(s->v, 0, np * 4));
  s->adam_t = 0;
  SGRET(refresh_weights(s, nullptr));
  SGCHK(hipDeviceSynchronize());
  return REFF_OK;
}

}  // namespace

namespace reffsg {

bool geometry_matches(reff_surrogate s, const reff_pdn_desc* d) {
  return s && d && d->n_tiers == s->nt && d->nx == s->nx && d->ny == s->ny;
}

reff_status predict_device(reff_surrogate s, const reff_pdn_desc* plans, int32_t n, double* R,
                           hipStream_t st) {
  const int64_t per = (int64_t)s->nt * s->nx * s->ny;
  std::vector<int32_t> idx;
  for (int32_t b0 = 0; b0 < n; b0 += 16) {
    const int B = std::min<int32_t>(16, n - b0);
    idx.resize(B);
    std::iota(idx.begin(), idx.end(), b0);
    SGRET(ensure_acts(s, B));
    SGRET(load_inputs(s, plans, idx.data(), B, st));
    SGRET(forward(s, B, st));
    SGCHK(predict_out(s->a.out, s->a.padm, B, s->nt, s->ny, s->nx, R + b0 * per, st));
  }
  return REFF_OK;
}

}  // namespace reffsg

extern "C" {

reff_status reff_surrogate_create(const reff_surrogate_config* cfg, int32_t device,
                                  reff_surrogate* out) {
  reff_surrogate_t* s = nullptr;
  SGRET(new_model(cfg, device, &s));
  // He-normal weights (fan-in K*K*Cin), zero biases.
  std::vector<float> h((size_t)s->n_params, 0.f);
  std::mt19937_64 rng(cfg->seed);
  for (const Layer& l : s->L) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)(l.k * l.k * l.cin)));
    for (int64_t i = 0; i < l.nw(); ++i) h[(size_t)(l.w_off + i)] = nd(rng);
  }
  reff_status rs = upload_params(s, h.data());
  if (rs != REFF_OK) {
    const std::string msg = reff_last_error();
    free_model(s);
    return host_fail(rs, msg);
  }
  *out = s;
  return REFF_OK;
}

void reff_surrogate_free(reff_surrogate s) { free_model(s); }

int64_t reff_surrogate_num_params(reff_surrogate s) { return s ? s->n_params : -1; }

reff_status reff_surrogate_get_params(reff_surrogate s, float* out) {
  if (!s || !out) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  SGCHK(hipSetDevice(s->device));
  SGCHK(hipMemcpy(out, s->p, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
  return REFF_OK;
}

reff_status reff_surrogate_set_params(reff_surrogate s, const float* in) {
  if (!s || !in) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  for (int64_t i = 0; i < s->n_params; ++i)
    if (!std::isfinite(in[i])) return host_fail(REFF_ERR_INVALID_ARG, "non-finite parameter");
  SGCHK(hipSetDevice(s->device));
  return upload_params(s, in);
}

reff_status reff_surrogate_loss_grad(reff_surrogate s, const reff_pdn_desc* plans,
                                     const reff_labels* labels, int32_t n_plans, double* loss,
                                     float* grad) {
  if (!s || !loss) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  SGRET(check_plans(s, plans, n_plans));
  SGRET(check_labels(s, labels, n_plans));
  if (n_plans < 1) return host_fail(REFF_ERR_INVALID_ARG, "n_plans must be >= 1");
  if (n_plans > MAX_BATCH) return host_fail(REFF_ERR_UNSUPPORTED, "more than 64 plans");
  SGCHK(hipSetDevice(s->device));
  std::vector<int32_t> idx((size_t)n_plans);
  std::iota(idx.begin(), idx.end(), 0);
  SGRET(step_grad(s, plans, labels, idx.data(), n_plans, loss, nullptr));
  if (grad) SGCHK(hipMemcpy(grad, s->g, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
  SGCHK(hipDeviceSynchronize());
  return REFF_OK;
}

reff_status reff_surrogate_train(reff_surrogate s, const reff_pdn_desc* plans,
                                 const reff_labels* labels, int32_t n_plans,
                                 const reff_train_opts* opts, double* epoch_loss) {
  if (!s) return host_fail(REFF_ERR_INVALID_ARG, "NULL model");
  reff_train_opts o{};
  if (opts) o = *opts;
  if (o.epochs < 0 || o.batch < 0 || !(o.lr >= 0.0) || !std::isfinite(o.lr))
    return host_fail(REFF_ERR_INVALID_ARG, "bad training options");
  const int epochs = o.epochs ? o.epochs : 1;
  const int batch = o.batch ? o.batch : 16;
  if (batch > MAX_BATCH) return host_fail(REFF_ERR_UNSUPPORTED, "batch above 64 plans");
  const float lr = o.lr > 0.0 ? (float)o.lr : 1e-3f;
  SGRET(check_plans(s, plans, n_plans));
  SGRET(check_labels(s, labels, n_plans));
  if (n_plans < 1) return host_fail(REFF_ERR_INVALID_ARG, "n_plans must be >= 1");
  SGCHK(hipSetDevice(s->device));
  std::vector<int32_t> order((size_t)n_plans);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 rng(o.seed);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int e = 0; e < epochs; ++e) {
    std::shuffle(order.begin(), order.end(), rng);
    double sum = 0.0;
    int steps = 0;
    for (int32_t b0 = 0; b0 < n_plans; b0 += batch) {
      const int B = std::min<int32_t>(batch, n_plans - b0);
      double loss = 0.0;
      SGRET(step_grad(s, plans, labels, order.data() + b0, B, &loss, nullptr));
      s->adam_t += 1;
      const float bc1 = 1.f - std::pow(b1, (float)s->adam_t);
      const float bc2 = 1.f - std::pow(b2, (float)s->adam_t);
      SGCHK(adam(s->p, s->g, s->m, s->v, s->n_params, lr, b1, b2, eps, bc1, bc2, nullptr));
      SGRET(refresh_weights(s, nullptr));
      sum += loss;
      ++steps;
    }
    if (epoch_loss) epoch_loss[e] = sum / std::max(steps, 1);
  }
  SGCHK(hipDeviceSynchronize());
  return REFF_OK;
}

reff_status reff_surrogate_predict(reff_surrogate s, const reff_pdn_desc* plans, int32_t n_plans,
                                   double* const* R_out, int32_t out_on_device) {
  if (!s) return host_fail(REFF_ERR_INVALID_ARG, "NULL model");
  if (out_on_device != 0 && out_on_device != 1)
    return host_fail(REFF_ERR_INVALID_ARG, "out_on_device must be 0 or 1");
  SGRET(check_plans(s, plans, n_plans));
  if (n_plans > 0 && !R_out) return host_fail(REFF_ERR_INVALID_ARG, "R_out is NULL");
  for (int32_t i = 0; i < n_plans; ++i)
    if (!R_out[i]) return host_fail(REFF_ERR_INVALID_ARG, "R_out[i] is NULL");
  SGCHK(hipSetDevice(s->device));
  const int64_t per = (int64_t)s->nt * s->nx * s->ny;
  for (int32_t b0 = 0; b0 < n_plans; b0 += 16) {
    const int B = std::min<int32_t>(16, n_plans - b0);
    SGRET(ensure_acts(s, B));
    SGRET(reffsg::predict_device(s, plans + b0, B, s->a.R, nullptr));
    for (int b = 0; b < B; ++b)
      SGCHK(hipMemcpy(R_out[b0 + b], s->a.R + b * per, (size_t)per * 8,
                      out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  }
  SGCHK(hipDeviceSynchronize());
  return REFF_OK;
}

reff_status reff_surrogate_save(reff_surrogate s, const char* path) {
  if (!s || !path) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> h((size_t)s->n_params);
  SGRET(reff_surrogate_get_params(s, h.data()));
  FILE* f = std::fopen(path, "wb");
  if (!f) return host_fail(REFF_ERR_INVALID_ARG, std::string("cannot open ") + path);
  const char magic[8] = {'R', 'E', 'F', 'F', 'S', 'G', '0', '1'};
  const int32_t dims[4] = {s->nt, s->nx, s->ny, s->C};
  const int64_t np = s->n_params;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, 4, 4, f) == 4 &&
            std::fwrite(&s->seed, 8, 1, f) == 1 && std::fwrite(&np, 8, 1, f) == 1 &&
            std::fwrite(h.data(), 4, h.size(), f) == h.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return host_fail(REFF_ERR_INVALID_ARG, std::string("write failed: ") + path);
  return REFF_OK;
}

reff_status reff_surrogate_load(const char* path, int32_t device, reff_surrogate* out) {
  if (!path || !out) return host_fail(REFF_ERR_INVALID_ARG, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return host_fail(REFF_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t dims[4];
  uint64_t seed = 0;
  int64_t np = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "REFFSG01", 8) == 0 &&
            std::fread(dims, 4, 4, f) == 4 && std::fread(&seed, 8, 1, f) == 1 &&
            std::fread(&np, 8, 1, f) == 1;
  reff_surrogate_config cfg{};
  if (ok) {
    cfg.n_tiers = dims[0];
    cfg.nx = dims[1];
    cfg.ny = dims[2];
    cfg.base_channels = dims[3];
    cfg.seed = seed;
  }
  reff_surrogate_t* s = nullptr;
  if (ok) {
    reff_status rs = new_model(&cfg, device, &s);
    if (rs != REFF_OK) {
      std::fclose(f);
      return rs;
    }
    ok = np == s->n_params;
  }
  std::vector<float> h;
  if (ok) {
    h.resize((size_t)np);
    ok = std::fread(h.data(), 4, h.size(), f) == h.size();
  }
  std::fclose(f);
  if (!ok) {
    free_model(s);
    return host_fail(REFF_ERR_INVALID_ARG, std::string("not a model file: ") + path);
  }
  reff_status rs = upload_params(s, h.data());
  if (rs != REFF_OK) {
    const std::string msg = reff_last_error();
    free_model(s);
    return host_fail(rs, msg);
  }
  *out = s;
  return REFF_OK;
}

}  // extern "C"
