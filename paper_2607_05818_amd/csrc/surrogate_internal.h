// Internal declarations of the screening model (surrogate_api.cpp and
// surrogate_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/reff_surrogate.h"

namespace reffsg {

// Screening support for reff_batch_plans: whether a plan has the model's
// geometry, and the predicted R of every node of n plans into the device
// buffer R [n][n_tiers*ny*nx] (pads 0), on stream st.
bool geometry_matches(reff_surrogate s, const reff_pdn_desc* d);
reff_status predict_device(reff_surrogate s, const reff_pdn_desc* plans, int32_t n, double* R,
                           hipStream_t st);

// C(m, n) = sum_k A(m, k) B(k, n) on the matrix cores (BF16 inputs, FP32
// accumulation), A(m, k) = A[m*sAm + k*sAk] (sAm == 1 or sAk == 1),
// B(k, n) = B[k*sBk + n].  With kchunk < K the K range is split over
// gridDim.z slices of kchunk (a multiple of 32) and slice z writes its FP32
// partial to (float*)C + z*M*ldc (no bias, no ReLU); otherwise
//   C(m, n) = relu?(acc + bias[n]) stored as FP32 or BF16 at C[m*ldc + n].
struct GemmArgs {
  const uint16_t* A;
  int64_t sAm, sAk;
  const uint16_t* B;
  int64_t sBk;
  int M, N, K;
  const float* bias;
  int relu;
  void* C;
  int64_t ldc;
  int c_fp32;
  int kchunk;
};

// One labelled node of a training batch: pixel (b*H + y)*W + x of the
// batch, tier t, target log R.
struct LabelRec {
  int32_t pix;
  int32_t t;
  float logR;
  float pad_;
};

hipError_t gemm(const GemmArgs& g, int nsplit, hipStream_t st);
// out[i] (=|+=) sum over z < nsplit of part[z*len + i]
hipError_t splitk_reduce(const float* part, int nsplit, int64_t len, float* out, int accumulate,
                         hipStream_t st);
// col[p][(kh*K + kw)*C + c] = X[p shifted by (kh - (K-1)/2, kw - (K-1)/2)][c]
// (0 outside the image); X has row stride ldx.
hipError_t im2col(const uint16_t* X, int64_t ldx, int C, int B, int H, int W, int K,
                  uint16_t* col, hipStream_t st);
hipError_t pool_fwd(const uint16_t* X, int64_t ldx, int C, int B, int H, int W, uint16_t* Y,
                    hipStream_t st);
// dX (row stride ldx) += dY routed to the first maximum of each 2x2 window
hipError_t pool_bwd(const uint16_t* X, int64_t ldx, const uint16_t* dY, int C, int B, int H,
                    int W, uint16_t* dX, hipStream_t st);
// depth-to-space: Y[(b, 2y+a, 2x+c)][ch] = S[(b, y, x)][(a*2+c)*C + ch]; H, W
// are the low-resolution sizes.  s2d is its adjoint (a gather).
hipError_t d2s(const uint16_t* S, int C, int B, int H, int W, uint16_t* Y, int64_t ldy,
               hipStream_t st);
hipError_t s2d(const uint16_t* Y, int64_t ldy, int C, int B, int H, int W, uint16_t* S,
               hipStream_t st);
// dY *= (Y > 0) over P rows of C channels
hipError_t relu_bwd(uint16_t* dY, int64_t lddy, const uint16_t* Y, int64_t ldy, int C, int64_t P,
                    hipStream_t st);
// db[c] = sum over P rows of dY[p][c]; part holds nblk*C floats
hipError_t colsum(const uint16_t* dY, int64_t ld, int C, int64_t P, float* part, int nblk,
                  float* db, hipStream_t st);
// Wb = bf16(W), Wt = bf16 of the flipped transpose used by the input gradient:
// Wt[(kh*K + kw)*Cout + co][ci] = W[((K-1-kh)*K + (K-1-kw))*Cin + ci][co]
hipError_t weight_copies(const float* W, int Cin, int Cout, int K, uint16_t* Wb, uint16_t* Wt,
                         hipStream_t st);
// dpred[pix][t] = 2 (pred - logR) / n for each label (dpred zeroed first);
// part[blockIdx] = partial sums of (pred - logR)^2
hipError_t masked_loss(const float* pred, int nt, const LabelRec* lab, int n, float inv_n,
                       uint16_t* dpred, double* part, int nblk, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, hipStream_t st);
hipError_t fill16(uint16_t* a, int64_t n, uint16_t val, hipStream_t st);
// R[(b*nt + t)*H*W + y*W + x] = pad ? 0 : exp(pred[((b*H + y)*W + x)*nt + t]);
// padm is the pad mask [b][H*W] (1 = pad)
hipError_t predict_out(const float* pred, const uint8_t* padm, int B, int nt, int H, int W,
                       double* R, hipStream_t st);

}  // namespace reffsg
