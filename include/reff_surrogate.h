/*
 * reff_surrogate.h -- learned screening model for batches of candidate TSV
 * plans (part of libreff; same conventions as reff.h).
 *
 * The paper motivates fast effective-resistance evaluation with TSV
 * placement and design-option exploration (Sec. I, Sec. IV-B), where many
 * plans of one stack geometry are compared.  This model maps a plan's
 * per-node conductance maps to log R_i for every node and tier (a BF16
 * U-Net run on the matrix cores); reff_batch_plans can use it to screen a
 * batch: predict every map, check a seeded fraction of each plan's nodes
 * with the solver, and fall back to the solver for any plan whose checked
 * error exceeds a threshold (reff_batch_opts.surrogate / spot_frac /
 * fallback_rel_err).  The paper itself has no learned model; the network
 * below is this library's design.
 *
 * Network (nx, ny divisible by 8; C = base_channels; NHWC BF16 activations,
 * FP32 accumulation, FP32 master weights):
 *   input  2*nt + 2 channels per (x,y): log gx per tier (0 on the last
 *          column), log gy per tier (0 on the last row), TSV column mask
 *          times log(1 + mean segment conductance), pad mask;
 *   encoder 4 levels of two 3x3 convolutions + ReLU with C, 2C, 4C, 8C
 *          channels, 2x2 max pooling between levels;
 *   decoder 2x2 stride-2 transposed convolution (no activation), channel
 *          concatenation [transposed-convolution output, then the encoder
 *          output of that level], two 3x3 convolutions + ReLU, for levels
 *          3, 2, 1 (the encoder output is that of the level's second
 *          convolution);
 *   head   1x1 convolution to nt channels = log R of the node (t, x, y).
 * Pads are reported as R = 0.
 *
 * Parameter vector (float32, the order of reff_surrogate_get_params): for
 * each layer in forward order (e1a, e1b, e2a, e2b, e3a, e3b, b1, b2, u3,
 * d3a, d3b, u2, d2a, d2b, u1, d1a, d1b, head), weights then biases:
 *   3x3 / 1x1 convolution: W[(kh*K + kw)*Cin + ci][Cout], b[Cout], where
 *          output (x, y) reads input (x + kw - (K-1)/2, y + kh - (K-1)/2);
 *   transposed convolution: W[ci][(a*2 + b)*Cout + co], b[(a*2 + b)*Cout +
 *          co] for output pixel (2x + b, 2y + a).
 */
#ifndef REFF_SURROGATE_H
#define REFF_SURROGATE_H

#include <stdint.h>

#include "reff.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct reff_surrogate_t* reff_surrogate;

typedef struct {
  int32_t n_tiers, nx, ny;  /* plan geometry the model accepts (nx, ny % 8 == 0) */
  int32_t base_channels;    /* C; 0 => 32                                     */
  uint64_t seed;            /* weight initialisation (He normal, zero biases)  */
} reff_surrogate_config;

/* Labelled nodes of one plan: R[i] = R_{nodes[i]} (> 0; pads are ignored). */
typedef struct {
  const int64_t* nodes;  /* host node ids t*nx*ny + y*nx + x               */
  int64_t n_nodes;
  const double* R;       /* host                                            */
} reff_labels;

typedef struct {
  int32_t epochs;   /* 0 => 1                                              */
  int32_t batch;    /* plans per step; 0 => 16                             */
  double lr;        /* Adam step size; 0 => 1e-3 (betas 0.9, 0.999, eps 1e-8) */
  uint64_t seed;    /* plan order shuffling                                */
} reff_train_opts;

/* New model with freshly initialised weights on `device`.
 * Errors: INVALID_ARG (dims), OUT_OF_MEMORY, DEVICE. */
reff_status reff_surrogate_create(const reff_surrogate_config* cfg, int32_t device,
                                  reff_surrogate* out);

/* Release a model.  NULL is ignored. */
void reff_surrogate_free(reff_surrogate s);

/* Length of the parameter vector, or -1 for NULL. */
int64_t reff_surrogate_num_params(reff_surrogate s);

/* Copy the float32 master parameters out (host float[num_params]) or in.
 * Setting also resets the Adam moments. */
reff_status reff_surrogate_get_params(reff_surrogate s, float* out);
reff_status reff_surrogate_set_params(reff_surrogate s, const float* in);

/*
 * Masked mean-squared error of log R over the labelled non-pad nodes of
 * n_plans plans (one forward and backward pass, no update):
 *   loss = sum over labels (pred - log R)^2 / (number of labels),
 * and its gradient with respect to the parameter vector (host
 * float[num_params], nullable).  Every plan must match the model geometry.
 * Errors: INVALID_ARG (geometry, ids, R <= 0), UNSUPPORTED (n_plans above
 * the model's batch capacity of 64), OUT_OF_MEMORY, DEVICE.
 */
reff_status reff_surrogate_loss_grad(reff_surrogate s, const reff_pdn_desc* plans,
                                     const reff_labels* labels, int32_t n_plans, double* loss,
                                     float* grad);

/*
 * Adam training on the masked loss above, opts->epochs passes over the
 * plans in seeded random order, opts->batch plans per step.  epoch_loss
 * (host double[epochs], nullable) receives the mean step loss per epoch.
 */
reff_status reff_surrogate_train(reff_surrogate s, const reff_pdn_desc* plans,
                                 const reff_labels* labels, int32_t n_plans,
                                 const reff_train_opts* opts, double* epoch_loss);

/*
 * Predicted R for every node of each plan: R_out[i] is float64
 * [n_tiers*ny*nx] in node-id order (host, or device memory if
 * out_on_device == 1); pads give 0.
 */
reff_status reff_surrogate_predict(reff_surrogate s, const reff_pdn_desc* plans,
                                   int32_t n_plans, double* const* R_out, int32_t out_on_device);

/* Save / load the configuration and float32 parameters (little-endian
 * binary file with a magic tag).  Errors: INVALID_ARG (path, bad file). */
reff_status reff_surrogate_save(reff_surrogate s, const char* path);
reff_status reff_surrogate_load(const char* path, int32_t device, reff_surrogate* out);

#ifdef __cplusplus
}
#endif

#endif /* REFF_SURROGATE_H */
