/*
 * snake_mlp.h - C ABI of the learned warm start's network on MI355X (gfx950).
 *
 * The network predicts initial multipliers of one constraint block from 32
 * features of that block (spec extension of the method; the features
 * are listed with sim_step_record in snake.h).  Shape 32 -> 64 -> 64 -> 3,
 * GELU (exact erf) after both hidden layers, inputs standardised per
 * feature.  Products run on BF16 MFMA with FP32 accumulation; parameters,
 * biases, activations' FP32 copies and the optimiser state are FP32.
 *
 * Parameters: one FP32 vector of mlp_param_count() = 6467 values,
 *   W1[64][32], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
 * (W[o][i] multiplies input i into output o).  mean_std holds the 32 means
 * followed by the 32 standard deviations.  Samples are row-major: x[n][32],
 * targets and outputs [n][3].
 *
 * Every pointer is device memory owned by the caller; calls are
 * asynchronous on `stream` (a hipStream_t, NULL = default stream).  Return
 * values are the SIM_* codes of snake.h; mlp_last_error() describes the
 * last failure of the calling thread.
 */
#ifndef SNAKE_MLP_H
#define SNAKE_MLP_H

#include <stdint.h>

#include "snake.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 6467 */
int mlp_param_count(void);

/* FP32 scratch that mlp_grad needs for a batch of n samples */
int64_t mlp_train_scratch_floats(int64_t n);

/* mean_std[0..31] = per-feature mean of x[n][32], [32..63] = standard
 * deviation sqrt(var + 1e-12), accumulated in double. */
int mlp_norm_stats(const float* x, int64_t n, float* mean_std, void* stream);

/* y[n][3] = network(standardised x) */
int mlp_forward(const float* params, const float* mean_std, const float* x, float* y, int64_t n,
                void* stream);

/* Mean-squared-error loss over the n x 3 outputs and its gradient with
 * respect to the parameters (grad[6467], loss[1]).  Deterministic: one
 * partial row per 64 samples, summed in order.  SIM_ENOMEM if scratch holds
 * fewer than mlp_train_scratch_floats(n) floats. */
int mlp_grad(const float* params, const float* mean_std, const float* x, const float* t, int64_t n,
             float* grad, float* loss, float* scratch, int64_t scratch_floats, void* stream);

/* For callers that cannot allocate (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mlp_grad without the
 * scratch argument.  The partial gradient rows live in a fixed device array
 * of the library sized for at most 4096 samples (3.3 MB per device, held
 * until the process ends); larger n gives SIM_EINVAL.  Allocates nothing.
 * Every call on one device uses the same array: calls that overlap on one
 * device (two streams, two threads) race and must be serialised by the
 * caller.  Same kernels, same results as mlp_grad. */
int mlp_grad_noalloc(const float* params, const float* mean_std, const float* x, const float* t, int64_t n,
                     float* grad, float* loss, void* stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected; t >= 1). */
int mlp_adam(float* params, float* m, float* v, const float* grad, int32_t t, float lr, void* stream);

const char* mlp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SNAKE_MLP_H */
