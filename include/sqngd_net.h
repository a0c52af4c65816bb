/*
 * sqngd_net.h - C ABI of the warm-start proposal network in libsqngd.so.
 *
 * The network is not part of the paper's method: the paper reparameterises
 * each design with its own ResNet and trains it for that design only
 * (Sec. III-A, eq. 17). Here a small network, trained once on converged runs
 * of the optimiser of Algorithm 1, maps seeded noise to starting logits for
 * that optimiser; plain N(0,1) logits remain the fallback.
 *
 * Network (1-D convolutions along the chip axis n, zero padding 2, output
 * length N; every weight and activation held in bfloat16, every product
 * accumulated in FP32 by gfx950 MFMA instructions):
 *   X0[b][n][c]  = noise[b][c][n] (c < M), cond0 (c = M), cond1 (c = M+1);
 *   Z_i[b][n][o] = bias_i[o] + sum_{tap<5} sum_c W_i[o][tap][c] X_i[b][n+tap-2][c];
 *   X_{i+1}      = relu(Z_i), i = 0, 1, 2 (64 channels each);
 *   logits[b][m][n][l] = Z_3[b][n][m*L + l]   (the [M][N][L] layout of z).
 * Loss of a training step: mean cross-entropy of softmax_l(logits[b][m][n][:])
 * against target levels t[b][m][n].
 *
 * Parameters: one flat FP32 array, per layer i = 0..3 W_i[cout][5][cin] then
 * bias_i[cout], with (cin, cout) = (M+2, 64), (64, 64), (64, 64), (64, M*L);
 * sqngd_net_param_count gives the length. Adam moments: 2 * count floats
 * (first moments, then second moments).
 *
 * Ownership: every array is a DEVICE pointer owned by the caller; the shape
 * and options are HOST pointers read during the call. Scratch (bfloat16
 * weights, activations, gradient partials) lives in the caller's workspace
 * (size from sqngd_net_workspace_size, 256-byte aligned); the library never
 * allocates. sqngd_net_backward uses the activations that the last
 * sqngd_net_forward on the same workspace left there. Calls only enqueue on
 * `stream` (a hipStream_t passed as void*) and issue no memset.
 *
 * Errors (checked on the host before any HIP call): SQNGD_E_INVALID_ARG for a
 * NULL required pointer, batch < 1 or a non-finite conditioning value;
 * SQNGD_E_UNSUPPORTED unless M + 2 <= 8, M*L is 16, 32 or 64, L is a multiple
 * of 4, N is a multiple of 64 with N <= 4096, batch <= 65536; SQNGD_E_WORKSPACE
 * for a short workspace; SQNGD_E_ALIGN for a misaligned pointer; SQNGD_E_HIP
 * for a failed launch.
 */
#ifndef SQNGD_NET_H
#define SQNGD_NET_H

#include <stddef.h>
#include <stdint.h>

#include "sqngd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t M, N, L;    /* waveforms, chips, phase levels of the designs proposed  */
  int32_t batch;      /* samples per call                                         */
  float cond0, cond1; /* conditioning inputs (for instance L / 8 and the Doppler span) */
  int32_t reserved[2]; /* must be 0                                                */
} sqngd_net_shape;

typedef struct {
  float lr, beta1, beta2, eps;
} sqngd_net_opt;

/* Number of FP32 parameters. */
int sqngd_net_param_count(const sqngd_net_shape* shape, int64_t* count);

/* Workspace bytes for `shape`. */
int sqngd_net_workspace_size(const sqngd_net_shape* shape, size_t* bytes);

/* logits[batch][M][N][L] (FP32) of noise[batch][M][N] (FP32). Converts the
   parameters to bfloat16 into the workspace and keeps every activation there
   for a following sqngd_net_backward. */
int sqngd_net_forward(const sqngd_net_shape* shape, const float* params, const float* noise, float* logits,
                      void* ws, size_t ws_bytes, void* stream);

/* Gradient of the loss with respect to the parameters (grad_params, FP32,
   overwritten) after a forward on the same workspace. With target
   ([batch][M][N] int32 levels) the loss is the mean cross-entropy of the
   forward's logits (passed again as `logits`), and *loss (device float,
   nullable) receives it; without target, grad_logits ([batch][M][N][L]) is
   the upstream gradient and `logits` and `loss` are ignored. */
int sqngd_net_backward(const sqngd_net_shape* shape, const float* logits, const int32_t* target,
                       const float* grad_logits, float* grad_params, float* loss, void* ws, size_t ws_bytes,
                       void* stream);

/* One Adam step (bias-corrected, step >= 1) on params with moments
   [2][count]: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
int sqngd_net_adam(const sqngd_net_shape* shape, const sqngd_net_opt* opt, int32_t step, float* params,
                   float* moments, const float* grad_params, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SQNGD_NET_H */
