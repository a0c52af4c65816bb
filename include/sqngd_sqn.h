/*
 * sqngd_sqn.h - C ABI of the paper's transmit parameterisation in libsqngd.so
 * (Sec. III-A): the ResNet f_theta that maps the fixed input y0 = vec(Y0)
 * (normalised discrete phases, eq. 15-16 and Algorithm 1's initialisation)
 * to continuous variables z (eq. 17), the copied tanh staircase Q_A with
 * trainable ordered thresholds rho (eq. 24) that gives the soft waveform
 * s = exp(j 2 pi Q_A(z)) (eq. 22-23), and the hard quantiser Q_R (eq. 43)
 * read as the staircase's limit: the number of thresholds at or below z,
 * mod B, as the phase index. The thresholds are kept ordered after every
 * transmit update (the projection Sec. III-C asks for).
 *
 * Network (D = M N inputs and outputs, width 128, 5 residual blocks):
 *   h_0 = tanh(W_in y0 + b_in),
 *   h_k = h_{k-1} + tanh(W2_k tanh(W1_k h_{k-1} + b1_k) + b2_k), k = 1..5,
 *   z   = sigmoid(W_out h_5 + b_out).
 * Parameters: one flat FP32 array theta, per dense layer W[out][in] then
 * b[out], in the order W_in, (W1_1, W2_1), ..., (W1_5, W2_5), W_out;
 * sqngd_sqn_param_count gives its length. Staircase: K = B * copies
 * thresholds rho (FP32, kept sorted), every transition of height 1/B and
 * steepness c: Q_A(z) = sum_i (tanh(c (z - rho_i)) + 1) / (2B).
 *
 * The AF, the loss and the waveform / filter gradients come from
 * sqngd_af_forward / sqngd_af_backward with wave_mode SQNGD_WAVE_GIVEN; these
 * calls carry the waveform gradient back to (theta, rho) and update them.
 *
 * Designs: a shape with designs = R describes R independent designs (random
 * restarts, each with its own y0, theta, rho): every per-design array is
 * stacked R times back to back (theta [R][count], y0 / z [R][M N], rho
 * [R][K], waveforms and gradients [R][M][N], the workspace R slices), the
 * layout of R equal problems in one sqngd batch. The hidden stack then runs
 * one workgroup per design, side by side.
 *
 * Ownership: every array is a DEVICE pointer owned by the caller; the shape is
 * a HOST pointer read during the call. The network's activations live in the
 * caller's workspace (size from sqngd_sqn_workspace_size, 256-byte aligned;
 * sqngd_sqn_forward also wants theta 16-byte aligned, as it reads the
 * hidden layers in 16-byte pieces):
 * sqngd_sqn_backward uses those the last sqngd_sqn_forward on the same
 * workspace left there. Calls only enqueue on `stream` (a hipStream_t passed
 * as void*), allocate nothing and issue no memset.
 *
 * Errors (checked on the host before any HIP call): SQNGD_E_INVALID_ARG for a
 * NULL required pointer, a non-positive size or a non-finite / non-positive
 * c; SQNGD_E_UNSUPPORTED unless M N <= 4096, 2 <= B <= 64,
 * B * copies <= 4096 and designs <= 65535; SQNGD_E_WORKSPACE for a short workspace; SQNGD_E_ALIGN
 * for a misaligned pointer; SQNGD_E_HIP for a failed launch.
 */
#ifndef SQNGD_SQN_H
#define SQNGD_SQN_H

#include <stddef.h>
#include <stdint.h>

#include "sqngd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t M, N;       /* waveforms and chips: D = M N network inputs and outputs */
  int32_t B;          /* phase levels (the problem's L)                         */
  int32_t copies;     /* r_n of the copying mechanism: K = B * copies thresholds */
  float c;            /* staircase steepness                                    */
  int32_t designs;    /* R independent designs of this shape, stacked (0 = 1)   */
  int32_t reserved[2]; /* must be 0                                              */
} sqngd_sqn_shape;

/* Length of theta for D = M N inputs. */
int sqngd_sqn_param_count(int32_t D, int64_t* count);

/* Workspace bytes of sqngd_sqn_forward / sqngd_sqn_backward. */
int sqngd_sqn_workspace_size(const sqngd_sqn_shape* shape, size_t* bytes);

/* z = f_theta(y0) (eq. 17); y0 and z are [M N] (waveform m at m N .. m N + N - 1). */
int sqngd_sqn_forward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, float* z, void* ws,
                      size_t ws_bytes, void* stream);

/* Soft waveform s[m][n] = exp(j 2 pi Q_A(z[m N + n])) (eq. 22-24). The phase is
   taken from Q_A mod 1 formed as (thresholds below z mod B + the fractional
   terms) / B, so its FP32 resolution does not degrade with the copy count. */
int sqngd_sqn_soft(const sqngd_sqn_shape* shape, const float* z, const float* rho, sqngd_c64* s, void* stream);

/* Hard waveform (Q_R, eq. 43): idx = #{i : rho_i <= z} mod B, x = exp(j 2 pi idx / B).
   Either output may be NULL. */
int sqngd_sqn_hard(const sqngd_sqn_shape* shape, const float* z, const float* rho, int32_t* idx, sqngd_c64* x,
                   void* stream);

/* Gradients of the loss with respect to theta and rho from the packed waveform
   gradient grad_s (dL/dRe + j dL/dIm, from sqngd_af_backward in mode GIVEN) at
   the soft waveform s of z: dL/dy1 = 2 pi Im(g conj(s)), through Q_A to z
   and rho, then through the network (whose activations the last
   sqngd_sqn_forward on ws left there; y0 is the input of that forward).
   g = grad_s, or grad_s + grad_h when grad_h (the packed filter gradient of
   the same sqngd_af_backward call) is given: matched filtering, the filters
   being the soft waveform itself, as in the AF extension of SQN the paper
   compares against (Sec. IV, no receive-filter optimisation). grad_theta and
   grad_rho are written. */
int sqngd_sqn_backward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, const float* z,
                       const float* rho, const sqngd_c64* s, const sqngd_c64* grad_s, const sqngd_c64* grad_h,
                       float* grad_theta, float* grad_rho, void* ws, size_t ws_bytes, void* stream);

/* sqngd_sqn_backward followed by sqngd_sqn_adam on theta, in the same
   launches: the weight gradients update theta (and its moments m_theta,
   v_theta, each the length of theta) in place instead of being written out;
   grad_rho is written as by sqngd_sqn_backward. The same results as the two
   calls. theta is read by the backward pass before the last launch updates
   it. */
int sqngd_sqn_backward_adam(const sqngd_sqn_shape* shape, float* theta, const float* y0, const float* z,
                            const float* rho, const sqngd_c64* s, const sqngd_c64* grad_s, const sqngd_c64* grad_h,
                            float* m_theta, float* v_theta, float* grad_rho, const int32_t* step, int32_t step_mul,
                            int32_t step_add, float lr, float beta1, float beta2, float eps, void* ws,
                            size_t ws_bytes, void* stream);

/* One bias-corrected Adam step on n floats: p -= lr mhat / (sqrt(vhat) + eps),
   with the moments m, v updated in place; used for theta, rho and the filters
   (as 2 M N floats, Re and Im interleaved). The step count is
   t = step_mul * (*step) + step_add, read on the device when step (a device
   int32, e.g. the outer-iteration counter) is given, so that a captured graph
   replays with the current count; else t = step_add (>= 1). */
int sqngd_sqn_adam(float* p, const float* g, float* m, float* v, int64_t n, const int32_t* step, int32_t step_mul,
                   int32_t step_add, float lr, float beta1, float beta2, float eps, void* stream);

/* sqngd_sqn_adam on rows filter rows of N complex values (g, m, v as 2 N
   floats per row, Re and Im interleaved) followed by the energy projection of
   each row (eq. 32), in one launch; the same results as sqngd_sqn_adam then
   sqngd_sqn_project. */
int sqngd_sqn_adam_project(int32_t rows, int32_t N, sqngd_c64* h, const sqngd_c64* g, float* m, float* v,
                           const int32_t* step, int32_t step_mul, int32_t step_add, float lr, float beta1,
                           float beta2, float eps, void* stream);

/* sqngd_sqn_adam on each of the `designs` rows of K thresholds followed by
   their ordered projection (the sort of sqngd_sqn_sort), in one launch; the
   same results as the two calls. */
int sqngd_sqn_adam_sort(float* rho, const float* g, float* m, float* v, int32_t K, int32_t designs,
                        const int32_t* step, int32_t step_mul, int32_t step_add, float lr, float beta1, float beta2,
                        float eps, void* stream);

/* *step += 1 on the device (the outer-iteration counter of the driver). */
int sqngd_sqn_count(int32_t* step, void* stream);

/* The projection of the thresholds onto an ordered set: sorts each of the
   `designs` rows rho[r][0..K) in place (ascending), K <= 4096. */
int sqngd_sqn_sort(float* rho, int32_t K, int32_t designs, void* stream);

/* Energy projection of the filters (eq. 32): h_m <- h_m sqrt(N / |h_m|^2),
   rows of N complex values (M R rows for R stacked designs). */
int sqngd_sqn_project(int32_t M, int32_t N, sqngd_c64* h, void* stream);

#ifdef __cplusplus
}
#endif

#endif
