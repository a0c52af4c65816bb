// sqn.hip - gfx950 kernels and C ABI of the paper's transmit parameterisation
// (Sec. III-A; declared in include/sqngd_sqn.h). Included by api.hip after
// its host helpers (one translation unit).
//
// The network runs on a single input vector, so every dense layer is a
// matrix-vector product bound by reading its weights once: one wavefront per
// output (lanes stride over the inputs, a DPP sum in lane order, so results
// are the same run to run). The backward pass mirrors the forward layer by
// layer: an outer-product kernel for the weight and bias gradients and a
// transposed product (one thread per input, outputs summed in order) for the
// gradient of the layer's input. The staircase, its gradient, the hard
// quantiser, Adam, the ordered projection of the thresholds (a bitonic sort in
// LDS) and the filters' energy projection are element- or row-wise kernels.
#include "../../include/sqngd_sqn.h"

namespace sqsqn {

using sq::wave_sum;

constexpr int kH = 128;       // hidden width
constexpr int kBlocks = 5;    // residual blocks
constexpr int kThreads = 256;
constexpr int kMaxD = 4096;
constexpr int kMaxK = 4096;

enum Act : int { ACT_TANH = 0, ACT_SIGMOID = 1 };

// a[o] = act(W[o][:] . in + b[o]); out[o] = res[o] + a[o] when res is given.
template <int ACT>
__global__ __launch_bounds__(kThreads) void k_dense_fwd(const float* __restrict__ in, int K,
                                                         const float* __restrict__ W, const float* __restrict__ b,
                                                         int O, const float* __restrict__ res, float* a_out,
                                                         float* out) {
  const int o = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= O) return;
  const float* w = W + (int64_t)o * K;
  float acc = 0.f;
  for (int k = lane; k < K; k += 64) acc += w[k] * in[k];
  acc = wave_sum(acc);
  if (lane == 0) {
    const float p = acc + b[o];
    const float a = ACT == ACT_TANH ? tanhf(p) : 1.0f / (1.0f + expf(-p));
    if (a_out) a_out[o] = a;
    if (out) out[o] = (res ? res[o] : 0.f) + a;
  }
}

__device__ __forceinline__ float act_grad(int act, float a) {
  return act == ACT_TANH ? 1.0f - a * a : a * (1.0f - a);
}

// dW[o][k] = dp[o] in[k], db[o] = dp[o], dp[o] = d_act[o] act'(a[o]).
__global__ __launch_bounds__(kThreads) void k_dense_bwd_w(const float* __restrict__ d_act,
                                                           const float* __restrict__ a, int act,
                                                           const float* __restrict__ in, int K, int O,
                                                           float* dW, float* db) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)O * K;
  if (i < n) {
    const int o = (int)(i / K), k = (int)(i - (int64_t)o * K);
    dW[i] = d_act[o] * act_grad(act, a[o]) * in[k];
  }
  if (i < O) db[i] = d_act[i] * act_grad(act, a[i]);
}

// din[k] = base[k] + sum_o W[o][k] dp[o], dp as above: a block owns 64
// inputs (one per lane); its 16 waves take the outputs o = w (mod 16) and
// their partial sums are added in wave order.
constexpr int kBwdWaves = 16;
__global__ __launch_bounds__(64 * kBwdWaves) void k_dense_bwd_in(const float* __restrict__ W,
                                                                  const float* __restrict__ d_act,
                                                                  const float* __restrict__ a, int act, int K, int O,
                                                                  const float* __restrict__ base, float* din) {
  __shared__ float part[kBwdWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  float acc = 0.f;
  if (k < K)
    for (int o = wv; o < O; o += kBwdWaves) acc += W[(int64_t)o * K + k] * (d_act[o] * act_grad(act, a[o]));
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && k < K) {
    float tot = base ? base[k] : 0.f;
    for (int w = 0; w < kBwdWaves; ++w) tot += part[w][lane];
    din[k] = tot;
  }
}

// One wave per chip, the K thresholds split over its lanes (sums in lane
// order). y1 = sum_i (tanh(c (z - rho_i)) + 1) / (2B); s = exp(j 2 pi y1).
__global__ __launch_bounds__(kThreads) void k_soft(const float* __restrict__ z, const float* __restrict__ rho,
                                                    int D, int K, int B, float c, float2* s) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D) return;
  const float zn = z[n];
  float acc = 0.f;
  for (int i = lane; i < K; i += 64) acc += tanhf(c * (zn - rho[i])) + 1.0f;
  acc = wave_sum(acc);
  if (lane == 0) {
    const float y1 = acc / (2.0f * (float)B);
    float sn, cs;
    sincospif(2.0f * y1, &sn, &cs);
    s[n] = make_float2(cs, sn);
  }
}

// dy = 2 pi Im(grad_s conj(s)); dz = dy sum_i c (1 - t_i^2) / (2B); one wave per chip.
__global__ __launch_bounds__(kThreads) void k_chain(const float* __restrict__ z, const float* __restrict__ rho,
                                                     const float2* __restrict__ s, const float2* __restrict__ gs,
                                                     int D, int K, int B, float c, float* dy_out, float* dz_out) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D) return;
  const float zn = z[n];
  float d = 0.f;
  for (int i = lane; i < K; i += 64) {
    const float t = tanhf(c * (zn - rho[i]));
    d += 1.0f - t * t;
  }
  d = wave_sum(d);
  if (lane == 0) {
    const float2 g = gs[n], sv = s[n];
    const float dy = 2.0f * 3.14159265358979f * (g.y * sv.x - g.x * sv.y);
    dy_out[n] = dy;
    dz_out[n] = dy * d * c / (2.0f * (float)B);
  }
}

// drho_i = -sum_n dy_n c (1 - tanh(c (z_n - rho_i))^2) / (2B): one block per
// threshold, chips in a fixed order.
__global__ __launch_bounds__(kThreads) void k_drho(const float* __restrict__ z, const float* __restrict__ rho,
                                                    const float* __restrict__ dy, int D, int B, float c,
                                                    float* drho) {
  __shared__ float sh[kThreads / 64];
  const int i = blockIdx.x;
  const float r = rho[i];
  float acc = 0.f;
  for (int n = threadIdx.x; n < D; n += kThreads) {
    const float t = tanhf(c * (z[n] - r));
    acc += dy[n] * (1.0f - t * t);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.f;
    for (int w = 0; w < kThreads / 64; ++w) tot += sh[w];
    drho[i] = -tot * c / (2.0f * (float)B);
  }
}

// One wave per chip: the count of thresholds at or below z, mod B.
__global__ __launch_bounds__(kThreads) void k_hard(const float* __restrict__ z, const float* __restrict__ rho,
                                                    int D, int K, int B, int32_t* idx, float2* x) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D) return;
  const float zn = z[n];
  int cnt = 0;
  for (int i = lane; i < K; i += 64) cnt += rho[i] <= zn ? 1 : 0;
  cnt = (int)wave_sum((float)cnt);  // exact: counts <= 4096
  if (lane == 0) {
    const int k = cnt % B;
    if (idx) idx[n] = k;
    if (x) {
      float sn, cs;
      sincospif(2.0f * (float)k / (float)B, &sn, &cs);
      x[n] = make_float2(cs, sn);
    }
  }
}

// Step count t = step_mul * (*step) + step_add when step is given (a device
// counter, so that a captured graph replays with the current count), else
// step_add.
__global__ __launch_bounds__(kThreads) void k_adam(float* p, const float* __restrict__ g, float* m, float* v,
                                                    int64_t n, float lr, float b1, float b2, float eps,
                                                    const int32_t* step, int32_t step_mul, int32_t step_add) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const float t = (float)((step ? step_mul * *step : 0) + step_add);
  const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_count(int32_t* step) {
  if (threadIdx.x == 0) *step += 1;
}

// Ascending bitonic sort of K <= 4096 values in LDS (padded with +inf).
__global__ __launch_bounds__(1024) void k_sort(float* rho, int K) {
  __shared__ float v[kMaxK];
  int Kp = 1;
  while (Kp < K) Kp <<= 1;
  for (int i = threadIdx.x; i < Kp; i += 1024) v[i] = i < K ? rho[i] : INFINITY;
  __syncthreads();
  for (int size = 2; size <= Kp; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < Kp; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const float a = v[i], bv = v[j];
          if ((a > bv) == up) {
            v[i] = bv;
            v[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < K; i += 1024) rho[i] = v[i];
}

// h_m <- h_m sqrt(N / |h_m|^2), one block per row.
__global__ __launch_bounds__(kThreads) void k_project(float2* h, int N) {
  __shared__ float sh[kThreads / 64];
  float2* row = h + (int64_t)blockIdx.x * N;
  float e = 0.f;
  for (int n = threadIdx.x; n < N; n += kThreads) e += row[n].x * row[n].x + row[n].y * row[n].y;
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  float tot = 0.f;
  for (int w = 0; w < kThreads / 64; ++w) tot += sh[w];
  const float sc = sqrtf((float)N / tot);
  for (int n = threadIdx.x; n < N; n += kThreads) row[n] = make_float2(row[n].x * sc, row[n].y * sc);
}

// Layer sizes and parameter offsets (floats) of theta for D inputs.
struct Layers {
  int in[2 * kBlocks + 2], out[2 * kBlocks + 2];
  int64_t w[2 * kBlocks + 2], b[2 * kBlocks + 2];
  int64_t total;
  explicit Layers(int D) {
    int64_t off = 0;
    for (int l = 0; l < 2 * kBlocks + 2; ++l) {
      in[l] = l == 0 ? D : kH;
      out[l] = l == 2 * kBlocks + 1 ? D : kH;
      w[l] = off;
      off += (int64_t)in[l] * out[l];
      b[l] = off;
      off += out[l];
    }
    total = off;
  }
};

// Workspace (floats): h[0..5][H], u[1..5][H], v[1..5][H], dh[2][H], du[H], dy[D], dz[D].
struct WsLayout {
  int64_t h, u, v, dh, du, dy, dz, total;
  explicit WsLayout(int D) {
    h = 0;
    u = h + (int64_t)(kBlocks + 1) * kH;
    v = u + (int64_t)kBlocks * kH;
    dh = v + (int64_t)kBlocks * kH;
    du = dh + 2 * kH;
    dy = du + kH;
    dz = dy + D;
    total = dz + D;
  }
};

inline int blocks_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

int validate(const sqngd_sqn_shape* s) {
  if (s == nullptr) return SQNGD_E_INVALID_ARG;
  if (s->M < 1 || s->N < 1 || s->B < 2 || s->copies < 1) return SQNGD_E_INVALID_ARG;
  if (!std::isfinite(s->c) || s->c <= 0.f) return SQNGD_E_INVALID_ARG;
  if (s->reserved[0] != 0 || s->reserved[1] != 0 || s->reserved[2] != 0) return SQNGD_E_INVALID_ARG;
  if ((int64_t)s->M * s->N > kMaxD || s->B > 64 || (int64_t)s->B * s->copies > kMaxK) return SQNGD_E_UNSUPPORTED;
  return SQNGD_OK;
}

}  // namespace sqsqn

extern "C" {

int sqngd_sqn_param_count(int32_t D, int64_t* count) {
  if (count == nullptr || D < 1) return SQNGD_E_INVALID_ARG;
  if (D > sqsqn::kMaxD) return SQNGD_E_UNSUPPORTED;
  *count = sqsqn::Layers(D).total;
  return SQNGD_OK;
}

int sqngd_sqn_workspace_size(const sqngd_sqn_shape* shape, size_t* bytes) {
  int rc = sqsqn::validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (bytes == nullptr) return SQNGD_E_INVALID_ARG;
  *bytes = align_up(4 * (size_t)sqsqn::WsLayout(shape->M * shape->N).total);
  return SQNGD_OK;
}

int sqngd_sqn_forward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, float* z, void* ws,
                      size_t ws_bytes, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (theta == nullptr || y0 == nullptr || z == nullptr || ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(theta, 4) || !aligned(y0, 4) || !aligned(z, 4) || !aligned(ws, kAlign))
    return SQNGD_E_ALIGN;
  const int D = shape->M * shape->N;
  const WsLayout L(D);
  if (ws_bytes < 4 * (size_t)L.total) return SQNGD_E_WORKSPACE;
  const Layers Y(D);
  hipStream_t s = (hipStream_t)stream;
  float* f = (float*)ws;
  float* h = f + L.h;
  const int wb = kThreads / 64;
  hipLaunchKernelGGL(k_dense_fwd<ACT_TANH>, dim3((kH + wb - 1) / wb), dim3(kThreads), 0, s, y0, D, theta + Y.w[0],
                     theta + Y.b[0], kH, (const float*)nullptr, (float*)nullptr, h);
  for (int k = 0; k < kBlocks; ++k) {
    const int l1 = 1 + 2 * k, l2 = 2 + 2 * k;
    float* u = f + L.u + (int64_t)k * kH;
    float* v = f + L.v + (int64_t)k * kH;
    hipLaunchKernelGGL(k_dense_fwd<ACT_TANH>, dim3((kH + wb - 1) / wb), dim3(kThreads), 0, s,
                       (const float*)(h + (int64_t)k * kH), kH, theta + Y.w[l1], theta + Y.b[l1], kH,
                       (const float*)nullptr, u, (float*)nullptr);
    hipLaunchKernelGGL(k_dense_fwd<ACT_TANH>, dim3((kH + wb - 1) / wb), dim3(kThreads), 0, s, (const float*)u, kH,
                       theta + Y.w[l2], theta + Y.b[l2], kH, (const float*)(h + (int64_t)k * kH), v,
                       h + (int64_t)(k + 1) * kH);
  }
  const int lo = 2 * kBlocks + 1;
  hipLaunchKernelGGL(k_dense_fwd<ACT_SIGMOID>, dim3((D + wb - 1) / wb), dim3(kThreads), 0, s,
                     (const float*)(h + (int64_t)kBlocks * kH), kH, theta + Y.w[lo], theta + Y.b[lo], D,
                     (const float*)nullptr, (float*)nullptr, z);
  return check_launch();
}

int sqngd_sqn_soft(const sqngd_sqn_shape* shape, const float* z, const float* rho, sqngd_c64* sw, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (z == nullptr || rho == nullptr || sw == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(rho, 4) || !aligned(sw, 8)) return SQNGD_E_ALIGN;
  const int D = shape->M * shape->N, K = shape->B * shape->copies;
  hipLaunchKernelGGL(k_soft, dim3(blocks_for(64 * (int64_t)D)), dim3(kThreads), 0, (hipStream_t)stream, z, rho, D, K, shape->B,
                     shape->c, (float2*)sw);
  return check_launch();
}

int sqngd_sqn_hard(const sqngd_sqn_shape* shape, const float* z, const float* rho, int32_t* idx, sqngd_c64* x,
                   void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (z == nullptr || rho == nullptr || (idx == nullptr && x == nullptr)) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(rho, 4) || !aligned(idx, 4) || !aligned(x, 8)) return SQNGD_E_ALIGN;
  const int D = shape->M * shape->N, K = shape->B * shape->copies;
  hipLaunchKernelGGL(k_hard, dim3(blocks_for(64 * (int64_t)D)), dim3(kThreads), 0, (hipStream_t)stream, z, rho, D, K, shape->B,
                     idx, (float2*)x);
  return check_launch();
}

int sqngd_sqn_backward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, const float* z,
                       const float* rho, const sqngd_c64* sw, const sqngd_c64* grad_s, float* grad_theta,
                       float* grad_rho, void* ws, size_t ws_bytes, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (theta == nullptr || y0 == nullptr || z == nullptr || rho == nullptr || sw == nullptr || grad_s == nullptr ||
      grad_theta == nullptr || grad_rho == nullptr || ws == nullptr)
    return SQNGD_E_INVALID_ARG;
  if (!aligned(theta, 4) || !aligned(y0, 4) || !aligned(z, 4) || !aligned(rho, 4) || !aligned(sw, 8) ||
      !aligned(grad_s, 8) || !aligned(grad_theta, 4) || !aligned(grad_rho, 4) ||
      !aligned(ws, kAlign))
    return SQNGD_E_ALIGN;
  const int D = shape->M * shape->N, K = shape->B * shape->copies, B = shape->B;
  const WsLayout L(D);
  if (ws_bytes < 4 * (size_t)L.total) return SQNGD_E_WORKSPACE;
  const Layers Y(D);
  hipStream_t s = (hipStream_t)stream;
  float* f = (float*)ws;
  float* h = f + L.h;
  float* dy = f + L.dy;
  float* dz = f + L.dz;
  float* dh[2] = {f + L.dh, f + L.dh + kH};
  float* du = f + L.du;
  // staircase: dL/dy1, dL/dz and dL/drho
  hipLaunchKernelGGL(k_chain, dim3(blocks_for(64 * (int64_t)D)), dim3(kThreads), 0, s, z, rho, (const float2*)sw,
                     (const float2*)grad_s, D, K, B, shape->c, dy, dz);
  hipLaunchKernelGGL(k_drho, dim3(K), dim3(kThreads), 0, s, z, rho, (const float*)dy, D, B, shape->c, grad_rho);
  // output layer: a = z (sigmoid), input h_5
  const int lo = 2 * kBlocks + 1;
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks_for((int64_t)D * kH)), dim3(kThreads), 0, s, (const float*)dz, z,
                     (int)ACT_SIGMOID, (const float*)(h + (int64_t)kBlocks * kH), kH, D, grad_theta + Y.w[lo],
                     grad_theta + Y.b[lo]);
  hipLaunchKernelGGL(k_dense_bwd_in, dim3((kH + 63) / 64), dim3(64 * kBwdWaves), 0, s, theta + Y.w[lo], (const float*)dz, z,
                     (int)ACT_SIGMOID, kH, D, (const float*)nullptr, dh[0]);
  int cur = 0;
  for (int k = kBlocks - 1; k >= 0; --k) {
    const int l1 = 1 + 2 * k, l2 = 2 + 2 * k;
    const float* u = f + L.u + (int64_t)k * kH;
    const float* v = f + L.v + (int64_t)k * kH;
    // residual branch, second layer: a = v, input u, upstream dh
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks_for((int64_t)kH * kH)), dim3(kThreads), 0, s,
                       (const float*)dh[cur], v, (int)ACT_TANH, u, kH, kH, grad_theta + Y.w[l2], grad_theta + Y.b[l2]);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3((kH + 63) / 64), dim3(64 * kBwdWaves), 0, s, theta + Y.w[l2],
                       (const float*)dh[cur], v, (int)ACT_TANH, kH, kH, (const float*)nullptr, du);
    // first layer: a = u, input h_{k}, upstream du; dh_new = dh + W1^T dp
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks_for((int64_t)kH * kH)), dim3(kThreads), 0, s, (const float*)du, u,
                       (int)ACT_TANH, (const float*)(h + (int64_t)k * kH), kH, kH, grad_theta + Y.w[l1],
                       grad_theta + Y.b[l1]);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3((kH + 63) / 64), dim3(64 * kBwdWaves), 0, s, theta + Y.w[l1], (const float*)du,
                       u, (int)ACT_TANH, kH, kH, (const float*)dh[cur], dh[cur ^ 1]);
    cur ^= 1;
  }
  // input layer: a = h_0, input y0 (its own gradient is not needed)
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks_for((int64_t)kH * D)), dim3(kThreads), 0, s, (const float*)dh[cur],
                     (const float*)h, (int)ACT_TANH, y0, D, kH, grad_theta + Y.w[0], grad_theta + Y.b[0]);
  return check_launch();
}

int sqngd_sqn_adam(float* p, const float* g, float* m, float* v, int64_t n, const int32_t* step, int32_t step_mul,
                   int32_t step_add, float lr, float beta1, float beta2, float eps, void* stream) {
  using namespace sqsqn;
  if (p == nullptr || g == nullptr || m == nullptr || v == nullptr || n < 1) return SQNGD_E_INVALID_ARG;
  if (step_mul < 0 || step_add < 0 || (step == nullptr && step_add < 1)) return SQNGD_E_INVALID_ARG;
  if (!std::isfinite(lr) || lr < 0.f || !(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f) ||
      !std::isfinite(eps) || eps <= 0.f)
    return SQNGD_E_INVALID_ARG;
  if (!aligned(p, 4) || !aligned(g, 4) || !aligned(m, 4) || !aligned(v, 4) || !aligned(step, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, p, g, m, v, n, lr, beta1,
                     beta2, eps, step, step_mul, step_add);
  return check_launch();
}

int sqngd_sqn_count(int32_t* step, void* stream) {
  using namespace sqsqn;
  if (step == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(step, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_count, dim3(1), dim3(64), 0, (hipStream_t)stream, step);
  return check_launch();
}

int sqngd_sqn_sort(float* rho, int32_t K, void* stream) {
  using namespace sqsqn;
  if (rho == nullptr || K < 1) return SQNGD_E_INVALID_ARG;
  if (K > kMaxK) return SQNGD_E_UNSUPPORTED;
  if (!aligned(rho, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_sort, dim3(1), dim3(1024), 0, (hipStream_t)stream, rho, (int)K);
  return check_launch();
}

int sqngd_sqn_project(int32_t M, int32_t N, sqngd_c64* h, void* stream) {
  using namespace sqsqn;
  if (h == nullptr || M < 1 || N < 1) return SQNGD_E_INVALID_ARG;
  if (!aligned(h, 8)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_project, dim3(M), dim3(kThreads), 0, (hipStream_t)stream, (float2*)h, (int)N);
  return check_launch();
}

}  // extern "C"
