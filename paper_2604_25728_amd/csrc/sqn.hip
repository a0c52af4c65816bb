// sqn.hip - gfx950 kernels and C ABI of the paper's transmit parameterisation
// (Sec. III-A; declared in include/sqngd_sqn.h). Included by api.hip after
// its host helpers (one translation unit).
//
// The network runs on a single input vector, so every dense layer is a
// matrix-vector product bound by reading its weights once. The wide input
// and output layers spread over the chip (one wavefront per output, lanes
// stride over the inputs, a DPP sum in lane order, so results are the same
// run to run); the ten 128 x 128 hidden layers run in one workgroup that
// keeps the activations in LDS, forward and backward, instead of twenty
// dependent launches. The weight and bias gradients of all layers are outer
// products, written by one launch over theta's layout. The staircase, its
// gradient and the hard quantiser take one wave per chip with the thresholds
// over the lanes; Adam, the ordered projection of the thresholds (a bitonic
// sort in LDS) and the filters' energy projection are element- or row-wise.
#include "../../include/sqngd_sqn.h"

namespace sqsqn {

using sq::wave_sum;

constexpr int kH = 128;       // hidden width
constexpr int kBlocks = 5;    // residual blocks
constexpr int kThreads = 256;
constexpr int kMaxD = 4096;
constexpr int kMaxK = 4096;

enum Act : int { ACT_TANH = 0, ACT_SIGMOID = 1, ACT_NONE = 2 };

// a[o] = act(W[o][:] . in + b[o]); out[o] = res[o] + a[o] when res is given.
// Design r = blockIdx.y: in, W / b and the outputs advance by their strides.
template <int ACT>
__global__ __launch_bounds__(kThreads) void k_dense_fwd(const float* __restrict__ in, int K,
                                                         const float* __restrict__ W, const float* __restrict__ b,
                                                         int O, const float* __restrict__ res, float* a_out,
                                                         float* out, int64_t in_str, int64_t w_str,
                                                         int64_t out_str) {
  const int o = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= O) return;
  const int64_t r = blockIdx.y;
  in += r * in_str;
  W += r * w_str;
  b += r * w_str;
  if (res) res += r * out_str;
  if (a_out) a_out += r * out_str;
  if (out) out += r * out_str;
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
  return act == ACT_TANH ? 1.0f - a * a : (act == ACT_SIGMOID ? a * (1.0f - a) : 1.0f);
}

// The ten hidden layers (five residual blocks) in one workgroup: activations
// stay in LDS, each layer's 128 x 128 weights stream from L2 once, and a wave
// owns 8 outputs (the same lane-strided dot product and DPP sum as
// k_dense_fwd). th points at the first hidden layer's weights; layers follow
// at kHidStride floats. h[0] holds the input-layer activation; h[1..5], u, v
// are written for the backward pass.
constexpr int kStackThreads = 1024;
constexpr int kStackWaves = kStackThreads / 64;
constexpr int kOutPerWave = kH / kStackWaves;
constexpr int64_t kHidStride = (int64_t)kH * kH + kH;
static_assert(kH == 128 && kOutPerWave * kStackWaves == kH, "hidden-stack tiling");

// A wave owns the 8 outputs o = 8 wv + j; lane 8 j + c computes the partial
// dot product of row o over the 16 inputs [16 c, 16 c + 16) (in order) and
// the 8 partials of a row are added by a DPP sum within the lane group, so a
// layer costs one short reduction per wave instead of one per output. The
// weights do not depend on the activations, so they are loaded kAhead - 1
// layers ahead of their use.
constexpr int kAhead = 5;
constexpr int kSeg = kH / 8;  // inputs per lane
struct StackW {
  float4 w[kSeg / 4];
  float b;
};
__device__ __forceinline__ StackW stack_load(const float* __restrict__ W, int wv, int lane) {
  StackW r;
  const int o = wv * kOutPerWave + (lane >> 3), c = lane & 7;
  const float4* row = (const float4*)(W + (int64_t)o * kH + c * kSeg);
#pragma unroll
  for (int q = 0; q < kSeg / 4; ++q) r.w[q] = row[q];
  r.b = W[(int64_t)kH * kH + o];
  return r;
}

__device__ __forceinline__ void stack_layer(const StackW& L, const float* in, int wv, int lane, float* res,
                                            float* a_lds, float* a_glob) {
  const int o = wv * kOutPerWave + (lane >> 3), c = lane & 7;
  const float4* x = (const float4*)(in + c * kSeg);
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < kSeg / 4; ++q) {
    const float4 xv = x[q];
    acc += L.w[q].x * xv.x;
    acc += L.w[q].y * xv.y;
    acc += L.w[q].z * xv.z;
    acc += L.w[q].w * xv.w;
  }
  // sum over the lane group 8 j .. 8 j + 7: after row_shr 1, 2, 4 its last
  // lane holds lanes 8 j .. 8 j + 7 (lanes shifted in from outside the row add 0)
  acc += sq::dpp_f<0x111, 0xF>(0.f, acc);
  acc += sq::dpp_f<0x112, 0xF>(0.f, acc);
  acc += sq::dpp_f<0x114, 0xF>(0.f, acc);
  acc = __shfl(acc, (lane & ~7) + 7);
  if (c == 0) {
    const float a = tanhf(acc + L.b);
    a_lds[o] = a;
    a_glob[o] = a;
    if (res) res[o] += a;
  }
}

__global__ __launch_bounds__(kStackThreads) void k_res_fwd(const float* __restrict__ th, float* h, float* u,
                                                            float* v, int64_t th_str, int64_t ws_str) {
  // one workgroup per design
  th += blockIdx.x * th_str;
  h += blockIdx.x * ws_str;
  u += blockIdx.x * ws_str;
  v += blockIdx.x * ws_str;
  __shared__ __align__(16) float xs[kH];
  __shared__ __align__(16) float us[kH];
  __shared__ float vs[kH];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the input activation is loaded first, so the barrier waits for it
  // alone while the first layers' weights are still in flight
  const float h0 = threadIdx.x < kH ? h[threadIdx.x] : 0.f;
  StackW buf[kAhead];
#pragma unroll
  for (int l = 0; l + 1 < kAhead; ++l) buf[l] = stack_load(th + l * kHidStride, wv, lane);
  if (threadIdx.x < kH) xs[threadIdx.x] = h0;
  __syncthreads();
#pragma unroll
  for (int l = 0; l < 2 * kBlocks; ++l) {
    if (l + kAhead - 1 < 2 * kBlocks)
      buf[(l + kAhead - 1) % kAhead] = stack_load(th + (l + kAhead - 1) * kHidStride, wv, lane);
    const int k = l >> 1;
    if ((l & 1) == 0) {
      stack_layer(buf[l % kAhead], xs, wv, lane, nullptr, us, u + k * kH);
      __syncthreads();
    } else {
      stack_layer(buf[l % kAhead], us, wv, lane, xs, vs, v + k * kH);
      __syncthreads();
      if (threadIdx.x < kH) h[(k + 1) * kH + threadIdx.x] = xs[threadIdx.x];
    }
  }
}

// out[k] = sum_o W[o][k] d[o] over the hidden width, 16 waves: wave w takes
// the inputs k = 64 (w & 1) + lane and the outputs o in [16 (w >> 1), +16);
// the eight partial sums per input are added in order by the caller. The
// weights are loaded kAhead - 1 layers ahead (stack_tload) like the forward's.
struct StackT {
  float w[16];
};
__device__ __forceinline__ StackT stack_tload(const float* __restrict__ W, int wv, int lane) {
  StackT r;
  const int kk = (wv & 1) * 64 + lane, g = wv >> 1;
#pragma unroll
  for (int j = 0; j < 16; ++j) r.w[j] = W[(int64_t)(g * 16 + j) * kH + kk];
  return r;
}
__device__ __forceinline__ void stack_transposed(const StackT& T, const float* d, int wv, int lane,
                                                 float (*red)[kH]) {
  const int kk = (wv & 1) * 64 + lane, g = wv >> 1;
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc += T.w[j] * d[g * 16 + j];
  red[g][kk] = acc;
}

// Backward through the hidden stack in one workgroup. The gradient into h_5
// arrives as S partial sums [S][H] (from k_dense_bwd_part); dp[l][:] receives
// the pre-activation gradient of layer l = 0..10 (layer 0 is the input layer)
// for k_dw_all.
__global__ __launch_bounds__(kStackThreads) void k_res_bwd(const float* __restrict__ th,
                                                            const float* __restrict__ part, int S,
                                                            const float* __restrict__ h, const float* __restrict__ u,
                                                            const float* __restrict__ v, float* dp, int64_t th_str,
                                                            int64_t ws_str) {
  // one workgroup per design
  th += blockIdx.x * th_str;
  part += blockIdx.x * ws_str;
  h += blockIdx.x * ws_str;
  u += blockIdx.x * ws_str;
  v += blockIdx.x * ws_str;
  dp += blockIdx.x * ws_str;
  __shared__ float dh[kH], ds[kH];
  __shared__ float red[8][kH];
  __shared__ float us[kBlocks * kH], vs[kBlocks * kH];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // the forward's activations are staged in LDS so the chain below waits on
  // no global load but the (prefetched) weights; all of these loads and the
  // first layers' weights are in flight together
  static_assert(kBlocks * kH <= kStackThreads, "one staged value per thread");
  const float uv = t < kBlocks * kH ? u[t] : 0.f, vv = t < kBlocks * kH ? v[t] : 0.f;
  const float h0 = t < kH ? h[t] : 0.f;
  float acc0 = 0.f;
  if (t < kH)
    for (int i = 0; i < S; ++i) acc0 += part[i * kH + t];
  // hidden layers from the last (10) down to 1; buffer i holds layer 10 - i
  StackT buf[kAhead];
#pragma unroll
  for (int i = 0; i + 1 < kAhead; ++i) buf[i] = stack_tload(th + (2 * kBlocks - 1 - i) * kHidStride, wv, lane);
  if (t < kBlocks * kH) {
    us[t] = uv;
    vs[t] = vv;
  }
  if (t < kH) dh[t] = acc0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2 * kBlocks; ++i) {
    const int l = 2 * kBlocks - i, k = (l - 1) >> 1;
    if (i + kAhead - 1 < 2 * kBlocks)
      buf[(i + kAhead - 1) % kAhead] = stack_tload(th + (l - kAhead) * kHidStride, wv, lane);
    if (t < kH) {
      // second layer of block k (a = v_k, upstream dh) or first (a = u_k, upstream du)
      float d;
      if ((l & 1) == 0) {
        d = dh[t] * act_grad(ACT_TANH, vs[k * kH + t]);
      } else {
        float du = 0.f;
        for (int g = 0; g < 8; ++g) du += red[g][t];
        d = du * act_grad(ACT_TANH, us[k * kH + t]);
      }
      ds[t] = d;
      dp[l * kH + t] = d;
    }
    __syncthreads();
    stack_transposed(buf[i % kAhead], ds, wv, lane, red);
    __syncthreads();
    if ((l & 1) == 1) {
      // dh_k = dh_{k+1} + W1^T dp1
      if (t < kH) {
        float acc = dh[t];
        for (int g = 0; g < 8; ++g) acc += red[g][t];
        dh[t] = acc;
      }
      __syncthreads();
    }
  }
  if (t < kH) dp[t] = dh[t] * act_grad(ACT_TANH, h0);
}

// part[s][k] = sum over o in chunk s of W[o][k] dp[o], dp[o] = d_act[o]
// act'(a[o]): blocks (input tile of 64, chunk s); the block's 16 waves stride
// over the chunk's outputs and are added in wave order.
constexpr int kBwdWaves = 16;
constexpr int kBwdSplit = 16;
__global__ __launch_bounds__(64 * kBwdWaves) void k_dense_bwd_part(const float* __restrict__ W,
                                                                    const float* __restrict__ d_act,
                                                                    const float* __restrict__ a, int act, int K,
                                                                    int O, float* part, int64_t w_str, int64_t d_str,
                                                                    int64_t a_str, int64_t part_str) {
  // design r = blockIdx.z
  const int64_t r = blockIdx.z;
  W += r * w_str;
  d_act += r * d_str;
  a += r * a_str;
  part += r * part_str;
  __shared__ float sh[kBwdWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const int chunk = (O + kBwdSplit - 1) / kBwdSplit;
  const int o0 = blockIdx.y * chunk, o1 = min(O, o0 + chunk);
  float acc = 0.f;
  if (k < K)
    for (int o = o0 + wv; o < o1; o += kBwdWaves) acc += W[(int64_t)o * K + k] * (d_act[o] * act_grad(act, a[o]));
  sh[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && k < K) {
    float tot = 0.f;
    for (int w = 0; w < kBwdWaves; ++w) tot += sh[w][lane];
    part[(int64_t)blockIdx.y * K + k] = tot;
  }
}

struct AdamArgs {
  float lr, b1, b2, eps;
  const int32_t* step;
  int32_t step_mul, step_add;
};
struct AdamBias {
  float bc1, bc2;
};
__device__ __forceinline__ AdamBias adam_bias(const AdamArgs& A) {
  const float t = (float)((A.step ? A.step_mul * *A.step : 0) + A.step_add);
  return {1.0f - powf(A.b1, t), 1.0f - powf(A.b2, t)};
}
// One element: moments updated in place, the new parameter returned.
__device__ __forceinline__ float adam_elem(float p, float gi, float* m, float* v, const AdamArgs& A,
                                           const AdamBias& c) {
  const float mi = A.b1 * *m + (1.0f - A.b1) * gi;
  const float vi = A.b2 * *v + (1.0f - A.b2) * gi * gi;
  *m = mi;
  *v = vi;
  return p - A.lr * (mi / c.bc1) / (sqrtf(vi / c.bc2) + A.eps);
}

// Weight and bias gradients of every layer in one launch over theta's
// layout: dW[o][k] = dp[o] x[k], db[o] = dp[o], with dp[o] = d[o] act'(a[o])
// (act = ACT_NONE when d already is the pre-activation gradient).
constexpr int kLayers = 2 * kBlocks + 2;
constexpr int kDwPer = 4;  // parameters per thread of k_dw_all
struct DwArgs {
  int64_t w[kLayers], b[kLayers];
  const float* d[kLayers];
  const float* a[kLayers];
  const float* x[kLayers];
  int64_t dstr[kLayers], astr[kLayers], xstr[kLayers];  // per-design strides of d, a, x
  int in[kLayers], act[kLayers];
  int bstart[kLayers + 1];  // first block of each layer (a block never spans two layers)
  float* g;
  int64_t total;  // parameters per design (the stride of g)
  // when theta is set, the gradient is not written: Adam updates theta (and
  // m, v) in place with it, the arithmetic of k_adam
  float* theta;
  float* m;
  float* v;
  AdamArgs adam;
};

__global__ __launch_bounds__(kThreads) void k_dw_all(DwArgs A) {
  // the layer is uniform per block (found from blockIdx, scalar work), so
  // each thread only splits its index into row and column
  const int bx = blockIdx.x;
  int l = 0;
#pragma unroll
  for (int q = 1; q < kLayers; ++q) l = bx >= A.bstart[q] ? q : l;
  int w = 0, b = 0, in = 1, act = ACT_NONE;
  const float *d = nullptr, *a = nullptr, *x = nullptr;
  int64_t dstr = 0, astr = 0, xstr = 0;
  int b0 = 0;
#pragma unroll
  for (int q = 0; q < kLayers; ++q)
    if (q == l) {
      w = (int)A.w[q];
      b = (int)A.b[q];
      in = A.in[q];
      act = A.act[q];
      d = A.d[q];
      a = A.a[q];
      x = A.x[q];
      dstr = A.dstr[q];
      astr = A.astr[q];
      xstr = A.xstr[q];
      b0 = A.bstart[q];
    }
  // layer l covers theta[w, b + out) with out = (b - w) / in; a block takes
  // kDwPer * kThreads consecutive parameters, a thread every kThreads-th
  const int end = b + (b - w) / in;
  const int64_t r = blockIdx.y;  // design
  d += r * dstr;
  if (a) a += r * astr;
  x += r * xstr;
  const AdamBias c = A.theta ? adam_bias(A.adam) : AdamBias{1.f, 1.f};
  const int i0 = w + (bx - b0) * (kDwPer * kThreads) + (int)threadIdx.x;
#pragma unroll
  for (int j = 0; j < kDwPer; ++j) {
    const int i = i0 + j * kThreads;
    if (i >= end) break;
    float gv;
    if (i < b) {
      const unsigned e = (unsigned)(i - w);
      const int o = (int)(e / (unsigned)in), k = (int)(e - (unsigned)o * (unsigned)in);
      gv = d[o] * act_grad(act, a ? a[o] : 0.f) * x[k];
    } else {
      const int o = i - b;
      gv = d[o] * act_grad(act, a ? a[o] : 0.f);
    }
    const int64_t gi = r * A.total + i;
    if (A.theta)
      A.theta[gi] = adam_elem(A.theta[gi], gv, A.m + gi, A.v + gi, A.adam, c);
    else
      A.g[gi] = gv;
  }
}

// Staircase term and slope of one threshold at u = c (z - rho_i), from
// e = exp(-2|u|) so that neither cancels where tanh(u) rounds to +-1:
//   tanh(u) + 1 = 2 [u > 0] + q_sgn,  q_sgn = -q (u > 0), +q (u <= 0),  q = 2e / (1 + e)
//   tanh'(u) = 1 - tanh(u)^2 = 4e / (1 + e)^2.
__device__ __forceinline__ float stair_e(float u) { return expf(-2.0f * fabsf(u)); }
__device__ __forceinline__ float stair_slope(float e) {
  const float d = 1.0f + e;
  return 4.0f * e / (d * d);
}

// One wave per chip, the K thresholds split over its lanes (sums in lane
// order). y1 = sum_i (tanh(c (z - rho_i)) + 1) / (2B) = (cnt + frac / 2) / B
// with cnt the thresholds below z (u > 0) and frac the signed q terms;
// s = exp(j 2 pi y1) takes the phase from (cnt mod B + frac / 2) / B, which
// keeps FP32's resolution of the fraction however many copies the staircase
// has (y1 itself reaches K / B turns).
// Chips n of all R designs in one range (design n / D, thresholds rho[r][:]).
__global__ __launch_bounds__(kThreads) void k_soft(const float* __restrict__ z, const float* __restrict__ rho,
                                                    int D, int R, int K, int B, float c, float2* s) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D * R) return;
  rho += (int64_t)(n / D) * K;
  const float zn = z[n];
  float frac = 0.f;
  int cnt = 0;
  for (int i = lane; i < K; i += 64) {
    const float u = c * (zn - rho[i]);
    const float e = stair_e(u);
    const float q = 2.0f * e / (1.0f + e);
    cnt += u > 0.f ? 1 : 0;
    frac += u > 0.f ? -q : q;
  }
  frac = wave_sum(frac);
  cnt = (int)wave_sum((float)cnt);  // exact: counts <= 4096
  if (lane == 0) {
    const float y1 = ((float)(cnt % B) + 0.5f * frac) / (float)B;
    float sn, cs;
    sincospif(2.0f * (y1 - rintf(y1)), &sn, &cs);
    s[n] = make_float2(cs, sn);
  }
}

// dy = 2 pi Im(g conj(s)) with g = gs (+ gh when given); dz = dy sum_i c
// tanh'(c (z - rho_i)) / (2B); one wave per chip.
__global__ __launch_bounds__(kThreads) void k_chain(const float* __restrict__ z, const float* __restrict__ rho,
                                                     const float2* __restrict__ s, const float2* __restrict__ gs,
                                                     const float2* __restrict__ gh, int D, int R, int K, int B,
                                                     float c, float* dy_out, float* dz_out, int64_t ws_str) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D * R) return;
  const int r = n / D;
  rho += (int64_t)r * K;
  dy_out += r * ws_str - (int64_t)r * D;  // dy_out[n] is design r's dy[n - r D]
  dz_out += r * ws_str - (int64_t)r * D;
  const float zn = z[n];
  float d = 0.f;
  for (int i = lane; i < K; i += 64) d += stair_slope(stair_e(c * (zn - rho[i])));
  d = wave_sum(d);
  if (lane == 0) {
    float2 g = gs[n];
    if (gh) g = make_float2(g.x + gh[n].x, g.y + gh[n].y);
    const float2 sv = s[n];
    const float dy = 2.0f * 3.14159265358979f * (g.y * sv.x - g.x * sv.y);
    dy_out[n] = dy;
    dz_out[n] = dy * d * c / (2.0f * (float)B);
  }
}

// drho_i = -sum_n dy_n c tanh'(c (z_n - rho_i)) / (2B): one block per
// threshold, chips in a fixed order.
__global__ __launch_bounds__(kThreads) void k_drho(const float* __restrict__ z, const float* __restrict__ rho,
                                                    const float* __restrict__ dy, int D, int B, float c,
                                                    float* drho, int K, int64_t ws_str) {
  __shared__ float sh[kThreads / 64];
  const int i = blockIdx.x;
  const int64_t dsg = blockIdx.y;  // design
  z += dsg * D;
  rho += dsg * K;
  dy += dsg * ws_str;
  drho += dsg * K;
  const float r = rho[i];
  float acc = 0.f;
  for (int n = threadIdx.x; n < D; n += kThreads) {
    acc += dy[n] * stair_slope(stair_e(c * (z[n] - r)));
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
                                                    int D, int R, int K, int B, int32_t* idx, float2* x) {
  const int n = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= D * R) return;
  rho += (int64_t)(n / D) * K;
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
// kDwPer elements per thread (the bias correction, two powf, once per thread)
__global__ __launch_bounds__(kThreads) void k_adam(float* p, const float* __restrict__ g, float* m, float* v,
                                                    int64_t n, AdamArgs A) {
  const int64_t i0 = (int64_t)blockIdx.x * (kDwPer * kThreads) + threadIdx.x;
  if (i0 >= n) return;
  const AdamBias c = adam_bias(A);
#pragma unroll
  for (int j = 0; j < kDwPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kThreads;
    if (i >= n) break;
    p[i] = adam_elem(p[i], g[i], m + i, v + i, A, c);
  }
}

// Adam on one filter row (2 N floats, Re and Im interleaved) followed by its
// energy projection: the same arithmetic and sum order as k_adam then
// k_project, in one launch (one block per row).
__global__ __launch_bounds__(kThreads) void k_adam_project(float2* h, const float2* __restrict__ g, float* m,
                                                            float* v, int N, AdamArgs A) {
  __shared__ float sh[kThreads / 64];
  const int64_t r0 = (int64_t)blockIdx.x * N;
  float2* row = h + r0;
  const AdamBias c = adam_bias(A);
  float e = 0.f;
  for (int n = threadIdx.x; n < N; n += kThreads) {
    const float2 gv = g[r0 + n], pv = row[n];
    const int64_t i = 2 * (r0 + n);
    const float2 q = make_float2(adam_elem(pv.x, gv.x, m + i, v + i, A, c), adam_elem(pv.y, gv.y, m + i + 1, v + i + 1, A, c));
    row[n] = q;
    e += q.x * q.x + q.y * q.y;
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  float tot = 0.f;
  for (int w = 0; w < kThreads / 64; ++w) tot += sh[w];
  const float sc = sqrtf((float)N / tot);
  for (int n = threadIdx.x; n < N; n += kThreads) row[n] = make_float2(row[n].x * sc, row[n].y * sc);
}

__global__ void k_count(int32_t* step) {
  if (threadIdx.x == 0) *step += 1;
}

// Ascending bitonic sort of K <= 4096 values in LDS (padded with +inf). A
// rank sort (each value placed by counting smaller keys) measured slower at
// the paper's K = 400: its K^2 comparisons run on the one CU.
__device__ __forceinline__ void bitonic_lds(float* v, int K, float* rho);

__global__ __launch_bounds__(1024) void k_sort(float* rho, int K) {
  rho += (int64_t)blockIdx.x * K;  // one workgroup per design
  __shared__ float v[kMaxK];
  int Kp = 1;
  while (Kp < K) Kp <<= 1;
  for (int i = threadIdx.x; i < Kp; i += 1024) v[i] = i < K ? rho[i] : INFINITY;
  __syncthreads();
  bitonic_lds(v, K, rho);
}

// Adam on one design's K thresholds, then the same bitonic sort (one launch).
__global__ __launch_bounds__(1024) void k_adam_sort(float* rho, const float* __restrict__ g, float* m, float* vv,
                                                     int K, AdamArgs A) {
  const int64_t r0 = (int64_t)blockIdx.x * K;
  rho += r0;
  g += r0;
  m += r0;
  vv += r0;
  __shared__ float v[kMaxK];
  int Kp = 1;
  while (Kp < K) Kp <<= 1;
  const AdamBias c = adam_bias(A);
  for (int i = threadIdx.x; i < Kp; i += 1024) v[i] = i < K ? adam_elem(rho[i], g[i], m + i, vv + i, A, c) : INFINITY;
  __syncthreads();
  bitonic_lds(v, K, rho);
}

// Ascending bitonic network over v[0..Kp) (Kp = K rounded up to a power of
// two, padded with +inf by the caller, then a barrier); the first K values go
// to rho. Every thread of the block calls it (it holds barriers).
__device__ __forceinline__ void bitonic_lds(float* v, int K, float* rho) {
  // thresholds after a small Adam step are mostly still in order: one
  // comparison pass skips the network then (a sorted array is its own sort)
  int unsorted = 0;
  for (int i = threadIdx.x; i + 1 < K; i += 1024) unsorted |= v[i] > v[i + 1] ? 1 : 0;
  if (__syncthreads_or(unsorted) == 0) {
    for (int i = threadIdx.x; i < K; i += 1024) rho[i] = v[i];
    return;
  }
  int Kp = 1;
  while (Kp < K) Kp <<= 1;
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

// Workspace (floats): h[0..5][H], u[1..5][H], v[1..5][H], dy[D], dz[D],
// dp[11][H] (pre-activation gradients of the input and hidden layers) and
// part[kBwdSplit][H] (split sums of the output layer's transposed product).
struct WsLayout {
  int64_t h, u, v, dy, dz, dp, part, total;
  explicit WsLayout(int D) {
    h = 0;
    u = h + (int64_t)(kBlocks + 1) * kH;
    v = u + (int64_t)kBlocks * kH;
    dy = v + (int64_t)kBlocks * kH;
    dz = dy + D;
    dp = dz + D;
    part = dp + (int64_t)(2 * kBlocks + 1) * kH;
    total = part + (int64_t)kBwdSplit * kH;
  }
};

inline int blocks_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

constexpr int kMaxDesigns = 65535;  // one grid dimension per design index

int validate(const sqngd_sqn_shape* s) {
  if (s == nullptr) return SQNGD_E_INVALID_ARG;
  if (s->M < 1 || s->N < 1 || s->B < 2 || s->copies < 1 || s->designs < 0) return SQNGD_E_INVALID_ARG;
  if (!std::isfinite(s->c) || s->c <= 0.f) return SQNGD_E_INVALID_ARG;
  if (s->reserved[0] != 0 || s->reserved[1] != 0) return SQNGD_E_INVALID_ARG;
  if ((int64_t)s->M * s->N > kMaxD || s->B > 64 || (int64_t)s->B * s->copies > kMaxK ||
      s->designs > kMaxDesigns)
    return SQNGD_E_UNSUPPORTED;
  return SQNGD_OK;
}

// Strides (floats) of the stacked per-design arrays.
struct Dims {
  int D, K, R;
  int64_t th, ws;  // parameters per design; workspace floats per design (a multiple of 64)
  explicit Dims(const sqngd_sqn_shape* s)
      : D(s->M * s->N), K(s->B * s->copies), R(s->designs > 0 ? s->designs : 1),
        th(Layers(s->M * s->N).total), ws((WsLayout(s->M * s->N).total + 63) & ~(int64_t)63) {}
  size_t ws_bytes() const { return 4 * (size_t)ws * (size_t)R; }
};

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
  *bytes = align_up(sqsqn::Dims(shape).ws_bytes());
  return SQNGD_OK;
}

int sqngd_sqn_forward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, float* z, void* ws,
                      size_t ws_bytes, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (theta == nullptr || y0 == nullptr || z == nullptr || ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(theta, 16) || !aligned(y0, 4) || !aligned(z, 4) || !aligned(ws, kAlign))
    return SQNGD_E_ALIGN;
  const Dims G(shape);
  const int D = G.D;
  const WsLayout L(D);
  if (ws_bytes < G.ws_bytes()) return SQNGD_E_WORKSPACE;
  const Layers Y(D);
  hipStream_t s = (hipStream_t)stream;
  float* f = (float*)ws;
  float* h = f + L.h;
  const int wb = kThreads / 64;
  hipLaunchKernelGGL(k_dense_fwd<ACT_TANH>, dim3((kH + wb - 1) / wb, G.R), dim3(kThreads), 0, s, y0, D,
                     theta + Y.w[0], theta + Y.b[0], kH, (const float*)nullptr, (float*)nullptr, h, (int64_t)D, G.th,
                     G.ws);
  hipLaunchKernelGGL(k_res_fwd, dim3(G.R), dim3(kStackThreads), 0, s, theta + Y.w[1], h, f + L.u, f + L.v, G.th,
                     G.ws);
  const int lo = 2 * kBlocks + 1;
  hipLaunchKernelGGL(k_dense_fwd<ACT_SIGMOID>, dim3((D + wb - 1) / wb, G.R), dim3(kThreads), 0, s,
                     (const float*)(h + (int64_t)kBlocks * kH), kH, theta + Y.w[lo], theta + Y.b[lo], D,
                     (const float*)nullptr, (float*)nullptr, z, G.ws, G.th, (int64_t)D);
  return check_launch();
}

int sqngd_sqn_soft(const sqngd_sqn_shape* shape, const float* z, const float* rho, sqngd_c64* sw, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (z == nullptr || rho == nullptr || sw == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(rho, 4) || !aligned(sw, 8)) return SQNGD_E_ALIGN;
  const Dims G(shape);
  hipLaunchKernelGGL(k_soft, dim3(blocks_for(64 * (int64_t)G.D * G.R)), dim3(kThreads), 0, (hipStream_t)stream, z,
                     rho, G.D, G.R, G.K, shape->B, shape->c, (float2*)sw);
  return check_launch();
}

int sqngd_sqn_hard(const sqngd_sqn_shape* shape, const float* z, const float* rho, int32_t* idx, sqngd_c64* x,
                   void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (z == nullptr || rho == nullptr || (idx == nullptr && x == nullptr)) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(rho, 4) || !aligned(idx, 4) || !aligned(x, 8)) return SQNGD_E_ALIGN;
  const Dims G(shape);
  hipLaunchKernelGGL(k_hard, dim3(blocks_for(64 * (int64_t)G.D * G.R)), dim3(kThreads), 0, (hipStream_t)stream, z,
                     rho, G.D, G.R, G.K, shape->B, idx, (float2*)x);
  return check_launch();
}

namespace sqsqn {
static int adam_args(const int32_t* step, int32_t step_mul, int32_t step_add, float lr, float beta1, float beta2, float eps,
              AdamArgs* A) {
  if (step_mul < 0 || step_add < 0 || (step == nullptr && step_add < 1)) return SQNGD_E_INVALID_ARG;
  if (!std::isfinite(lr) || lr < 0.f || !(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f) ||
      !std::isfinite(eps) || eps <= 0.f)
    return SQNGD_E_INVALID_ARG;
  if (!aligned(step, 4)) return SQNGD_E_ALIGN;
  *A = AdamArgs{lr, beta1, beta2, eps, step, step_mul, step_add};
  return SQNGD_OK;
}

// The backward pass; with adam set, the weight gradients update theta by Adam
// instead of being written to grad_theta.
static int backward_impl(const sqngd_sqn_shape* shape, const float* theta, const float* y0, const float* z,
                  const float* rho, const sqngd_c64* sw, const sqngd_c64* grad_s, const sqngd_c64* grad_h,
                  float* grad_theta, float* grad_rho, void* ws, size_t ws_bytes, void* stream, float* theta_w,
                  float* m_theta, float* v_theta, const AdamArgs* adam) {
  const Dims G(shape);
  const int D = G.D, K = G.K, B = shape->B;
  const WsLayout L(D);
  if (ws_bytes < G.ws_bytes()) return SQNGD_E_WORKSPACE;
  const Layers Y(D);
  hipStream_t s = (hipStream_t)stream;
  float* f = (float*)ws;
  float* h = f + L.h;
  float* dy = f + L.dy;
  float* dz = f + L.dz;
  float* dp = f + L.dp;
  float* part = f + L.part;
  // staircase: dL/dy1, dL/dz and dL/drho
  hipLaunchKernelGGL(k_chain, dim3(blocks_for(64 * (int64_t)D * G.R)), dim3(kThreads), 0, s, z, rho,
                     (const float2*)sw, (const float2*)grad_s, (const float2*)grad_h, D, G.R, K, B, shape->c, dy, dz,
                     G.ws);
  hipLaunchKernelGGL(k_drho, dim3(K, G.R), dim3(kThreads), 0, s, z, rho, (const float*)dy, D, B, shape->c, grad_rho,
                     K, G.ws);
  // output layer (a = z, sigmoid): gradient into h_5 as split sums
  const int lo = 2 * kBlocks + 1;
  hipLaunchKernelGGL(k_dense_bwd_part, dim3((kH + 63) / 64, kBwdSplit, G.R), dim3(64 * kBwdWaves), 0, s,
                     theta + Y.w[lo], (const float*)dz, z, (int)ACT_SIGMOID, kH, D, part, G.th, G.ws, (int64_t)D,
                     G.ws);
  // hidden stack and input layer: pre-activation gradients dp[0..10]
  hipLaunchKernelGGL(k_res_bwd, dim3(G.R), dim3(kStackThreads), 0, s, theta + Y.w[1], (const float*)part, kBwdSplit,
                     (const float*)h, (const float*)(f + L.u), (const float*)(f + L.v), dp, G.th, G.ws);
  // weight and bias gradients of all layers
  DwArgs A{};
  for (int l = 0; l < kLayers; ++l) {
    A.w[l] = Y.w[l];
    A.b[l] = Y.b[l];
    A.in[l] = Y.in[l];
    if (l == lo) {
      A.d[l] = dz;
      A.dstr[l] = G.ws;
      A.a[l] = z;
      A.astr[l] = D;
      A.act[l] = ACT_SIGMOID;
    } else {
      A.d[l] = dp + (int64_t)l * kH;
      A.dstr[l] = G.ws;
      A.a[l] = nullptr;
      A.astr[l] = 0;
      A.act[l] = ACT_NONE;
    }
    // inputs: y0 for layer 0, u_k for the second layer of block k, h_k for
    // the first, h_5 for the output layer
    A.xstr[l] = l == 0 ? (int64_t)D : G.ws;
    if (l == 0) A.x[l] = y0;
    else if (l == lo) A.x[l] = h + (int64_t)kBlocks * kH;
    else if (l % 2 == 1) A.x[l] = h + (int64_t)((l - 1) / 2) * kH;
    else A.x[l] = f + L.u + (int64_t)((l - 2) / 2) * kH;
  }
  A.g = grad_theta;
  A.total = Y.total;
  A.theta = adam ? theta_w : nullptr;
  A.m = m_theta;
  A.v = v_theta;
  if (adam) A.adam = *adam;
  int nb = 0;
  for (int l = 0; l < kLayers; ++l) {
    A.bstart[l] = nb;
    nb += (int)(((int64_t)Y.in[l] * Y.out[l] + Y.out[l] + kDwPer * kThreads - 1) / (kDwPer * kThreads));
  }
  A.bstart[kLayers] = nb;
  hipLaunchKernelGGL(k_dw_all, dim3(nb, G.R), dim3(kThreads), 0, s, A);
  return check_launch();
}
}  // namespace sqsqn

int sqngd_sqn_backward(const sqngd_sqn_shape* shape, const float* theta, const float* y0, const float* z,
                       const float* rho, const sqngd_c64* sw, const sqngd_c64* grad_s, const sqngd_c64* grad_h,
                       float* grad_theta, float* grad_rho, void* ws, size_t ws_bytes, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (theta == nullptr || y0 == nullptr || z == nullptr || rho == nullptr || sw == nullptr || grad_s == nullptr ||
      grad_theta == nullptr || grad_rho == nullptr || ws == nullptr)
    return SQNGD_E_INVALID_ARG;
  if (!aligned(theta, 4) || !aligned(y0, 4) || !aligned(z, 4) || !aligned(rho, 4) || !aligned(sw, 8) ||
      !aligned(grad_s, 8) || !aligned(grad_h, 8) || !aligned(grad_theta, 4) || !aligned(grad_rho, 4) ||
      !aligned(ws, kAlign))
    return SQNGD_E_ALIGN;
  return backward_impl(shape, theta, y0, z, rho, sw, grad_s, grad_h, grad_theta, grad_rho, ws, ws_bytes, stream,
                       nullptr, nullptr, nullptr, nullptr);
}

int sqngd_sqn_backward_adam(const sqngd_sqn_shape* shape, float* theta, const float* y0, const float* z,
                            const float* rho, const sqngd_c64* sw, const sqngd_c64* grad_s, const sqngd_c64* grad_h,
                            float* m_theta, float* v_theta, float* grad_rho, const int32_t* step, int32_t step_mul,
                            int32_t step_add, float lr, float beta1, float beta2, float eps, void* ws,
                            size_t ws_bytes, void* stream) {
  using namespace sqsqn;
  int rc = validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (theta == nullptr || y0 == nullptr || z == nullptr || rho == nullptr || sw == nullptr || grad_s == nullptr ||
      m_theta == nullptr || v_theta == nullptr || grad_rho == nullptr || ws == nullptr)
    return SQNGD_E_INVALID_ARG;
  AdamArgs ad;
  rc = adam_args(step, step_mul, step_add, lr, beta1, beta2, eps, &ad);
  if (rc != SQNGD_OK) return rc;
  if (!aligned(theta, 4) || !aligned(y0, 4) || !aligned(z, 4) || !aligned(rho, 4) || !aligned(sw, 8) ||
      !aligned(grad_s, 8) || !aligned(grad_h, 8) || !aligned(m_theta, 4) || !aligned(v_theta, 4) ||
      !aligned(grad_rho, 4) || !aligned(ws, kAlign))
    return SQNGD_E_ALIGN;
  return backward_impl(shape, theta, y0, z, rho, sw, grad_s, grad_h, nullptr, grad_rho, ws, ws_bytes, stream, theta,
                       m_theta, v_theta, &ad);
}


int sqngd_sqn_adam(float* p, const float* g, float* m, float* v, int64_t n, const int32_t* step, int32_t step_mul,
                   int32_t step_add, float lr, float beta1, float beta2, float eps, void* stream) {
  using namespace sqsqn;
  if (p == nullptr || g == nullptr || m == nullptr || v == nullptr || n < 1) return SQNGD_E_INVALID_ARG;
  AdamArgs A;
  int rc = adam_args(step, step_mul, step_add, lr, beta1, beta2, eps, &A);
  if (rc != SQNGD_OK) return rc;
  if (!aligned(p, 4) || !aligned(g, 4) || !aligned(m, 4) || !aligned(v, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_adam, dim3((int)((n + kDwPer * kThreads - 1) / (kDwPer * kThreads))), dim3(kThreads), 0,
                     (hipStream_t)stream, p, g, m, v, n, A);
  return check_launch();
}

int sqngd_sqn_adam_project(int32_t rows, int32_t N, sqngd_c64* h, const sqngd_c64* g, float* m, float* v,
                           const int32_t* step, int32_t step_mul, int32_t step_add, float lr, float beta1,
                           float beta2, float eps, void* stream) {
  using namespace sqsqn;
  if (h == nullptr || g == nullptr || m == nullptr || v == nullptr || rows < 1 || N < 1) return SQNGD_E_INVALID_ARG;
  AdamArgs A;
  int rc = adam_args(step, step_mul, step_add, lr, beta1, beta2, eps, &A);
  if (rc != SQNGD_OK) return rc;
  if (!aligned(h, 8) || !aligned(g, 8) || !aligned(m, 4) || !aligned(v, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_adam_project, dim3(rows), dim3(kThreads), 0, (hipStream_t)stream, (float2*)h,
                     (const float2*)g, m, v, (int)N, A);
  return check_launch();
}

int sqngd_sqn_adam_sort(float* rho, const float* g, float* m, float* v, int32_t K, int32_t designs,
                        const int32_t* step, int32_t step_mul, int32_t step_add, float lr, float beta1, float beta2,
                        float eps, void* stream) {
  using namespace sqsqn;
  if (rho == nullptr || g == nullptr || m == nullptr || v == nullptr || K < 1 || designs < 1)
    return SQNGD_E_INVALID_ARG;
  if (K > kMaxK || designs > kMaxDesigns) return SQNGD_E_UNSUPPORTED;
  AdamArgs A;
  int rc = adam_args(step, step_mul, step_add, lr, beta1, beta2, eps, &A);
  if (rc != SQNGD_OK) return rc;
  if (!aligned(rho, 4) || !aligned(g, 4) || !aligned(m, 4) || !aligned(v, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_adam_sort, dim3(designs), dim3(1024), 0, (hipStream_t)stream, rho, g, m, v, (int)K, A);
  return check_launch();
}

int sqngd_sqn_count(int32_t* step, void* stream) {
  using namespace sqsqn;
  if (step == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(step, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_count, dim3(1), dim3(64), 0, (hipStream_t)stream, step);
  return check_launch();
}

int sqngd_sqn_sort(float* rho, int32_t K, int32_t designs, void* stream) {
  using namespace sqsqn;
  if (rho == nullptr || K < 1 || designs < 1) return SQNGD_E_INVALID_ARG;
  if (K > kMaxK || designs > kMaxDesigns) return SQNGD_E_UNSUPPORTED;
  if (!aligned(rho, 4)) return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_sort, dim3(designs), dim3(1024), 0, (hipStream_t)stream, rho, (int)K);
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
