// net.hip - gfx950 kernels and C ABI of the warm-start proposal network
// (declared in include/sqngd_net.h). Included by api.hip after its host
// helpers (one translation unit).
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16:
//   forward / input gradient: D[o][pos] = sum_k W[o][k] X'[k][pos] with
//     k = tap * CIN + c and X'[k][pos] = X[pos + tap - 2][c]; a block owns 64
//     positions of one sample (4 waves x 16), stages the 72 input rows it
//     needs and the bfloat16 weights in LDS, and keeps all COUT outputs of
//     its 16 positions in each wave's accumulators. The input gradient of a
//     layer is the same product with the weights transposed and the taps
//     flipped, W'[c][tap'][o] = W[o][4 - tap'][c], followed by the ReLU mask
//     of the layer below.
//   weight gradient: D[o][(tap, c)] = sum_pos dZ[pos][o] X[pos + tap - 2][c];
//     a block stages dZ transposed and X in five tap-shifted copies (so every
//     operand is a 16-byte LDS read), accumulates over a run of 64-position
//     chunks and writes one FP32 partial; a second kernel sums the partials
//     in block order (deterministic).
// MFMA operand layout (16x16x32): lane l holds A row (l mod 16), B column
// (l mod 16), both for k = 8 (l / 16) .. +7; D column (l mod 16), rows
// 4 (l / 16) .. +3.
#include "../../include/sqngd_net.h"

namespace sqnet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int kC = 64;          // hidden channels
constexpr int kTaps = 5;        // kernel width
constexpr int kPos = 64;        // positions per block
constexpr int kRows = kPos + 8; // staged input rows (taps up to 7 with zero-padded weights)
constexpr int kThreads = 256;
constexpr int kDwChunks = 16;   // 64-position chunks per weight-gradient block
constexpr int kXin = 8;         // padded input channels of layer 0

__host__ __device__ constexpr int round32(int k) { return (k + 31) / 32 * 32; }

__device__ __forceinline__ u16 to_bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(u16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool positive(u16 h) { return h != 0 && (h & 0x8000u) == 0; }

__device__ __forceinline__ f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

enum ConvMode : int { CONV_RELU = 0, CONV_LOGITS = 1, CONV_BACK = 2 };

struct ConvArgs {
  const u16* x;       // [B][N][CIN]
  const u16* w;       // [COUT][round32(5 CIN)], k = tap * CIN + c, zero for tap >= 5
  const float* bias;  // [COUT] (forward modes)
  const u16* ref;     // CONV_BACK: [B][N][COUT], output kept where ref > 0
  u16* y;             // CONV_RELU / CONV_BACK: [B][N][COUT]
  float* z;           // CONV_LOGITS: [B][M][N][L]
  int N, M, L;
};

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(kThreads) void k_conv(ConvArgs a) {
  constexpr int KP = round32(kTaps * CIN);
  constexpr int KS = KP + 8;  // LDS row stride of the weights (bank spread)
  constexpr int NT = COUT / 16;
  __shared__ __attribute__((aligned(16))) u16 xs[kRows * CIN];
  __shared__ __attribute__((aligned(16))) u16 ws[COUT * KS];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
  const int bpr = a.N / kPos;
  const int b = blockIdx.x / bpr, n0 = (blockIdx.x - b * bpr) * kPos;
  for (int i = tid; i < COUT * KP / 8; i += kThreads) {
    const int o = i / (KP / 8), q = i - o * (KP / 8);
    *(uint4*)(ws + o * KS + q * 8) = *(const uint4*)(a.w + (size_t)o * KP + q * 8);
  }
  for (int i = tid; i < kRows * CIN / 8; i += kThreads) {
    const int r = i / (CIN / 8), q = i - r * (CIN / 8);
    const int n = n0 - 2 + r;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (n >= 0 && n < a.N) v = *(const uint4*)(a.x + ((size_t)b * a.N + n) * CIN + q * 8);
    *(uint4*)(xs + r * CIN + q * 8) = v;
  }
  __syncthreads();
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kk = 0; kk < KP / 32; ++kk) {
    const int k0 = kk * 32 + kq * 8;
    const int tap = k0 / CIN, c0 = k0 - tap * CIN;
    const uint4 bv = *(const uint4*)(xs + (wv * 16 + col + tap) * CIN + c0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma(*(const uint4*)(ws + (t * 16 + col) * KS + k0), bv, acc[t]);
  }
  const int n = n0 + wv * 16 + col;
  const size_t row = (size_t)b * a.N + n;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int o0 = t * 16 + 4 * kq;
    float v[4] = {acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
    if constexpr (MODE == CONV_LOGITS) {
      const int m = o0 / a.L, l0 = o0 - m * a.L;
      *(float4*)(a.z + (((size_t)b * a.M + m) * a.N + n) * a.L + l0) =
          make_float4(v[0] + a.bias[o0], v[1] + a.bias[o0 + 1], v[2] + a.bias[o0 + 2], v[3] + a.bias[o0 + 3]);
    } else {
      u16 h[4];
      if constexpr (MODE == CONV_RELU) {
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = to_bf16(fmaxf(v[i] + a.bias[o0 + i], 0.f));
      } else {
        const uint2 rv = *(const uint2*)(a.ref + row * COUT + o0);
        const u16 rr[4] = {(u16)(rv.x & 0xFFFFu), (u16)(rv.x >> 16), (u16)(rv.y & 0xFFFFu), (u16)(rv.y >> 16)};
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = to_bf16(positive(rr[i]) ? v[i] : 0.f);
      }
      *(uint2*)(a.y + row * COUT + o0) =
          make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    }
  }
}

struct DwArgs {
  const u16* dz;  // [B][N][COUT]
  const u16* x;   // [B][N][CIN]
  float* part;    // [blocks][COUT * 5 * CIN + COUT]
  int N, chunks;
};

template <int CIN, int COUT>
__global__ __launch_bounds__(kThreads) void k_conv_dw(DwArgs a) {
  constexpr int KW = kTaps * CIN;
  constexpr int NR = COUT / 16, NC = (KW + 15) / 16, NTILE = NR * NC, TPW = (NTILE + 3) / 4;
  constexpr int RS = kPos + 8;  // LDS row stride (positions)
  __shared__ __attribute__((aligned(16))) u16 dzt[COUT * RS];
  __shared__ __attribute__((aligned(16))) u16 xsh[kTaps * CIN * RS];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
  const int bpr = a.N / kPos;
  f32x4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbias = 0.f;
  const int c_begin = blockIdx.x * kDwChunks;
  const int c_end = min(c_begin + kDwChunks, a.chunks);
  for (int c = c_begin; c < c_end; ++c) {
    const int b = c / bpr, n0 = (c - b * bpr) * kPos;
    for (int i = tid; i < kPos * COUT / 8; i += kThreads) {
      const int p = i / (COUT / 8), q = i - p * (COUT / 8);
      const uint4 v = *(const uint4*)(a.dz + ((size_t)b * a.N + n0 + p) * COUT + q * 8);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) dzt[(q * 8 + e) * RS + p] = (u16)(w4[e >> 1] >> (16 * (e & 1)));
    }
    for (int i = tid; i < (kPos + 4) * CIN / 8; i += kThreads) {
      const int r = i / (CIN / 8), q = i - r * (CIN / 8);
      const int n = n0 - 2 + r;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (n >= 0 && n < a.N) v = *(const uint4*)(a.x + ((size_t)b * a.N + n) * CIN + q * 8);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int tap = 0; tap < kTaps; ++tap) {
        const int p = r - tap;
        if (p < 0 || p >= kPos) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e) xsh[(tap * CIN + q * 8 + e) * RS + p] = (u16)(w4[e >> 1] >> (16 * (e & 1)));
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kPos / 32; ++kk) {
      const int k0 = kk * 32 + kq * 8;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int tile = wv + 4 * i;
        if (tile >= NTILE) break;
        const int rt = tile / NC, ct = tile - rt * NC;
        const int cc = ct * 16 + col;
        uint4 bv = make_uint4(0u, 0u, 0u, 0u);
        if (cc < KW) {
          const int tap = cc / CIN, ci = cc - tap * CIN;
          bv = *(const uint4*)(xsh + (tap * CIN + ci) * RS + k0);
        }
        acc[i] = mfma(*(const uint4*)(dzt + (rt * 16 + col) * RS + k0), bv, acc[i]);
      }
    }
    if (tid < COUT)
      for (int p = 0; p < kPos; ++p) dbias += from_bf16(dzt[tid * RS + p]);
    __syncthreads();
  }
  float* out = a.part + (size_t)blockIdx.x * (COUT * KW + COUT);
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tile = wv + 4 * i;
    if (tile >= NTILE) break;
    const int rt = tile / NC, ct = tile - rt * NC;
    const int cc = ct * 16 + col;
    if (cc < KW) {
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(rt * 16 + 4 * kq + e) * KW + cc] = acc[i][e];
    }
  }
  if (tid < COUT) out[COUT * KW + tid] = dbias;
}

// Sum of the weight-gradient partials in block order into the flat FP32
// gradient of one layer (true input channels cin <= the padded CINP).
struct ReduceArgs {
  const float* part;
  int blocks, cinp, cin, cout;
  float* grad;
};
__global__ __launch_bounds__(256) void k_dw_reduce(ReduceArgs a) {
  const int nw = a.cout * kTaps * a.cin;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nw + a.cout) return;
  int src;
  if (idx < nw) {
    const int o = idx / (kTaps * a.cin), rem = idx - o * kTaps * a.cin;
    const int tap = rem / a.cin, c = rem - tap * a.cin;
    src = o * kTaps * a.cinp + tap * a.cinp + c;
  } else {
    src = a.cout * kTaps * a.cinp + (idx - nw);
  }
  const size_t stride = (size_t)a.cout * kTaps * a.cinp + a.cout;
  float s = 0.f;
  for (int k = 0; k < a.blocks; ++k) s += a.part[k * stride + src];
  a.grad[idx] = s;
}

// bfloat16 weights of one layer: wf[o][k] (k = tap * cinp + c) and, when wt
// is set, the transposed and tap-flipped wt[c][k'] (k' = tap' * cout + o)
// of the input-gradient product.
struct NetPrepArgs {
  const float* w;  // [cout][5][cin]
  int cin, cinp, cout;
  u16* wf;
  u16* wt;
};
__global__ __launch_bounds__(256) void k_net_prep(NetPrepArgs a) {
  const int kp = round32(kTaps * a.cinp);
  const int nf = a.cout * kp;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < nf) {
    const int o = idx / kp, k = idx - o * kp;
    const int tap = k / a.cinp, c = k - tap * a.cinp;
    const float v = (tap < kTaps && c < a.cin) ? a.w[(o * kTaps + tap) * a.cin + c] : 0.f;
    a.wf[idx] = to_bf16(v);
  }
  if (a.wt != nullptr) {
    const int kt = round32(kTaps * a.cout);
    const int j = idx - nf;
    if (j >= 0 && j < a.cin * kt) {
      const int c = j / kt, k = j - c * kt;
      const int tp = k / a.cout, o = k - tp * a.cout;
      const float v = tp < kTaps ? a.w[(o * kTaps + (kTaps - 1 - tp)) * a.cin + c] : 0.f;
      a.wt[j] = to_bf16(v);
    }
  }
}

// X0[b][n][c]: the noise rows, the two conditioning values, zero padding.
struct InputArgs {
  const float* noise;
  int B, M, N;
  float cond0, cond1;
  u16* x0;
};
__global__ __launch_bounds__(256) void k_net_input(InputArgs a) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.B * a.N) return;
  const int b = idx / a.N, n = idx - b * a.N;
  u16 h[kXin];
  for (int c = 0; c < kXin; ++c) {
    float v = 0.f;
    if (c < a.M) v = a.noise[((size_t)b * a.M + c) * a.N + n];
    else if (c == a.M) v = a.cond0;
    else if (c == a.M + 1) v = a.cond1;
    h[c] = to_bf16(v);
  }
  *(uint4*)(a.x0 + (size_t)idx * kXin) =
      make_uint4((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                 (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16));
}

// Logit gradient fed to the last layer, dZ3[b][n][m L + l] in bfloat16: the
// cross-entropy gradient (softmax - one-hot) / count with per-block partial
// losses, or a given upstream gradient.
struct CeArgs {
  const float* z;       // [B][M][N][L]
  const int32_t* t;     // [B][M][N] or null
  const float* dz_in;   // [B][M][N][L] when t is null
  u16* dz;              // [B][N][M L]
  float* lpart;         // [blocks]
  int B, M, N, L;
};
__global__ __launch_bounds__(256) void k_net_ce(CeArgs a) {
  __shared__ float red[256];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int total = a.B * a.M * a.N;
  const float inv_cnt = 1.0f / (float)total;
  float lsum = 0.f;
  if (idx < total) {
    const int n = idx % a.N, bm = idx / a.N, m = bm % a.M, b = bm / a.M;
    const float* zr = a.z + (size_t)idx * a.L;
    u16* out = a.dz + ((size_t)b * a.N + n) * (a.M * a.L) + m * a.L;
    if (a.t != nullptr) {
      float zm = zr[0];
      for (int l = 1; l < a.L; ++l) zm = fmaxf(zm, zr[l]);
      float s = 0.f;
      for (int l = 0; l < a.L; ++l) s += expf(zr[l] - zm);
      const int tl = a.t[idx];
      lsum = zm + logf(s) - zr[tl];
      const float inv_s = 1.0f / s;
      for (int l = 0; l < a.L; ++l) {
        const float g = (expf(zr[l] - zm) * inv_s - (l == tl ? 1.0f : 0.0f)) * inv_cnt;
        out[l] = to_bf16(g);
      }
    } else {
      const float* gr = a.dz_in + (size_t)idx * a.L;
      for (int l = 0; l < a.L; ++l) out[l] = to_bf16(gr[l]);
    }
  }
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.lpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(64) void k_net_loss(const float* lpart, int blocks, float scale, float* loss) {
  if (threadIdx.x != 0) return;
  float s = 0.f;
  for (int k = 0; k < blocks; ++k) s += lpart[k];
  *loss = s * scale;
}

struct AdamArgs {
  float* p;
  float* m;
  float* v;
  const float* g;
  int64_t n;
  float lr, b1, b2, eps, bc1, bc2;
};
__global__ __launch_bounds__(256) void k_net_adam(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const float g = a.g[i];
  const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.p[i] -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

// ------------------------------------------------------------------ host side

struct NetLayout {
  int M, N, L, B, ML;
  int cin[4], cinp[4], cout[4];
  int64_t poff[4], nparam;
  size_t wf[4], wt[4], x[4], dz[2], part, lpart, total;
  int dw_blocks, ce_blocks;
};

inline size_t up256(size_t v) { return (v + 255) / 256 * 256; }

int net_validate(const sqngd_net_shape* s) {
  if (s == nullptr) return SQNGD_E_INVALID_ARG;
  if (s->M < 1 || s->N < 1 || s->L < 2 || s->batch < 1 || s->reserved[0] != 0 || s->reserved[1] != 0)
    return SQNGD_E_INVALID_ARG;
  if (!std::isfinite(s->cond0) || !std::isfinite(s->cond1)) return SQNGD_E_INVALID_ARG;
  const int ml = s->M * s->L;
  if (s->M + 2 > kXin || (ml != 16 && ml != 32 && ml != 64) || s->L % 4 != 0 || s->N % kPos != 0 || s->N > 4096 ||
      s->batch > 65536)
    return SQNGD_E_UNSUPPORTED;
  return SQNGD_OK;
}

NetLayout net_layout(const sqngd_net_shape& s) {
  NetLayout g{};
  g.M = s.M;
  g.N = s.N;
  g.L = s.L;
  g.B = s.batch;
  g.ML = s.M * s.L;
  const int cin[4] = {s.M + 2, kC, kC, kC}, cinp[4] = {kXin, kC, kC, kC}, cout[4] = {kC, kC, kC, g.ML};
  int64_t off = 0;
  size_t w = 0;
  for (int i = 0; i < 4; ++i) {
    g.cin[i] = cin[i];
    g.cinp[i] = cinp[i];
    g.cout[i] = cout[i];
    g.poff[i] = off;
    off += (int64_t)cout[i] * kTaps * cin[i] + cout[i];
  }
  g.nparam = off;
  for (int i = 0; i < 4; ++i) {
    g.wf[i] = w;
    w = up256(w + 2 * (size_t)cout[i] * round32(kTaps * cinp[i]));
    g.wt[i] = w;
    if (i > 0) w = up256(w + 2 * (size_t)cin[i] * round32(kTaps * cout[i]));
  }
  const size_t pos = (size_t)s.batch * s.N;
  for (int i = 0; i < 4; ++i) {
    g.x[i] = w;
    w = up256(w + 2 * pos * cinp[i]);
  }
  for (int i = 0; i < 2; ++i) {
    g.dz[i] = w;
    w = up256(w + 2 * pos * kC);
  }
  const int chunks = (int)(pos / kPos);
  g.dw_blocks = (chunks + kDwChunks - 1) / kDwChunks;
  size_t stride = 0;
  for (int i = 0; i < 4; ++i) stride = std::max(stride, (size_t)cout[i] * kTaps * cinp[i] + cout[i]);
  g.part = w;
  w = up256(w + 4 * stride * g.dw_blocks);
  g.ce_blocks = (int)((pos * s.M + 255) / 256);
  g.lpart = w;
  w = up256(w + 4 * (size_t)g.ce_blocks);
  g.total = w;
  return g;
}

template <int CIN, int COUT, int MODE>
void launch_conv(const ConvArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), dim3(blocks), dim3(kThreads), 0, s, a);
}

}  // namespace sqnet

extern "C" {

int sqngd_net_param_count(const sqngd_net_shape* shape, int64_t* count) {
  int rc = sqnet::net_validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (count == nullptr) return SQNGD_E_INVALID_ARG;
  *count = sqnet::net_layout(*shape).nparam;
  return SQNGD_OK;
}

int sqngd_net_workspace_size(const sqngd_net_shape* shape, size_t* bytes) {
  int rc = sqnet::net_validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (bytes == nullptr) return SQNGD_E_INVALID_ARG;
  *bytes = sqnet::net_layout(*shape).total;
  return SQNGD_OK;
}

int sqngd_net_forward(const sqngd_net_shape* shape, const float* params, const float* noise, float* logits, void* ws,
                      size_t ws_bytes, void* stream) {
  using namespace sqnet;
  int rc = net_validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (params == nullptr || noise == nullptr || logits == nullptr || ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(params, 4) || !aligned(noise, 4) || !aligned(logits, 16) || !aligned(ws, 256)) return SQNGD_E_ALIGN;
  const NetLayout g = net_layout(*shape);
  if (ws_bytes < g.total) return SQNGD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  auto U = [&](size_t off) { return (u16*)(base + off); };
  for (int i = 0; i < 4; ++i) {
    NetPrepArgs pa{params + g.poff[i], g.cin[i], g.cinp[i], g.cout[i], U(g.wf[i]), i > 0 ? U(g.wt[i]) : nullptr};
    const int n = g.cout[i] * round32(kTaps * g.cinp[i]) + (i > 0 ? g.cin[i] * round32(kTaps * g.cout[i]) : 0);
    hipLaunchKernelGGL(k_net_prep, dim3((n + 255) / 256), dim3(256), 0, s, pa);
  }
  InputArgs ia{noise, g.B, g.M, g.N, shape->cond0, shape->cond1, U(g.x[0])};
  hipLaunchKernelGGL(k_net_input, dim3((g.B * g.N + 255) / 256), dim3(256), 0, s, ia);
  const int blocks = g.B * g.N / kPos;
  for (int i = 0; i < 4; ++i) {
    ConvArgs ca{};
    ca.x = U(g.x[i]);
    ca.w = U(g.wf[i]);
    ca.bias = params + g.poff[i] + (int64_t)g.cout[i] * kTaps * g.cin[i];
    ca.N = g.N;
    ca.M = g.M;
    ca.L = g.L;
    if (i < 3) {
      ca.y = U(g.x[i + 1]);
      if (i == 0) launch_conv<kXin, kC, CONV_RELU>(ca, blocks, s);
      else launch_conv<kC, kC, CONV_RELU>(ca, blocks, s);
    } else {
      ca.z = logits;
      if (g.ML == 16) launch_conv<kC, 16, CONV_LOGITS>(ca, blocks, s);
      else if (g.ML == 32) launch_conv<kC, 32, CONV_LOGITS>(ca, blocks, s);
      else launch_conv<kC, 64, CONV_LOGITS>(ca, blocks, s);
    }
  }
  return check_launch();
}

int sqngd_net_backward(const sqngd_net_shape* shape, const float* logits, const int32_t* target,
                       const float* grad_logits, float* grad_params, float* loss, void* ws, size_t ws_bytes,
                       void* stream) {
  using namespace sqnet;
  int rc = net_validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (grad_params == nullptr || ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (target != nullptr ? logits == nullptr : grad_logits == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(logits, 4) || !aligned(target, 4) || !aligned(grad_logits, 4) || !aligned(grad_params, 4) ||
      !aligned(loss, 4) || !aligned(ws, 256))
    return SQNGD_E_ALIGN;
  const NetLayout g = net_layout(*shape);
  if (ws_bytes < g.total) return SQNGD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  auto U = [&](size_t off) { return (u16*)(base + off); };
  float* part = (float*)(base + g.part);
  float* lpart = (float*)(base + g.lpart);
  CeArgs ce{logits, target, grad_logits, U(g.dz[0]), lpart, g.B, g.M, g.N, g.L};
  hipLaunchKernelGGL(k_net_ce, dim3(g.ce_blocks), dim3(256), 0, s, ce);
  if (target != nullptr && loss != nullptr)
    hipLaunchKernelGGL(k_net_loss, dim3(1), dim3(64), 0, s, (const float*)lpart, g.ce_blocks,
                       1.0f / (float)((int64_t)g.B * g.M * g.N), loss);
  const int chunks = g.B * g.N / kPos;
  int cur = 0;  // dz buffer holding dZ_i
  for (int i = 3; i >= 0; --i) {
    DwArgs da{U(g.dz[cur]), U(g.x[i]), part, g.N, chunks};
    if (i == 0) hipLaunchKernelGGL((k_conv_dw<kXin, kC>), dim3(g.dw_blocks), dim3(kThreads), 0, s, da);
    else if (i < 3) hipLaunchKernelGGL((k_conv_dw<kC, kC>), dim3(g.dw_blocks), dim3(kThreads), 0, s, da);
    else if (g.ML == 16) hipLaunchKernelGGL((k_conv_dw<kC, 16>), dim3(g.dw_blocks), dim3(kThreads), 0, s, da);
    else if (g.ML == 32) hipLaunchKernelGGL((k_conv_dw<kC, 32>), dim3(g.dw_blocks), dim3(kThreads), 0, s, da);
    else hipLaunchKernelGGL((k_conv_dw<kC, 64>), dim3(g.dw_blocks), dim3(kThreads), 0, s, da);
    ReduceArgs ra{part, g.dw_blocks, g.cinp[i], g.cin[i], g.cout[i], grad_params + g.poff[i]};
    const int nred = g.cout[i] * kTaps * g.cin[i] + g.cout[i];
    hipLaunchKernelGGL(k_dw_reduce, dim3((nred + 255) / 256), dim3(256), 0, s, ra);
    if (i == 0) break;
    ConvArgs ca{};
    ca.x = U(g.dz[cur]);
    ca.w = U(g.wt[i]);
    ca.ref = U(g.x[i]);
    ca.y = U(g.dz[1 - cur]);
    ca.N = g.N;
    if (i < 3) launch_conv<kC, kC, CONV_BACK>(ca, chunks, s);
    else if (g.ML == 16) launch_conv<16, kC, CONV_BACK>(ca, chunks, s);
    else if (g.ML == 32) launch_conv<32, kC, CONV_BACK>(ca, chunks, s);
    else launch_conv<64, kC, CONV_BACK>(ca, chunks, s);
    cur = 1 - cur;
  }
  return check_launch();
}

int sqngd_net_adam(const sqngd_net_shape* shape, const sqngd_net_opt* opt, int32_t step, float* params,
                   float* moments, const float* grad_params, void* stream) {
  using namespace sqnet;
  int rc = net_validate(shape);
  if (rc != SQNGD_OK) return rc;
  if (opt == nullptr || params == nullptr || moments == nullptr || grad_params == nullptr || step < 1)
    return SQNGD_E_INVALID_ARG;
  if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
      !(opt->eps > 0.f))
    return SQNGD_E_INVALID_ARG;
  if (!aligned(params, 4) || !aligned(moments, 4) || !aligned(grad_params, 4)) return SQNGD_E_ALIGN;
  const NetLayout g = net_layout(*shape);
  AdamArgs a{params, moments, moments + g.nparam, grad_params, g.nparam, opt->lr, opt->beta1, opt->beta2, opt->eps,
             (float)(1.0 - std::pow((double)opt->beta1, step)), (float)(1.0 - std::pow((double)opt->beta2, step))};
  hipLaunchKernelGGL(k_net_adam, dim3((unsigned)((g.nparam + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  return check_launch();
}

}  // extern "C"
