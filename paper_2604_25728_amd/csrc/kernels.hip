// kernels.hip - gfx950 kernels of the SQNGD hot path.
//
//   k_prep    waveform quantisation (soft / hard) and the spectra of the
//             partner sequences (one wave-local FFT per row);
//   k_pass    the fused pass: per unit (self row w, Doppler bin f) the
//             Doppler-modulated FFT of the self sequence, then for every
//             partner g the correlation IFFT (eq. 36), the ROI statistics
//             and p-norm partial sums (eq. 7-9, 37 as a p-norm) and, for the
//             gradient, the FFT of the scaled adjoint and its accumulation;
//             one inverse FFT and the Doppler demodulation per unit. The AF
//             cube never leaves registers and LDS;
//   k_final   deterministic reduction of the unit partials, the SNRL penalty
//             (eq. 38-41), the loss (eq. 42), the statistics (eq. 8-10, 48),
//             the gradient rows, the chain rule to the logits and the
//             optimiser updates (Adam, eq. 32 projection);
//   k_hardq   hard quantisation of the logits.
//
// Orientation. A pass runs with a "self" sequence that is Doppler-modulated
// and differentiated and "partner" sequences whose spectra are shared by all
// units. Orientation 0: self = waveforms, partners = filters; this is eq. 6
// itself and yields the waveform gradient. Orientation 1: self = filters,
// partners = waveforms, with the Doppler and delay axes negated; since
// |A_{x,h}(tau, nu)| = |A_{h,x}(-tau, -nu)| every ROI magnitude, hence the loss,
// is the same, and the self gradient is the filter gradient.
#include "../../include/sqngd.h"
#include "fft_wave.hpp"
#include "plan.hpp"

namespace sq {

// ---------------------------------------------------------------- helpers

// exp(j 2 pi n nu / N), phase reduced to [-1/2, 1/2] turns before sincospi.
__device__ __forceinline__ float2 phasor(int n, float nu, float invN) {
  float ph = (float)n * nu * invN;
  ph -= rintf(ph);
  float s, c;
  sincospif(2.0f * ph, &s, &c);
  return make_float2(c, s);
}

__device__ __forceinline__ unsigned long long make_key(float q, uint32_t cell) {
  return ((unsigned long long)__float_as_uint(q) << 32) | (unsigned long long)(0xFFFFFFFFu - cell);
}
__device__ __forceinline__ float key_q(unsigned long long k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_cell(unsigned long long k) { return 0xFFFFFFFFu - (uint32_t)k; }
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

template <int TF>
__device__ __forceinline__ float slot_sum(float v) {
#pragma unroll
  for (int off = TF / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
template <int TF>
__device__ __forceinline__ unsigned long long slot_max_key(unsigned long long v) {
#pragma unroll
  for (int off = TF / 2; off > 0; off >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)v, off), hi = __shfl_xor((uint32_t)(v >> 32), off);
    v = umax64(v, ((unsigned long long)hi << 32) | lo);
  }
  return v;
}

// x^(PH-1) and x^PH for PH = p/2. PHLOG >= 0: PH = 2^PHLOG (exact products);
// PHLOG < 0: any p through exp2/log2.
template <int PHLOG>
__device__ __forceinline__ void pow_ph(float x, float phm1, float& y_m1, float& y) {
  if constexpr (PHLOG >= 0) {
    float a = 1.0f, s = x;
#pragma unroll
    for (int i = 0; i < PHLOG; ++i) {
      a *= s;
      s *= s;
    }
    y_m1 = a;  // x^(2^PHLOG - 1)
    y = s;     // x^(2^PHLOG)
  } else {
    y_m1 = x > 0.0f ? exp2f(phm1 * log2f(x)) : (phm1 == 0.0f ? 1.0f : 0.0f);
    y = y_m1 * x;
  }
}

__device__ __forceinline__ float temperature_at(const sqngd_opt& o, int t) {
  if (o.total_iters <= 1) return o.T0;
  float frac = fminf((float)t, (float)(o.total_iters - 1)) / (float)(o.total_iters - 1);
  return o.T0 * powf(o.T1 / o.T0, frac);
}

// Soft-quantised chip from its L logits (softmax at temperature T).
__device__ __forceinline__ float2 soft_chip(const float* zc, int L, float T, int mode) {
  float zm = zc[0];
  for (int l = 1; l < L; ++l) zm = fmaxf(zm, zc[l]);
  const float invT = 1.0f / T;
  float sum = 0.f, ybar = 0.f, re = 0.f, im = 0.f;
  for (int l = 0; l < L; ++l) {
    float e = expf((zc[l] - zm) * invT);
    sum += e;
    if (mode == SQNGD_SQ_PHASE_MEAN) {
      ybar += (float)l * e;
    } else {
      float s, c;
      sincospif(2.0f * (float)l / (float)L, &s, &c);
      re += e * c;
      im += e * s;
    }
  }
  const float inv = 1.0f / sum;
  if (mode == SQNGD_SQ_PHASE_MEAN) {
    float s, c;
    sincospif(2.0f * ybar * inv / (float)L, &s, &c);
    return make_float2(c, s);
  }
  return make_float2(re * inv, im * inv);
}

__device__ __forceinline__ int hard_chip(const float* zc, int L) {
  int best = 0;
  float bv = zc[0];
  for (int l = 1; l < L; ++l)
    if (zc[l] > bv) {
      bv = zc[l];
      best = l;
    }
  return best;
}

__device__ __forceinline__ float2 level_phasor(int l, int L) {
  float s, c;
  sincospif(2.0f * (float)l / (float)L, &s, &c);
  return make_float2(c, s);
}

__device__ __forceinline__ int find_entry(const int32_t* base, int n, int wave) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= wave) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ k_prep

enum PrepMode : int32_t {
  PREP_B_SOFT = 0,   // self = soft(z) -> wself; partners = h
  PREP_B_HARD = 1,   // self = hard(z) -> wself; partners = h
  PREP_B_GIVEN = 2,  // self = s_given -> wself; partners = h
  PREP_A_HARD = 3,   // partners = hard(z) -> wpart (self = h)
  PREP_A_SELF = 4,   // partners = wself (self = h)
};

struct PrepArgs {
  const ProbPlan* plans;
  const int32_t* gprob;
  const int32_t* grwave;
  int32_t gn;
  int32_t mode;
  int32_t use_schedule;  // temperature from opt and *counter instead of the plan
  int32_t pad;
  sqngd_opt opt;
  const int32_t* counter;
  const float* z;
  const float2* s_given;
  const float2* h;
  float2* wself;
  float2* wpart;
  float2* spec;
  float4* snrl;  // per row: (Re, Im) of sum_n conj(part(n)) self(n), |self|^2, |part|^2
};

template <int P>
__global__ __launch_bounds__(64) void k_prep(PrepArgs a) {
  using G = Geom<P>;
  constexpr int E = G::E, TF = G::TF, EH = E / 2;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x, slot = lane / TF, t = lane % TF;
  const int entry = find_entry(a.grwave, a.gn, blockIdx.x);
  const ProbPlan pl = a.plans[a.gprob[entry]];
  const int row = (blockIdx.x - a.grwave[entry]) * G::SLOTS + slot;
  const bool active = row < pl.M;
  const int g = active ? row : pl.M - 1;
  const int N = pl.N, L = pl.L;
  const int64_t rbase = pl.off_w + (int64_t)g * N;
  const float* zr = a.z ? a.z + pl.off_z + (int64_t)g * N * L : nullptr;
  float T = pl.temperature;
  if (a.use_schedule) T = temperature_at(a.opt, *a.counter);

  // X: the partner row (transformed below); the self row only enters the
  // mainlobe inner product c' = sum_n conj(part(n)) self(n) of eq. 38.
  float2 X[E];
  float cr = 0.f, ci = 0.f, es = 0.f, ep = 0.f;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const int n = t + TF * e;
    float2 v = make_float2(0.f, 0.f), s = make_float2(0.f, 0.f);
    if (e < EH && n < N) {
      switch (a.mode) {
        case PREP_B_SOFT:
        case PREP_B_HARD:
        case PREP_B_GIVEN: {
          if (a.mode == PREP_B_SOFT) s = soft_chip(zr + (int64_t)n * L, L, T, pl.sq_mode);
          else if (a.mode == PREP_B_HARD) s = level_phasor(hard_chip(zr + (int64_t)n * L, L), L);
          else s = a.s_given[rbase + n];
          if (active) a.wself[rbase + n] = s;
          v = a.h[rbase + n];
          break;
        }
        case PREP_A_HARD: {
          v = level_phasor(hard_chip(zr + (int64_t)n * L, L), L);
          if (active) a.wpart[rbase + n] = v;
          s = a.h[rbase + n];
          break;
        }
        default:
          v = a.wself[rbase + n];
          s = a.h[rbase + n];
          break;
      }
    }
    cr += v.x * s.x + v.y * s.y;
    ci += v.x * s.y - v.y * s.x;
    es += s.x * s.x + s.y * s.y;
    ep += v.x * v.x + v.y * v.y;
    X[e] = v;
  });
  cr = slot_sum<TF>(cr);
  ci = slot_sum<TF>(ci);
  es = slot_sum<TF>(es);
  ep = slot_sum<TF>(ep);
  if (active && t == 0) a.snrl[pl.row0 + g] = make_float4(cr, ci, es, ep);
  WaveTwiddles<P> W;
  W.init(t);
  fft_forward<P>(X, lds + slot * P, t, W);
  if (active) {
    float2* sp = a.spec + pl.ws_spec + (int64_t)g * P;
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      sp[e * TF + t] = X[e];
    });
  }
}

// ------------------------------------------------------------------ k_pass

struct PassArgs {
  const ProbPlan* plans;
  const int32_t* gprob;
  const int32_t* gwave;
  int32_t gn;
  int32_t orient;
  int32_t want_grad;
  int32_t pad;
  const float2* self_w;
  const float2* spec;
  UnitStat* ustat;
  float2* upart;
  float2* cube;  // orientation 0 only, may be null
};

template <int P, int PHLOG>
__global__ __launch_bounds__(64) void k_pass(PassArgs a) {
  using G = Geom<P>;
  constexpr int E = G::E, TF = G::TF, EH = E / 2;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x, slot = lane / TF, t = lane % TF;
  float2* buf = lds + slot * P;
  const int entry = find_entry(a.gwave, a.gn, blockIdx.x);
  const ProbPlan pl = a.plans[a.gprob[entry]];
  const int M = pl.M, N = pl.N, F = pl.F;
  const int unit = (blockIdx.x - a.gwave[entry]) * G::SLOTS + slot;
  const bool active = unit < pl.units;
  const int u = active ? unit : pl.units - 1;
  const int w = u / F, f = u - w * F;
  const float invN = 1.0f / (float)N;
  const float nu = (a.orient ? -1.0f : 1.0f) * (pl.nu_min + (float)f * pl.dnu);
  const int wlo = a.orient ? -pl.tau_hi : pl.tau_lo;
  const int whi = a.orient ? -pl.tau_lo : pl.tau_hi;
  const float phm1 = 0.5f * pl.p - 1.0f;
  const bool grad = a.want_grad != 0;

  WaveTwiddles<P> W;
  W.init(t);

  // Doppler-modulated self sequence, zero-padded to P (eq. 33, 35), and its FFT.
  float2 X[E];
  const float2* sw = a.self_w + pl.off_w + (int64_t)w * N;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    X[e] = make_float2(0.f, 0.f);
    if constexpr (e < EH) {
      const int n = t + TF * e;
      if (n < N) X[e] = cmul(sw[n], phasor(n, nu, invN));
    }
  });
  fft_forward<P>(X, buf, t, W);

  float2 U[E];
  static_for<E>([&](auto ec) { U[decltype(ec)::value] = make_float2(0.f, 0.f); });
  float sigma = 0.f, S = 0.f;
  unsigned long long kauto = 0, kcross = 0;
  const float2* spec = a.spec + pl.ws_spec;
  float2* cube = a.cube ? a.cube + pl.off_cube : nullptr;
  const float invP = 1.0f / (float)P;
  const int T2 = 2 * N - 1;

  for (int g = 0; g < M; ++g) {
    const float2* sg = spec + (int64_t)g * P;
    float2 R[E];
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      R[e] = cmulc(X[e], sg[e * TF + t]);
    });
    fft_inverse<P>(R, buf, t, W);  // R[e] = P * A(tau') at r-index k = t + TF e

    // ROI cells: r-index k holds tau' = -k (k < N) or P - k (k > P - N).
    uint32_t vmask = 0;
    unsigned long long key = 0;
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const int k = t + TF * e;
      int tp = 0;
      bool inr = false;
      if (k <= N - 1) {
        tp = -k;
        inr = true;
      } else if (k >= P - N + 1) {
        tp = P - k;
        inr = true;
      }
      const bool valid = inr && tp >= wlo && tp <= whi && !(g == w && tp == 0);
      if (valid) {
        vmask |= 1u << e;
        const float q = R[e].x * R[e].x + R[e].y * R[e].y;
        key = umax64(key, make_key(q, (uint32_t)(((int64_t)u * M + g) * P + k)));
      }
      if (cube != nullptr && active && inr)
        cube[((int64_t)(w * M + g) * F + f) * T2 + tp + N - 1] = cscale(R[e], invP);
    });
    key = slot_max_key<TF>(key);
    if (g == w) kauto = umax64(kauto, key);
    else kcross = umax64(kcross, key);
    const float mu = sqrtf(key_q(key));
    if (mu > sigma) {  // new running scale: rescale the partial sums (online max)
      const float c = sigma / mu;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);  // (c^2)^(p/2 - 1), (c^2)^(p/2)
      S *= cp;
      if (grad) {
        const float cpm1 = cm1 * c;  // c^(p-1)
        static_for<E>([&](auto ec) { U[decltype(ec)::value] = cscale(U[decltype(ec)::value], cpm1); });
      }
      sigma = mu;
    }
    const float inv_s = sigma > 0.f ? 1.0f / sigma : 0.f;
    const float inv_s2 = inv_s * inv_s;
    // a/sigma = x^(1/2), x = |r|^2 / sigma^2:  S += x^(p/2);  G~ = x^(p/2 - 1) r / sigma
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      if (vmask & (1u << e)) {
        const float x = (R[e].x * R[e].x + R[e].y * R[e].y) * inv_s2;
        float ym1, y;
        pow_ph<PHLOG>(x, phm1, ym1, y);
        S += y;
        R[e] = cscale(R[e], ym1 * inv_s);
      } else {
        R[e] = make_float2(0.f, 0.f);
      }
    });
    if (grad) {
      fft_forward<P>(R, buf, t, W);
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        U[e] = cadd(U[e], cmul(R[e], sg[e * TF + t]));
      });
    }
  }

  if (grad) {
    fft_inverse<P>(U, buf, t, W);
    if (active) {
      float2* up = a.upart + pl.ws_upart + (int64_t)u * N;
      static_for<EH>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        const int n = t + TF * e;
        if (n < N) up[n] = cmulc(U[e], phasor(n, nu, invN));
      });
    }
  }
  S = slot_sum<TF>(S);
  if (active && t == 0) {
    UnitStat st;
    st.sigma = sigma;
    st.S = S;
    st.pad0 = st.pad1 = 0;
    st.key_auto = kauto;
    st.key_cross = kcross;
    a.ustat[pl.ws_unit + u] = st;
  }
}

// ------------------------------------------------------------------ k_final

enum FinMode : int32_t {
  FIN_STATS = 0,   // statistics only
  FIN_GRAD = 1,    // statistics and gradient outputs (scaled by grad_loss)
  FIN_STEP_A = 2,  // Adam on the filters, then the energy projection
  FIN_STEP_B = 3,  // chain rule to the logits, Adam on the logits
};

struct FinArgs {
  const ProbPlan* plans;
  const int32_t* row_prob;
  int32_t nrows;
  int32_t orient;
  int32_t mode;
  int32_t inner;        // index of the inner step (Adam step count t * n + inner + 1)
  int32_t count_step;   // this launch ends the outer iteration: advance *counter
  int32_t wave_mode;    // SOFT / HARD / GIVEN for the logit chain of FIN_GRAD
  const float2* self_w;
  const float2* part_w;
  const UnitStat* ustat;
  const float2* upart;
  const float4* snrl;
  sqngd_stats* stats;
  const float* grad_loss;
  float2* grad_w;
  float* grad_z;
  float* z;     // logits: read for the chain, updated by FIN_STEP_B
  float2* h;    // filters updated by FIN_STEP_A
  float* adam;
  int32_t* counter;
  int32_t* done;
  sqngd_opt opt;
};

constexpr int kFinThreads = 256;

template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, T* sh, Op op) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off));
  __syncthreads();
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  T r = sh[0];
  for (int i = 1; i < kFinThreads / 64; ++i) r = op(r, sh[i]);
  return r;
}

__device__ __forceinline__ unsigned long long block_max_key(unsigned long long v, unsigned long long* sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)v, off), hi = __shfl_xor((uint32_t)(v >> 32), off);
    v = umax64(v, ((unsigned long long)hi << 32) | lo);
  }
  __syncthreads();
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  unsigned long long r = sh[0];
  for (int i = 1; i < kFinThreads / 64; ++i) r = umax64(r, sh[i]);
  return r;
}

struct FMax {
  __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct FSum {
  __device__ float operator()(float a, float b) const { return a + b; }
};
struct IOr {
  __device__ int operator()(int a, int b) const { return a | b; }
};

__global__ __launch_bounds__(kFinThreads) void k_final(FinArgs a) {
  __shared__ float shf[kFinThreads / 64];
  __shared__ int shi[kFinThreads / 64];
  __shared__ unsigned long long shk[kFinThreads / 64];
  __shared__ float fac[4096];
  __shared__ float2 csnrl[16];
  __shared__ float pm_sh[16];
  const int tid = threadIdx.x;
  const int r = blockIdx.x;
  const int pid = a.row_prob[r];
  const ProbPlan pl = a.plans[pid];
  const int M = pl.M, N = pl.N, F = pl.F, L = pl.L, P = pl.P;
  const int m = r - pl.row0;
  if (a.mode == FIN_STATS && m != 0) return;
  const UnitStat* us = a.ustat + pl.ws_unit;
  const float p = pl.p;

  // L_p = (sum over units of sigma_u^p S_u)^(1/p), evaluated relative to the largest sigma.
  float smax = 0.f;
  unsigned long long ka = 0, kc = 0;
  for (int i = tid; i < pl.units; i += kFinThreads) {
    smax = fmaxf(smax, us[i].sigma);
    ka = umax64(ka, us[i].key_auto);
    kc = umax64(kc, us[i].key_cross);
  }
  smax = block_reduce(smax, shf, FMax());
  ka = block_max_key(ka, shk);
  kc = block_max_key(kc, shk);
  float acc = 0.f;
  if (smax > 0.f)
    for (int i = tid; i < pl.units; i += kFinThreads) acc += powf(us[i].sigma / smax, p) * us[i].S;
  acc = block_reduce(acc, shf, FSum());
  const float lp_raw = smax > 0.f ? smax * powf(acc, 1.0f / p) : 0.f;
  const float lp = lp_raw * pl.inv_NP;

  // SNRL penalty (eq. 38-41): c'_k = sum_n conj(part_k(n)) self_k(n).
  float l_snrl = 0.f, snrl_max = -INFINITY, p_min = INFINITY;
  for (int k = 0; k < M; ++k) {
    const float4 c4 = a.snrl[pl.row0 + k];
    const float mag = sqrtf(c4.x * c4.x + c4.y * c4.y);
    const float pk = mag / (float)N;
    l_snrl += (pk - pl.p_tar) * (pk - pl.p_tar) / (float)M;
    snrl_max = fmaxf(snrl_max, 10.0f * log10f(c4.z * c4.w / (mag * mag)));
    p_min = fminf(p_min, pk);
    if (tid == 0) {
      csnrl[k] = make_float2(c4.x, c4.y);
      pm_sh[k] = pk;
    }
  }
  const float loss = pl.w_psl * lp + pl.w_snrl * l_snrl;
  const bool bad = !isfinite(loss);

  if (m == 0 && tid == 0 && a.stats != nullptr) {
    sqngd_stats st;
    st.loss = loss;
    st.lp = lp;
    st.l_snrl = l_snrl;
    const float invP = 1.0f / (float)P;
    st.psl_auto = sqrtf(key_q(ka)) * invP;
    st.psl_cross = sqrtf(key_q(kc)) * invP;
    const float psl = fmaxf(st.psl_auto, st.psl_cross);
    st.pslr_db = 20.0f * log10f(psl / (float)N);
    st.snrl_db_max = snrl_max;
    st.p_min = p_min;
    const unsigned long long kb = key_q(ka) >= key_q(kc) ? ka : kc;
    const uint32_t cell = key_cell(kb);
    const int kk = (int)(cell % (uint32_t)P);
    const uint32_t rest = cell / (uint32_t)P;
    const int gg = (int)(rest % (uint32_t)M);
    const int uu = (int)(rest / (uint32_t)M);
    const int ww = uu / F, ff = uu % F;
    const int tp = kk <= N - 1 ? -kk : P - kk;
    if (a.orient == 0) {
      st.arg_m = ww;
      st.arg_l = gg;
      st.arg_tau = tp;
    } else {
      st.arg_m = gg;
      st.arg_l = ww;
      st.arg_tau = -tp;
    }
    st.arg_f = ff;
    st.nonfinite = bad ? 1u : 0u;
    st.reserved[0] = st.reserved[1] = st.reserved[2] = 0;
    a.stats[pid] = st;
  }
  if (a.mode == FIN_STATS) return;
  __syncthreads();

  // Gradient of row m of the self sequence:
  //   sum_f (w_psl / (N P)) (sigma_u / lp_raw)^(p-1) partial_u  +  G'_S part_m
  for (int ff = tid; ff < F; ff += kFinThreads) {
    const float su = us[m * F + ff].sigma;
    fac[ff] = lp_raw > 0.f ? pl.w_psl / ((float)N * (float)P) * powf(su / lp_raw, p - 1.0f) : 0.f;
  }
  __syncthreads();
  const float gl = a.grad_loss ? a.grad_loss[pid] : 1.0f;
  const float2 cm = csnrl[m];
  const float magm = sqrtf(cm.x * cm.x + cm.y * cm.y);
  float2 gS = make_float2(0.f, 0.f);
  if (magm > 0.f) gS = cscale(cm, pl.w_snrl * (2.0f / (float)M) * (pm_sh[m] - pl.p_tar) / ((float)N * magm));
  constexpr int kMaxPer = 1024 / kFinThreads;
  float2 gr[kMaxPer];
  int rowbad = 0;
  const float2* up = a.upart + pl.ws_upart + (int64_t)m * F * N;
  const float2* pw = a.part_w + pl.off_w + (int64_t)m * N;
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) {
    const int n = tid + i * kFinThreads;
    float2 g = make_float2(0.f, 0.f);
    if (n < N) {
      for (int ff = 0; ff < F; ++ff) {
        const float2 v = up[(int64_t)ff * N + n];
        g.x += fac[ff] * v.x;
        g.y += fac[ff] * v.y;
      }
      g = cadd(g, cmul(gS, pw[n]));
      g = cscale(g, gl);
      if (!isfinite(g.x) || !isfinite(g.y)) rowbad = 1;
    }
    gr[i] = g;
  }
  rowbad = block_reduce(rowbad, shi, IOr());
  const bool skip = bad || rowbad;

  const int64_t wrow = pl.off_w + (int64_t)m * N;
  if (a.mode == FIN_GRAD) {
    if (a.grad_w) {
#pragma unroll
      for (int i = 0; i < kMaxPer; ++i) {
        const int n = tid + i * kFinThreads;
        if (n < N) a.grad_w[wrow + n] = gr[i];
      }
    }
    if (a.grad_z && a.orient == 0) {
      const float T = pl.temperature;
#pragma unroll
      for (int i = 0; i < kMaxPer; ++i) {
        const int n = tid + i * kFinThreads;
        if (n >= N) continue;
        float* gz = a.grad_z + pl.off_z + (wrow - pl.off_w + n) * L;
        const float* zc = a.z + pl.off_z + (wrow - pl.off_w + n) * L;
        if (a.wave_mode != SQNGD_WAVE_SOFT) {
          for (int l = 0; l < L; ++l) gz[l] = 0.f;
          continue;
        }
        float zm = zc[0];
        for (int l = 1; l < L; ++l) zm = fmaxf(zm, zc[l]);
        float sum = 0.f, ybar = 0.f;
        for (int l = 0; l < L; ++l) {
          float e = expf((zc[l] - zm) / T);
          sum += e;
          ybar += (float)l * e;
        }
        ybar /= sum;
        const float2 s = a.self_w[wrow + n];
        const float2 g = gr[i];
        if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
          const float dphi = g.y * s.x - g.x * s.y;  // Im(g conj(s))
          const float c = dphi * 2.0f * 3.14159265358979f / ((float)L * T);
          for (int l = 0; l < L; ++l) gz[l] = c * (expf((zc[l] - zm) / T) / sum) * ((float)l - ybar);
        } else {
          for (int l = 0; l < L; ++l) {
            const float pi_l = expf((zc[l] - zm) / T) / sum;
            const float2 ul = level_phasor(l, L);
            gz[l] = pi_l / T * (g.x * (ul.x - s.x) + g.y * (ul.y - s.y));
          }
        }
      }
    }
  } else if (a.mode == FIN_STEP_A) {
    const int tstep = *a.counter;
    const int k = tstep * a.opt.n_h + a.inner + 1;
    const float b1 = a.opt.beta1, b2 = a.opt.beta2;
    const float bc1 = 1.0f - powf(b1, (float)k), bc2 = 1.0f - powf(b2, (float)k);
    const bool sgd = (a.opt.flags & SQNGD_OPT_SGD) != 0;
    float* mh = a.adam + pl.off_state + 2 * (int64_t)M * N * L + 2 * (wrow - pl.off_w);
    float* vh = mh + 2 * (int64_t)M * N;
    float2 hn[kMaxPer];
    float e2 = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const int n = tid + i * kFinThreads;
      hn[i] = make_float2(0.f, 0.f);
      if (n >= N) continue;
      float2 hv = a.h[wrow + n];
      if (!skip) {
        const float g2[2] = {gr[i].x, gr[i].y};
        float hv2[2] = {hv.x, hv.y};
        for (int c = 0; c < 2; ++c) {
          if (sgd) {
            hv2[c] -= a.opt.lr_h * g2[c];
          } else {
            float mm = b1 * mh[2 * n + c] + (1.0f - b1) * g2[c];
            float vv = b2 * vh[2 * n + c] + (1.0f - b2) * g2[c] * g2[c];
            mh[2 * n + c] = mm;
            vh[2 * n + c] = vv;
            hv2[c] -= a.opt.lr_h * (mm / bc1) / (sqrtf(vv / bc2) + a.opt.eps);
          }
        }
        hv = make_float2(hv2[0], hv2[1]);
      }
      hn[i] = hv;
      e2 += hv.x * hv.x + hv.y * hv.y;
    }
    e2 = block_reduce(e2, shf, FSum());
    const float sc = skip ? 1.0f : sqrtf((float)N / e2);  // eq. 32
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const int n = tid + i * kFinThreads;
      if (n < N) a.h[wrow + n] = cscale(hn[i], sc);
    }
  } else if (a.mode == FIN_STEP_B) {
    const int tstep = *a.counter;
    const int k = tstep * a.opt.n_x + a.inner + 1;
    const float b1 = a.opt.beta1, b2 = a.opt.beta2;
    const float bc1 = 1.0f - powf(b1, (float)k), bc2 = 1.0f - powf(b2, (float)k);
    const bool sgd = (a.opt.flags & SQNGD_OPT_SGD) != 0;
    const float T = temperature_at(a.opt, tstep);
    float* mz = a.adam + pl.off_state;
    float* vz = mz + (int64_t)M * N * L;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const int n = tid + i * kFinThreads;
      if (n >= N || skip) continue;
      const int64_t zoff = pl.off_z + (wrow - pl.off_w + n) * L;
      const int64_t soff = (wrow - pl.off_w + n) * L;
      float* zc = a.z + zoff;
      float zm = zc[0];
      for (int l = 1; l < L; ++l) zm = fmaxf(zm, zc[l]);
      float sum = 0.f, ybar = 0.f;
      for (int l = 0; l < L; ++l) {
        float e = expf((zc[l] - zm) / T);
        sum += e;
        ybar += (float)l * e;
      }
      ybar /= sum;
      const float2 s = a.self_w[wrow + n];
      const float2 g = gr[i];
      const float dphi = g.y * s.x - g.x * s.y;
      const float c = dphi * 2.0f * 3.14159265358979f / ((float)L * T);
      for (int l = 0; l < L; ++l) {
        const float pi_l = expf((zc[l] - zm) / T) / sum;
        float gv;
        if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
          gv = c * pi_l * ((float)l - ybar);
        } else {
          const float2 ul = level_phasor(l, L);
          gv = pi_l / T * (g.x * (ul.x - s.x) + g.y * (ul.y - s.y));
        }
        if (sgd) {
          zc[l] -= a.opt.lr_z * gv;
        } else {
          float mm = b1 * mz[soff + l] + (1.0f - b1) * gv;
          float vv = b2 * vz[soff + l] + (1.0f - b2) * gv * gv;
          mz[soff + l] = mm;
          vz[soff + l] = vv;
          zc[l] -= a.opt.lr_z * (mm / bc1) / (sqrtf(vv / bc2) + a.opt.eps);
        }
      }
    }
  }

  if (a.count_step) {
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const int old = atomicAdd(a.done, 1);
      if (old == a.nrows - 1) {
        atomicExch(a.done, 0);
        atomicAdd(a.counter, 1);
      }
    }
  }
}

// ------------------------------------------------------------------ k_hardq

struct HardArgs {
  const ProbPlan* plans;
  const int32_t* row_prob;
  const float* z;
  int32_t* idx;
  float2* x;
};

__global__ __launch_bounds__(256) void k_hardq(HardArgs a) {
  const int r = blockIdx.x;
  const ProbPlan pl = a.plans[a.row_prob[r]];
  const int m = r - pl.row0;
  for (int n = threadIdx.x; n < pl.N; n += 256) {
    const int64_t c = (int64_t)m * pl.N + n;
    const int l = hard_chip(a.z + pl.off_z + c * pl.L, pl.L);
    if (a.idx) a.idx[pl.off_w + c] = l;
    if (a.x) a.x[pl.off_w + c] = level_phasor(l, pl.L);
  }
}

__global__ void k_zero_i32(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

}  // namespace sq
