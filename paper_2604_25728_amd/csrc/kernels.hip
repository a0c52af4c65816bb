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

// exp(j 2 pi n nu / N) (the Doppler modulation of eq. 33): the phase in turns
// is formed and reduced to [-1/2, 1/2] in FP64 -- on a wide Doppler span
// (|nu| up to N / 2) it holds hundreds of whole turns, and an FP32 product
// would keep only about 1e-5 of a turn of its fraction -- then one FP32
// sincospi. Two calls per lane and unit, so the FP64 cost is negligible.
__device__ __forceinline__ float2 phasor(int n, double nu, double invN) {
  double ph = (double)n * nu * invN;
  ph -= rint(ph);
  float s, c;
  sincospif(2.0f * (float)ph, &s, &c);
  return make_float2(c, s);
}

// Doppler frequency of bin f, negated in orientation 1 (the role swap).
__device__ __forceinline__ double doppler_nu(const ProbPlan& pl, int f, int orient) {
  const double nu = pl.nu_min + (double)f * pl.dnu;
  return orient ? -nu : nu;
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
  return o.T0 * exp2f(frac * log2f(o.T1 / o.T0));
}

// 1 - b^k for the Adam bias corrections (0 < b < 1, k >= 1).
__device__ __forceinline__ float bias_corr(float b, int k) { return 1.0f - exp2f((float)k * log2f(b)); }

// phasor(n, nu, invN) for n = t + TF e, e < EH: one sincospi for n = t, one
// for the step TF, then products (the step's rounding grows by one ulp per e).
template <int EH, int TF>
__device__ __forceinline__ void phasor_row(int t, double nu, double invN, float2 (&ph)[EH]) {
  ph[0] = phasor(t, nu, invN);
  if constexpr (EH > 1) {
    const float2 st = phasor(TF, nu, invN);
    static_for<EH - 1>([&](auto ec) {
      constexpr int e = decltype(ec)::value + 1;
      ph[e] = cmul(ph[e - 1], st);
    });
  }
}

// The region-of-interest cells of one AF row held as R[e] = P A(tau') at
// r-index k = t + TF e, as two runs of r-index: k in
// [a0, a0 + na] holds tau' = -k (k <= N - 1), k in [b0, b0 + nb] holds tau' =
// P - k (k >= P - N + 1), each clipped to [wlo, whi]; an empty run starts at
// 2^30 with length 0, past every index. Cell k is inside when the unsigned
// (k - a0) <= na or (k - b0) <= nb: the same for every partner of a unit.
struct RoiRuns {
  int a0, na, b0, nb;
};
template <int P>
__device__ __forceinline__ RoiRuns roi_runs(int N, int wlo, int whi) {
  RoiRuns r;
  const int alo = max(0, -whi), ahi = min(N - 1, -wlo);
  const int blo = max(P - N + 1, P - whi), bhi = min(P - 1, P - wlo);
  r.a0 = alo <= ahi ? alo : (1 << 30);
  r.na = alo <= ahi ? ahi - alo : 0;
  r.b0 = blo <= bhi ? blo : (1 << 30);
  r.nb = blo <= bhi ? bhi - blo : 0;
  return r;
}

// The membership bits of lane t's cells k = t + TF e; with drop0 the cell
// k = 0 (tau' = 0) is left out.
template <int TF, int E>
__device__ __forceinline__ uint32_t roi_bits(const RoiRuns& r, int t, bool drop0) {
  uint32_t v = 0;
  const int ta = t - r.a0, tb = t - r.b0;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const bool in = (uint32_t)(ta + TF * e) <= (uint32_t)r.na || (uint32_t)(tb + TF * e) <= (uint32_t)r.nb;
    v |= in ? (1u << e) : 0u;
  });
  return drop0 && t == 0 ? v & ~1u : v;
}

// In-ROI scan of a row over the membership bits vmask: cells outside the
// region are set to 0 (so that the scaling after it needs no mask), and the
// lane's largest |r|^2 is found with its lowest index.
template <int TF, int E>
__device__ __forceinline__ void roi_scan_bits(float2 (&R)[E], int t, uint32_t vmask, float& qmax, int& kbest) {
  qmax = 0.f;
  kbest = 0;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const bool valid = (vmask >> e) & 1u;
    R[e] = valid ? R[e] : make_float2(0.f, 0.f);
    const float q = R[e].x * R[e].x + R[e].y * R[e].y;
    const bool better = q > qmax;
    qmax = better ? q : qmax;
    kbest = better ? t + TF * e : kbest;
  });
}

// S += sum over the cells of x^(p/2), x = |r|^2 / sigma^2, and the scaled
// adjoint r <- x^(p/2 - 1) r / sigma. Cells outside the region hold 0 (from
// roi_scan_bits): they add 0 and stay 0 for every p.
template <int PHLOG, int E>
__device__ __forceinline__ void roi_scale(float2 (&R)[E], float inv_s, float phm1, float& S) {
  const float inv_s2 = inv_s * inv_s;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const float x = (R[e].x * R[e].x + R[e].y * R[e].y) * inv_s2;
    float ym1, y;
    pow_ph<PHLOG>(x, phm1, ym1, y);
    S += y;
    R[e] = cscale(R[e], ym1 * inv_s);
  });
}

// ROI weights w(tau, f) of eq. 8-9 applied to a row held as R[e] (r-index
// k = t + TF e holds tau' = -k or P - k of the pass's orientation; the table
// row wrow = w(., f) is indexed by the original delay tau + N - 1, with
// tau = tau' in orientation 0 and -tau' in the role-swapped orientation 1).
// Cells that hold no delay get 0.
template <int P, int TF, int E>
__device__ __forceinline__ void roi_weigh(float2 (&R)[E], int t, int N, int orient, const float* wrow) {
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const int k = t + TF * e;
    const bool lo = k <= N - 1, hi = k >= P - N + 1;
    const int tp = lo ? -k : P - k;
    const int tau = orient ? -tp : tp;
    const float wv = (lo || hi) ? wrow[tau + N - 1] : 0.f;
    R[e] = cscale(R[e], wv);
  });
}

// The same with the weights of the lane's cells already in registers.
template <int E>
__device__ __forceinline__ void roi_weigh_reg(float2 (&R)[E], const float (&wr)[E]) {
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    R[e] = cscale(R[e], wr[e]);
  });
}

// The ROI weights of lane t's cells from the table row wrow = w(., f) (the
// indexing of roi_weigh), 0 where a cell holds no delay; every load issued.
template <int P, int TF, int E>
__device__ __forceinline__ void roi_weights_load(float (&wr)[E], int t, int N, int orient, const float* wrow) {
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const int k = t + TF * e;
    const bool lo = k <= N - 1, hi = k >= P - N + 1;
    const int tp = lo ? -k : P - k;
    const int tau = orient ? -tp : tp;
    const float v = wrow[(lo || hi) ? tau + N - 1 : 0];
    wr[e] = (lo || hi) ? v : 0.f;
  });
}

// AF cells of one row into the cube [w][g][f][tau + N - 1] (scaled by 1/P).
template <int P, int TF, int E>
__device__ __forceinline__ void cube_store(const float2 (&R)[E], int t, int N, float2* row) {
  const float invP = 1.0f / (float)P;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const int k = t + TF * e;
    if (k <= N - 1) row[N - 1 - k] = cscale(R[e], invP);
    else if (k >= P - N + 1) row[P - k + N - 1] = cscale(R[e], invP);
  });
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

// Waves per block of the throughput pass launched for one FFT length: four
// (one unit per wave up to P = 512, one unit at 2048), two at 1024 (one
// unit), eight sharing one unit at 4096. In the one-launch form of several
// groups every block has four waves (two units of two waves at 1024).
__host__ __device__ constexpr int pass_waves(int P) { return P >= 4096 ? 8 : (P == 1024 ? 2 : 4); }
// FFT geometry of the throughput pass: wave-local up to P = 512; from 1024
// on one transform spans the block's waves with 8 elements per lane (128
// lanes at 1024, 256 at 2048, 512 at 4096; three LDS exchanges). With the
// exchange buffers padded against bank conflicts this runs three waves per
// SIMD at P = 1024 and 2048 (168 VGPRs; 250 with one wave and 16 elements
// per lane held only two), measured 23% faster per pass on both.
__host__ __device__ constexpr int pass_tf(int P) {
  return P >= 4096 ? 512 : (P >= 2048 ? 256 : (P >= 1024 ? 128 : (P >= 512 ? 64 : P / 8)));
}
template <int P>
using PassGeom = GeomT<P, pass_tf(P)>;
// Waves per SIMD the throughput pass is compiled for: three at P = 1024 and
// 2048 (the register budget of 168 per lane; the compiler keeps a few values
// in scratch at 2048). The weighted instantiations keep their registers and
// run two.
__host__ __device__ constexpr int pass_min_waves(int P) { return P == 1024 || P == 2048 ? 3 : 1; }
// Doppler bins (units) per throughput-pass block of BW waves
__host__ __device__ constexpr int pass_upb(int P, int BW) { return BW * 64 / pass_tf(P); }
__host__ __device__ constexpr int pass_upb(int P) { return pass_upb(P, pass_waves(P)); }
// Where a producer's spectral bin k lands in the partner-spectrum rows the
// pass reads: the throughput pass's own layout, or (spec_wave, a problem
// whose group runs the latency pass) the one-wave layout the producers and
// the latency pass share, so neither side scatters.
template <int P>
__device__ __forceinline__ int pass_spec_slot(int t, int e) {
  using GP = Geom<P>;
  using GC = PassGeom<P>;
  if constexpr (GP::TF == GC::TF) return e * GP::TF + t;
  else return GC::spec_index(GP::spec_bin(t, e));
}
template <int P>
__device__ __forceinline__ int spec_slot(const ProbPlan& pl, int t, int e) {
  return pl.spec_wave ? e * Geom<P>::TF + t : pass_spec_slot<P>(t, e);
}

// Reductions over the lanes of one FFT of geometry G, the result in all of
// them; a transform spread over several waves combines the waves' values
// through red[] (one entry per wave of the block) in wave order.
// kLead = false drops the barrier that orders the previous reads of red[]
// before the new writes: for callers whose every wave has passed a block
// barrier since it last read red[] (a multi-wave transform's exchanges are).
template <class G, class Op, bool kLead = true>
__device__ __forceinline__ float fft_lanes_reduce(float v, float ident, Op op, float* red) {
  if constexpr (G::WAVES == 1) {
    return slot_reduce<G::TF>(v, ident, op);
  } else {
    v = slot_reduce<64>(v, ident, op);
    if constexpr (kLead) block_lds_sync();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    block_lds_sync();
    const int w0 = (threadIdx.x / G::TF) * G::WAVES;
    float r = red[w0];
    for (int i = 1; i < G::WAVES; ++i) r = op(r, red[w0 + i]);
    return r;
  }
}
template <class G>
__device__ __forceinline__ unsigned long long fft_lanes_max_key(unsigned long long v, unsigned long long* red) {
  if constexpr (G::WAVES == 1) {
    return slot_max_key<G::TF>(v);
  } else {
    v = slot_max_key<64>(v);
    block_lds_sync();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    block_lds_sync();
    const int w0 = (threadIdx.x / G::TF) * G::WAVES;
    unsigned long long r = red[w0];
    for (int i = 1; i < G::WAVES; ++i) r = umax64(r, red[w0 + i]);
    return r;
  }
}

// At P >= 2048 the partner spectra are computed by k_rowspec (the pass's own
// two- or eight-wave transform) after the kernel that writes their rows,
// instead of by one wave of k_prep / k_final (32 or 64 elements per lane).
__host__ __device__ constexpr bool spec_by_rowspec(int P) { return P >= 2048; }

struct RowSpecArgs {
  const ProbPlan* plans;
  const int32_t* rows;      // batch rows of this launch, one block each
  const int32_t* row_prob;  // problem of every batch row
  const float2* src;        // rows [off_w + m N .. + N) to transform
  float2* spec;             // partner spectra, the pass's layout
  int32_t single;
  ProbPlan one;
};

// Spectrum of one row of src (zero-padded to P) in the throughput pass's
// layout, one block of the pass's transform width per row.
template <int P>
__global__ __launch_bounds__(64 * PassGeom<P>::WAVES) void k_rowspec(RowSpecArgs a) {
  using G = PassGeom<P>;
  constexpr int E = G::E, TF = G::TF;
  __shared__ float2 buf[G::SPAN];
  int r, pid;
  ProbPlan pl;
  if (a.single) {
    r = a.rows[blockIdx.x];
    pid = 0;
    pl = a.one;
  } else {
    r = a.rows[blockIdx.x];
    pid = a.row_prob[r];
    pl = a.plans[pid];
  }
  (void)pid;
  const int m = r - pl.row0, N = pl.N, t = threadIdx.x;
  const float2* row = a.src + pl.off_w + (int64_t)m * N;
  float2 X[E];
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    const int n = t + TF * e;
    X[e] = n < N ? row[n] : make_float2(0.f, 0.f);
  });
  TwiddlesG<G> W;
  W.init(t);
  fft_forward_g<G>(X, buf, t, W);
  float2* out = a.spec + pl.ws_spec + (int64_t)m * P;
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    out[e * TF + t] = X[e];
  });
}

// ------------------------------------------------------------------ k_prep

enum PrepMode : int32_t {
  PREP_B_SOFT = 0,   // self = soft(z) -> wself; partners = h
  PREP_B_HARD = 1,   // self = hard(z) -> wself; partners = h
  PREP_B_GIVEN = 2,  // self = s_given -> wself; partners = h
  PREP_A_HARD = 3,   // partners = hard(z) -> wpart (self = h)
  PREP_A_SELF = 4,   // partners = wself (self = h)
  PREP_A_GIVEN = 5,  // partners = s_given (self = h)
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
  const int32_t* rows;      // k_prep_row: the group's batch rows, one block each
  const int32_t* row_prob;  // k_prep_row: problem of each batch row
  int32_t single;  // one problem: its plan is `one`, no table lookups
  ProbPlan one;
};

// One chip n of the first pass's inputs: the partner sample v (the row that
// is transformed into the partner spectrum) and the self sample s, with the
// waveform the mode derives written to its buffer when the row is active.
__device__ __forceinline__ void prep_chip(const PrepArgs& a, const ProbPlan& pl, int64_t rbase, const float* zr,
                                          int n, float T, bool active, float2& v, float2& s) {
  const int L = pl.L;
  v = s = make_float2(0.f, 0.f);
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
    case PREP_A_GIVEN:
      v = a.s_given[rbase + n];
      s = a.h[rbase + n];
      break;
    default:
      v = a.wself[rbase + n];
      s = a.h[rbase + n];
      break;
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_prep(PrepArgs a) {
  using G = Geom<P>;
  constexpr int E = G::E, TF = G::TF, EH = E / 2;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x, slot = lane / TF, t = lane % TF;
  int base = 0;
  ProbPlan pl;
  if (a.single) {
    pl = a.one;
  } else {
    const int entry = find_entry(a.grwave, a.gn, blockIdx.x);
    pl = a.plans[a.gprob[entry]];
    base = a.grwave[entry];
  }
  const int row = (blockIdx.x - base) * G::SLOTS + slot;
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
    if (e < EH && n < N) prep_chip(a, pl, rbase, zr, n, T, active, v, s);
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
  if constexpr (!spec_by_rowspec(P)) {
    WaveTwiddles<P> W;
    W.init(t);
    fft_forward<P>(X, lds + slot * G::SPAN, t, W);
    if (active) {
      float2* sp = a.spec + pl.ws_spec + (int64_t)g * P;
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        sp[spec_slot<P>(pl, t, e)] = X[e];
      });
    }
  }
}

// Maximum and sum over a wave's 64 lanes (every lane gets the result).
__device__ __forceinline__ float wave_max(float v) { return slot_reduce<64>(v, 0.0f, OpMax()); }
__device__ __forceinline__ float wave_sum(float v) { return slot_reduce<64>(v, 0.0f, OpAdd()); }

// Block sums of four products and a flag, in wave order (the same in every
// thread) over NW waves; sh holds 5 * NW floats.
template <int NW>
__device__ __forceinline__ void block_sum5(float (&v)[5], float* sh) {
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = wave_sum(v[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 5; ++i) sh[i * NW + (threadIdx.x >> 6)] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float r = 0.f;
    for (int w = 0; w < NW; ++w) r += sh[i * NW + w];
    v[i] = r;
  }
}

// The first pass's inputs at the FFT lengths whose partner spectra k_rowspec
// computes (P >= 2048): one 1024-thread block per batch row, a thread per chip
// (two at N > 1024), the row's mainlobe and energy products (eq. 38) summed
// over the block in wave order.
constexpr int kPrepRowThreads = 1024;
__global__ __launch_bounds__(kPrepRowThreads) void k_prep_row(PrepArgs a) {
  constexpr int NW = kPrepRowThreads / 64;
  __shared__ float sh[5 * NW];
  int r;
  ProbPlan pl;
  if (a.single) {
    r = blockIdx.x;
    pl = a.one;
  } else {
    r = a.rows[blockIdx.x];
    pl = a.plans[a.row_prob[r]];
  }
  const int g = r - pl.row0;
  const int N = pl.N, L = pl.L;
  const int64_t rbase = pl.off_w + (int64_t)g * N;
  const float* zr = a.z ? a.z + pl.off_z + (int64_t)g * N * L : nullptr;
  float T = pl.temperature;
  if (a.use_schedule) T = temperature_at(a.opt, *a.counter);
  float q[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  for (int n = threadIdx.x; n < N; n += kPrepRowThreads) {
    float2 v, s;
    prep_chip(a, pl, rbase, zr, n, T, true, v, s);
    q[0] += v.x * s.x + v.y * s.y;
    q[1] += v.x * s.y - v.y * s.x;
    q[2] += s.x * s.x + s.y * s.y;
    q[3] += v.x * v.x + v.y * v.y;
  }
  block_sum5<NW>(q, sh);
  if (threadIdx.x == 0) a.snrl[r] = make_float4(q[0], q[1], q[2], q[3]);
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
  int32_t* bump;  // if set, block 0 advances this step counter (deferred by the previous finalize)
  const float* roi_w;  // ROI weights [F][2N-1] per problem (plan offset off_rw), or null for w = 1
  const float2* self_w;
  const float2* spec;
  UnitStat* ustat;
  float2* upart;
  float2* cube;  // orientation 0 only, may be null
  int32_t single;  // one problem: its plan is `one`, no table lookups
  ProbPlan one;
};


// LDS of one throughput-pass block. The accumulated adjoint spectra U and the
// self spectrum X live in the slot's LDS slice instead of registers: three
// E-element arrays per lane plus the partner spectrum would cap the occupancy.
template <int P, int BW>
struct PassSmem {
  static constexpr int UPB = pass_upb(P, BW), W = BW;
  float2 lds[UPB * PassGeom<P>::SPAN];  // FFT exchange buffers (padded), then the demodulated partials
  float2 ulds[UPB * P];                 // accumulated adjoint spectra U
  float2 xlds[UPB * P];                 // self spectrum X
  float u_sig[UPB], u_S[UPB];
  unsigned long long u_ka[UPB], u_kc[UPB];
  float red_f[W];
  unsigned long long red_k[W];
};

// One block of the throughput pass: block `blk` of the FFT-length group the
// tables of `a` describe. WT: the launch carries ROI weights (a separate
// instantiation, so that the unweighted pass keeps its registers).
template <int P, int PHLOG, bool WT, int BW>
__device__ __forceinline__ void pass_block(const PassArgs& a, int blk, PassSmem<P, BW>& sm) {
  using G = PassGeom<P>;
  constexpr int kPassWaves = BW;
  constexpr int E = G::E, TF = G::TF, EH = E / 2;
  constexpr int UPB = pass_upb(P, BW);  // units (Doppler bins of one row) per block
  static_assert(UPB * TF == 64 * kPassWaves, "the units fill the block");
  constexpr bool kUL = true;
  constexpr bool kXL = true;
  float2* const lds = sm.lds;
  float2* const ulds = sm.ulds;
  float2* const xlds = sm.xlds;
  float* const u_sig = sm.u_sig;
  float* const u_S = sm.u_S;
  unsigned long long* const u_ka = sm.u_ka;
  unsigned long long* const u_kc = sm.u_kc;
  float* const red_f = sm.red_f;
  unsigned long long* const red_k = sm.red_k;
  // uslot: the block's unit this lane works on; t: its lane within the FFT
  const int uslot = threadIdx.x / TF, t = threadIdx.x % TF;
  if (a.bump != nullptr && blk == 0 && threadIdx.x == 0) atomicAdd(a.bump, 1);
  float2* buf = lds + uslot * G::SPAN;
  int base = 0;
  ProbPlan pl;
  if (a.single) {
    pl = a.one;
  } else {
    const int entry = find_entry(a.gwave, a.gn, blk);
    pl = a.plans[a.gprob[entry]];
    base = a.gwave[entry];
  }
  const int M = pl.M, N = pl.N, F = pl.F;
  // blocks of a problem: wpr per row, rows in order; a block covers UPB
  // consecutive Doppler bins of one row, one per slot
  const int lb = blk - base;
  const int w = lb / pl.wpr;
  const int grp = lb - w * pl.wpr;
  const int fs = grp * UPB + uslot;
  const bool active = fs < F;
  const int f = active ? fs : F - 1;
  const int u = w * F + f;
  const double invN = 1.0 / (double)N;
  const double nu = doppler_nu(pl, f, a.orient);
  const int wlo = a.orient ? -pl.tau_hi : pl.tau_lo;
  const int whi = a.orient ? -pl.tau_lo : pl.tau_hi;
  const float phm1 = 0.5f * pl.p - 1.0f;
  const bool grad = a.want_grad != 0;
  const float* wrow = WT ? a.roi_w + pl.off_rw + (int64_t)f * (2 * N - 1) : nullptr;

  TwiddlesG<G> W;
  W.init(t);

  // The pass is a sequence of 2M+2 transforms (M+1 without the gradient):
  //   SELF  forward FFT of the Doppler-modulated self sequence (eq. 33, 35)
  //   PAIR  inverse FFT of X conj(H_g): the AF row of partner g (eq. 36)
  //   ADJ   forward FFT of the scaled adjoint of that row
  //   UINV  inverse FFT of the accumulated adjoint spectra
  // run as one loop over a single forward and a single inverse transform, so
  // the code each wave streams through the instruction cache stays small.
  enum Op { OP_SELF, OP_PAIR, OP_ADJ, OP_UINV };
  constexpr bool kKeepSG = E <= 8 && !kXL;  // the partner spectrum stays in registers for both uses
  const float2* spec = a.spec + pl.ws_spec;
  const float2* sw = a.self_w + pl.off_w + (int64_t)w * N;
  float2* cube = a.cube ? a.cube + pl.off_cube : nullptr;
  const int T2 = 2 * N - 1;
  float2 X[kXL ? 1 : E], U[kUL ? 1 : E], R[E], SG[kKeepSG ? E : 1];
  float2* ub = ulds + uslot * P;
  float2* xb = xlds + (kXL ? uslot * P : 0);
  {
    float2 ph[EH];
    phasor_row<EH, TF>(t, nu, invN, ph);
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      R[e] = make_float2(0.f, 0.f);
      if constexpr (kUL) ub[e * TF + t] = make_float2(0.f, 0.f);
      else U[e] = make_float2(0.f, 0.f);
      if constexpr (e < EH) {
        const int n = t + TF * e;
        if (n < N) R[e] = cmul(sw[n], ph[e]);
      }
    });
  }
  float sigma = 0.f, S = 0.f;
  unsigned long long kauto = 0, kcross = 0;  // per lane; reduced once per unit
  const RoiRuns runs = roi_runs<P>(N, wlo, whi);
  const bool cut0 = f >= pl.cut_lo && f < pl.cut_hi;  // the auto pair drops its tau = 0 cell
  int g = 0;
  const float2* sg = spec;
  auto start_pair = [&]() {  // R = X conj(H_g)
    sg = spec + (int64_t)g * P;
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const float2 xe = kXL ? xb[e * TF + t] : X[kXL ? 0 : e];
      if constexpr (kKeepSG) {
        SG[e] = sg[e * TF + t];
        R[e] = cmulc(xe, SG[e]);
      } else {
        R[e] = cmulc(xe, sg[e * TF + t]);
      }
    });
  };
  for (int op = OP_SELF;;) {
    if (op == OP_PAIR || op == OP_UINV) fft_inverse_g<G>(R, buf, t, W);
    else fft_forward_g<G>(R, buf, t, W);
    if (op == OP_UINV) break;
    if (op == OP_SELF) {
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        if constexpr (kXL) xb[e * TF + t] = R[e];
        else X[e] = R[e];
      });
      start_pair();
      op = OP_PAIR;
      continue;
    }
    if (op == OP_ADJ) {
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        if constexpr (kUL) ub[e * TF + t] = cadd(ub[e * TF + t], cmul(R[e], sg[e * TF + t]));
        else if constexpr (kKeepSG) U[e] = cadd(U[e], cmul(R[e], SG[e]));
        else U[e] = cadd(U[e], cmul(R[e], sg[e * TF + t]));
      });
      if (++g < M) {
        start_pair();
        op = OP_PAIR;
      } else {
        static_for<E>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          if constexpr (kUL) R[e] = ub[e * TF + t];
          else R[e] = U[e];
        });
        op = OP_UINV;
      }
      continue;
    }
    // OP_PAIR: R[e] = P * A(tau') at r-index k = t + TF e; ROI cells hold
    // tau' = -k (k < N) or P - k (k > P - N).
    uint32_t vmask;
    float qmax;
    int kbest;
    if (cube != nullptr && active) cube_store<P, TF, E>(R, t, N, cube + ((int64_t)(w * M + g) * F + f) * T2);
    if constexpr (WT) roi_weigh<P, TF, E>(R, t, N, a.orient, wrow);  // a = w |A| / N from here on
    vmask = roi_bits<TF, E>(runs, t, g == w && cut0);
    roi_scan_bits<TF, E>(R, t, vmask, qmax, kbest);
    // this lane's largest cell of the pair (lowest index among equal values)
    const unsigned long long key = vmask ? make_key(qmax, (uint32_t)(((int64_t)u * M + g) * P + kbest)) : 0ull;
    if (g == w) kauto = umax64(kauto, key);
    else kcross = umax64(kcross, key);
    // every wave has passed this pair's inverse transform (block barriers
    // between its exchanges) since the previous pair's reduction read red_f
    qmax = fft_lanes_reduce<G, OpMax, false>(qmax, 0.0f, OpMax(), red_f);
    const float mu = sqrtf(qmax);
    if (mu > sigma) {  // new running scale: rescale the partial sums (online max)
      const float c = sigma / mu;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);  // (c^2)^(p/2 - 1), (c^2)^(p/2)
      S *= cp;
      const float cpm1 = cm1 * c;  // c^(p-1)
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        if constexpr (kUL) ub[e * TF + t] = cscale(ub[e * TF + t], cpm1);
        else U[e] = cscale(U[e], cpm1);
      });
      sigma = mu;
    }
    // a/sigma = x^(1/2), x = |r|^2 / sigma^2:  S += x^(p/2);  G~ = x^(p/2 - 1) r / sigma
    // v_rcp (1 ulp) suffices for the inverse scale: every partial sum and
    // gradient partial of the unit is taken relative to the same scale
    roi_scale<PHLOG, E>(R, sigma > 0.f ? __builtin_amdgcn_rcpf(sigma) : 0.f, phm1, S);
    if constexpr (WT) roi_weigh<P, TF, E>(R, t, N, a.orient, wrow);  // d(w|r|)^p / dr carries w^2
    if (grad) {
      op = OP_ADJ;
    } else if (++g < M) {
      start_pair();
    } else {
      break;
    }
  }

  // Unit results: statistics to the block's tables, the demodulated gradient
  // partial into this slot's LDS region (unscaled, with the unit scale sigma).
  S = fft_lanes_reduce<G>(S, 0.0f, OpAdd(), red_f);
  kauto = fft_lanes_max_key<G>(kauto, red_k);
  kcross = fft_lanes_max_key<G>(kcross, red_k);
  if (t == 0) {
    u_sig[uslot] = active ? sigma : 0.f;
    u_S[uslot] = active ? S : 0.f;
    u_ka[uslot] = active ? kauto : 0ull;
    u_kc[uslot] = active ? kcross : 0ull;
  }
  if (grad) {
    float2 ph[EH];
    phasor_row<EH, TF>(t, nu, invN, ph);
    fft_sync<G>();
    static_for<EH>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const int n = t + TF * e;
      if (n < N) buf[n] = active ? cmulc(R[e], ph[e]) : make_float2(0.f, 0.f);
    });
  }
  block_lds_sync();

  // Block combine: one statistics entry and one partial per block, both
  // relative to the block's largest unit scale (unit order fixed).
  float sb = 0.f;
  for (int j = 0; j < UPB; ++j) sb = fmaxf(sb, u_sig[j]);
  const float inv_b = sb > 0.f ? 1.0f / sb : 0.f;
  const int64_t ent = (int64_t)w * pl.wpr + grp;
  if (threadIdx.x == 0) {
    float Sb = 0.f;
    unsigned long long ka = 0, kc = 0;
    for (int j = 0; j < UPB; ++j) {
      const float c = u_sig[j] * inv_b;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);
      Sb += cp * u_S[j];
      ka = umax64(ka, u_ka[j]);
      kc = umax64(kc, u_kc[j]);
    }
    UnitStat st;
    st.sigma = sb;
    st.S = Sb;
    st.pad0 = st.pad1 = 0;
    st.key_auto = ka;
    st.key_cross = kc;
    a.ustat[pl.ws_unit + ent] = st;
  }
  if (grad) {
    float fac[UPB];
#pragma unroll
    for (int j = 0; j < UPB; ++j) {
      const float c = u_sig[j] * inv_b;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);
      fac[j] = cm1 * c;  // (sigma_j / sigma_block)^(p-1)
    }
    float2* up = a.upart + pl.ws_upart + ent * N;
    for (int n = threadIdx.x; n < N; n += 64 * kPassWaves) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < UPB; ++j) {
        const float2 v = lds[j * G::SPAN + n];
        acc.x += fac[j] * v.x;
        acc.y += fac[j] * v.y;
      }
      up[n] = acc;
    }
  }
}


template <int P, int PHLOG, bool WT>
__global__ __launch_bounds__(64 * pass_waves(P), WT ? 1 : pass_min_waves(P)) void k_pass(PassArgs a) {
  constexpr int BW = pass_waves(P);
  __shared__ __align__(16) unsigned char smem[sizeof(PassSmem<P, BW>)];
  pass_block<P, PHLOG, WT, BW>(a, blockIdx.x, *reinterpret_cast<PassSmem<P, BW>*>(smem));
}

// The throughput pass of several FFT-length groups (P = 128 .. 2048) of an
// uneven batch in one launch. Every group's block has four waves (two units
// of two waves at P = 1024) and about 50 KB of LDS, so one block shape and
// one LDS region serve them all. The
// segments are ordered longest first (by FFT length): the dispatcher hands
// out blocks in index order to whichever compute unit has room, which makes
// the grid a work queue served longest-job-first, and the short blocks of
// the small FFT lengths fill the tail the long ones leave.
constexpr int kMultiMax = 5;
struct MultiArgs {
  PassArgs a;
  int32_t nseg;
  int32_t logp[kMultiMax];      // FFT length (log2) of each segment, decreasing
  int32_t base[kMultiMax + 1];  // first block of each segment; base[nseg] = grid size
  const int32_t* gprob[kMultiMax];
  const int32_t* gwave[kMultiMax];
  int32_t gn[kMultiMax];
};

template <int... Ps>
constexpr size_t max_pass_smem() {
  size_t m = 0;
  ((m = sizeof(PassSmem<Ps, 4>) > m ? sizeof(PassSmem<Ps, 4>) : m), ...);
  return m;
}
constexpr size_t kMultiSmem = max_pass_smem<128, 256, 512, 1024, 2048>();

template <int PHLOG, bool WT>
__global__ __launch_bounds__(256, WT ? 2 : 3) void k_pass_multi(MultiArgs m) {
  __shared__ __align__(16) unsigned char smem[kMultiSmem];
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < m.nseg && b >= m.base[i + 1]) ++i;
  PassArgs a = m.a;
  a.gprob = m.gprob[i];
  a.gwave = m.gwave[i];
  a.gn = m.gn[i];
  if (i != 0) a.bump = nullptr;  // block 0 of the first segment advances the step counter
  const int lb = b - m.base[i];
  switch (m.logp[i]) {
    case 11: pass_block<2048, PHLOG, WT, 4>(a, lb, *reinterpret_cast<PassSmem<2048, 4>*>(smem)); break;
    case 10: pass_block<1024, PHLOG, WT, 4>(a, lb, *reinterpret_cast<PassSmem<1024, 4>*>(smem)); break;
    case 9: pass_block<512, PHLOG, WT, 4>(a, lb, *reinterpret_cast<PassSmem<512, 4>*>(smem)); break;
    case 8: pass_block<256, PHLOG, WT, 4>(a, lb, *reinterpret_cast<PassSmem<256, 4>*>(smem)); break;
    default: pass_block<128, PHLOG, WT, 4>(a, lb, *reinterpret_cast<PassSmem<128, 4>*>(smem)); break;
  }
}

// ------------------------------------------------------------------ k_final

// x^p and x^(p-1) for 0 <= x <= 1: exact repeated squaring when p/2 is a
// power of two (ph_log >= 0), exp2 / log2 otherwise.
__device__ __forceinline__ float pow_p(float x, const ProbPlan& pl) {
  if (pl.ph_log >= 0) {
    float y = x * x;
    for (int i = 0; i < pl.ph_log; ++i) y *= y;
    return y;
  }
  return x > 0.f ? exp2f(pl.p * log2f(x)) : 0.f;
}
__device__ __forceinline__ float pow_pm1(float x, const ProbPlan& pl) {
  if (pl.ph_log >= 0) {
    float a = 1.0f, s = x * x;  // a = x^(p-2) after the loop
    for (int i = 0; i < pl.ph_log; ++i) {
      a *= s;
      s *= s;
    }
    return a * x;
  }
  return x > 0.f ? exp2f((pl.p - 1.0f) * log2f(x)) : 0.f;
}

enum FinMode : int32_t {
  FIN_STATS = 0,   // statistics only (the first row of each problem works)
  FIN_GRAD = 1,    // statistics and gradient outputs (scaled by grad_loss)
  FIN_STEP_A = 2,  // Adam on the filters, then the energy projection
  FIN_STEP_B = 3,  // chain rule to the logits, Adam on the logits
};

// What k_final prepares for the pass that follows it.
enum NextPrep : int32_t {
  NEXT_NONE = 0,
  NEXT_B_FULL = 1,  // after a filter update: soft waveform, filter spectrum, mainlobe products
  NEXT_A_SNRL = 2,  // after a filter update, another filter step: mainlobe products only
  NEXT_A_FULL = 3,  // after a logit update: hard waveform, its spectrum, mainlobe products
  NEXT_B_SOFT = 4,  // after a logit update, another logit step: soft waveform, mainlobe products
};

struct FinArgs {
  const ProbPlan* plans;
  const int32_t* rows;      // batch rows of this launch, one block each
  const int32_t* row_prob;  // problem of every batch row
  int32_t nrows_total;      // rows of the whole batch (blocks of all launches of one step)
  int32_t orient;
  int32_t mode;
  int32_t inner;            // index of the inner step (Adam step count t * n + inner + 1)
  int32_t count_step;       // this launch ends the outer iteration: advance *counter
  int32_t wave_mode;        // SOFT / HARD / GIVEN for the logit chain of FIN_GRAD
  int32_t next;             // NextPrep
  int32_t next_t_offset;    // temperature of NEXT_B_SOFT at step t + offset
  const float2* self_w;
  const float2* part_w;
  const UnitStat* ustat;
  const float2* upart;
  const float4* snrl;       // mainlobe inner products of the pass just run
  float4* snrl_next;        // ... of the prepared pass
  sqngd_stats* stats;
  const float* grad_loss;
  float2* grad_w;
  float* grad_z;
  float* z;     // logits: read for the chain, updated by FIN_STEP_B
  float2* h;    // filters updated by FIN_STEP_A
  float* adam;
  float2* wself;  // prepared soft waveforms
  float2* wpart;  // prepared hard waveforms
  float2* spec;   // prepared partner spectra
  int32_t* counter;
  int32_t* done;
  sqngd_opt opt;
  float2* gbuf;         // gradient rows (k_grad -> k_step)
  const float2* grad_in;  // k_final: gradient rows already reduced by k_grad (skips the partial sums)
  int32_t* pflag;       // per problem: the loss is not finite (k_grad -> k_step)
  const int32_t* frozen;  // per problem, optimiser steps: nonzero keeps the parameters (stopped design), or null
  int32_t grad_chunks;  // k_grad blocks per row
  int32_t grad_nprob;   // problems of the launch (one statistics block each)
  const int32_t* gprob; // their ids
  int32_t split;        // k_step2 blocks per row
  int32_t* rowcnt;      // k_step2: per row of the launch, blocks done (zero between launches)
  float4* rowpart;      // k_step2: per row of the launch, kStep2MaxSplit partial products
  int32_t single;  // one problem: its plan is `one`, rows are the block indices
  ProbPlan one;
};

constexpr int kFinThreads = 1024;
constexpr int kFinWaves = kFinThreads / 64;

__device__ __forceinline__ float block_max(float v, float* sh) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < kFinWaves; ++i) r = fmaxf(r, sh[i]);
  return r;
}
__device__ __forceinline__ float block_sum(float v, float* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < kFinWaves; ++i) r += sh[i];
  return r;
}
__device__ __forceinline__ unsigned long long block_max_key(unsigned long long v, unsigned long long* sh) {
  v = slot_max_key<64>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long r = sh[0];
  for (int i = 1; i < kFinWaves; ++i) r = umax64(r, sh[i]);
  return r;
}

// dL/dz of one chip from the packed waveform gradient g by the chain rule
// through the soft quantiser at temperature T; fn(l, dL/dz_l) is called in
// order l = 0 .. L-1 after the softmax statistics have been read.
template <class Fn>
__device__ __forceinline__ void logit_chain(const float* zc, int L, float T, int mode, float2 s, float2 g,
                                            Fn&& fn) {
  float zm = zc[0];
  for (int l = 1; l < L; ++l) zm = fmaxf(zm, zc[l]);
  const float invT = 1.0f / T;
  float sum = 0.f, ybar = 0.f;
  for (int l = 0; l < L; ++l) {
    const float e = expf((zc[l] - zm) * invT);
    sum += e;
    ybar += (float)l * e;
  }
  const float inv = 1.0f / sum;
  ybar *= inv;
  if (mode == SQNGD_SQ_PHASE_MEAN) {
    const float dphi = g.y * s.x - g.x * s.y;  // Im(g conj(s)) = dL/dphi
    const float c = dphi * 2.0f * 3.14159265358979f / (float)L * invT;
    for (int l = 0; l < L; ++l) fn(l, c * expf((zc[l] - zm) * invT) * inv * ((float)l - ybar));
  } else {
    for (int l = 0; l < L; ++l) {
      const float2 ul = level_phasor(l, L);
      fn(l, expf((zc[l] - zm) * invT) * inv * invT * (g.x * (ul.x - s.x) + g.y * (ul.y - s.y)));
    }
  }
}

// Spectrum of one row (value v of chip n; threads n >= N pass zero) in the
// spectral layout of the fused pass, computed by wave 0 of the block; fbuf
// holds the staged row and then serves as that wave's exchange buffer.
template <int P, int CH>
__device__ __forceinline__ void row_spectrum(const float2 (&v)[CH], int N, float2* fbuf, float2* out,
                                             const ProbPlan& pl) {
  using G = Geom<P>;
  constexpr int E = G::E, TF = G::TF;
  const int tid = threadIdx.x;
  for (int i = tid; i < P; i += kFinThreads) fbuf[i] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int c = 0; c < CH; ++c)
    if (tid + c * kFinThreads < N) fbuf[tid + c * kFinThreads] = v[c];
  __syncthreads();
  if (tid < 64) {
    const int slot = tid / TF, t = tid % TF;
    float2 X[E];
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      X[e] = slot == 0 ? fbuf[t + TF * e] : make_float2(0.f, 0.f);
    });
    WaveTwiddles<P> W;
    W.init(t);
    fft_forward<P>(X, fbuf + slot * G::SPAN, t, W);
    if (slot == 0) {
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        out[spec_slot<P>(pl, t, e)] = X[e];
      });
    }
  }
}

// Mainlobe inner product c' = sum_n conj(part(n)) self(n) and the two
// energies (eq. 10, 38) of one row (CH chips per thread), written by thread 0
// (one LDS round).
template <int CH>
__device__ __forceinline__ void row_snrl(const float2 (&self)[CH], const float2 (&part)[CH], float* sh, float4* out) {
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < CH; ++c) {
    v[0] += part[c].x * self[c].x + part[c].y * self[c].y;
    v[1] += part[c].x * self[c].y - part[c].y * self[c].x;
    v[2] += self[c].x * self[c].x + self[c].y * self[c].y;
    v[3] += part[c].x * part[c].x + part[c].y * part[c].y;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 4; ++i) sh[i * kFinWaves + (threadIdx.x >> 6)] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    float r[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 4; ++i)
      for (int w = 0; w < kFinWaves; ++w) r[i] += sh[i * kFinWaves + w];
    *out = make_float4(r[0], r[1], r[2], r[3]);
  }
}

// Segmented reductions over aligned groups of LP lanes (LP a power of two <= 64).
__device__ __forceinline__ float seg_max(float v, int LP) {
  for (int off = LP >> 1; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ float seg_sum(float v, int LP) {
  for (int off = LP >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
// largest value and its lowest index
__device__ __forceinline__ void seg_argmax(float& v, int& idx, int LP) {
  for (int off = LP >> 1; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}


// Statistics record of one problem (eq. 8-10, 48): loss terms, the auto and
// cross PSL with the cell that holds the peak, the PSLR and the SNRL of the
// worst waveform, from the reduced maximum keys and the mainlobe products of
// the problem's M rows.
__device__ __forceinline__ void stats_record(sqngd_stats* out, const ProbPlan& pl, int orient, float loss,
                                          float lp_raw, float l_snrl, unsigned long long ka,
                                          unsigned long long kc, const float4* snrl_rows, bool bad) {
  const int M = pl.M, N = pl.N, F = pl.F, Pl = pl.P;
  float snrl_max = -INFINITY, p_min = INFINITY;
  for (int k = 0; k < M; ++k) {
    const float4 c4 = snrl_rows[k];
    const float mag = sqrtf(c4.x * c4.x + c4.y * c4.y);
    snrl_max = fmaxf(snrl_max, 10.0f * log10f(c4.z * c4.w / (mag * mag)));
    p_min = fminf(p_min, mag / (float)N);
  }
  sqngd_stats& st = *out;
  st.loss = loss;
  st.lp = lp_raw * pl.inv_NP;
  st.l_snrl = l_snrl;
  const float invP = 1.0f / (float)Pl;
  st.psl_auto = sqrtf(key_q(ka)) * invP;
  st.psl_cross = sqrtf(key_q(kc)) * invP;
  st.pslr_db = 20.0f * log10f(fmaxf(st.psl_auto, st.psl_cross) / (float)N);
  st.snrl_db_max = snrl_max;
  st.p_min = p_min;
  const unsigned long long kb = key_q(ka) >= key_q(kc) ? ka : kc;
  const uint32_t cell = key_cell(kb);
  const int kk = (int)(cell % (uint32_t)Pl);
  const uint32_t rest = cell / (uint32_t)Pl;
  const int gg = (int)(rest % (uint32_t)M);
  const int uu = (int)(rest / (uint32_t)M);
  const int ww = uu / F, ff = uu % F;
  const int tp = kk <= N - 1 ? -kk : Pl - kk;
  st.arg_m = orient == 0 ? ww : gg;
  st.arg_l = orient == 0 ? gg : ww;
  st.arg_tau = orient == 0 ? tp : -tp;
  st.arg_f = ff;
  st.nonfinite = bad ? 1u : 0u;
  st.reserved[0] = st.reserved[1] = st.reserved[2] = 0;
}

// One block per row of the batch. The block
//  1. issues every load that does not wait for a reduction;
//  2. reduces the problem's unit statistics to L_p (every row of a problem
//     does the same, in the same order) and the SNRL penalty;
//  3. sums the row's per-block gradient partials over the Doppler bins (in
//     bin order within each of FS interleaved splits, then over the splits);
//  4. applies the filter update (one thread per chip), or writes the gradient;
//  5. runs the logit side one thread per (chip, level): the chain rule through
//     the soft quantiser, the logit update and the quantisation that prepares
//     the next pass, with per-chip softmax statistics from lane shuffles;
//  6. forms the next pass's mainlobe products and partner spectrum;
//  7. writes the statistics record.
// CH chips per thread: two at P = 4096 (N up to 2048), where the gradient
// rows always come reduced from k_grad (grad_in).
template <int P>
__global__ __launch_bounds__(kFinThreads) void k_final(FinArgs a) {
  constexpr int CH = P >= 4096 ? 2 : 1;
  __shared__ float shf[kFinWaves * 4];
  __shared__ unsigned long long shk[kFinWaves * 2];
  __shared__ float fac[4096];
  __shared__ float2 part[kFinThreads];
  __shared__ float2 gsh[CH * kFinThreads];  // row gradient of each chip
  __shared__ float2 nsh[CH * kFinThreads];  // quantised waveform of each chip for the next pass
  __shared__ float4 snrl_sh[16];
  __shared__ float2 fbuf[Geom<P>::LDS];
  const int tid = threadIdx.x;
  int r, pid;
  ProbPlan pl;
  if (a.single) {
    r = blockIdx.x;
    pid = 0;
    pl = a.one;
  } else {
    r = a.rows[blockIdx.x];
    pid = a.row_prob[r];
    pl = a.plans[pid];
  }
  const int M = pl.M, N = pl.N, F = pl.F, L = pl.L;
  const int m = r - pl.row0;
  if (a.mode == FIN_STATS && m != 0) return;
  const UnitStat* us = a.ustat + pl.ws_unit;
  const float p = pl.p;
  const int n = tid;  // chip of slot c: n + c * kFinThreads
  const bool on = n < N;
  const bool upd = a.mode != FIN_STATS;
  const int64_t wrow = pl.off_w + (int64_t)m * N;
  const int64_t crow = (int64_t)m * N;
  const int NE = pl.wpr;  // statistics entries / partials per row (one per fused-pass block)
  const bool chain_out = a.mode == FIN_GRAD && a.grad_z != nullptr && a.orient == 0;
  const bool zstep = a.mode == FIN_STEP_B;
  const bool next_soft = a.next == NEXT_B_FULL || a.next == NEXT_B_SOFT;
  const bool next_hard = a.next == NEXT_A_FULL;
  const bool elem = chain_out || zstep || next_soft || next_hard;
  int LP = 1, lg = 0;
  while (LP < L) {
    LP <<= 1;
    ++lg;
  }

  // ---- 1. loads
  float2 pw = make_float2(0.f, 0.f), hv[CH];
  float4 mvh[CH];
  float* mh = a.adam + pl.off_state + 2 * (int64_t)M * N * L + 2 * crow;
  float* vh = mh + 2 * (int64_t)M * N;
  if (upd && on) pw = a.part_w[wrow + n];
  for (int c = 0; c < CH; ++c) {
    const int nc = n + c * kFinThreads;
    hv[c] = make_float2(0.f, 0.f);
    mvh[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (upd && nc < N) {
      if (a.mode == FIN_STEP_A || a.mode == FIN_STEP_B) hv[c] = a.h[wrow + nc];
      if (a.mode == FIN_STEP_A) {
        const float2 m2 = *(const float2*)(mh + 2 * nc), v2 = *(const float2*)(vh + 2 * nc);
        mvh[c] = make_float4(m2.x, m2.y, v2.x, v2.y);
      }
    }
  }
  const float fsig = upd && tid < NE ? us[m * NE + tid].sigma : 0.f;
  const float4 sn = tid < M ? a.snrl[pl.row0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
  const int tstep = (a.mode == FIN_STEP_A || a.mode == FIN_STEP_B) ? *a.counter : 0;
  constexpr int kBatch = 8;
  const int Nc = (N + 63) & ~63;
  const int FS = kFinThreads / Nc;
  const int nn = tid % Nc, fsi = tid / Nc;
  const bool red = upd && fsi < FS && nn < N && a.grad_in == nullptr;
  const float2* up = a.upart + pl.ws_upart + (int64_t)m * NE * N + nn;
  float2 v[kBatch];
#pragma unroll
  for (int j = 0; j < kBatch; ++j) {
    const int ff = fsi + j * FS;
    v[j] = red && ff < NE ? up[(int64_t)ff * N] : make_float2(0.f, 0.f);
  }
  // this thread's first logit element (chip i >> lg, level i & (LP-1))
  float zv0 = 0.f, m0 = 0.f, v0 = 0.f;
  float2 s0 = make_float2(0.f, 0.f);
  {
    const int en = tid >> lg, el = tid & (LP - 1);
    if (elem && en < N && el < L) {
      zv0 = a.z[pl.off_z + (crow + en) * L + el];
      if (zstep) {
        m0 = a.adam[pl.off_state + (crow + en) * L + el];
        v0 = a.adam[pl.off_state + (int64_t)M * N * L + (crow + en) * L + el];
      }
      if (zstep || chain_out) s0 = a.self_w[wrow + en];
    }
  }
  // online (max, rescaled sum) of this thread's unit statistics
  float mx = 0.f, sx = 0.f;
  unsigned long long ka = 0, kc = 0;
  for (int i = tid; i < pl.units; i += kFinThreads) {
    const UnitStat u = us[i];
    ka = umax64(ka, u.key_auto);
    kc = umax64(kc, u.key_cross);
    if (u.sigma > mx) {
      sx = (mx > 0.f ? sx * pow_p(mx / u.sigma, pl) : 0.f) + u.S;
      mx = u.sigma;
    } else if (u.sigma > 0.f) {
      sx += u.S * pow_p(u.sigma / mx, pl);
    }
  }
  if (tid < NE) fac[tid] = fsig;
  for (int j = tid + kFinThreads; upd && j < NE; j += kFinThreads) fac[j] = us[m * NE + j].sigma;
  if (tid < M) snrl_sh[tid] = sn;

  // ---- 2. L_p and the SNRL penalty
  {
    const float wm = wave_max(mx);
    float s = mx > 0.f ? sx * pow_p(mx / wm, pl) : 0.f;
    s = wave_sum(s);
    ka = slot_max_key<64>(ka);
    kc = slot_max_key<64>(kc);
    if ((tid & 63) == 0) {
      shf[tid >> 6] = wm;
      shf[kFinWaves + (tid >> 6)] = s;
      shk[tid >> 6] = ka;
      shk[kFinWaves + (tid >> 6)] = kc;
    }
  }
  __syncthreads();
  float smax = 0.f;
  for (int w = 0; w < kFinWaves; ++w) {
    smax = fmaxf(smax, shf[w]);
    ka = umax64(ka, shk[w]);
    kc = umax64(kc, shk[kFinWaves + w]);
  }
  float acc = 0.f;
  for (int w = 0; w < kFinWaves; ++w)
    if (shf[w] > 0.f) acc += shf[kFinWaves + w] * pow_p(shf[w] / smax, pl);
  const float lp_raw = smax > 0.f ? smax * powf(acc, 1.0f / p) : 0.f;
  float l_snrl = 0.f;
  for (int k = 0; k < M; ++k) {
    const float4 c4 = snrl_sh[k];
    const float pk = sqrtf(c4.x * c4.x + c4.y * c4.y) / (float)N;
    l_snrl += (pk - pl.p_tar) * (pk - pl.p_tar) / (float)M;
  }
  const float loss = pl.w_psl * lp_raw * pl.inv_NP + pl.w_snrl * l_snrl;
  const bool bad = !isfinite(loss);

  float2 g[CH];
  for (int c = 0; c < CH; ++c) g[c] = make_float2(0.f, 0.f);
  bool skip = true;
  if (upd) {
    // ---- 3. row gradient: sum_f (w_psl/(N P)) (sigma_u/lp_raw)^(p-1) partial_u + G'_S part_m
    // (or the rows k_grad reduced already, SNRL term included)
    if (a.grad_in != nullptr) {
      const float gl = a.grad_loss ? a.grad_loss[pid] : 1.0f;
      for (int c = 0; c < CH; ++c) {
        const int nc = n + c * kFinThreads;
        if (nc < N) {
          g[c] = cscale(a.grad_in[wrow + nc], gl);
          gsh[nc] = g[c];
        }
      }
    } else {
    for (int j = tid; j < NE; j += kFinThreads)
      fac[j] = lp_raw > 0.f ? pl.w_psl / ((float)N * (float)pl.P) * pow_pm1(fac[j] / lp_raw, pl) : 0.f;
    __syncthreads();
    {
      float2 gp = make_float2(0.f, 0.f);
      if (red) {
        for (int f0 = fsi;; f0 += kBatch * FS) {
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const int ff = f0 + j * FS;
            const float c = ff < NE ? fac[ff] : 0.f;
            gp.x += c * v[j].x;
            gp.y += c * v[j].y;
          }
          const int f1 = f0 + kBatch * FS;
          if (f1 >= NE) break;
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const int ff = f1 + j * FS;
            v[j] = ff < NE ? up[(int64_t)ff * N] : make_float2(0.f, 0.f);
          }
        }
      }
      part[tid] = gp;
    }
    __syncthreads();
    const float gl = a.grad_loss ? a.grad_loss[pid] : 1.0f;
    const float4 cm = snrl_sh[m];
    const float magm = sqrtf(cm.x * cm.x + cm.y * cm.y);
    float2 gS = make_float2(0.f, 0.f);
    if (magm > 0.f)
      gS = cscale(make_float2(cm.x, cm.y),
                  pl.w_snrl * (2.0f / (float)M) * (magm / (float)N - pl.p_tar) / ((float)N * magm));
    if (on) {
      for (int s = 0; s < FS; ++s) g[0] = cadd(g[0], part[s * Nc + n]);
      g[0] = cscale(cadd(g[0], cmul(gS, pw)), gl);
      gsh[n] = g[0];
    }
    }
    bool chipbad = false;
    for (int c = 0; c < CH; ++c)
      chipbad |= n + c * kFinThreads < N && (!isfinite(g[c].x) || !isfinite(g[c].y));
    const int rowbad = __syncthreads_or(chipbad);
    skip = bad || rowbad || (a.frozen != nullptr && a.frozen[pid] != 0);

    // ---- 4. per chip
    for (int c = 0; c < CH; ++c)
      if (a.mode == FIN_GRAD && n + c * kFinThreads < N && a.grad_w) a.grad_w[wrow + n + c * kFinThreads] = g[c];
    if (a.mode == FIN_STEP_A) {
      // Adam on (Re h, Im h), then h <- h sqrt(N / |h|^2) (eq. 32)
      const int k = tstep * a.opt.n_h + a.inner + 1;
      const float b1 = a.opt.beta1, b2 = a.opt.beta2;
      const float bc1 = 1.0f - powf(b1, (float)k), bc2 = 1.0f - powf(b2, (float)k);
      float esum = 0.f;
      for (int c = 0; c < CH; ++c) {
        const int nc = n + c * kFinThreads;
        if (nc < N && !skip) {
          if (a.opt.flags & SQNGD_OPT_SGD) {
            hv[c].x -= a.opt.lr_h * g[c].x;
            hv[c].y -= a.opt.lr_h * g[c].y;
          } else {
            const float mx2 = b1 * mvh[c].x + (1.0f - b1) * g[c].x, my2 = b1 * mvh[c].y + (1.0f - b1) * g[c].y;
            const float vx = b2 * mvh[c].z + (1.0f - b2) * g[c].x * g[c].x;
            const float vy = b2 * mvh[c].w + (1.0f - b2) * g[c].y * g[c].y;
            *(float2*)(mh + 2 * nc) = make_float2(mx2, my2);
            *(float2*)(vh + 2 * nc) = make_float2(vx, vy);
            hv[c].x -= a.opt.lr_h * (mx2 / bc1) / (sqrtf(vx / bc2) + a.opt.eps);
            hv[c].y -= a.opt.lr_h * (my2 / bc1) / (sqrtf(vy / bc2) + a.opt.eps);
          }
        }
        esum += hv[c].x * hv[c].x + hv[c].y * hv[c].y;
      }
      const float e2 = block_sum(esum, shf);
      for (int c = 0; c < CH; ++c) {
        hv[c] = cscale(hv[c], skip ? 1.0f : sqrtf((float)N / e2));
        if (n + c * kFinThreads < N) a.h[wrow + n + c * kFinThreads] = hv[c];
      }
    }

    // ---- 5. logit side, one thread per (chip, level)
    if (elem) {
      const bool zupd = zstep && !skip;
      const int kz = tstep * a.opt.n_x + a.inner + 1;
      const float b1 = a.opt.beta1, b2 = a.opt.beta2;
      const float bc1 = zupd ? 1.0f - powf(b1, (float)kz) : 1.0f;
      const float bc2 = zupd ? 1.0f - powf(b2, (float)kz) : 1.0f;
      const float Tc = zstep ? temperature_at(a.opt, tstep) : pl.temperature;
      const float Tn = temperature_at(a.opt, tstep + (a.next == NEXT_B_SOFT ? a.next_t_offset : 0));
      const bool soft_grad = chain_out ? a.wave_mode == SQNGD_WAVE_SOFT : zupd;
      const float tw = 2.0f * 3.14159265358979f / (float)L;
      // the next round's loads are issued before this round's arithmetic
      // (a round's elements are disjoint from every other round's, and each
      // is written only by the thread that reads it)
      float zq = zv0, mq = m0, vq = v0;
      float2 sq0 = s0;
      for (int base = 0; base < N * LP; base += kFinThreads) {
        const int i = base + tid, en = i >> lg, el = i & (LP - 1);
        const bool ok = en < N && el < L;
        float zv = zq, mm = mq, vv = vq;
        float2 s = sq0;
        const int64_t zi = pl.off_z + (crow + en) * L + el;
        {
          const int i2 = i + kFinThreads, en2 = i2 >> lg, el2 = i2 & (LP - 1);
          if (en2 < N && el2 < L) {
            zq = a.z[pl.off_z + (crow + en2) * L + el2];
            if (zstep) {
              mq = a.adam[pl.off_state + (crow + en2) * L + el2];
              vq = a.adam[pl.off_state + (int64_t)M * N * L + (crow + en2) * L + el2];
            }
            if (zstep || chain_out) sq0 = a.self_w[wrow + en2];
          }
        }
        if (chain_out || zupd) {
          // dL/dz through the soft quantiser at Tc (chip softmax from the L lanes)
          const float zm = seg_max(ok ? zv : -INFINITY, LP);
          const float e = ok ? expf((zv - zm) / Tc) : 0.f;
          const float sum = seg_sum(e, LP);
          const float yb = seg_sum((float)el * e, LP) / sum;
          const float2 gc = ok ? gsh[en] : make_float2(0.f, 0.f);
          const float pi = e / sum;
          float gv;
          if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
            gv = (gc.y * s.x - gc.x * s.y) * tw / Tc * pi * ((float)el - yb);
          } else {
            const float2 ul = level_phasor(el, L);
            gv = pi / Tc * (gc.x * (ul.x - s.x) + gc.y * (ul.y - s.y));
          }
          if (!soft_grad) gv = 0.f;
          if (chain_out && ok) a.grad_z[zi] = gv;
          if (zupd && ok) {
            if (a.opt.flags & SQNGD_OPT_SGD) {
              zv -= a.opt.lr_z * gv;
            } else {
              mm = b1 * mm + (1.0f - b1) * gv;
              vv = b2 * vv + (1.0f - b2) * gv * gv;
              a.adam[pl.off_state + (crow + en) * L + el] = mm;
              a.adam[pl.off_state + (int64_t)M * N * L + (crow + en) * L + el] = vv;
              zv -= a.opt.lr_z * (mm / bc1) / (sqrtf(vv / bc2) + a.opt.eps);
            }
            a.z[zi] = zv;
          }
        }
        if (next_soft) {  // soft waveform of the next pass at Tn
          const float zm = seg_max(ok ? zv : -INFINITY, LP);
          const float e = ok ? expf((zv - zm) / Tn) : 0.f;
          const float sum = seg_sum(e, LP);
          float2 sq;
          if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
            const float yb = seg_sum((float)el * e, LP) / sum;
            float sn_, cs_;
            sincospif(2.0f * yb / (float)L, &sn_, &cs_);
            sq = make_float2(cs_, sn_);
          } else {
            const float2 ul = level_phasor(el, L);
            sq = make_float2(seg_sum(e * ul.x, LP) / sum, seg_sum(e * ul.y, LP) / sum);
          }
          if (el == 0 && en < N) nsh[en] = sq;
        } else if (next_hard) {  // hard waveform of the next pass
          float bv = ok ? zv : -INFINITY;
          int bi = el;
          seg_argmax(bv, bi, LP);
          if (el == 0 && en < N) nsh[en] = level_phasor(bi, L);
        }
      }
    }
  }

  // ---- 6. inputs of the next pass
  if (a.next != NEXT_NONE) {
    __syncthreads();
    float2 self[CH], prt[CH], sp[CH];
    for (int c = 0; c < CH; ++c) {
      const int nc = n + c * kFinThreads;
      const bool onc = nc < N;
      self[c] = prt[c] = sp[c] = hv[c];
      if (next_soft) {
        self[c] = onc ? nsh[nc] : make_float2(0.f, 0.f);
        if (onc) a.wself[wrow + nc] = self[c];
      } else if (next_hard) {
        prt[c] = onc ? nsh[nc] : make_float2(0.f, 0.f);
        sp[c] = prt[c];
        if (onc) a.wpart[wrow + nc] = prt[c];
      } else {  // NEXT_A_SNRL
        prt[c] = onc ? a.wpart[wrow + nc] : make_float2(0.f, 0.f);
      }
    }
    row_snrl<CH>(self, prt, shf, a.snrl_next + r);
    if constexpr (!spec_by_rowspec(P))
      if (a.next == NEXT_B_FULL || next_hard)
        row_spectrum<P, CH>(sp, N, fbuf, a.spec + pl.ws_spec + (int64_t)m * P, pl);
  }

  // ---- 7. statistics record
  if (m == 0 && tid == 0 && a.stats != nullptr)
    stats_record(a.stats + pid, pl, a.orient, loss, lp_raw, l_snrl, ka, kc, snrl_sh, bad);
  if (a.mode == FIN_STATS) return;

  if (a.count_step) {
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const int old = atomicAdd(a.done, 1);
      if (old == a.nrows_total - 1) {
        atomicExch(a.done, 0);
        atomicAdd(a.counter, 1);
      }
    }
  }
}

// ------------------------------------------------------------------ k_grad / k_step

// The finalize of an optimiser step (Algorithm 1; step A: filter update and
// projection, eq. 31-32; step B: chain rule through the soft quantiser and
// logit update) for problems with P <= 1024 runs as two latency-oriented
// kernels instead of k_final's one block per row:
//   k_grad  many blocks per row: every block reduces the problem's unit
//           statistics to L_p and the loss (all in the same order, so all
//           agree), then the gradient of its chips: the Doppler partials
//           scaled by (w_psl / (N P)) (sigma_u / L_p)^(p-1), 16 lanes per
//           chip, plus the SNRL term. The row's partials are read by many
//           compute units at once instead of one.
//   k_step  one block per row: the update, the next pass's waveform samples,
//           their energy and mainlobe sums, the partner spectrum. TPC
//           consecutive lanes own one chip (quad DPP between them), so the
//           chain rule's per-chip softmax, the Adam updates and the
//           quantisation stay in the chip's lanes; one block barrier for the
//           row sums. The projection scale of eq. 32 is known only after it,
//           so it is applied to the sums and, by linearity, to the spectrum
//           of the unscaled row. A non-finite loss or gradient (rare) is
//           handled after the barrier by redoing the next-pass inputs from
//           the unchanged state.

constexpr int kStepThreads = 512;  // below P = 2048
constexpr int kStepWaves = kStepThreads / 64;
// threads of a k_step block: 512, or 1024 at P = 2048 (one lane per chip)
__host__ __device__ constexpr int step_threads(int P) { return P >= 2048 ? 2 * kStepThreads : kStepThreads; }

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
// Sums / maxima over the TPC lanes of a chip (aligned groups of TPC lanes);
// every lane of the group gets the same value.
template <int TPC>
__device__ __forceinline__ float chip_sum(float v) {
  if constexpr (TPC >= 2) v += dpp_f<0xB1, 0xF>(0.f, v);  // quad_perm [1,0,3,2]
  if constexpr (TPC >= 4) v += dpp_f<0x4E, 0xF>(0.f, v);  // quad_perm [2,3,0,1]
  if constexpr (TPC >= 8) v += __shfl_xor(v, 4);
  return v;
}
template <int TPC>
__device__ __forceinline__ float chip_max(float v) {
  if constexpr (TPC >= 2) v = fmaxf(v, dpp_f<0xB1, 0xF>(0.f, v));
  if constexpr (TPC >= 4) v = fmaxf(v, dpp_f<0x4E, 0xF>(0.f, v));
  if constexpr (TPC >= 8) v = fmaxf(v, __shfl_xor(v, 4));
  return v;
}
// largest value, lowest level among equal values
__device__ __forceinline__ void argmax_merge(float& v, int& l, float ov, int ol) {
  if (ov > v || (ov == v && ol < l)) {
    v = ov;
    l = ol;
  }
}
template <int TPC>
__device__ __forceinline__ void chip_argmax(float& v, int& l) {
  if constexpr (TPC >= 2) argmax_merge(v, l, dpp_f<0xB1, 0xF>(0.f, v), dpp_i<0xB1>(l));
  if constexpr (TPC >= 4) argmax_merge(v, l, dpp_f<0x4E, 0xF>(0.f, v), dpp_i<0x4E>(l));
  if constexpr (TPC >= 8) argmax_merge(v, l, __shfl_xor(v, 4), __shfl_xor(l, 4));
}

// Next-pass waveform sample of one chip from its logits zc (levels
// sub + TPC k, invalid ones -inf): soft at temperature T or hard.
template <int TPC, int LVMAX>
__device__ __forceinline__ float2 chip_quantise(const float (&zc)[LVMAX], int sub, int L, bool hard, float T,
                                                int sq_mode) {
  if (hard) {
    float bv = -INFINITY;
    int bl = 0x7FFFFFFF;
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) argmax_merge(bv, bl, zc[k], sub + TPC * k);
    chip_argmax<TPC>(bv, bl);
    return level_phasor(bl < L ? bl : 0, L);
  }
  float zm = -INFINITY;
#pragma unroll
  for (int k = 0; k < LVMAX; ++k) zm = fmaxf(zm, zc[k]);
  zm = chip_max<TPC>(zm);
  const float invT = 1.0f / T;
  float se = 0.f, sy = 0.f, sc = 0.f, ss = 0.f;
#pragma unroll
  for (int k = 0; k < LVMAX; ++k) {
    const int l = sub + TPC * k;
    const float e = l < L ? expf((zc[k] - zm) * invT) : 0.f;
    se += e;
    if (sq_mode == SQNGD_SQ_PHASE_MEAN) {
      sy += (float)l * e;
    } else if (l < L) {
      const float2 u = level_phasor(l, L);
      sc += e * u.x;
      ss += e * u.y;
    }
  }
  se = chip_sum<TPC>(se);
  if (sq_mode == SQNGD_SQ_PHASE_MEAN) {
    sy = chip_sum<TPC>(sy);
    float sn, cs;
    sincospif(2.0f * (sy / se) / (float)L, &sn, &cs);
    return make_float2(cs, sn);
  }
  sc = chip_sum<TPC>(sc);
  ss = chip_sum<TPC>(ss);
  return make_float2(sc / se, ss / se);
}

constexpr int kGradThreads = 256;
constexpr int kGradWaves = kGradThreads / 64;
constexpr int kGradK = 8;                         // Doppler partials a lane loads per round
constexpr int kGradMaxNE = 4096;                  // partial rows per row: at most F (one per Doppler bin)
// k_grad row blocks per batch row of FFT length P (N <= P / 2 chips), LPC
// lanes per chip
__host__ __device__ constexpr int grad_chunks(int P, int LPC) {
  return P / 2 > kGradThreads / LPC ? P / 2 / (kGradThreads / LPC) : 1;
}

// Per problem of the launch, after the row blocks: one statistics block
// (L_p, maxima, loss, the record and the non-finite flag).
template <int NT>
__device__ __forceinline__ void grad_units(const ProbPlan& pl, const UnitStat* us, bool keys, float& mx, float& sx,
                                           unsigned long long& ka, unsigned long long& kc) {
  // four units per thread and round, loads first
  for (int i0 = threadIdx.x; i0 < pl.units; i0 += 4 * NT) {
    UnitStat u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + q * NT;
      if (i < pl.units) {
        u[q] = us[i];
      } else {
        u[q].sigma = 0.f;
        u[q].S = 0.f;
        u[q].key_auto = u[q].key_cross = 0ull;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (keys) {
        ka = umax64(ka, u[q].key_auto);
        kc = umax64(kc, u[q].key_cross);
      }
      if (u[q].sigma > mx) {
        sx = (mx > 0.f ? sx * pow_p(mx / u[q].sigma, pl) : 0.f) + u[q].S;
        mx = u[q].sigma;
      } else if (u[q].sigma > 0.f) {
        sx += u[q].S * pow_p(u[q].sigma / mx, pl);
      }
    }
  }
}

// Gradient rows from the fused pass's per-block partial rows (eq. 37-42 by
// the adjoint): LPC lanes per chip n sum the row's NE partials, lane `sub`
// of a chip taking j = sub, sub + LPC, ... , each weighted by
// (sigma_j / L_p)^(p-1) (one factor per partial, from LDS); the LPC lane sums
// are then added in a fixed butterfly order. A wave's lanes with the same sub
// read 64 / LPC consecutive chips of one partial row (whole cache lines).
// Large batches take one lane per chip (few, long rows of loads per lane);
// small ones 4 or 16, which shortens each lane's chain of dependent load
// rounds. One more block per problem writes the statistics.
template <int LPC>
__global__ __launch_bounds__(kGradThreads) void k_grad(FinArgs a) {
  constexpr int CPW = 64 / LPC;            // chips per wave
  constexpr int CPB = kGradThreads / LPC;  // chips per block
  __shared__ float shw[2 * kGradWaves];
  __shared__ unsigned long long shk[2 * kGradWaves];
  __shared__ float4 snrl_sh[16];
  __shared__ float fj_sh[kGradMaxNE];
  const int tid = threadIdx.x;
  const int nrb = gridDim.x - a.grad_nprob;  // row blocks
  const bool stat_block = (int)blockIdx.x >= nrb;
  int r = 0, pid, chunk = 0;
  ProbPlan pl;
  if (stat_block) {
    pid = a.single ? 0 : a.gprob[blockIdx.x - nrb];
    pl = a.single ? a.one : a.plans[pid];
  } else {
    const int rb = blockIdx.x / a.grad_chunks;
    chunk = blockIdx.x - rb * a.grad_chunks;
    if (a.single) {
      r = rb;
      pid = 0;
      pl = a.one;
    } else {
      r = a.rows[rb];
      pid = a.row_prob[r];
      pl = a.plans[pid];
    }
  }
  const int M = pl.M, N = pl.N, NE = pl.wpr;
  const int m = stat_block ? 0 : r - pl.row0;
  if (!stat_block && chunk * CPB >= N) return;  // whole block beyond the row
  const int lane = tid & 63, sub = lane / CPW;
  const int n = chunk * CPB + (tid >> 6) * CPW + lane % CPW;
  const bool on = !stat_block && n < N;
  const int64_t wrow = pl.off_w + (int64_t)m * N;

  // ---- loads: the first round of partials, then the statistics they wait on
  const UnitStat* us = a.ustat + pl.ws_unit;
  const float2* up = a.upart + pl.ws_upart + (int64_t)m * NE * N + (on ? n : 0);
  float2 v[kGradK];
#pragma unroll
  for (int k = 0; k < kGradK; ++k) {
    const int j = sub + LPC * k;
    v[k] = on && j < NE ? up[(int64_t)j * N] : make_float2(0.f, 0.f);
  }
  const float2 pw = on ? a.part_w[wrow + n] : make_float2(0.f, 0.f);
  if (tid < M) snrl_sh[tid] = a.snrl[pl.row0 + tid];
  float mx = 0.f, sx = 0.f;
  unsigned long long ka = 0, kc = 0;
  grad_units<kGradThreads>(pl, us, stat_block, mx, sx, ka, kc);

  // ---- L_p, the SNRL penalty and the loss (eq. 37-42)
  {
    const float wm = wave_max(mx);
    float s = mx > 0.f ? sx * pow_p(mx / wm, pl) : 0.f;
    s = wave_sum(s);
    if ((tid & 63) == 0) {
      shw[tid >> 6] = wm;
      shw[kGradWaves + (tid >> 6)] = s;
    }
    if (stat_block) {
      ka = slot_max_key<64>(ka);
      kc = slot_max_key<64>(kc);
      if ((tid & 63) == 0) {
        shk[tid >> 6] = ka;
        shk[kGradWaves + (tid >> 6)] = kc;
      }
    }
  }
  __syncthreads();
  float smax = 0.f;
  for (int w = 0; w < kGradWaves; ++w) smax = fmaxf(smax, shw[w]);
  float acc = 0.f;
  for (int w = 0; w < kGradWaves; ++w)
    if (shw[w] > 0.f) acc += shw[kGradWaves + w] * pow_p(shw[w] / smax, pl);
  const float lp_raw = smax > 0.f ? smax * exp2f(log2f(acc) / pl.p) : 0.f;
  if (stat_block) {
    if (tid == 0) {
      float l_snrl = 0.f;
      for (int k = 0; k < M; ++k) {
        const float4 c4 = snrl_sh[k];
        const float pk = sqrtf(c4.x * c4.x + c4.y * c4.y) / (float)N;
        l_snrl += (pk - pl.p_tar) * (pk - pl.p_tar) / (float)M;
      }
      const float loss = pl.w_psl * lp_raw * pl.inv_NP + pl.w_snrl * l_snrl;
      const bool bad = !isfinite(loss);
      for (int w = 0; w < kGradWaves; ++w) {
        ka = umax64(ka, shk[w]);
        kc = umax64(kc, shk[kGradWaves + w]);
      }
      if (a.stats != nullptr) stats_record(a.stats + pid, pl, a.orient, loss, lp_raw, l_snrl, ka, kc, snrl_sh, bad);
      a.pflag[pid] = bad ? 1 : 0;
    }
    return;
  }

  // ---- the partials' factors (sigma_j / L_p)^(p-1), once per row block
  const float cfac = pl.w_psl / ((float)N * (float)pl.P);
  const float inv_lp = lp_raw > 0.f ? 1.0f / lp_raw : 0.f;
  for (int j = tid; j < NE; j += kGradThreads)
    fj_sh[j] = lp_raw > 0.f ? cfac * pow_pm1(us[m * NE + j].sigma * inv_lp, pl) : 0.f;
  __syncthreads();

  // ---- gradient of the chip: each lane its partials in order, then the
  // chip's LPC lanes
  float2 g = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < kGradK; ++k) {
    const int j = sub + LPC * k;
    const float f = j < NE ? fj_sh[j] : 0.f;
    g.x += f * v[k].x;
    g.y += f * v[k].y;
  }
  for (int j0 = LPC * kGradK; j0 < NE; j0 += LPC * kGradK) {
#pragma unroll
    for (int k = 0; k < kGradK; ++k) {
      const int j = j0 + sub + LPC * k;
      v[k] = on && j < NE ? up[(int64_t)j * N] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < kGradK; ++k) {
      const int j = j0 + sub + LPC * k;
      const float f = j < NE ? fj_sh[j] : 0.f;
      g.x += f * v[k].x;
      g.y += f * v[k].y;
    }
  }
#pragma unroll
  for (int off = CPW; off < 64; off <<= 1) {
    g.x += __shfl_xor(g.x, off);
    g.y += __shfl_xor(g.y, off);
  }
  const float4 cm = snrl_sh[m];
  const float magm = sqrtf(cm.x * cm.x + cm.y * cm.y);
  if (magm > 0.f) {
    const float2 gS = cscale(make_float2(cm.x, cm.y),
                             pl.w_snrl * (2.0f / (float)M) * (magm / (float)N - pl.p_tar) / ((float)N * magm));
    g = cadd(g, cmul(gS, pw));
  }
  if (on && sub == 0) a.gbuf[wrow + n] = g;
}

// Lanes per chip in k_step, and the Doppler partials a lane loads per round
// when k_step reduces the gradient rows itself (FG).
__host__ __device__ constexpr int step_tpc(int P) { return P >= 256 ? 2 * step_threads(P) / P : 8; }
__host__ __device__ constexpr int step_fg_loads(int P) {
  return step_tpc(P) < 1 ? 0 : (48 / step_tpc(P) < 32 ? 48 / step_tpc(P) : 32);
}

// FG: the block also does k_grad's work for its row (the problem's L_p and
// loss from the unit statistics, in every block in the same order; the
// record by the problem's first row; the chip gradients from the Doppler
// partials, TPC lanes per chip), so one kernel ends the inner step. Used
// when a row's partials take at most two load rounds per lane.
template <int P, int MODE, int LVMAX, bool FG>
__global__ __launch_bounds__(step_threads(P)) void k_step(FinArgs a) {
  constexpr int NT = step_threads(P), NW = NT / 64;
  constexpr int TPC = step_tpc(P);  // lanes per chip: N <= P/2 chips fill the block
  constexpr bool kA = MODE == FIN_STEP_A;
  using G = Geom<P>;
  __shared__ float shr[2 * 5 * NW];
  __shared__ float2 rowbuf[P];
  __shared__ float2 fbuf[G::LDS];
  __shared__ float shw[FG ? 2 * NW : 1];
  __shared__ unsigned long long shk[FG ? 2 * NW : 1];
  __shared__ float4 snrl_sh[FG ? 16 : 1];
  const int tid = threadIdx.x;
  int r, pid;
  ProbPlan pl;
  if (a.single) {
    r = blockIdx.x;
    pid = 0;
    pl = a.one;
  } else {
    r = a.rows[blockIdx.x];
    pid = a.row_prob[r];
    pl = a.plans[pid];
  }
  const int M = pl.M, N = pl.N, L = pl.L;
  const int m = r - pl.row0;
  const int n = tid / TPC, sub = tid % TPC;
  const bool on = n < N, lead = on && sub == 0;
  const int64_t wrow = pl.off_w + (int64_t)m * N;
  const int64_t crow = (int64_t)m * N;
  const int next = a.next;
  const bool want_spec = next == NEXT_B_FULL || next == NEXT_A_FULL;
  const bool want_soft = next == NEXT_B_FULL || next == NEXT_B_SOFT;
  const bool need_z = !kA || want_soft;
  const bool sgd = (a.opt.flags & SQNGD_OPT_SGD) != 0;
  const float2 zero2 = make_float2(0.f, 0.f);

  // ---- loads
  const int tstep = *a.counter;
  constexpr int KL = FG ? step_fg_loads(P) : 1;
  const int NE = pl.wpr;
  const UnitStat* us = a.ustat + pl.ws_unit;
  const float2* up = a.upart + pl.ws_upart + (int64_t)m * NE * N + n;
  float sj[KL];
  float2 vj[KL];
  float2 pw = zero2;
  if constexpr (FG) {
    // first round of the chip's Doppler partials: lane sub takes sub + TPC k
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int j = sub + TPC * k;
      const bool ok = on && j < NE;
      sj[k] = ok ? us[m * NE + j].sigma : 0.f;
      vj[k] = ok ? up[(int64_t)j * N] : zero2;
    }
    pw = on ? a.part_w[wrow + n] : zero2;
    if (tid < M) snrl_sh[tid] = a.snrl[pl.row0 + tid];
  }
  float2 hv = zero2, sv = zero2, xv = zero2;
  float4 mvh = make_float4(0.f, 0.f, 0.f, 0.f);
  float* mh = a.adam + pl.off_state + 2 * (int64_t)M * N * L + 2 * crow;
  float* vh = mh + 2 * (int64_t)M * N;
  if (lead) {
    hv = a.h[wrow + n];
    if (kA && !sgd) {
      const float2 m2 = *(const float2*)(mh + 2 * n), v2 = *(const float2*)(vh + 2 * n);
      mvh = make_float4(m2.x, m2.y, v2.x, v2.y);
    }
    if (kA && next == NEXT_A_SNRL) xv = a.wpart[wrow + n];
  }
  if (!kA && on) sv = a.self_w[wrow + n];
  const int64_t zrow = pl.off_z + (crow + n) * L;
  float* amz = a.adam + pl.off_state + (crow + n) * L;
  float* avz = amz + (int64_t)M * N * L;
  float zl[LVMAX], mz[LVMAX], vz[LVMAX];
  // one lane per chip with L a multiple of 4 and aligned rows: the chip's
  // logits and moments move as 16-byte vectors (a quarter of the accesses,
  // each lane's 4 L bytes contiguous)
  const bool vec4 = TPC == 1 && LVMAX % 4 == 0 && (L & 3) == 0 && ((pl.off_z | pl.off_state) & 3) == 0 &&
                    (((uintptr_t)a.z | (uintptr_t)a.adam) & 15) == 0;
  if (vec4) {
#pragma unroll
    for (int k4 = 0; k4 < LVMAX / 4; ++k4) {
      const bool ok = on && 4 * k4 < L && need_z;
      const bool okm = ok && !kA && !sgd;
      const float4 z4 = ok ? *(const float4*)(a.z + zrow + 4 * k4)
                           : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
      const float4 m4 = okm ? *(const float4*)(amz + 4 * k4) : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 v4 = okm ? *(const float4*)(avz + 4 * k4) : make_float4(0.f, 0.f, 0.f, 0.f);
      zl[4 * k4] = z4.x, zl[4 * k4 + 1] = z4.y, zl[4 * k4 + 2] = z4.z, zl[4 * k4 + 3] = z4.w;
      mz[4 * k4] = m4.x, mz[4 * k4 + 1] = m4.y, mz[4 * k4 + 2] = m4.z, mz[4 * k4 + 3] = m4.w;
      vz[4 * k4] = v4.x, vz[4 * k4 + 1] = v4.y, vz[4 * k4 + 2] = v4.z, vz[4 * k4 + 3] = v4.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) {
      const int l = sub + TPC * k;
      const bool ok = on && l < L && need_z;
      zl[k] = ok ? a.z[zrow + l] : -INFINITY;
      mz[k] = ok && !kA && !sgd ? amz[l] : 0.f;
      vz[k] = ok && !kA && !sgd ? avz[l] : 0.f;
    }
  }
  if (want_spec)
    for (int i = N + tid; i < P; i += NT) rowbuf[i] = zero2;

  bool bad;
  float2 g;
  if constexpr (FG) {
    // ---- L_p, the SNRL penalty and the loss (eq. 37-42), as in k_grad
    float mx = 0.f, sx = 0.f;
    unsigned long long ka = 0, kc = 0;
    const bool keys = m == 0;
    grad_units<NT>(pl, us, keys, mx, sx, ka, kc);
    {
      const float wm = wave_max(mx);
      float sw = mx > 0.f ? sx * pow_p(mx / wm, pl) : 0.f;
      sw = wave_sum(sw);
      if ((tid & 63) == 0) {
        shw[tid >> 6] = wm;
        shw[NW + (tid >> 6)] = sw;
      }
      if (keys) {
        ka = slot_max_key<64>(ka);
        kc = slot_max_key<64>(kc);
        if ((tid & 63) == 0) {
          shk[tid >> 6] = ka;
          shk[NW + (tid >> 6)] = kc;
        }
      }
    }
    __syncthreads();
    float smax = 0.f;
    for (int w = 0; w < NW; ++w) smax = fmaxf(smax, shw[w]);
    float acc = 0.f;
    for (int w = 0; w < NW; ++w)
      if (shw[w] > 0.f) acc += shw[NW + w] * pow_p(shw[w] / smax, pl);
    const float lp_raw = smax > 0.f ? smax * exp2f(log2f(acc) / pl.p) : 0.f;
    float l_snrl = 0.f;
    for (int k = 0; k < M; ++k) {
      const float4 c4 = snrl_sh[k];
      const float pk = sqrtf(c4.x * c4.x + c4.y * c4.y) / (float)N;
      l_snrl += (pk - pl.p_tar) * (pk - pl.p_tar) / (float)M;
    }
    const float loss = pl.w_psl * lp_raw * pl.inv_NP + pl.w_snrl * l_snrl;
    bad = !isfinite(loss);
    if (keys && tid == 0 && a.stats != nullptr) {
      for (int w = 0; w < NW; ++w) {
        ka = umax64(ka, shk[w]);
        kc = umax64(kc, shk[NW + w]);
      }
      stats_record(a.stats + pid, pl, a.orient, loss, lp_raw, l_snrl, ka, kc, snrl_sh, bad);
    }
    // ---- gradient of the chip: Doppler partials scaled by
    // (w_psl / (N P)) (sigma_u / L_p)^(p-1), then the SNRL term
    g = zero2;
    if (lp_raw > 0.f) {
      const float cfac = pl.w_psl / ((float)N * (float)pl.P);
      const float inv_lp = 1.0f / lp_raw;
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const float f = cfac * pow_pm1(sj[k] * inv_lp, pl);
        g.x += f * vj[k].x;
        g.y += f * vj[k].y;
      }
      for (int j0 = TPC * KL; j0 < NE; j0 += TPC * KL) {
#pragma unroll
        for (int k = 0; k < KL; ++k) {
          const int j = j0 + sub + TPC * k;
          const bool ok = on && j < NE;
          sj[k] = ok ? us[m * NE + j].sigma : 0.f;
          vj[k] = ok ? up[(int64_t)j * N] : zero2;
        }
#pragma unroll
        for (int k = 0; k < KL; ++k) {
          const float f = cfac * pow_pm1(sj[k] * inv_lp, pl);
          g.x += f * vj[k].x;
          g.y += f * vj[k].y;
        }
      }
    }
    g.x = chip_sum<TPC>(g.x);
    g.y = chip_sum<TPC>(g.y);
    const float4 cm = snrl_sh[m];
    const float magm = sqrtf(cm.x * cm.x + cm.y * cm.y);
    if (magm > 0.f) {
      const float2 gS = cscale(make_float2(cm.x, cm.y),
                               pl.w_snrl * (2.0f / (float)M) * (magm / (float)N - pl.p_tar) / ((float)N * magm));
      g = cadd(g, cmul(gS, pw));
    }
    if (!on) g = zero2;
  } else {
    bad = a.pflag[pid] != 0;
    g = on ? a.gbuf[wrow + n] : zero2;
  }
  const float flag = lead && !(isfinite(g.x) && isfinite(g.y)) ? 1.0f : 0.0f;
  const float b1 = a.opt.beta1, b2 = a.opt.beta2;
  // a stopped design keeps its parameters: the step runs as a skipped one
  const bool hold = a.frozen != nullptr && a.frozen[pid] != 0;

  // ---- the update candidate and the next pass's waveform sample
  float2 hu = hv;   // step A: updated, unprojected filter chip (lead lanes)
  float2 nx = zero2;  // next pass: soft self sample or hard partner sample
  float4 mvn = mvh;
  if constexpr (kA) {
    if (lead && !bad && !hold) {
      if (sgd) {
        hu.x -= a.opt.lr_h * g.x;
        hu.y -= a.opt.lr_h * g.y;
      } else {
        const int k = tstep * a.opt.n_h + a.inner + 1;
        const float bc1 = bias_corr(b1, k), bc2 = bias_corr(b2, k);
        mvn.x = b1 * mvh.x + (1.0f - b1) * g.x;
        mvn.y = b1 * mvh.y + (1.0f - b1) * g.y;
        mvn.z = b2 * mvh.z + (1.0f - b2) * g.x * g.x;
        mvn.w = b2 * mvh.w + (1.0f - b2) * g.y * g.y;
        hu.x -= a.opt.lr_h * (mvn.x / bc1) / (sqrtf(mvn.z / bc2) + a.opt.eps);
        hu.y -= a.opt.lr_h * (mvn.y / bc1) / (sqrtf(mvn.w / bc2) + a.opt.eps);
      }
    }
    if (next == NEXT_B_FULL) nx = chip_quantise<TPC, LVMAX>(zl, sub, L, false, temperature_at(a.opt, tstep), pl.sq_mode);
  } else {
    // dL/dz through the soft quantiser at the temperature of this step, then Adam
    const float Tc = temperature_at(a.opt, tstep);
    const float invT = 1.0f / Tc;
    float zm = -INFINITY;
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) zm = fmaxf(zm, zl[k]);
    zm = chip_max<TPC>(zm);
    float e[LVMAX];
    float se = 0.f, sy = 0.f;
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) {
      const int l = sub + TPC * k;
      e[k] = on && l < L ? expf((zl[k] - zm) * invT) : 0.f;
      se += e[k];
      sy += (float)l * e[k];
    }
    se = chip_sum<TPC>(se);
    sy = chip_sum<TPC>(sy);
    const float yb = sy / se;
    const int kz = tstep * a.opt.n_x + a.inner + 1;
    const float bc1 = sgd ? 1.0f : bias_corr(b1, kz), bc2 = sgd ? 1.0f : bias_corr(b2, kz);
    const float dphi = (g.y * sv.x - g.x * sv.y) * (2.0f * 3.14159265358979f / (float)L) * invT;
    const bool upd = !bad && !hold;
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) {
      const int l = sub + TPC * k;
      if (!(on && l < L) || !upd) continue;
      const float pi = e[k] / se;
      float gv;
      if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
        gv = dphi * pi * ((float)l - yb);
      } else {
        const float2 ul = level_phasor(l, L);
        gv = pi * invT * (g.x * (ul.x - sv.x) + g.y * (ul.y - sv.y));
      }
      if (sgd) {
        e[k] = zl[k] - a.opt.lr_z * gv;
      } else {
        mz[k] = b1 * mz[k] + (1.0f - b1) * gv;
        vz[k] = b2 * vz[k] + (1.0f - b2) * gv * gv;
        e[k] = zl[k] - a.opt.lr_z * (mz[k] / bc1) / (sqrtf(vz[k] / bc2) + a.opt.eps);
      }
    }
    // e[] now holds the updated logits of the valid levels
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) {
      const int l = sub + TPC * k;
      if (!(on && l < L)) e[k] = -INFINITY;
      else if (!upd) e[k] = zl[k];
    }
    if (next == NEXT_A_FULL || next == NEXT_B_SOFT)
      nx = chip_quantise<TPC, LVMAX>(e, sub, L, next == NEXT_A_FULL,
                                     temperature_at(a.opt, tstep + (next == NEXT_B_SOFT ? a.next_t_offset : 0)),
                                     pl.sq_mode);
    // keep the updated logits in zl for the writes after the barrier; the
    // unchanged ones are reloaded if the step is skipped
#pragma unroll
    for (int k = 0; k < LVMAX; ++k) zl[k] = e[k];
  }

  // ---- energy and mainlobe products of the next pass (eq. 10, 32, 38),
  // summed over the row together with the count of non-finite gradient
  // chips: slots 0-1 Re, Im of sum conj(partner) self; 2 |self|^2;
  // 3 |partner|^2; 4 the count. In step A the filter chips are the
  // unprojected hcur, whose energy is slot 2 or 3 (slot 3 without a next pass).
  auto products = [&](float2 hcur, float2 nxt, float* sh, float4& prod, float& nbad) {
    float q[5] = {0.f, 0.f, 0.f, 0.f, flag};
    float2 self, part;
    if (kA) {
      self = next == NEXT_B_FULL ? nxt : hcur;
      part = next == NEXT_B_FULL ? hcur : (next == NEXT_A_SNRL ? xv : hcur);
    } else {
      self = next == NEXT_A_FULL ? hv : nxt;
      part = next == NEXT_A_FULL ? nxt : hv;
    }
    if (lead) {
      q[0] = part.x * self.x + part.y * self.y;
      q[1] = part.x * self.y - part.y * self.x;
      q[2] = self.x * self.x + self.y * self.y;
      q[3] = part.x * part.x + part.y * part.y;
    }
    block_sum5<NW>(q, sh);
    prod = make_float4(q[0], q[1], q[2], q[3]);
    nbad = q[4];
  };
  if (want_spec && lead) rowbuf[n] = kA ? hu : nx;
  float4 prod;
  float nbad;
  products(hu, nx, shr, prod, nbad);
  const bool skip = bad || hold || nbad > 0.f;
  float cs = 1.0f;  // scale of the prepared spectrum

  // ---- writes
  if (!skip) {
    if constexpr (kA) {
      const float e2 = next == NEXT_A_SNRL ? prod.z : prod.w;
      const float c = sqrtf((float)N / e2);
      if (lead) {
        if (!sgd) {
          *(float2*)(mh + 2 * n) = make_float2(mvn.x, mvn.y);
          *(float2*)(vh + 2 * n) = make_float2(mvn.z, mvn.w);
        }
        a.h[wrow + n] = cscale(hu, c);
      }
      if (next == NEXT_B_FULL) prod = make_float4(c * prod.x, c * prod.y, prod.z, c * c * prod.w);
      if (next == NEXT_A_SNRL) prod = make_float4(c * prod.x, c * prod.y, c * c * prod.z, prod.w);
      cs = c;
    } else if (vec4) {
#pragma unroll
      for (int k4 = 0; k4 < LVMAX / 4; ++k4) {
        if (on && 4 * k4 < L) {
          *(float4*)(a.z + zrow + 4 * k4) = make_float4(zl[4 * k4], zl[4 * k4 + 1], zl[4 * k4 + 2], zl[4 * k4 + 3]);
          if (!sgd) {
            *(float4*)(amz + 4 * k4) = make_float4(mz[4 * k4], mz[4 * k4 + 1], mz[4 * k4 + 2], mz[4 * k4 + 3]);
            *(float4*)(avz + 4 * k4) = make_float4(vz[4 * k4], vz[4 * k4 + 1], vz[4 * k4 + 2], vz[4 * k4 + 3]);
          }
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < LVMAX; ++k) {
        const int l = sub + TPC * k;
        if (on && l < L) {
          a.z[zrow + l] = zl[k];
          if (!sgd) {
            amz[l] = mz[k];
            avz[l] = vz[k];
          }
        }
      }
    }
  } else {
    // no update: the next pass is prepared from the unchanged state
    if constexpr (kA) {
      hu = hv;
    } else {
#pragma unroll
      for (int k = 0; k < LVMAX; ++k) {
        const int l = sub + TPC * k;
        zl[k] = on && l < L ? a.z[zrow + l] : -INFINITY;
      }
      if (next == NEXT_A_FULL || next == NEXT_B_SOFT)
        nx = chip_quantise<TPC, LVMAX>(zl, sub, L, next == NEXT_A_FULL,
                                       temperature_at(a.opt, tstep + (next == NEXT_B_SOFT ? a.next_t_offset : 0)),
                                       pl.sq_mode);
    }
    if (want_spec && lead) rowbuf[n] = kA ? hu : nx;
    products(hu, nx, shr + 5 * NW, prod, nbad);
  }
  if (lead) {
    if (next == NEXT_B_FULL || next == NEXT_B_SOFT) a.wself[wrow + n] = nx;
    if (next == NEXT_A_FULL) a.wpart[wrow + n] = nx;
  }
  if (tid == 0 && next != NEXT_NONE) a.snrl_next[r] = prod;

  // ---- spectrum of the next pass's partner row (wave 0; k_rowspec at P >= 2048)
  if constexpr (!spec_by_rowspec(P)) {
  if (want_spec && tid < 64) {
    constexpr int E = G::E, TF = G::TF;
    const int slot = tid / TF, t = tid % TF;
    float2 X[E];
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      X[e] = slot == 0 ? rowbuf[t + TF * e] : zero2;
    });
    WaveTwiddles<P> W;
    W.init(t);
    fft_forward<P>(X, fbuf + slot * G::SPAN, t, W);
    if (slot == 0) {
      float2* out = a.spec + pl.ws_spec + (int64_t)m * P;
      static_for<E>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        out[spec_slot<P>(pl, t, e)] = cscale(X[e], cs);
      });
    }
  }
  }

  if (a.count_step) {
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const int old = atomicAdd(a.done, 1);
      if (old == a.nrows_total - 1) {
        atomicExch(a.done, 0);
        atomicAdd(a.counter, 1);
      }
    }
  }
}

// ------------------------------------------------------------ k_step2

// k_step for FFT lengths 2048 and 4096 (up to 1024 / 2048 chips per row): a
// row is split over ceil(N / 256) blocks of 256 threads, one chip per thread,
// with the gradient rows from k_grad. Every block reads the whole row's
// gradient for the row's skip decision (a non-finite loss, a stopped design or
// a non-finite gradient chip), so each chip's new logits and moments are
// written as soon as they are formed. The row's products for the next pass
// (and in step A the filter's energy) are summed by the row's last block, or
// by k_step2_rows one launch later, from the blocks' partial sums in block
// order; in step A that block then projects the whole filter row (eq. 32),
// which the other blocks have written unprojected. Same arithmetic per chip
// as k_step with one lane per chip.
constexpr int kStep2Threads = 256;
constexpr int kStep2MaxSplit = 8;  // 2048 chips

// The end of a row's step, by one block of kStep2Threads once every block of
// the row has written its partial products: their sum in block order, the
// projection of the filter row (step A, eq. 32) and the next pass's mainlobe
// products.
template <bool kA>
__device__ __forceinline__ void step2_finish(const FinArgs& a, const float4* part, int nblk, bool skip, int r,
                                             int64_t wrow, int N) {
  constexpr int NT = kStep2Threads;
  const int next = a.next;
  float4 prod = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int j = 0; j < nblk; ++j) {
    const float4 pj = part[j];
    prod = make_float4(prod.x + pj.x, prod.y + pj.y, prod.z + pj.z, prod.w + pj.w);
  }
  if constexpr (kA) {
    // h <- h sqrt(N / |h|^2) over the row, and the products of the projected chips
    if (!skip) {
      const float e2 = next == NEXT_A_SNRL ? prod.z : prod.w;
      const float cn = sqrtf((float)N / e2);
      for (int j = threadIdx.x; j < N; j += NT) a.h[wrow + j] = cscale(a.h[wrow + j], cn);
      if (next == NEXT_B_FULL) prod = make_float4(cn * prod.x, cn * prod.y, prod.z, cn * cn * prod.w);
      if (next == NEXT_A_SNRL) prod = make_float4(cn * prod.x, cn * prod.y, cn * cn * prod.z, prod.w);
    }
  }
  if (threadIdx.x == 0 && next != NEXT_NONE) a.snrl_next[r] = prod;
  if (a.count_step) {
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const int old = atomicAdd(a.done, 1);
      if (old == a.nrows_total - 1) {
        atomicExch(a.done, 0);
        atomicAdd(a.counter, 1);
      }
    }
  }
}

// The row's skip decision over its whole gradient row (every thread of the
// block gets it), and this thread's chip's gradient when the chip is n.
__device__ __forceinline__ bool step2_skip(const FinArgs& a, int pid, int64_t wrow, int N, int n, float2& gc) {
  bool flag = false;
  for (int j = threadIdx.x; j < N; j += kStep2Threads) {
    const float2 gj = a.gbuf[wrow + j];
    flag |= !(isfinite(gj.x) && isfinite(gj.y));
    if (j == n) gc = gj;
  }
  const bool hold = a.frozen != nullptr && a.frozen[pid] != 0;
  return __syncthreads_or(flag) != 0 || a.pflag[pid] != 0 || hold;
}

// LAST: the row's last block (a per-row arrival counter, device-scope fences)
// finishes the row; otherwise k_step2_rows does, one launch later (no fence
// per block: each one writes back the L2's dirty lines, which large batches
// pay for every block).
template <int MODE, int LVMAX, bool LAST>
__global__ __launch_bounds__(kStep2Threads) void k_step2(FinArgs a) {
  constexpr int NT = kStep2Threads, NW = NT / 64;
  constexpr bool kA = MODE == FIN_STEP_A;
  __shared__ float shr[5 * NW];
  __shared__ int last_sh;
  const int tid = threadIdx.x;
  const int rb = blockIdx.x / a.split, blk = blockIdx.x - rb * a.split;  // row of the launch, block of the row
  int r, pid;
  ProbPlan pl;
  if (a.single) {
    r = rb;
    pid = 0;
    pl = a.one;
  } else {
    r = a.rows[rb];
    pid = a.row_prob[r];
    pl = a.plans[pid];
  }
  const int M = pl.M, N = pl.N, L = pl.L;
  const int nblk = (N + NT - 1) / NT;
  if (blk >= nblk) return;  // the row has fewer blocks than the launch's longest
  const int m = r - pl.row0;
  const int64_t wrow = pl.off_w + (int64_t)m * N;
  const int64_t crow = (int64_t)m * N;
  const int next = a.next;
  const bool sgd = (a.opt.flags & SQNGD_OPT_SGD) != 0;
  const float2 zero2 = make_float2(0.f, 0.f);
  const int tstep = *a.counter;
  float* mh = a.adam + pl.off_state + 2 * (int64_t)M * N * L + 2 * crow;
  float* vh = mh + 2 * (int64_t)M * N;
  const int n = blk * NT + tid;  // this thread's chip
  const bool on = n < N;

  // ---- the row's skip decision from its whole gradient row; this chip's gradient
  float2 gc = zero2;
  const bool skip = step2_skip(a, pid, wrow, N, n, gc);
  const float b1 = a.opt.beta1, b2 = a.opt.beta2;
  const bool vec4 = LVMAX % 4 == 0 && (L & 3) == 0 && ((pl.off_z | pl.off_state) & 3) == 0 &&
                    (((uintptr_t)a.z | (uintptr_t)a.adam) & 15) == 0;

  // the chip's logits (invalid levels -inf) and, for the z step, its moments
  auto load_z = [&](float (&zl)[LVMAX], float (&mz)[LVMAX], float (&vz)[LVMAX], bool moments) {
    const int64_t zrow = pl.off_z + (crow + n) * L;
    const float* amz = a.adam + pl.off_state + (crow + n) * L;
    const float* avz = amz + (int64_t)M * N * L;
    if (vec4) {
#pragma unroll
      for (int k4 = 0; k4 < LVMAX / 4; ++k4) {
        const bool ok = 4 * k4 < L;
        const float4 z4 = ok ? *(const float4*)(a.z + zrow + 4 * k4)
                             : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
        const float4 m4 = ok && moments ? *(const float4*)(amz + 4 * k4) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 v4 = ok && moments ? *(const float4*)(avz + 4 * k4) : make_float4(0.f, 0.f, 0.f, 0.f);
        zl[4 * k4] = z4.x, zl[4 * k4 + 1] = z4.y, zl[4 * k4 + 2] = z4.z, zl[4 * k4 + 3] = z4.w;
        mz[4 * k4] = m4.x, mz[4 * k4 + 1] = m4.y, mz[4 * k4 + 2] = m4.z, mz[4 * k4 + 3] = m4.w;
        vz[4 * k4] = v4.x, vz[4 * k4 + 1] = v4.y, vz[4 * k4 + 2] = v4.z, vz[4 * k4 + 3] = v4.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < LVMAX; ++k) {
        const bool ok = k < L;
        zl[k] = ok ? a.z[zrow + k] : -INFINITY;
        mz[k] = ok && moments ? amz[k] : 0.f;
        vz[k] = ok && moments ? avz[k] : 0.f;
      }
    }
  };
  // energy and mainlobe products of the next pass (eq. 10, 32, 38): Re, Im
  // of conj(partner) self, |self|^2, |partner|^2
  float q[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  auto product = [&](float2 self, float2 part) {
    q[0] = part.x * self.x + part.y * self.y;
    q[1] = part.x * self.y - part.y * self.x;
    q[2] = self.x * self.x + self.y * self.y;
    q[3] = part.x * part.x + part.y * part.y;
  };

  if (on) {
    const float2 hv = a.h[wrow + n];
    if constexpr (kA) {
      // Adam on (Re h, Im h); the row's last block projects it
      float2 h1 = hv;
      if (!skip) {
        if (sgd) {
          h1.x -= a.opt.lr_h * gc.x;
          h1.y -= a.opt.lr_h * gc.y;
        } else {
          const float2 m2 = *(const float2*)(mh + 2 * n), v2 = *(const float2*)(vh + 2 * n);
          const int k = tstep * a.opt.n_h + a.inner + 1;
          const float bc1 = bias_corr(b1, k), bc2 = bias_corr(b2, k);
          const float mx = b1 * m2.x + (1.0f - b1) * gc.x, my = b1 * m2.y + (1.0f - b1) * gc.y;
          const float vx = b2 * v2.x + (1.0f - b2) * gc.x * gc.x, vy = b2 * v2.y + (1.0f - b2) * gc.y * gc.y;
          h1.x -= a.opt.lr_h * (mx / bc1) / (sqrtf(vx / bc2) + a.opt.eps);
          h1.y -= a.opt.lr_h * (my / bc1) / (sqrtf(vy / bc2) + a.opt.eps);
          *(float2*)(mh + 2 * n) = make_float2(mx, my);
          *(float2*)(vh + 2 * n) = make_float2(vx, vy);
        }
        a.h[wrow + n] = h1;
      }
      if (next == NEXT_B_FULL) {
        float zl[LVMAX], mz[LVMAX], vz[LVMAX];
        load_z(zl, mz, vz, false);
        const float2 nx = chip_quantise<1, LVMAX>(zl, 0, L, false, temperature_at(a.opt, tstep), pl.sq_mode);
        a.wself[wrow + n] = nx;
        product(nx, h1);
      } else {
        product(h1, next == NEXT_A_SNRL ? a.wpart[wrow + n] : h1);
      }
    } else {
      const float2 sv = a.self_w[wrow + n];
      float zl[LVMAX], mz[LVMAX], vz[LVMAX];
      load_z(zl, mz, vz, !skip && !sgd);
      if (!skip) {
        // dL/dz through the soft quantiser at the temperature of this step, then Adam
        const float Tc = temperature_at(a.opt, tstep);
        const float invT = 1.0f / Tc;
        float zm = -INFINITY;
#pragma unroll
        for (int k = 0; k < LVMAX; ++k) zm = fmaxf(zm, zl[k]);
        float e[LVMAX];
        float se = 0.f, sy = 0.f;
#pragma unroll
        for (int k = 0; k < LVMAX; ++k) {
          e[k] = k < L ? expf((zl[k] - zm) * invT) : 0.f;
          se += e[k];
          sy += (float)k * e[k];
        }
        // one division per chip and per step instead of three per level
        const float inv_se = 1.0f / se;
        const float yb = sy * inv_se;
        const int kz = tstep * a.opt.n_x + a.inner + 1;
        const float ibc1 = sgd ? 1.0f : 1.0f / bias_corr(b1, kz), ibc2 = sgd ? 1.0f : 1.0f / bias_corr(b2, kz);
        const float dphi = (gc.y * sv.x - gc.x * sv.y) * (2.0f * 3.14159265358979f / (float)L) * invT;
#pragma unroll
        for (int k = 0; k < LVMAX; ++k) {
          if (k >= L) continue;
          const float pi = e[k] * inv_se;
          float gv;
          if (pl.sq_mode == SQNGD_SQ_PHASE_MEAN) {
            gv = dphi * pi * ((float)k - yb);
          } else {
            const float2 ul = level_phasor(k, L);
            gv = pi * invT * (gc.x * (ul.x - sv.x) + gc.y * (ul.y - sv.y));
          }
          if (sgd) {
            zl[k] -= a.opt.lr_z * gv;
          } else {
            mz[k] = b1 * mz[k] + (1.0f - b1) * gv;
            vz[k] = b2 * vz[k] + (1.0f - b2) * gv * gv;
            zl[k] -= a.opt.lr_z * (mz[k] * ibc1) / (sqrtf(vz[k] * ibc2) + a.opt.eps);
          }
        }
        const int64_t zrow = pl.off_z + (crow + n) * L;
        float* amz = a.adam + pl.off_state + (crow + n) * L;
        float* avz = amz + (int64_t)M * N * L;
        if (vec4) {
#pragma unroll
          for (int k4 = 0; k4 < LVMAX / 4; ++k4) {
            if (4 * k4 < L) {
              *(float4*)(a.z + zrow + 4 * k4) = make_float4(zl[4 * k4], zl[4 * k4 + 1], zl[4 * k4 + 2], zl[4 * k4 + 3]);
              if (!sgd) {
                *(float4*)(amz + 4 * k4) = make_float4(mz[4 * k4], mz[4 * k4 + 1], mz[4 * k4 + 2], mz[4 * k4 + 3]);
                *(float4*)(avz + 4 * k4) = make_float4(vz[4 * k4], vz[4 * k4 + 1], vz[4 * k4 + 2], vz[4 * k4 + 3]);
              }
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < LVMAX; ++k) {
            if (k < L) {
              a.z[zrow + k] = zl[k];
              if (!sgd) {
                amz[k] = mz[k];
                avz[k] = vz[k];
              }
            }
          }
        }
      }
      float2 nx = zero2;
      if (next == NEXT_A_FULL || next == NEXT_B_SOFT)
        nx = chip_quantise<1, LVMAX>(zl, 0, L, next == NEXT_A_FULL,
                                     temperature_at(a.opt, tstep + (next == NEXT_B_SOFT ? a.next_t_offset : 0)),
                                     pl.sq_mode);
      if (next == NEXT_B_SOFT) a.wself[wrow + n] = nx;
      if (next == NEXT_A_FULL) a.wpart[wrow + n] = nx;
      if (next == NEXT_A_FULL) product(hv, nx);
      else product(nx, hv);
    }
  }

  // ---- the block's partial products; the row's last block, or k_step2_rows, sums them
  block_sum5<NW>(q, shr);
  float4* part = a.rowpart + (int64_t)rb * kStep2MaxSplit;
  if constexpr (!LAST) {
    if (tid == 0) part[blk] = make_float4(q[0], q[1], q[2], q[3]);
    return;
  }
  if (tid == 0) {
    part[blk] = make_float4(q[0], q[1], q[2], q[3]);
    __threadfence();  // release: the partials and this block's filter chips
    last_sh = atomicAdd(a.rowcnt + rb, 1) == nblk - 1;
  }
  __syncthreads();
  if (!last_sh) return;
  __threadfence();  // acquire: every block's partials and filter chips
  if (tid == 0) atomicExch(a.rowcnt + rb, 0);
  step2_finish<kA>(a, part, nblk, skip, r, wrow, N);
}

// The rows' ends after k_step2<..., false>: one block of kStep2Threads per row.
template <int MODE>
__global__ __launch_bounds__(kStep2Threads) void k_step2_rows(FinArgs a) {
  const int rb = blockIdx.x;
  int r, pid;
  ProbPlan pl;
  if (a.single) {
    r = rb;
    pid = 0;
    pl = a.one;
  } else {
    r = a.rows[rb];
    pid = a.row_prob[r];
    pl = a.plans[pid];
  }
  const int N = pl.N;
  const int64_t wrow = pl.off_w + (int64_t)(r - pl.row0) * N;
  float2 gc = make_float2(0.f, 0.f);
  const bool skip = step2_skip(a, pid, wrow, N, -1, gc);
  step2_finish<MODE == FIN_STEP_A>(a, a.rowpart + (int64_t)rb * kStep2MaxSplit, (N + kStep2Threads - 1) / kStep2Threads,
                                   skip, r, wrow, N);
}

// ------------------------------------------------------------ k_pass_split

// Latency variant of the fused pass for small batches: one wave per
// (Doppler bin, partner) pair instead of one wave per Doppler bin looping
// over the partners. A block holds UB = WV / M units of one row, all M
// partners of each; the partners' adjoint spectra and statistics are
// combined per unit in LDS (relative to the unit's largest pair scale), then
// the units per block as in k_pass. Every wave computes its unit's modulated
// spectrum itself. Needs one FFT per wave (P >= 512) and M <= WV.
template <int P, int PHLOG, int WV, bool WT>
__global__ __launch_bounds__(64 * WV) void k_pass_split(PassArgs a) {
  // padding every 32 elements keeps two blocks per CU at P = 1024 with 8 waves
  using G = GeomT<P, 64, 5>;
  static_assert(G::TF == 64, "one FFT per wave");
  constexpr int E = G::E, EH = E / 2;
  __shared__ float2 lds[WV * G::SPAN];
  // tables the block computes once: W_P^k, and per unit exp(j 2 pi t nu / N)
  // for t < 64 with the step t = 64 in the last column
  __shared__ float2 tw_tab[P];
  __shared__ float2 ph_tab[WV][65];
  __shared__ float g_sig[WV], g_S[WV];
  __shared__ unsigned long long g_ka[WV], g_kc[WV];
  __shared__ float u_sig[WV], u_S[WV];
  __shared__ unsigned long long u_ka[WV], u_kc[WV];
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  if (a.bump != nullptr && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.bump, 1);
  float2* buf = lds + wv * G::SPAN;
  int base = 0;
  ProbPlan pl;
  if (a.single) {
    pl = a.one;
  } else {
    const int entry = find_entry(a.gwave, a.gn, blockIdx.x);
    pl = a.plans[a.gprob[entry]];
    base = a.gwave[entry];
  }
  const int M = pl.M, N = pl.N, F = pl.F;
  const int UB = WV / M;
  const int j = wv / M, g = wv - (wv / M) * M;
  // the unit's leader wave (it combines the partners and runs the unit's
  // inverse transform): partner j mod M, so that the leaders of a block's
  // units sit on different SIMDs (a block's waves go round-robin over them)
  const int lead = j % M;
  const bool wave_on = j < UB;
  const int lb = blockIdx.x - base;
  const int w = lb / pl.wpr;
  const int grp = lb - w * pl.wpr;
  const int fs = grp * UB + j;
  const bool active = wave_on && fs < F;
  const int f = fs < F ? fs : F - 1;
  const int u = w * F + f;
  const double invN = 1.0 / (double)N;
  const double nu = doppler_nu(pl, f, a.orient);
  const int wlo = a.orient ? -pl.tau_hi : pl.tau_lo;
  const int whi = a.orient ? -pl.tau_lo : pl.tau_hi;
  const float phm1 = 0.5f * pl.p - 1.0f;
  const bool grad = a.want_grad != 0;
  const float* wrow = WT ? a.roi_w + pl.off_rw + (int64_t)f * (2 * N - 1) : nullptr;

  // global loads first, in the order they are needed (a wave's loads complete
  // in issue order): the self row, the partner spectrum, the ROI weights;
  // then the arithmetic that hides their latency
  const float2* sg = a.spec + pl.ws_spec + (int64_t)(wave_on ? g : 0) * P;
  const float2* sw = a.self_w + pl.off_w + (int64_t)w * N;
  float2 SG[E], X[E];
  float WR[WT ? E : 1];  // ROI weights of this lane's cells (0 where a cell holds no delay)
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    X[e] = make_float2(0.f, 0.f);
    if constexpr (e < EH) {  // every load issued (clamped index), the tail zeroed after
      const int n = t + 64 * e;
      X[e] = sw[n < N ? n : N - 1];
    }
  });
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    SG[e] = sg[e * 64 + t];  // the one-wave layout (spec_wave) at P = 1024; the same as the pass layout below
  });
  if constexpr (WT) {
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const int k = t + 64 * e;
      const bool lo = k <= N - 1, hi = k >= P - N + 1;
      const int tp = lo ? -k : P - k;
      const int tau = a.orient ? -tp : tp;
      WR[e] = wrow[(lo || hi) ? tau + N - 1 : 0];
    });
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the table arithmetic
  if constexpr (WT) {
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const int k = t + 64 * e;
      if (!(k <= N - 1 || k >= P - N + 1)) WR[e] = 0.f;
    });
  }
  for (int i = threadIdx.x; i < P; i += 64 * WV) tw_tab[i] = tw_exact<P>(i);
  for (int i = threadIdx.x; i < UB * 65; i += 64 * WV) {
    const int jj = i / 65, tt = i - jj * 65;
    const int fj = min(grp * UB + jj, F - 1);
    ph_tab[jj][tt] = phasor(tt, doppler_nu(pl, fj, a.orient), invN);
  }
  block_lds_sync();
  TwiddlesG<G> W;
  W.init_table(t, tw_tab);
  auto phasor_row_tab = [&](float2 (&ph)[EH]) {
    ph[0] = ph_tab[wave_on ? j : 0][t];
    const float2 st = ph_tab[wave_on ? j : 0][64];
    static_for<EH - 1>([&](auto ec) {
      constexpr int e = decltype(ec)::value + 1;
      ph[e] = cmul(ph[e - 1], st);
    });
  };
  {
    float2 ph[EH];
    phasor_row_tab(ph);
    static_for<EH>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      X[e] = t + 64 * e < N ? cmul(X[e], ph[e]) : make_float2(0.f, 0.f);
    });
  }
  fft_forward_g<G>(X, buf, t, W);

  // this wave's pair (unit j, partner g)
  float2 R[E];
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    R[e] = cmulc(X[e], SG[e]);
  });
  fft_inverse_g<G>(R, buf, t, W);
  uint32_t vmask;
  float qmax;
  int kbest;
  if (a.cube != nullptr && active)
    cube_store<P, 64, E>(R, t, N, a.cube + pl.off_cube + ((int64_t)(w * M + g) * F + f) * (2 * N - 1));
  if constexpr (WT) roi_weigh_reg<E>(R, WR);  // a = w |A| / N from here on
  vmask = roi_bits<64, E>(roi_runs<P>(N, wlo, whi), t, g == w && f >= pl.cut_lo && f < pl.cut_hi);
  roi_scan_bits<64, E>(R, t, vmask, qmax, kbest);
  // wave maximum, and its cell from the lowest lane that holds it
  const float qw = wave_max(qmax);
  const unsigned long long holders = __ballot(vmask != 0 && qmax == qw);
  const int src = holders ? __ffsll((long long)holders) - 1 : 0;
  const int kb = __builtin_amdgcn_readlane(kbest, src);
  const unsigned long long key = holders ? make_key(qw, (uint32_t)(((int64_t)u * M + g) * P + kb)) : 0ull;
  const float sigma = sqrtf(qw);
  float S = 0.f;
  roi_scale<PHLOG, E>(R, sigma > 0.f ? __builtin_amdgcn_rcpf(sigma) : 0.f, phm1, S);
  if constexpr (WT) roi_weigh_reg<E>(R, WR);  // d(w|r|)^p / dr carries w^2
  S = wave_sum(S);
  if (t == 0) {
    g_sig[wv] = active ? sigma : 0.f;
    g_S[wv] = active ? S : 0.f;
    g_ka[wv] = active && g == w ? key : 0ull;
    g_kc[wv] = active && g != w ? key : 0ull;
  }
  if (grad) {
    fft_forward_g<G>(R, buf, t, W);
    wave_lds_sync();
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      buf[e * 64 + t] = cmul(R[e], SG[e]);
    });
  }
  block_lds_sync();

  // per unit: the partner waves combined by the unit's leader
  if (wave_on && g == lead) {
    float su = 0.f;
    for (int gg = 0; gg < M; ++gg) su = fmaxf(su, g_sig[j * M + gg]);
    const float inv_u = su > 0.f ? 1.0f / su : 0.f;
    float Su = 0.f;
    unsigned long long ka = 0, kc = 0;
    float2 U[E];
    static_for<E>([&](auto ec) { U[decltype(ec)::value] = make_float2(0.f, 0.f); });
    for (int gg = 0; gg < M; ++gg) {
      const int src = j * M + gg;
      const float c = g_sig[src] * inv_u;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);
      Su += cp * g_S[src];
      ka = umax64(ka, g_ka[src]);
      kc = umax64(kc, g_kc[src]);
      if (grad) {
        const float fc = cm1 * c;  // (sigma_g / sigma_u)^(p-1)
        static_for<E>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          const float2 v = lds[src * G::SPAN + e * 64 + t];
          U[e].x += fc * v.x;
          U[e].y += fc * v.y;
        });
      }
    }
    if (t == 0) {
      u_sig[j] = su;
      u_S[j] = Su;
      u_ka[j] = ka;
      u_kc[j] = kc;
    }
    if (grad) {
      fft_inverse_g<G>(U, buf, t, W);
      float2 ph[EH];
      phasor_row_tab(ph);
      wave_lds_sync();
      static_for<EH>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        const int n = t + 64 * e;
        if (n < N) buf[n] = active ? cmulc(U[e], ph[e]) : make_float2(0.f, 0.f);
      });
    }
  }
  block_lds_sync();

  // block combine over the UB units (unit order fixed)
  float sb = 0.f;
  for (int jj = 0; jj < UB; ++jj) sb = fmaxf(sb, u_sig[jj]);
  const float inv_b = sb > 0.f ? 1.0f / sb : 0.f;
  const int64_t ent = (int64_t)w * pl.wpr + grp;
  if (threadIdx.x == 0) {
    float Sb = 0.f;
    unsigned long long ka = 0, kc = 0;
    for (int jj = 0; jj < UB; ++jj) {
      const float c = u_sig[jj] * inv_b;
      float cm1, cp;
      pow_ph<PHLOG>(c * c, phm1, cm1, cp);
      Sb += cp * u_S[jj];
      ka = umax64(ka, u_ka[jj]);
      kc = umax64(kc, u_kc[jj]);
    }
    UnitStat st;
    st.sigma = sb;
    st.S = Sb;
    st.pad0 = st.pad1 = 0;
    st.key_auto = ka;
    st.key_cross = kc;
    a.ustat[pl.ws_unit + ent] = st;
  }
  if (grad) {
    float2* up = a.upart + pl.ws_upart + ent * N;
    for (int n = threadIdx.x; n < N; n += 64 * WV) {
      float2 acc = make_float2(0.f, 0.f);
      for (int jj = 0; jj < UB; ++jj) {
        const float c = u_sig[jj] * inv_b;
        float cm1, cp;
        pow_ph<PHLOG>(c * c, phm1, cm1, cp);
        const float fc = cm1 * c;
        const float2 v = lds[(jj * M + jj % M) * G::SPAN + n];
        acc.x += fc * v.x;
        acc.y += fc * v.y;
      }
      up[n] = acc;
    }
  }
}

// ------------------------------------------------------------- k_pass_pair

// Latency form of the pass at the FFT lengths whose transform spans a whole
// block (P >= 2048): one block per (row w, Doppler bin f, partner g) pair.
// The block computes the modulated self spectrum, the pair's AF row, its ROI
// statistics, the adjoint and that partner's own share of the gradient row
// (the inverse transform of adjoint x partner spectrum, demodulated): four
// transforms in sequence where the throughput pass runs 2M + 2 per unit. The
// pairs' statistics and gradient partial rows are separate entries, each
// relative to its own scale (the finalize combines any number of them), so
// no partial sum over partners is held and the block needs one exchange
// buffer of LDS. For single designs whose units barely exceed the compute
// units (M=2 N=1200 F=129: 258 units, 516 pairs), where one block of the
// throughput pass per unit leaves a second round of whole units.
template <int P, int PHLOG, bool WT>
__global__ __launch_bounds__(64 * PassGeom<P>::WAVES, 4) void k_pass_pair(PassArgs a) {
  using G = PassGeom<P>;
  static_assert(G::WAVES >= 4, "a transform spans the block");
  constexpr int E = G::E, TF = G::TF, EH = E / 2;
  __shared__ float2 lds[G::SPAN];
  __shared__ float red_f[G::WAVES];
  __shared__ unsigned long long red_k[G::WAVES];
  const int t = threadIdx.x;
  const int blk = blockIdx.x;
  if (a.bump != nullptr && blk == 0 && t == 0) atomicAdd(a.bump, 1);
  int base = 0;
  ProbPlan pl;
  if (a.single) {
    pl = a.one;
  } else {
    const int entry = find_entry(a.gwave, a.gn, blk);
    pl = a.plans[a.gprob[entry]];
    base = a.gwave[entry];
  }
  const int M = pl.M, N = pl.N, F = pl.F;
  // blocks of a problem: wpr = F M per row, rows in order; within a row
  // Doppler bin major, partner minor
  const int lb = blk - base;
  const int w = lb / pl.wpr;
  const int rem = lb - w * pl.wpr;
  const int f = rem / M, g = rem - (rem / M) * M;
  const int u = w * F + f;
  const double invN = 1.0 / (double)N;
  const double nu = doppler_nu(pl, f, a.orient);
  const int wlo = a.orient ? -pl.tau_hi : pl.tau_lo;
  const int whi = a.orient ? -pl.tau_lo : pl.tau_hi;
  const float phm1 = 0.5f * pl.p - 1.0f;
  const bool grad = a.want_grad != 0;

  // global loads first, in the order they are needed
  const float2* sw = a.self_w + pl.off_w + (int64_t)w * N;
  const float2* sg = a.spec + pl.ws_spec + (int64_t)g * P;
  float2 R[E];
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    R[e] = make_float2(0.f, 0.f);
    if constexpr (e < EH) {
      const int n = t + TF * e;
      R[e] = sw[n < N ? n : N - 1];
    }
  });
  float WR[WT ? E : 1];
  if constexpr (WT) roi_weights_load<P, TF, E>(WR, t, N, a.orient, a.roi_w + pl.off_rw + (int64_t)f * (2 * N - 1));
  TwiddlesG<G> W;
  W.init(t);
  {
    float2 ph[EH];
    phasor_row<EH, TF>(t, nu, invN, ph);
    static_for<EH>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      R[e] = t + TF * e < N ? cmul(R[e], ph[e]) : make_float2(0.f, 0.f);
    });
  }
  fft_forward_g<G>(R, lds, t, W);  // X, the modulated self spectrum
  static_for<E>([&](auto ec) {
    constexpr int e = decltype(ec)::value;
    R[e] = cmulc(R[e], sg[e * TF + t]);
  });
  fft_inverse_g<G>(R, lds, t, W);  // P A(tau') of the pair at r-index k = t + TF e
  if (a.cube != nullptr)
    cube_store<P, TF, E>(R, t, N, a.cube + pl.off_cube + ((int64_t)(w * M + g) * F + f) * (2 * N - 1));
  if constexpr (WT) roi_weigh_reg<E>(R, WR);  // a = w |A| / N from here on
  uint32_t vmask;
  float qmax;
  int kbest;
  vmask = roi_bits<TF, E>(roi_runs<P>(N, wlo, whi), t, g == w && f >= pl.cut_lo && f < pl.cut_hi);
  roi_scan_bits<TF, E>(R, t, vmask, qmax, kbest);
  unsigned long long key = vmask ? make_key(qmax, (uint32_t)(((int64_t)u * M + g) * P + kbest)) : 0ull;
  key = fft_lanes_max_key<G>(key, red_k);
  qmax = fft_lanes_reduce<G>(qmax, 0.0f, OpMax(), red_f);
  const float sigma = sqrtf(qmax);
  float S = 0.f;
  roi_scale<PHLOG, E>(R, sigma > 0.f ? __builtin_amdgcn_rcpf(sigma) : 0.f, phm1, S);
  if constexpr (WT) roi_weigh_reg<E>(R, WR);  // d(w|r|)^p / dr carries w^2
  S = fft_lanes_reduce<G>(S, 0.0f, OpAdd(), red_f);
  const int64_t ent = (int64_t)w * pl.wpr + rem;
  if (t == 0) {
    UnitStat st;
    st.sigma = sigma;
    st.S = S;
    st.pad0 = st.pad1 = 0;
    st.key_auto = g == w ? key : 0ull;
    st.key_cross = g == w ? 0ull : key;
    a.ustat[pl.ws_unit + ent] = st;
  }
  if (grad) {
    fft_forward_g<G>(R, lds, t, W);  // the adjoint's spectrum
    static_for<E>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      R[e] = cmul(R[e], sg[e * TF + t]);
    });
    fft_inverse_g<G>(R, lds, t, W);  // this partner's share of the self gradient
    float2 ph[EH];
    phasor_row<EH, TF>(t, nu, invN, ph);
    float2* up = a.upart + pl.ws_upart + ent * N;
    static_for<EH>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      const int n = t + TF * e;
      if (n < N) up[n] = cmulc(R[e], ph[e]);
    });
  }
}

// ------------------------------------------------------------------ k_stop

// The stopping criterion of Algorithm 1, one thread per design: the hard
// WPSL of the checkpoint (dB) against the best so far; a checkpoint that does
// not lower it by more than min_gain counts as a stall, and `patience`
// consecutive stalls stop the design at the current outer iteration.
__global__ void k_stop(int32_t n, const sqngd_stats* __restrict__ st, float min_gain, int32_t patience,
                       const int32_t* __restrict__ step, float* best, int32_t* stall, int32_t* stopped,
                       int32_t* stop_iter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || stopped[i] != 0) return;
  const float w = st[i].pslr_db;
  if ((double)w < (double)best[i] - (double)min_gain) {  // the comparison in FP64, as the host rule makes it
    best[i] = w;
    stall[i] = 0;
  } else if (++stall[i] >= patience) {
    stopped[i] = 1;
    stop_iter[i] = step != nullptr ? *step : 0;
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

}  // namespace sq
