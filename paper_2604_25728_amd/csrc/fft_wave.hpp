// fft_wave.hpp - wave-local complex64 FFTs of length P = 128 .. 2048 for gfx950.
//
// One FFT lives in TF lanes, E = P / TF elements per lane in registers. The
// default geometry (Geom) keeps it inside one 64-lane wave (TF = 64 for
// P >= 512, else P / 8, so E >= 8), and a wave runs 64 / TF independent FFTs
// side by side ("slots"); every exchange of data between lanes stays inside
// the wave, so no workgroup barrier is needed: an exchange is a write of the
// slot's elements to its private LDS region, a wave-scope fence, and a read
// back in the next stage's order. A geometry with TF = 128 spreads one FFT
// over two waves of a workgroup (half the registers per lane); its exchanges
// synchronise the workgroup instead.
//
// Factorisation (Cooley-Tukey four-step, P = E * TF with TF = A * B):
//   natural index n = t + TF * e            (lane t, register e)
//   1. length-E DFT over the registers of each lane           -> k1
//   2. twiddle W_P^(t k1)
//   3a. LDS exchange, length-A DFTs over alpha (n2 = B alpha + beta)  -> gamma,
//       twiddle W_TF^(beta gamma)
//   3b. LDS exchange, length-B DFTs over beta                          -> delta
//   output "spectral layout": lane t, register j2*B + delta holds bin
//       k = k1 + E (gamma + A delta),  gamma = t % A,  k1 = j2*B + t / A.
// The inverse transform runs the same stages mirrored, from the spectral
// layout back to the natural layout, with conjugate twiddles. Neither
// transform scales by 1/P.
//
// Products of two spectra are formed element by element in the spectral
// layout, so a forward FFT, a pointwise product and an inverse FFT never
// reorder data through memory beyond the four exchanges.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace sq {

// ----------------------------------------------------------------- utilities

template <int... Is, class Fn>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, Fn&& fn) {
  (fn(std::integral_constant<int, Is>{}), ...);
}
template <int Count, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  static_for_impl(std::make_integer_sequence<int, Count>{}, static_cast<Fn&&>(fn));
}

// Compile-time sine and cosine (Taylor series after reduction to [-pi, pi]),
// used only to form constant twiddles of the in-register DFTs.
constexpr double cx_pi = 3.14159265358979323846264338327950288;
constexpr double cx_sin(double x) {
  while (x > cx_pi) x -= 2.0 * cx_pi;
  while (x < -cx_pi) x += 2.0 * cx_pi;
  double term = x, sum = x;
  for (int i = 1; i < 30; ++i) {
    term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) { return cx_sin(x + 0.5 * cx_pi); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Multiply by the constant W = exp(DIR * 2 pi i J / LEN), DIR = -1 forward, +1 inverse.
template <int J, int LEN, int DIR>
__device__ __forceinline__ float2 twiddle_const(float2 v) {
  constexpr int j = ((J % LEN) + LEN) % LEN;
  if constexpr (j == 0) {
    return v;
  } else if constexpr (4 * j == LEN) {  // W = DIR * i
    return DIR < 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  } else if constexpr (2 * j == LEN) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * j == 3 * LEN) {  // W = -DIR * i
    return DIR < 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  } else {
    constexpr double ang = 2.0 * cx_pi * (double)j / (double)LEN;
    constexpr float c = (float)cx_cos(ang);
    constexpr float s = (float)(DIR * cx_sin(ang));
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

constexpr int cx_log2(int v) { return v <= 1 ? 0 : 1 + cx_log2(v / 2); }
constexpr int cx_bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register DFT of length R on x[OFF .. OFF+R) (natural order in and out):
// radix-2 decimation in time after a compile-time bit reversal (a register
// renaming, free at run time).
template <int R, int DIR, int OFF, int CAP>
__device__ __forceinline__ void dft_reg(float2 (&x)[CAP]) {
  if constexpr (R == 1) {
    return;
  } else {
    constexpr int LB = cx_log2(R);
    float2 y[R];
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      y[cx_bitrev(i, LB)] = x[OFF + i];
    });
    static_for<LB>([&](auto sc) {
      constexpr int half = 1 << decltype(sc)::value;
      constexpr int len = 2 * half;
      static_for<R / len>([&](auto bc) {
        constexpr int base = decltype(bc)::value * len;
        static_for<half>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          float2 u = y[base + j];
          float2 v = twiddle_const<j, len, DIR>(y[base + j + half]);
          y[base + j] = cadd(u, v);
          y[base + j + half] = csub(u, v);
        });
      });
    });
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      x[OFF + i] = y[i];
    });
  }
}

// Reductions over the TF lanes of a slot with DPP row operations (VALU
// speed); the result is returned in every lane of the slot.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}
template <int TF, class Op>
__device__ __forceinline__ float slot_reduce(float v, float ident, Op op) {
  static_assert(TF == 16 || TF == 32 || TF == 64, "slot_reduce spans whole 16-lane rows");
  v = op(v, dpp_f<0x111, 0xF>(ident, v));  // row_shr:1
  v = op(v, dpp_f<0x112, 0xF>(ident, v));  // row_shr:2
  v = op(v, dpp_f<0x114, 0xF>(ident, v));  // row_shr:4
  v = op(v, dpp_f<0x118, 0xF>(ident, v));  // row_shr:8  -> lane 15 of each row holds the row
  if constexpr (TF >= 32) v = op(v, dpp_f<0x142, 0xA>(ident, v));  // row_bcast:15 -> lanes 31, 63
  if constexpr (TF >= 64) {
    v = op(v, dpp_f<0x143, 0xC>(ident, v));  // row_bcast:31 -> lane 63
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  } else {
    const int lane = __lane_id();
    return __shfl(v, (lane & ~(TF - 1)) + TF - 1);
  }
}
struct OpMax {
  __device__ __forceinline__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct OpAdd {
  __device__ __forceinline__ float operator()(float a, float b) const { return a + b; }
};

// Wave-scope ordering of LDS traffic: every lane's earlier LDS accesses are
// complete and visible to the wave before any later one starts.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS traffic only: every wave's earlier LDS
// accesses are complete and visible to the workgroup before any later one
// starts. Global loads in flight stay in flight across it (a full
// __syncthreads would wait for them), so a kernel that reads only inputs no
// wave of it writes can issue its global loads early and cross barriers
// before they land.
__device__ __forceinline__ void block_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ twiddles

// ------------------------------------------------------------------ geometry

// Exchange buffers carry one float2 of padding after every 2^PS elements:
// element i of an FFT's buffer lives at G::ix(i) = i + (i >> PS). The
// exchanges read with lane strides of 8 or 16 elements across rows of TF
// elements; unpadded, a wave's 64 lanes then fall on 4 to 16 times fewer LDS
// banks than they span (up to 16-way conflicts at P = 2048), padded every
// 16 elements (PS = 4) they spread over all banks. A kernel short of LDS may
// pad every 32 (PS = 5: the second exchange's reads become conflict-free,
// the first keeps part of its conflicts). The padding changes no layout
// outside the exchange buffer. Every exchange access is a lane-dependent
// part plus a compile-time part whose low PS bits never carry into the lane
// part's, so G::ix(lane + c) = G::ix(lane) + G::ix(c): the stages form one
// padded base pointer per lane and address from it with immediate offsets.

template <int P_, int TF_, int PS_ = 4>
struct GeomT {
  static constexpr int P = P_;
  static constexpr int TF = TF_;                     // lanes per FFT
  static constexpr int PS = PS_;                     // exchange-buffer padding: one float2 per 2^PS
  static constexpr int E = P / TF;                   // elements per lane
  static constexpr int A = TF >= 32 ? 8 : 4;
  // The length-TF DFT over the lanes runs as radix-A then radix-B stages
  // (two LDS exchanges) when every lane's E elements tile both radices, else
  // as radix-A, radix-B = E and radix-C stages (three exchanges).
  static constexpr bool THREE = E % (TF / A) != 0;
  static constexpr int B = THREE ? E : TF / A;
  static constexpr int C = THREE ? TF / (A * B) : 1;
  static constexpr int BC = B * C;
  static constexpr int SLOTS = TF <= 64 ? 64 / TF : 1;  // FFTs per wave
  static constexpr int WAVES = TF > 64 ? TF / 64 : 1;   // waves per FFT
  static constexpr int SPAN = P + (P >> PS);        // float2 of one FFT's padded exchange buffer
  static constexpr int LDS = SLOTS * SPAN;           // float2 of a wave's exchange buffers (wave-local)
  __host__ __device__ static constexpr int ix(int i) { return i + (i >> PS); }
  static_assert(A * B * C == TF, "the lane radices factor TF");
  static_assert(E % A == 0 && E % B == 0 && E % C == 0, "register blocks must tile E");
  static_assert(TF <= 64 ? 64 % TF == 0 : TF % 64 == 0, "an FFT fills whole waves or divides one");
  // spectral-layout bin of lane t, register e (unsigned arithmetic: every
  // index is non-negative and every radix a power of two, so the divisions
  // and remainders are shifts and masks)
  __device__ static constexpr int spec_bin(int t_, int e_) {
    const unsigned t = (unsigned)t_, e = (unsigned)e_;
    constexpr unsigned uA = A, uB = B, uC = C, uE = E;
    if constexpr (!THREE) {
      const unsigned gamma = t % uA, k1 = (e / uB) * uB + t / uA, delta = e % uB;
      return (int)(k1 + uE * (gamma + uA * delta));
    } else {
      const unsigned q3 = t / (uA * uB), gamma = (t % (uA * uB)) / uB, zeta = t % uB;
      const unsigned k1 = (e / uC) * uC + q3, eta = e % uC;
      return (int)(k1 + uE * (gamma + uA * (zeta + uB * eta)));
    }
  }
  // the inverse: storage index e * TF + t of bin k
  __device__ static constexpr int spec_index(int k_) {
    const unsigned k = (unsigned)k_;
    constexpr unsigned uA = A, uB = B, uC = C, uE = E, uTF = TF;
    const unsigned k1 = k % uE, r = k / uE, gamma = r % uA;
    if constexpr (!THREE) {
      const unsigned delta = r / uA;
      return (int)(((k1 / uB) * uB + delta) * uTF + (k1 % uB) * uA + gamma);
    } else {
      const unsigned r2 = r / uA, zeta = r2 % uB, eta = r2 / uB;
      return (int)(((k1 / uC) * uC + eta) * uTF + (k1 % uC) * (uA * uB) + gamma * uB + zeta);
    }
  }
};
template <int P>
using Geom = GeomT<P, (P >= 512 ? 64 : P / 8)>;

// LDS ordering between the stages of one FFT: the wave for a wave-local
// geometry, the workgroup for one spread over several waves.
template <class G>
__device__ __forceinline__ void fft_sync() {
  if constexpr (G::WAVES > 1) block_lds_sync();
  else wave_lds_sync();
}

// exp(-2 pi i k / P) for an integer k, from one sincospi of the reduced angle.
template <int P>
__device__ __forceinline__ float2 tw_exact(int k) {
  float s, c;
  sincospif(2.0f * (float)(k & (P - 1)) / (float)P, &s, &c);
  return make_float2(c, -s);
}

// w[k] = w1^k for k < K, each power the product of two lower ones
// (w[k] = w[k/2] w[k - k/2]): one sincospi per twiddle set instead of one
// per power; the error grows with the product depth, a few ulp at K = 8.
template <int K>
__device__ __forceinline__ void tw_powers(float2 (&w)[K], float2 w1) {
  w[0] = make_float2(1.f, 0.f);
  if constexpr (K > 1) w[1] = w1;
  static_for<K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k >= 2) w[k] = cmul(w[k >> 1], w[k - (k >> 1)]);
  });
}

// Per-lane twiddles reused by every FFT of the wave: each set the powers of
// one sincospi value, so no table is read from memory at kernel start.
template <class G_>
struct TwiddlesG {
  using G = G_;
  static constexpr int P = G::P;
  static constexpr int NLO = G::E < 8 ? G::E : 8;
  static constexpr int NHI = G::E / NLO;
  float2 lo[NLO];  // W_P^(t b),        b < NLO
  float2 hi[NHI];  // W_P^(t NLO a),    a < NHI     (W_P^(t k1) = lo[k1 % NLO] hi[k1 / NLO])
  float2 col[G::A];  // W_TF^(beta gamma), gamma < A, beta = t % (B C)
  float2 col2[G::THREE ? G::B : 1];  // three stages: W_(B C)^(c zeta), zeta < B, c = t % C
  // Powers 1, 2 and 4 of each set from sincospi, the others as products:
  // the FFT-length-2048 throughput geometry (256 lanes) runs its pass about
  // 1% faster with these than with the single-sincospi powers (measured on
  // the uneven batch; the other geometries are faster with the powers).
  __device__ __forceinline__ void init_exact(int t) {
    // lo: powers 1, 2, 4 exact; 3, 5, 6, 7 as products
    lo[0] = make_float2(1.f, 0.f);
    if constexpr (NLO > 1) lo[1] = tw_exact<P>(t);
    if constexpr (NLO > 2) lo[2] = tw_exact<P>(2 * t);
    if constexpr (NLO > 3) lo[3] = cmul(lo[2], lo[1]);
    if constexpr (NLO > 4) {
      lo[4] = tw_exact<P>(4 * t);
      lo[5] = cmul(lo[4], lo[1]);
      lo[6] = cmul(lo[4], lo[2]);
      lo[7] = cmul(lo[4], lo[3]);
    }
    hi[0] = make_float2(1.f, 0.f);
    for (int a = 1; a < NHI; ++a) hi[a] = tw_exact<P>(t * NLO * a);
    const int beta = (unsigned)t % G::BC;
    col[0] = make_float2(1.f, 0.f);
    if constexpr (G::A > 1) col[1] = tw_exact<P>(beta * G::E);
    if constexpr (G::A > 2) col[2] = tw_exact<P>(2 * beta * G::E);
    if constexpr (G::A > 3) col[3] = cmul(col[2], col[1]);
    if constexpr (G::A > 4) {
      col[4] = tw_exact<P>(4 * beta * G::E);
      col[5] = cmul(col[4], col[1]);
      col[6] = cmul(col[4], col[2]);
      col[7] = cmul(col[4], col[3]);
    }
    if constexpr (G::THREE) {
      // powers 1, 2, 4 exact; 3, 5, 6, 7 as products (as lo and col)
      const int c = (unsigned)t % G::C;
      constexpr int step = G::E * G::A;
      col2[0] = make_float2(1.f, 0.f);
      if constexpr (G::B == 8) {
        col2[1] = tw_exact<P>(c * step);
        col2[2] = tw_exact<P>(2 * c * step);
        col2[3] = cmul(col2[2], col2[1]);
        col2[4] = tw_exact<P>(4 * c * step);
        col2[5] = cmul(col2[4], col2[1]);
        col2[6] = cmul(col2[4], col2[2]);
        col2[7] = cmul(col2[4], col2[3]);
      } else {
        for (int z = 1; z < G::B; ++z) col2[z] = tw_exact<P>(c * z * step);
      }
    }
  }  __device__ __forceinline__ void init(int t) {
    if constexpr (G::P == 2048 && G::TF == 256) {
      init_exact(t);
      return;
    }
    tw_powers<NLO>(lo, NLO > 1 ? tw_exact<P>(t) : make_float2(1.f, 0.f));
    tw_powers<NHI>(hi, NHI > 1 ? tw_exact<P>(t * NLO) : make_float2(1.f, 0.f));
    const int beta = (unsigned)t % G::BC;
    tw_powers<G::A>(col, G::A > 1 ? tw_exact<P>(beta * G::E) : make_float2(1.f, 0.f));
    if constexpr (G::THREE) {
      const int c = (unsigned)t % G::C;
      tw_powers<G::B>(col2, tw_exact<P>(c * G::E * G::A));
    }
  }
  // The same twiddles read from a table tab[k] = W_P^k, k < P (a block
  // computes the table once instead of every wave its own sincospi values).
  __device__ __forceinline__ void init_table(int t, const float2* tab) {
    lo[0] = make_float2(1.f, 0.f);
    for (int b = 1; b < NLO; ++b) lo[b] = tab[(t * b) & (P - 1)];
    hi[0] = make_float2(1.f, 0.f);
    for (int a = 1; a < NHI; ++a) hi[a] = tab[(t * NLO * a) & (P - 1)];
    const int beta = (unsigned)t % G::BC;
    col[0] = make_float2(1.f, 0.f);
    for (int g = 1; g < G::A; ++g) col[g] = tab[(g * beta * G::E) & (P - 1)];
    if constexpr (G::THREE) {
      const int c = (unsigned)t % G::C;
      col2[0] = make_float2(1.f, 0.f);
      for (int z = 1; z < G::B; ++z) col2[z] = tab[(c * z * G::E * G::A) & (P - 1)];
    }
  }
  template <int K1>
  __device__ __forceinline__ float2 step2(float2 v, bool inverse) const {
    constexpr int b = K1 % NLO, a = K1 / NLO;
    float2 w = lo[b];
    if constexpr (a > 0) w = cmul(w, hi[a]);
    return inverse ? cmulc(v, w) : cmul(v, w);
  }
};

template <int P>
using WaveTwiddles = TwiddlesG<Geom<P>>;

// Three-exchange forms (G::THREE): the lane index t = BC alpha + tau with
// tau = C beta + c; radix-A DFT over alpha (-> gamma), twiddle W_TF^(tau
// gamma); radix-B DFT over beta (-> zeta), twiddle W_BC^(c zeta); radix-C
// DFT over c (-> eta). Spectral layout: lane t = q3 A B + gamma B + zeta,
// register j3 C + eta holds bin k1 + E (gamma + A (zeta + B eta)) with
// k1 = j3 C + q3.
template <class G>
__device__ __forceinline__ void fft3_forward(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  constexpr int E = G::E, TF = G::TF, A = G::A, B = G::B, C = G::C, BC = G::BC;
  dft_reg<E, -1, 0>(x);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    x[k1] = W.template step2<k1>(x[k1], false);
  });
  fft_sync<G>();
  float2* const bt = buf + G::ix(t);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    bt[G::ix(k1 * TF)] = x[k1];
  });
  fft_sync<G>();
  {  // radix A over alpha: lane (q, tau), k1 = j A + q
    const int tau = (unsigned)t % BC, q = (unsigned)t / BC;
    float2* const bq = buf + G::ix(q * TF + tau);
    static_for<E / A>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      static_for<A>([&](auto ac) {
        constexpr int al = decltype(ac)::value;
        x[j * A + al] = bq[G::ix(j * A * TF + BC * al)];
      });
      dft_reg<A, -1, j * A>(x);
      static_for<A>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if constexpr (g > 0) x[j * A + g] = cmul(x[j * A + g], W.col[g]);
      });
    });
    fft_sync<G>();
    static_for<E / A>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      static_for<A>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        bq[G::ix(j * A * TF + g * BC)] = x[j * A + g];
      });
    });
    fft_sync<G>();
  }
  {  // radix B over beta: lane (q2, gamma, c), k1 = j2 B + q2
    const int q2 = (unsigned)t / (A * C), gamma = ((unsigned)t % (A * C)) / C, c = (unsigned)t % C;
    float2* const bq2 = buf + G::ix(q2 * TF + gamma * BC + c);
    static_for<E / B>([&](auto jc) {
      constexpr int j2 = decltype(jc)::value;
      static_for<B>([&](auto bc) {
        constexpr int be = decltype(bc)::value;
        x[j2 * B + be] = bq2[G::ix(j2 * B * TF + C * be)];
      });
      dft_reg<B, -1, j2 * B>(x);
      static_for<B>([&](auto zc) {
        constexpr int z = decltype(zc)::value;
        if constexpr (z > 0) x[j2 * B + z] = cmul(x[j2 * B + z], W.col2[z]);
      });
    });
    fft_sync<G>();
    static_for<E / B>([&](auto jc) {
      constexpr int j2 = decltype(jc)::value;
      static_for<B>([&](auto zc) {
        constexpr int z = decltype(zc)::value;
        bq2[G::ix(j2 * B * TF + z * C)] = x[j2 * B + z];
      });
    });
    fft_sync<G>();
  }
  {  // radix C over c: lane (q3, gamma, zeta), k1 = j3 C + q3
    const int q3 = (unsigned)t / (A * B), gamma = ((unsigned)t % (A * B)) / B, zeta = (unsigned)t % B;
    float2* const bq3 = buf + G::ix(q3 * TF + gamma * BC + zeta * C);
    static_for<E / C>([&](auto jc) {
      constexpr int j3 = decltype(jc)::value;
      static_for<C>([&](auto cc) {
        constexpr int ci = decltype(cc)::value;
        x[j3 * C + ci] = bq3[G::ix(j3 * C * TF + ci)];
      });
      dft_reg<C, -1, j3 * C>(x);
    });
  }
}

template <class G>
__device__ __forceinline__ void fft3_inverse(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  constexpr int E = G::E, TF = G::TF, A = G::A, B = G::B, C = G::C, BC = G::BC;
  {  // radix C over eta -> c
    const int q3 = (unsigned)t / (A * B), gamma = ((unsigned)t % (A * B)) / B, zeta = (unsigned)t % B;
    float2* const bq3 = buf + G::ix(q3 * TF + gamma * BC + zeta * C);
    static_for<E / C>([&](auto jc) {
      constexpr int j3 = decltype(jc)::value;
      dft_reg<C, +1, j3 * C>(x);
    });
    fft_sync<G>();
    static_for<E / C>([&](auto jc) {
      constexpr int j3 = decltype(jc)::value;
      static_for<C>([&](auto cc) {
        constexpr int ci = decltype(cc)::value;
        bq3[G::ix(j3 * C * TF + ci)] = x[j3 * C + ci];
      });
    });
    fft_sync<G>();
  }
  {  // radix B over zeta -> beta
    const int q2 = (unsigned)t / (A * C), gamma = ((unsigned)t % (A * C)) / C, c = (unsigned)t % C;
    float2* const bq2 = buf + G::ix(q2 * TF + gamma * BC + c);
    static_for<E / B>([&](auto jc) {
      constexpr int j2 = decltype(jc)::value;
      static_for<B>([&](auto zc) {
        constexpr int z = decltype(zc)::value;
        float2 v = bq2[G::ix(j2 * B * TF + z * C)];
        if constexpr (z > 0) v = cmulc(v, W.col2[z]);
        x[j2 * B + z] = v;
      });
      dft_reg<B, +1, j2 * B>(x);
    });
    fft_sync<G>();
    static_for<E / B>([&](auto jc) {
      constexpr int j2 = decltype(jc)::value;
      static_for<B>([&](auto bc) {
        constexpr int be = decltype(bc)::value;
        bq2[G::ix(j2 * B * TF + C * be)] = x[j2 * B + be];
      });
    });
    fft_sync<G>();
  }
  {  // radix A over gamma -> alpha
    const int tau = (unsigned)t % BC, q = (unsigned)t / BC;
    float2* const bq = buf + G::ix(q * TF + tau);
    static_for<E / A>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      static_for<A>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        float2 v = bq[G::ix(j * A * TF + g * BC)];
        if constexpr (g > 0) v = cmulc(v, W.col[g]);
        x[j * A + g] = v;
      });
      dft_reg<A, +1, j * A>(x);
    });
    fft_sync<G>();
    static_for<E / A>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      static_for<A>([&](auto ac) {
        constexpr int al = decltype(ac)::value;
        bq[G::ix(j * A * TF + BC * al)] = x[j * A + al];
      });
    });
    fft_sync<G>();
  }
  float2* const bt = buf + G::ix(t);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    x[k1] = W.template step2<k1>(bt[G::ix(k1 * TF)], true);
  });
  dft_reg<E, +1, 0>(x);
}

// Forward FFT of one slot, two exchanges: x in natural layout -> x in spectral
// layout. buf points at this slot's P-element LDS region; t is the lane within
// the slot.
template <class G>
__device__ __forceinline__ void fft2_forward(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  constexpr int E = G::E, TF = G::TF, A = G::A, B = G::B;
  dft_reg<E, -1, 0>(x);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    x[k1] = W.template step2<k1>(x[k1], false);
  });
  // exchange 1: [k1][n2]
  fft_sync<G>();
  float2* const bt = buf + G::ix(t);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    bt[G::ix(k1 * TF)] = x[k1];
  });
  fft_sync<G>();
  const int beta = (unsigned)t % B, q = (unsigned)t / B;
  float2* const bq = buf + G::ix(q * TF + beta);
  static_for<E / A>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    static_for<A>([&](auto ac) {
      constexpr int al = decltype(ac)::value;
      x[j * A + al] = bq[G::ix(j * A * TF + B * al)];
    });
    dft_reg<A, -1, j * A>(x);
    static_for<A>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g > 0) x[j * A + g] = cmul(x[j * A + g], W.col[g]);
    });
  });
  // exchange 2: [k1][gamma * B + beta]
  fft_sync<G>();
  static_for<E / A>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    static_for<A>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      bq[G::ix(j * A * TF + g * B)] = x[j * A + g];
    });
  });
  fft_sync<G>();
  const int gamma = (unsigned)t % A, q2 = (unsigned)t / A;
  float2* const bq2 = buf + G::ix(q2 * TF + gamma * B);
  static_for<E / B>([&](auto jc) {
    constexpr int j2 = decltype(jc)::value;
    static_for<B>([&](auto bc) {
      constexpr int be = decltype(bc)::value;
      x[j2 * B + be] = bq2[G::ix(j2 * B * TF + be)];
    });
    dft_reg<B, -1, j2 * B>(x);
  });
}

// Inverse FFT of one slot, two exchanges (unscaled): x in spectral layout -> x
// in natural layout.
template <class G>
__device__ __forceinline__ void fft2_inverse(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  constexpr int E = G::E, TF = G::TF, A = G::A, B = G::B;
  const int gamma = (unsigned)t % A, q2 = (unsigned)t / A;
  float2* const bq2 = buf + G::ix(q2 * TF + gamma * B);
  static_for<E / B>([&](auto jc) {
    constexpr int j2 = decltype(jc)::value;
    dft_reg<B, +1, j2 * B>(x);
  });
  fft_sync<G>();
  static_for<E / B>([&](auto jc) {
    constexpr int j2 = decltype(jc)::value;
    static_for<B>([&](auto bc) {
      constexpr int be = decltype(bc)::value;
      bq2[G::ix(j2 * B * TF + be)] = x[j2 * B + be];
    });
  });
  fft_sync<G>();
  const int beta = (unsigned)t % B, q = (unsigned)t / B;
  float2* const bq = buf + G::ix(q * TF + beta);
  static_for<E / A>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    static_for<A>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      float2 v = bq[G::ix(j * A * TF + g * B)];
      if constexpr (g > 0) v = cmulc(v, W.col[g]);
      x[j * A + g] = v;
    });
    dft_reg<A, +1, j * A>(x);
  });
  fft_sync<G>();
  static_for<E / A>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    static_for<A>([&](auto ac) {
      constexpr int al = decltype(ac)::value;
      bq[G::ix(j * A * TF + B * al)] = x[j * A + al];
    });
  });
  fft_sync<G>();
  float2* const bt = buf + G::ix(t);
  static_for<E>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    x[k1] = W.template step2<k1>(bt[G::ix(k1 * TF)], true);
  });
  dft_reg<E, +1, 0>(x);
}

template <class G>
__device__ __forceinline__ void fft_forward_g(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  if constexpr (G::THREE) fft3_forward<G>(x, buf, t, W);
  else fft2_forward<G>(x, buf, t, W);
}
template <class G>
__device__ __forceinline__ void fft_inverse_g(float2 (&x)[G::E], float2* buf, int t, const TwiddlesG<G>& W) {
  if constexpr (G::THREE) fft3_inverse<G>(x, buf, t, W);
  else fft2_inverse<G>(x, buf, t, W);
}

template <int P>
__device__ __forceinline__ void fft_forward(float2 (&x)[Geom<P>::E], float2* buf, int t, const WaveTwiddles<P>& W) {
  fft_forward_g<Geom<P>>(x, buf, t, W);
}
template <int P>
__device__ __forceinline__ void fft_inverse(float2 (&x)[Geom<P>::E], float2* buf, int t, const WaveTwiddles<P>& W) {
  fft_inverse_g<Geom<P>>(x, buf, t, W);
}

}  // namespace sq
