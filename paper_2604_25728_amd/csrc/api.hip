// api.hip - host side of libsqngd.so: argument validation, the batch plan
// kept in the caller's workspace, and the launch sequences of the C ABI
// declared in include/sqngd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "kernels.hip"

using namespace sq;

namespace {

std::atomic<int> g_last_hip{0};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fft_len(int N) {
  int P = 128;
  while (P < 2 * N - 1) P *= 2;
  return P;
}
int log2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

bool finite(float v) { return std::isfinite(v); }

// waves per block of the latency variant of the fused pass
// Latency variant of the fused pass: waves per block (M partners x units per
// block) are chosen per FFT length among the compiled shapes; the LDS of a
// block holds one P-point exchange buffer per wave (<= 64 KiB).
// (the automatic rule picks among these; a SPLIT hint may also ask for the
// smaller shapes below, kSplitExtra512 / kSplitExtra1024)
// (measured at M=2 N=512 F=129 with ROI weights: 19.1 us per pass with 8
// waves per block, 15.9 with 4, 17.5 with 2)
constexpr int kSplitShapes512[] = {8, 12, 16};
constexpr int kSplitShapes1024[] = {4, 8};
constexpr int kSplitExtra512[] = {4};
constexpr int kSplitExtra1024[] = {2};
constexpr int kMaxSplitWaves = 16;
// Pair form of the pass (one block per (row, Doppler bin, partner)) at FFT
// lengths 2048 and 4096: the rule takes it for groups of at most this many
// pairs (a few rounds of the chip), where one throughput block per unit
// would leave a partial second round of whole units; and at 4096 for groups
// whose problems have at most kPairMaxM4096 partners at any size: there the
// throughput pass holds one 8-wave block per CU (100 KB of LDS) and the pair
// form two, which outweighs its extra transform per pair (measured, M=2
// N=1200 F=129, 64 designs: pass 1405 -> 1198 us, iteration 3071 -> 2788 us;
// M=3, 16 designs: 1433 -> 1328 us; at M=4 the larger gradient reduction of
// F M partial rows per row cancels the faster pass).
constexpr int64_t kPairMaxBlocks = 2048;
// k_step2 launches of at most this many blocks finish each row in its last
// block; larger ones in a second launch (no device-scope fence per block).
// Measured at M=2 N=1200 L=16 F=129: 1-4 designs (10-40 blocks) 2-4 us per
// iteration faster in the last block, 8 designs (80) even, 16 (160) 18 us
// and 64 (640) 95 us faster with the second launch.
constexpr int64_t kStep2LastMaxBlocks = 96;
constexpr int kPairMaxM4096 = 3;
constexpr double kSplitMaxWaves = 8192.0;
constexpr int kNumCUs = 256;  // MI355X compute units: one block per CU is the aim
// the gradient reduction moves into k_step for groups of at least this many
// rows, or whose rows hold at most this many bytes of Doppler partials
constexpr int kFuseRows = kNumCUs / 2;
// throughput groups below this many blocks count as small for the one-launch rule
constexpr int kFuseSmallBlocks = 2 * 3 * kNumCUs;
constexpr int64_t kFuseRowBytes = 16384;

// Waves per split block for the problems of one FFT length: the compiled
// shape minimising (rounds of kNumCUs blocks) x (waves per block), i.e. the
// per-SIMD wave count of the slowest compute unit; ties go to fewer waves.
int choose_split_waves(int P, const sqngd_problem* probs, const std::vector<int>& ids, int forced) {
  std::vector<int> shapes;
  if (P == 512) shapes.assign(std::begin(kSplitShapes512), std::end(kSplitShapes512));
  else shapes.assign(std::begin(kSplitShapes1024), std::end(kSplitShapes1024));
  if (forced != 0) {
    if (P == 512) shapes.insert(shapes.end(), std::begin(kSplitExtra512), std::end(kSplitExtra512));
    else shapes.insert(shapes.end(), std::begin(kSplitExtra1024), std::end(kSplitExtra1024));
  }
  int best = 0;
  double best_cost = 0.0;
  for (size_t k = 0; k < shapes.size(); ++k) {
    const int wv = shapes[k];
    if (forced != 0 && wv != forced) continue;
    int64_t blocks = 0;
    bool fits = true;
    for (int id : ids) {
      const int M = probs[id].M;
      if (M > wv) fits = false;
      else blocks += (int64_t)M * ((probs[id].F + wv / M - 1) / (wv / M));
    }
    if (!fits) continue;
    const double cost = (double)((blocks + kNumCUs - 1) / kNumCUs) * wv;
    if (best == 0 || cost < best_cost) {
      best = wv;
      best_cost = cost;
    }
  }
  return best;
}

int validate_problem(const sqngd_problem& p) {
  if (p.M < 1 || p.N < 2 || p.L < 2 || p.F < 1) return SQNGD_E_INVALID_ARG;
  if (p.M > 16 || p.N > 2048 || p.L > 64 || p.F > 4096) return SQNGD_E_UNSUPPORTED;
  const double P = fft_len(p.N);
  if ((double)p.M * p.M * p.F * P >= 4294967296.0) return SQNGD_E_UNSUPPORTED;
  if (!finite(p.nu_min) || !finite(p.nu_max) || p.nu_min > p.nu_max) return SQNGD_E_INVALID_ARG;
  if (p.tau_lo < -(p.N - 1) || p.tau_hi > p.N - 1 || p.tau_lo > p.tau_hi) return SQNGD_E_INVALID_ARG;
  if (!finite(p.p) || p.p < 2.0f || p.p > 64.0f) return SQNGD_E_INVALID_ARG;
  if (!finite(p.snrl_target_db) || p.snrl_target_db < 0.0f) return SQNGD_E_INVALID_ARG;
  if (!finite(p.w_psl) || !finite(p.w_snrl) || p.w_psl < 0.0f || p.w_snrl < 0.0f) return SQNGD_E_INVALID_ARG;
  if (!finite(p.temperature) || p.temperature <= 0.0f) return SQNGD_E_INVALID_ARG;
  if (p.sq_mode != SQNGD_SQ_PHASE_MEAN && p.sq_mode != SQNGD_SQ_PHASOR_MEAN) return SQNGD_E_INVALID_ARG;
  if (p.auto_mask != SQNGD_MASK_TAU0 && p.auto_mask != SQNGD_MASK_MAINLOBE) return SQNGD_E_INVALID_ARG;
  if (p.schedule != SQNGD_SCHED_AUTO && p.schedule != SQNGD_SCHED_THROUGHPUT && p.schedule != SQNGD_SCHED_SPLIT2 &&
      p.schedule != SQNGD_SCHED_SPLIT4 && p.schedule != SQNGD_SCHED_SPLIT8 && p.schedule != SQNGD_SCHED_SPLIT12 &&
      p.schedule != SQNGD_SCHED_SPLIT16 && p.schedule != SQNGD_SCHED_GROUPED && p.schedule != SQNGD_SCHED_FUSED &&
      p.schedule != SQNGD_SCHED_PAIR)
    return SQNGD_E_INVALID_ARG;
  return SQNGD_OK;
}

int validate_batch(const sqngd_problem* probs, int32_t nprob) {
  if (probs == nullptr || nprob < 1 || nprob > (1 << 20)) return SQNGD_E_INVALID_ARG;
  for (int i = 0; i < nprob; ++i) {
    int rc = validate_problem(probs[i]);
    if (rc != SQNGD_OK) return rc;
  }
  return SQNGD_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Host copy of a batch plan: the bytes uploaded to the start of the workspace.
struct Plan {
  WsHeader hdr{};
  std::vector<char> bytes;  // [0, hdr.spec): header, plans, tables
  std::vector<ProbPlan> plans;
  int group_phlog[kNumPGroups];
  int group_wv[kNumPGroups];  // waves per block of the latency variant (split groups)
  bool group_split[kNumPGroups];  // the group's pass runs as k_pass_split
  bool group_pair[kNumPGroups];   // ... as k_pass_pair (one block per pair)
  // finalize of the optimiser steps: 0 = k_final, else k_step with this
  // bound on the logit levels per lane
  int group_step[kNumPGroups];
  bool group_fuse[kNumPGroups];  // k_step reduces the gradient rows itself (no k_grad launch)
  bool all_step = true;  // every group runs k_step: the step counter advances in the next pass
  int step2_split[kNumPGroups] = {};  // k_step2 blocks per row (FFT lengths 2048, 4096): longest row in 256-chip blocks
  int maxN = 0;
  // throughput groups (bit g: FFT length 128 << g) that share one launch
  // (k_pass_multi), 0 for one launch per group
  int fuse_mask = 0;
  uint64_t hash = 0;
  std::vector<sqngd_problem> src;  // the descriptors the plan was built from
  // ROI weights attached by sqngd_set_roi_weights (device, packed per
  // problem), or null for w = 1; read when a pass is enqueued
  mutable const float* roi_w = nullptr;
  // per-problem stop mask attached by sqngd_set_stop_mask (device), or null;
  // read when an optimiser step is enqueued
  mutable const int32_t* frozen = nullptr;
};

uint64_t fnv1a(const void* data, size_t n) {
  const unsigned char* c = (const unsigned char*)data;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::unique_ptr<Plan> build_plan(const sqngd_problem* probs, int32_t nprob) {
  auto pl = std::make_unique<Plan>();
  WsHeader& H = pl->hdr;
  H.magic = kWsMagic;
  H.nprob = nprob;
  pl->plans.resize(nprob);
  std::vector<int> gprob[kNumPGroups];
  // Each FFT-length group takes the throughput pass or, at P = 512 or 1024,
  // the latency variant (one wave per Doppler bin and partner). A group's
  // hint is the first non-AUTO schedule among its problems. AUTO: the latency
  // variant for small groups, and at P = 1024 for groups whose problems all
  // have M <= 2 (the throughput pass amortises its per-unit self and adjoint
  // transforms over only two partners there; 64 M=2 N=512 designs: 12.0
  // against 16.2 ms per transmit-side iteration, 64 M=4 N=512: 2.15 against
  // 1.81 ms).
  std::vector<int> ids_p[kNumPGroups];
  for (int i = 0; i < nprob; ++i) ids_p[log2i(fft_len(probs[i].N)) - kMinLogP].push_back(i);
  bool ask_grouped = false, ask_fused = false;
  for (int i = 0; i < nprob; ++i) {
    ask_grouped |= probs[i].schedule == SQNGD_SCHED_GROUPED;
    ask_fused |= probs[i].schedule == SQNGD_SCHED_FUSED;
  }
  for (int g = 0; g < kNumPGroups; ++g) {
    pl->group_wv[g] = 0;
    pl->group_split[g] = false;
    pl->group_pair[g] = false;
    if (ids_p[g].empty()) continue;
    const int P = 1 << (g + kMinLogP);
    int hint = SQNGD_SCHED_AUTO;
    bool can = P == 512 || P == 1024, pairs2 = P == 1024;
    int mmax = 0;
    double pair_waves = 0.0;
    for (int id : ids_p[g]) {
      if (hint == SQNGD_SCHED_AUTO) hint = probs[id].schedule;
      if (probs[id].M > kMaxSplitWaves) can = false;
      if (probs[id].M > 2) pairs2 = false;
      mmax = std::max(mmax, (int)probs[id].M);
      pair_waves += (double)probs[id].M * probs[id].M * probs[id].F;
    }
    if (P >= 2048) {
      // pair blocks: every problem's F M partial rows must fit the finalize
      bool fit = true;
      for (int id : ids_p[g]) fit = fit && (int64_t)probs[id].F * probs[id].M <= 4096;
      // a latency-variant hint (FFT length 512 / 1024 only) acts as AUTO here
      const bool rule = hint == SQNGD_SCHED_AUTO || (hint >= SQNGD_SCHED_SPLIT2 && hint <= SQNGD_SCHED_SPLIT16);
      const bool few = pair_waves <= (double)kPairMaxBlocks || (P == 4096 && mmax <= kPairMaxM4096);
      pl->group_pair[g] = fit && (hint == SQNGD_SCHED_PAIR || (rule && few));
      continue;
    }
    bool split = can;
    if (hint == SQNGD_SCHED_AUTO) split = can && (pair_waves <= kSplitMaxWaves || pairs2);
    if (hint == SQNGD_SCHED_THROUGHPUT || hint == SQNGD_SCHED_GROUPED || hint == SQNGD_SCHED_FUSED) split = false;
    if (!split) continue;
    // a forced shape that does not apply falls back to the rule's shape
    const int forced = hint >= SQNGD_SCHED_SPLIT2 && hint <= SQNGD_SCHED_SPLIT16 ? hint : 0;
    int wv = choose_split_waves(P, probs, ids_p[g], forced);
    if (wv == 0 && forced != 0) wv = choose_split_waves(P, probs, ids_p[g], 0);
    pl->group_wv[g] = wv;
    pl->group_split[g] = wv != 0;
  }
  // One launch for the throughput groups of FFT length <= 2048 when asked
  // (FUSED), or by the rule when every such group is small (fewer blocks
  // than two rounds of the chip at three blocks per CU: its launch would run
  // mostly as a tail); GROUPED keeps one launch per group. The groups must
  // agree on the p-norm's instantiation.
  {
    int mask = 0, phl = -2, nseg = 0;
    bool small = true, same = true;
    for (int g = 0; g < kNumPGroups - 1; ++g) {
      if (ids_p[g].empty() || pl->group_split[g] || pl->group_pair[g]) continue;
      const int P = 1 << (g + kMinLogP);
      int64_t blocks = 0;
      int gphl = -2;
      for (int id : ids_p[g]) {
        int k = -1;
        for (int e = 0; e <= 5; ++e)
          if (probs[id].p == 2.0f * (float)(1 << e)) k = e;
        gphl = (gphl == -2 || gphl == k) ? k : -1;
        blocks += (int64_t)probs[id].M * ((probs[id].F + pass_upb(P) - 1) / pass_upb(P));
      }
      if (blocks >= (int64_t)kFuseSmallBlocks) small = false;
      if (phl != -2 && phl != gphl) same = false;
      phl = gphl;
      mask |= 1 << g;
      ++nseg;
    }
    const bool fuse = nseg >= 2 && same && !ask_grouped && (ask_fused || small);
    pl->fuse_mask = fuse ? mask : 0;
  }
  int64_t off_z = 0, off_w = 0, off_state = 0, off_cube = 0, off_rw = 0, spec = 0, unit = 0, upart = 0;
  int rows = 0;
  for (int i = 0; i < nprob; ++i) {
    const sqngd_problem& p = probs[i];
    ProbPlan& q = pl->plans[i];
    std::memset(&q, 0, sizeof(q));
    q.M = p.M;
    q.N = p.N;
    q.L = p.L;
    q.F = p.F;
    q.P = fft_len(p.N);
    q.logP = log2i(q.P);
    q.tau_lo = p.tau_lo;
    q.tau_hi = p.tau_hi;
    q.nu_min = (double)p.nu_min;
    q.dnu = p.F > 1 ? ((double)p.nu_max - (double)p.nu_min) / (double)(p.F - 1) : 0.0;
    q.cut_lo = 0;
    q.cut_hi = p.F;
    if (p.auto_mask == SQNGD_MASK_MAINLOBE) {
      // the bins the pass modulates with |nu_f| < 1 (nu_f increases with f,
      // so they are one run [cut_lo, cut_hi), possibly empty)
      q.cut_lo = q.cut_hi = 0;
      for (int f = 0; f < p.F; ++f)
        if (std::fabs(q.nu_min + (double)f * q.dnu) < 1.0) {
          if (q.cut_hi == 0) q.cut_lo = f;
          q.cut_hi = f + 1;
        }
    }
    q.p = p.p;
    q.p_tar = (float)std::pow(10.0, -(double)p.snrl_target_db / 20.0);
    q.w_psl = p.w_psl;
    q.w_snrl = p.w_snrl;
    q.temperature = p.temperature;
    q.inv_NP = (float)(1.0 / ((double)p.N * (double)q.P));
    q.sq_mode = p.sq_mode;
    q.ph_log = -1;
    for (int k = 0; k <= 5; ++k)
      if (p.p == 2.0f * (float)(1 << k)) q.ph_log = k;
    q.units = p.M * p.F;
    q.row0 = rows;
    {
      int upb;  // Doppler bins per fused-pass block
      if (pl->group_pair[q.logP - kMinLogP]) {
        upb = 0;  // one block per (Doppler bin, partner): wpr = F M below
      } else if (pl->group_split[q.logP - kMinLogP]) {
        upb = pl->group_wv[q.logP - kMinLogP] / p.M;
      } else if ((pl->fuse_mask >> (q.logP - kMinLogP)) & 1) {
        upb = pass_upb(q.P, 4);  // four-wave blocks of the one-launch pass
      } else {
        upb = pass_upb(q.P);
      }
      q.wpr = upb == 0 ? p.F * p.M : (p.F + upb - 1) / upb;
      // the latency pass reads the spectra in the one-wave layout the
      // producers compute them in (the layouts coincide below P = 1024)
      q.spec_wave = pl->group_split[q.logP - kMinLogP] && q.P >= 1024 ? 1 : 0;
    }
    q.units = p.M * q.wpr;
    q.off_z = off_z;
    q.off_w = off_w;
    q.off_state = off_state;
    q.off_cube = off_cube;
    q.off_rw = off_rw;
    q.ws_spec = spec;
    q.ws_unit = unit;
    q.ws_upart = upart;
    off_z += (int64_t)p.M * p.N * p.L;
    off_w += (int64_t)p.M * p.N;
    off_state += SQNGD_ADAM_FLOATS(p.M, p.N, p.L);
    off_cube += (int64_t)p.M * p.M * p.F * (2 * p.N - 1);
    off_rw += (int64_t)p.F * (2 * p.N - 1);
    spec += (int64_t)p.M * q.P;
    unit += q.units;
    upart += (int64_t)q.units * p.N;  // one partial row per fused-pass block
    rows += p.M;
    gprob[q.logP - kMinLogP].push_back(i);
  }
  H.nrows = rows;
  // table region
  size_t off = align_up(sizeof(WsHeader));
  H.plans = (int64_t)off;
  off = align_up(off + sizeof(ProbPlan) * nprob);
  std::vector<std::vector<int32_t>> wave(kNumPGroups), rwave(kNumPGroups);
  for (int g = 0; g < kNumPGroups; ++g) {
    const int P = 1 << (g + kMinLogP);
    const int TF = P >= 512 ? 64 : P / 8;
    const int slots = 64 / TF;
    H.group_n[g] = (int32_t)gprob[g].size();
    int wsum = 0, rsum = 0;
    int phl = -2;
    for (int id : gprob[g]) {
      wave[g].push_back(wsum);
      rwave[g].push_back(rsum);
      wsum += pl->plans[id].M * pl->plans[id].wpr;
      rsum += (pl->plans[id].M + slots - 1) / slots;
      phl = (phl == -2 || phl == pl->plans[id].ph_log) ? pl->plans[id].ph_log : -1;
    }
    wave[g].push_back(wsum);
    rwave[g].push_back(rsum);
    H.group_waves[g] = wsum;
    H.group_rwaves[g] = rsum;
    pl->group_phlog[g] = phl;
    {
      // k_step holds N <= P / 2 chips with tpc lanes each (P <= 1024),
      // k_step2 one chip per lane, a row over 256-chip blocks (P >= 2048);
      // rows with more than 16 logit levels per lane use k_final
      const int tpc = P >= 2048 ? 1 : step_tpc(P);
      int lv = 0;
      for (int id : gprob[g]) lv = std::max(lv, tpc > 0 ? (pl->plans[id].L + tpc - 1) / tpc : 1 << 30);
      const int mode = tpc < 1 ? 0 : (lv <= 4 ? 4 : (lv <= 16 ? 16 : 0));
      if (P >= 2048)
        for (int id : gprob[g])
          pl->step2_split[g] = std::max(pl->step2_split[g], (pl->plans[id].N + kStep2Threads - 1) / kStep2Threads);
      pl->group_step[g] = mode;
      if (!gprob[g].empty() && mode == 0) pl->all_step = false;
      // k_step reduces the rows' Doppler partials itself when that takes at
      // most two load rounds per lane and either the rows alone fill half the
      // chip or a row's partials are small (one block reading a large row is
      // slower than k_grad's many blocks reading it together), and only with
      // at most 4 logit levels per lane: with 16 the fused form holds about
      // 210 VGPRs, one block per CU, and k_grad + k_step measured faster
      // (uneven 64 x 8 batch: 14.695 -> 14.66 ms per step)
      int ne = 0, nr = 0;
      int64_t row_bytes = 0;
      for (int id : gprob[g]) {
        const ProbPlan& q = pl->plans[id];
        ne = std::max(ne, q.wpr);
        nr += q.M;
        row_bytes = std::max(row_bytes, (int64_t)8 * q.wpr * q.N);
      }
      pl->group_fuse[g] = mode == 4 && P <= 1024 && ne <= 2 * step_tpc(P) * step_fg_loads(P) &&
                          (nr >= kFuseRows || row_bytes <= kFuseRowBytes);
    }
    H.group_prob[g] = (int64_t)off;
    off = align_up(off + 4 * gprob[g].size());
    H.group_wave[g] = (int64_t)off;
    off = align_up(off + 4 * wave[g].size());
    H.group_rwave[g] = (int64_t)off;
    off = align_up(off + 4 * rwave[g].size());
    int nr = 0;
    for (int id : gprob[g]) nr += pl->plans[id].M;
    H.group_nrows[g] = nr;
    H.group_rows[g] = (int64_t)off;
    off = align_up(off + 4 * (size_t)nr);
  }
  H.row_prob = (int64_t)off;
  off = align_up(off + 4 * (size_t)rows);
  // counters live in the uploaded table region, so the upload zeroes them
  H.counters = (int64_t)off;
  off = align_up(off + 4 * kNumCounters);
  // k_step2's per-row scratch, shared by the FFT-length-2048 and -4096 groups (stream-ordered launches)
  const int rows_split = std::max(H.group_nrows[kNumPGroups - 1], H.group_nrows[kNumPGroups - 2]);
  H.rowsync = (int64_t)off;
  off = align_up(off + 4 * (size_t)rows_split);
  const size_t table_bytes = off;
  H.spec = (int64_t)off;
  off = align_up(off + 8 * (size_t)spec);
  H.wself = (int64_t)off;
  off = align_up(off + 8 * (size_t)off_w);
  H.wpart = (int64_t)off;
  off = align_up(off + 8 * (size_t)off_w);
  H.ustat = (int64_t)off;
  off = align_up(off + sizeof(UnitStat) * (size_t)unit);
  H.upart = (int64_t)off;
  off = align_up(off + 8 * (size_t)upart);
  H.snrl = (int64_t)off;
  off = align_up(off + 2 * 16 * (size_t)rows);
  H.gbuf = (int64_t)off;
  off = align_up(off + 8 * (size_t)off_w);
  H.pflag = (int64_t)off;
  off = align_up(off + 4 * (size_t)nprob);
  H.rowpart = (int64_t)off;
  off = align_up(off + 16 * (size_t)kStep2MaxSplit * rows_split);
  H.total = (int64_t)off;
  int maxN = 0;
  for (int i = 0; i < nprob; ++i) maxN = probs[i].N > maxN ? probs[i].N : maxN;
  pl->maxN = maxN;

  pl->bytes.assign(table_bytes, 0);
  char* b = pl->bytes.data();
  std::memcpy(b + H.plans, pl->plans.data(), sizeof(ProbPlan) * nprob);
  for (int g = 0; g < kNumPGroups; ++g) {
    if (!gprob[g].empty()) std::memcpy(b + H.group_prob[g], gprob[g].data(), 4 * gprob[g].size());
    std::memcpy(b + H.group_wave[g], wave[g].data(), 4 * wave[g].size());
    std::memcpy(b + H.group_rwave[g], rwave[g].data(), 4 * rwave[g].size());
    std::vector<int32_t> gr;
    for (int id : gprob[g])
      for (int m = 0; m < pl->plans[id].M; ++m) gr.push_back(pl->plans[id].row0 + m);
    if (!gr.empty()) std::memcpy(b + H.group_rows[g], gr.data(), 4 * gr.size());
  }
  std::vector<int32_t> rp(rows);
  for (int i = 0; i < nprob; ++i)
    for (int m = 0; m < probs[i].M; ++m) rp[pl->plans[i].row0 + m] = i;
  std::memcpy(b + H.row_prob, rp.data(), 4 * rp.size());
  std::memcpy(b, &H, sizeof(WsHeader));
  pl->hash = fnv1a(b, table_bytes);
  pl->src.assign(probs, probs + nprob);
  return pl;
}

// Workspace registry: the plan each workspace was last initialised for. The
// device copy of a plan is written through kernel arguments (put_plan), so no
// host buffer has to outlive the call that uploads it: re-initialising a
// workspace frees its previous plan, and sqngd_workspace_release drops it.
std::mutex g_mu;
std::unordered_map<const void*, std::unique_ptr<Plan>> g_ws;

int hip_fail(hipError_t e) {
  g_last_hip.store((int)e);
  return SQNGD_E_HIP;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SQNGD_OK : hip_fail(e);
}

// Bytes carried by value in a kernel's arguments: the runtime copies the
// arguments at launch, so the host buffer they came from may go away at once
// (no host-memory lifetime to track, no copy engine, nothing allocated).
constexpr int kPutWords = 960;
struct PutArgs {
  uint32_t* dst;
  int32_t nwords, pad;
  uint32_t w[kPutWords];
};
static_assert(sizeof(PutArgs) <= 4096, "kernel argument limit");

__global__ __launch_bounds__(256) void k_put_words(PutArgs a) {
  for (int i = threadIdx.x; i < a.nwords; i += 256) a.dst[i] = a.w[i];
}

// Writes the plan's table bytes (header, problem plans, work tables, zeroed
// counters) to the start of the workspace `dst` on `s`.
int put_plan(const Plan& pl, void* dst, hipStream_t s) {
  const size_t nb = pl.bytes.size();  // a multiple of the 256-byte alignment
  const uint32_t* src = (const uint32_t*)pl.bytes.data();
  const size_t nw = nb / 4;
  for (size_t off = 0; off < nw; off += kPutWords) {
    PutArgs a;
    a.dst = (uint32_t*)dst + off;
    a.nwords = (int32_t)std::min<size_t>(kPutWords, nw - off);
    a.pad = 0;
    std::memcpy(a.w, src + off, 4 * (size_t)a.nwords);
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, a);
  }
  return check_launch();
}

// Validates the batch and the workspace; on success *out is the plan the
// workspace holds. The descriptors are compared with the ones the workspace
// was initialised with (no plan is rebuilt per call).
int lookup(const sqngd_problem* probs, int32_t nprob, void* ws, size_t ws_bytes, const Plan** out) {
  int rc = validate_batch(probs, nprob);
  if (rc != SQNGD_OK) return rc;
  if (ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(ws, kAlign)) return SQNGD_E_ALIGN;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(ws);
  if (it == g_ws.end()) return SQNGD_E_WORKSPACE;
  const Plan& pl = *it->second;
  if (pl.src.size() != (size_t)nprob || std::memcmp(pl.src.data(), probs, sizeof(sqngd_problem) * nprob) != 0)
    return SQNGD_E_WORKSPACE;
  if (ws_bytes < (size_t)pl.hdr.total) return SQNGD_E_WORKSPACE;
  *out = &pl;
  return SQNGD_OK;
}

struct Ptrs {
  char* base;
  const ProbPlan* plans;
  const int32_t* row_prob;
  int32_t* counters;
  float2* spec;
  float2* wself;
  float2* wpart;
  UnitStat* ustat;
  float2* upart;
  float4* snrl;
  float2* gbuf;
  int32_t* pflag;
  int32_t* rowsync;
  float4* rowpart;
};

Ptrs ptrs(const Plan& pl, void* ws) {
  char* b = (char*)ws;
  const WsHeader& H = pl.hdr;
  return Ptrs{b,
              (const ProbPlan*)(b + H.plans),
              (const int32_t*)(b + H.row_prob),
              (int32_t*)(b + H.counters),
              (float2*)(b + H.spec),
              (float2*)(b + H.wself),
              (float2*)(b + H.wpart),
              (UnitStat*)(b + H.ustat),
              (float2*)(b + H.upart),
              (float4*)(b + H.snrl),
              (float2*)(b + H.gbuf),
              (int32_t*)(b + H.pflag),
              (int32_t*)(b + H.rowsync),
              (float4*)(b + H.rowpart)};
}

// ----------------------------------------------------------- launch helpers

template <int P>
void launch_prep_p(const PrepArgs& a, int waves, hipStream_t s) {
  hipLaunchKernelGGL(k_prep<P>, dim3(waves), dim3(64), 0, s, a);
}

// Partner spectra of a group whose spectra k_rowspec computes (P >= 2048).
template <int P>
void launch_rowspec_p(const Plan& pl, const Ptrs& w, int g, const float2* src, hipStream_t s) {
  RowSpecArgs r{};
  r.plans = w.plans;
  r.rows = (const int32_t*)(w.base + pl.hdr.group_rows[g]);
  r.row_prob = w.row_prob;
  r.src = src;
  r.spec = w.spec;
  r.single = pl.hdr.nprob == 1;
  r.one = pl.plans[0];
  hipLaunchKernelGGL(k_rowspec<P>, dim3(pl.hdr.group_nrows[g]), dim3(64 * PassGeom<P>::WAVES), 0, s, r);
}
void launch_rowspec(const Plan& pl, const Ptrs& w, int g, const float2* src, hipStream_t s) {
  if (g + kMinLogP == 11) launch_rowspec_p<2048>(pl, w, g, src, s);
  else launch_rowspec_p<4096>(pl, w, g, src, s);
}

void launch_prep(const Plan& pl, const Ptrs& w, PrepArgs a, hipStream_t s) {
  a.plans = w.plans;
  a.spec = w.spec;
  a.wself = w.wself;
  a.wpart = w.wpart;
  if (a.snrl == nullptr) a.snrl = w.snrl;
  a.single = pl.hdr.nprob == 1;
  a.one = pl.plans[0];
  for (int g = 0; g < kNumPGroups; ++g) {
    if (pl.hdr.group_n[g] == 0) continue;
    a.gprob = (const int32_t*)(w.base + pl.hdr.group_prob[g]);
    a.grwave = (const int32_t*)(w.base + pl.hdr.group_rwave[g]);
    a.gn = pl.hdr.group_n[g];
    const int waves = pl.hdr.group_rwaves[g];
    switch (g) {
      case 0: launch_prep_p<128>(a, waves, s); break;
      case 1: launch_prep_p<256>(a, waves, s); break;
      case 2: launch_prep_p<512>(a, waves, s); break;
      case 3: launch_prep_p<1024>(a, waves, s); break;
      default:  // P >= 2048: a block per row; the spectra by k_rowspec below
        a.rows = (const int32_t*)(w.base + pl.hdr.group_rows[g]);
        a.row_prob = w.row_prob;
        hipLaunchKernelGGL(k_prep_row, dim3(pl.hdr.group_nrows[g]), dim3(kPrepRowThreads), 0, s, a);
        break;
    }
    if (g + kMinLogP >= 11)
      launch_rowspec(pl, w, g,
                     a.mode == PREP_A_HARD    ? w.wpart
                     : a.mode == PREP_A_SELF  ? w.wself
                     : a.mode == PREP_A_GIVEN ? a.s_given
                                              : a.h,
                     s);
  }
}

// Measurement hook state (see sqngd_profile_enable).
struct Profiler {
  std::mutex mu;
  std::vector<hipEvent_t> ev;  // 2 per launch
  std::vector<int32_t> mask;   // per launch: bit g set for each FFT-length group (P = 128 << g) it covers
  int max = 0, used = 0, repeat = 1;
} g_prof;

// A profiling slot for the next pass launch on s (-1: not profiled); records
// the start event.
int prof_begin(hipStream_t s, int32_t mask);
void prof_end(int slot, hipStream_t s);

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Weighted launches (ROI weights attached) have p = 16 (squarings) and
// general-p instantiations.
template <int P, int WV>
void launch_split_wv(const PassArgs& a, int phlog, int blocks, hipStream_t s) {
  const dim3 block(64 * WV);
  if (a.roi_w != nullptr && phlog == 3)
    hipLaunchKernelGGL((k_pass_split<P, 3, WV, true>), dim3(blocks), block, 0, s, a);
  else if (a.roi_w != nullptr) hipLaunchKernelGGL((k_pass_split<P, -1, WV, true>), dim3(blocks), block, 0, s, a);
  else if (phlog == 3) hipLaunchKernelGGL((k_pass_split<P, 3, WV, false>), dim3(blocks), block, 0, s, a);
  else if (phlog == 2) hipLaunchKernelGGL((k_pass_split<P, 2, WV, false>), dim3(blocks), block, 0, s, a);
  else hipLaunchKernelGGL((k_pass_split<P, -1, WV, false>), dim3(blocks), block, 0, s, a);
}

void launch_split(int P, int wv, const PassArgs& a, int phlog, int blocks, hipStream_t s) {
  if (P == 1024) {
    if (wv == 2) launch_split_wv<1024, 2>(a, phlog, blocks, s);
    else if (wv == 4) launch_split_wv<1024, 4>(a, phlog, blocks, s);
    else launch_split_wv<1024, 8>(a, phlog, blocks, s);
  } else if (wv == 4) launch_split_wv<512, 4>(a, phlog, blocks, s);
  else if (wv == 12) launch_split_wv<512, 12>(a, phlog, blocks, s);
  else if (wv == 16) launch_split_wv<512, 16>(a, phlog, blocks, s);
  else launch_split_wv<512, 8>(a, phlog, blocks, s);
}

template <int P>
void launch_pair_p(const PassArgs& a, int phlog, int blocks, hipStream_t s) {
  const dim3 block(64 * PassGeom<P>::WAVES);
  if (a.roi_w != nullptr && phlog == 3) hipLaunchKernelGGL((k_pass_pair<P, 3, true>), dim3(blocks), block, 0, s, a);
  else if (a.roi_w != nullptr) hipLaunchKernelGGL((k_pass_pair<P, -1, true>), dim3(blocks), block, 0, s, a);
  else if (phlog == 3) hipLaunchKernelGGL((k_pass_pair<P, 3, false>), dim3(blocks), block, 0, s, a);
  else if (phlog == 2) hipLaunchKernelGGL((k_pass_pair<P, 2, false>), dim3(blocks), block, 0, s, a);
  else hipLaunchKernelGGL((k_pass_pair<P, -1, false>), dim3(blocks), block, 0, s, a);
}

template <int P>
void launch_pass_p(const PassArgs& a, int phlog, int waves, hipStream_t s) {
  const dim3 block(64 * pass_waves(P));
  if (a.roi_w != nullptr && phlog == 3) hipLaunchKernelGGL((k_pass<P, 3, true>), dim3(waves), block, 0, s, a);
  else if (a.roi_w != nullptr) hipLaunchKernelGGL((k_pass<P, -1, true>), dim3(waves), block, 0, s, a);
  else if (phlog == 3) hipLaunchKernelGGL((k_pass<P, 3, false>), dim3(waves), block, 0, s, a);
  else if (phlog == 2) hipLaunchKernelGGL((k_pass<P, 2, false>), dim3(waves), block, 0, s, a);
  else hipLaunchKernelGGL((k_pass<P, -1, false>), dim3(waves), block, 0, s, a);
}

void launch_multi(const MultiArgs& m, int phl, hipStream_t s) {
  const dim3 grid(m.base[m.nseg]), block(256);
  // weighted launches have p = 16 (squarings) and general-p instantiations
  if (m.a.roi_w != nullptr && phl == 3) hipLaunchKernelGGL((k_pass_multi<3, true>), grid, block, 0, s, m);
  else if (m.a.roi_w != nullptr) hipLaunchKernelGGL((k_pass_multi<-1, true>), grid, block, 0, s, m);
  else if (phl == 3) hipLaunchKernelGGL((k_pass_multi<3, false>), grid, block, 0, s, m);
  else if (phl == 2) hipLaunchKernelGGL((k_pass_multi<2, false>), grid, block, 0, s, m);
  else hipLaunchKernelGGL((k_pass_multi<-1, false>), grid, block, 0, s, m);
}

int prof_begin(hipStream_t s, int32_t mask) {
  int slot = -1;
  if (g_prof.max > 0 && !stream_capturing(s)) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (g_prof.used < g_prof.max) {
      slot = g_prof.used++;
      g_prof.mask[slot] = mask;
    }
  }
  if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot], s);
  return slot;
}

void prof_end(int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], s);
}

void launch_pass(const Plan& pl, const Ptrs& w, PassArgs a, hipStream_t s) {
  a.plans = w.plans;
  a.roi_w = pl.roi_w;
  a.spec = w.spec;
  a.ustat = w.ustat;
  a.upart = w.upart;
  a.single = pl.hdr.nprob == 1;
  a.one = pl.plans[0];
  // The throughput groups the plan fused share one launch, longest FFT
  // length first.
  int32_t multi_mask = 0;
  MultiArgs m{};
  if (pl.fuse_mask != 0) {
    int phl = -2, nseg = 0, blocks = 0;
    for (int g = 4; g >= 0; --g) {
      if (!((pl.fuse_mask >> g) & 1)) continue;
      phl = pl.group_phlog[g];
      m.logp[nseg] = g + kMinLogP;
      m.base[nseg] = blocks;
      m.gprob[nseg] = (const int32_t*)(w.base + pl.hdr.group_prob[g]);
      m.gwave[nseg] = (const int32_t*)(w.base + pl.hdr.group_wave[g]);
      m.gn[nseg] = pl.hdr.group_n[g];
      blocks += pl.hdr.group_waves[g];
      ++nseg;
    }
    if (nseg >= 2) {
      m.nseg = nseg;
      m.base[nseg] = blocks;
      for (int i = 0; i < nseg; ++i) multi_mask |= 1 << (m.logp[i] - kMinLogP);
      m.a = a;
      m.a.single = 0;
      const int slot = prof_begin(s, multi_mask);
      const int reps = slot >= 0 ? g_prof.repeat : 1;
      for (int rep = 0; rep < reps; ++rep, m.a.bump = nullptr) launch_multi(m, phl, s);
      prof_end(slot, s);
      a.bump = nullptr;
    }
  }
  for (int g = 0; g < kNumPGroups; ++g) {
    if (pl.hdr.group_n[g] == 0 || (multi_mask >> g) & 1) continue;
    a.gprob = (const int32_t*)(w.base + pl.hdr.group_prob[g]);
    a.gwave = (const int32_t*)(w.base + pl.hdr.group_wave[g]);
    a.gn = pl.hdr.group_n[g];
    const int waves = pl.hdr.group_waves[g];
    const int phl = pl.group_phlog[g];
    const int slot = prof_begin(s, 1 << g);
    const int reps = slot >= 0 ? g_prof.repeat : 1;
    for (int rep = 0; rep < reps; ++rep, a.bump = nullptr) {
      if (pl.group_pair[g]) {
        if (g + kMinLogP == 11) launch_pair_p<2048>(a, phl, waves, s);
        else launch_pair_p<4096>(a, phl, waves, s);
      } else if (pl.group_split[g]) {
        launch_split(1 << (g + kMinLogP), pl.group_wv[g], a, phl, waves, s);
      } else {
        switch (g) {
          case 0: launch_pass_p<128>(a, phl, waves, s); break;
          case 1: launch_pass_p<256>(a, phl, waves, s); break;
          case 2: launch_pass_p<512>(a, phl, waves, s); break;
          case 3: launch_pass_p<1024>(a, phl, waves, s); break;
          case 4: launch_pass_p<2048>(a, phl, waves, s); break;
          default: launch_pass_p<4096>(a, phl, waves, s); break;
        }
      }
    }
    prof_end(slot, s);
    a.bump = nullptr;  // the first kernel of the pass advances the counter
  }
}

template <int P, bool FG>
void launch_step_pf(const FinArgs& a, int lv, dim3 grid, hipStream_t s) {
  const dim3 block(step_threads(P));
  if (a.mode == FIN_STEP_A) {
    if (lv == 4) hipLaunchKernelGGL((k_step<P, FIN_STEP_A, 4, FG>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step<P, FIN_STEP_A, 16, FG>), grid, block, 0, s, a);
  } else {
    if (lv == 4) hipLaunchKernelGGL((k_step<P, FIN_STEP_B, 4, FG>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step<P, FIN_STEP_B, 16, FG>), grid, block, 0, s, a);
  }
}
// FFT lengths 2048 and 4096: each row over split blocks of 256 chips, gradient rows
// from k_grad; the row's last block finishes it when the launch has at most
// kStep2LastMaxBlocks blocks, else k_step2_rows in a second launch.
template <int MODE, bool LAST>
void launch_step2_m(const FinArgs& a, int lv, dim3 grid, hipStream_t s) {
  if (lv == 4) hipLaunchKernelGGL((k_step2<MODE, 4, LAST>), grid, dim3(kStep2Threads), 0, s, a);
  else hipLaunchKernelGGL((k_step2<MODE, 16, LAST>), grid, dim3(kStep2Threads), 0, s, a);
}
void launch_step2(const FinArgs& a, int lv, int nrows, hipStream_t s) {
  const dim3 grid(nrows * a.split);
  const bool last = (int64_t)nrows * a.split <= kStep2LastMaxBlocks;
  if (a.mode == FIN_STEP_A) {
    if (last) launch_step2_m<FIN_STEP_A, true>(a, lv, grid, s);
    else launch_step2_m<FIN_STEP_A, false>(a, lv, grid, s);
  } else {
    if (last) launch_step2_m<FIN_STEP_B, true>(a, lv, grid, s);
    else launch_step2_m<FIN_STEP_B, false>(a, lv, grid, s);
  }
  if (!last) {
    if (a.mode == FIN_STEP_A) hipLaunchKernelGGL(k_step2_rows<FIN_STEP_A>, dim3(nrows), dim3(kStep2Threads), 0, s, a);
    else hipLaunchKernelGGL(k_step2_rows<FIN_STEP_B>, dim3(nrows), dim3(kStep2Threads), 0, s, a);
  }
}
template <int P>
void launch_step_p(const FinArgs& a, int lv, bool fuse, dim3 grid, hipStream_t s) {
  if constexpr (P <= 1024) {
    if (fuse) {
      launch_step_pf<P, true>(a, lv, grid, s);
      return;
    }
  }
  launch_step_pf<P, false>(a, lv, grid, s);
}

// k_grad over the rows of one FFT-length group: lanes per chip by the
// group's chip count (one lane per chip from 65536 chips, 4 from 8192, else
// 16), one statistics block per problem after the row blocks.
void launch_grad(FinArgs& a, int nrows, int P, int nprob, const int32_t* gprob, hipStream_t s) {
  const int64_t chips = (int64_t)nrows * (P / 2);
  const int lpc = chips >= 65536 ? 1 : (chips >= 8192 ? 4 : 16);
  a.grad_chunks = grad_chunks(P, lpc);
  a.grad_nprob = nprob;
  a.gprob = gprob;
  const dim3 grid(nrows * a.grad_chunks + nprob), block(kGradThreads);
  if (lpc == 1) hipLaunchKernelGGL(k_grad<1>, grid, block, 0, s, a);
  else if (lpc == 4) hipLaunchKernelGGL(k_grad<4>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_grad<16>, grid, block, 0, s, a);
}

void launch_final(const Plan& pl, const Ptrs& w, FinArgs a, hipStream_t s) {
  a.plans = w.plans;
  a.row_prob = w.row_prob;
  a.nrows_total = pl.hdr.nrows;
  a.ustat = w.ustat;
  a.upart = w.upart;
  a.wself = w.wself;
  a.wpart = w.wpart;
  a.spec = w.spec;
  a.done = w.counters;
  a.gbuf = w.gbuf;
  a.pflag = w.pflag;
  a.frozen = (a.mode == FIN_STEP_A || a.mode == FIN_STEP_B) ? pl.frozen : nullptr;
  a.single = pl.hdr.nprob == 1;
  a.one = pl.plans[0];
  for (int g = 0; g < kNumPGroups; ++g) {
    if (pl.hdr.group_nrows[g] == 0) continue;
    a.rows = (const int32_t*)(w.base + pl.hdr.group_rows[g]);
    const dim3 grid(pl.hdr.group_nrows[g]), block(kFinThreads);
    if ((a.mode == FIN_STEP_A || a.mode == FIN_STEP_B) && pl.group_step[g] != 0) {
      const int lv = pl.group_step[g];
      const bool fuse = pl.group_fuse[g];
      if (!fuse) {
        launch_grad(a, pl.hdr.group_nrows[g], 1 << (g + kMinLogP), pl.hdr.group_n[g],
                    (const int32_t*)(w.base + pl.hdr.group_prob[g]), s);
      }
      switch (g) {
        case 0: launch_step_p<128>(a, lv, fuse, grid, s); break;
        case 1: launch_step_p<256>(a, lv, fuse, grid, s); break;
        case 2: launch_step_p<512>(a, lv, fuse, grid, s); break;
        case 3: launch_step_p<1024>(a, lv, fuse, grid, s); break;
        default: {  // P >= 2048
          FinArgs a2 = a;
          a2.split = pl.step2_split[g];
          a2.rowcnt = w.rowsync;
          a2.rowpart = w.rowpart;
          launch_step2(a2, lv, pl.hdr.group_nrows[g], s);
          break;
        }
      }
      if (g + kMinLogP >= 11) {  // partner spectra of the next pass
        if (a.next == NEXT_B_FULL) launch_rowspec(pl, w, g, a.h, s);
        if (a.next == NEXT_A_FULL) launch_rowspec(pl, w, g, w.wpart, s);
      }
      continue;
    }
    FinArgs af = a;
    // k_final at P = 4096 holds two chips per thread and always takes its
    // gradient rows from k_grad
    if (a.mode == FIN_STEP_A || a.mode == FIN_STEP_B || (a.mode == FIN_GRAD && g + kMinLogP >= 12)) {
      // gradient rows by the wide kernel first; k_final then skips the partial sums
      launch_grad(af, pl.hdr.group_nrows[g], 1 << (g + kMinLogP), pl.hdr.group_n[g],
                  (const int32_t*)(w.base + pl.hdr.group_prob[g]), s);
      af.grad_in = w.gbuf;
    }
    switch (g) {
      case 0: hipLaunchKernelGGL(k_final<128>, grid, block, 0, s, af); break;
      case 1: hipLaunchKernelGGL(k_final<256>, grid, block, 0, s, af); break;
      case 2: hipLaunchKernelGGL(k_final<512>, grid, block, 0, s, af); break;
      case 3: hipLaunchKernelGGL(k_final<1024>, grid, block, 0, s, af); break;
      case 4: hipLaunchKernelGGL(k_final<2048>, grid, block, 0, s, af); break;
      default: hipLaunchKernelGGL(k_final<4096>, grid, block, 0, s, af); break;
    }
    if (g + kMinLogP >= 11) {
      if (af.next == NEXT_B_FULL) launch_rowspec(pl, w, g, af.h, s);
      if (af.next == NEXT_A_FULL) launch_rowspec(pl, w, g, w.wpart, s);
    }
  }
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char* sqngd_status_string(int status) {
  switch (status) {
    case SQNGD_OK: return "ok";
    case SQNGD_E_INVALID_ARG: return "invalid argument";
    case SQNGD_E_UNSUPPORTED: return "unsupported problem size";
    case SQNGD_E_WORKSPACE: return "workspace too small or not initialised for this batch";
    case SQNGD_E_ALIGN: return "misaligned pointer";
    case SQNGD_E_HIP: return "HIP launch failure";
    case SQNGD_E_SCRATCH: return "batch needs more scratch than the static array of the no-allocation entry point";
    default: return "unknown status";
  }
}

int sqngd_last_hip_error(void) { return g_last_hip.load(); }

int sqngd_profile_enable(int32_t max_launches, int32_t repeat) {
  if (max_launches < 0 || max_launches > (1 << 16) || repeat < 1 || repeat > 1000) return SQNGD_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  while ((int)g_prof.ev.size() < 2 * max_launches) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return hip_fail(err);
    g_prof.ev.push_back(e);
  }
  if ((int)g_prof.mask.size() < max_launches) g_prof.mask.resize(max_launches, 0);
  g_prof.max = max_launches;
  g_prof.used = 0;
  g_prof.repeat = repeat;
  return SQNGD_OK;
}

int sqngd_profile_groups(int32_t* masks, int32_t capacity, int32_t* count) {
  if (count == nullptr || (masks == nullptr && capacity > 0) || capacity < 0) return SQNGD_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  const int n = g_prof.used < capacity ? g_prof.used : capacity;
  for (int i = 0; i < n; ++i) masks[i] = g_prof.mask[i];
  *count = g_prof.used;
  return SQNGD_OK;
}

int sqngd_profile_read(float* ms, int32_t capacity, int32_t* count) {
  if (count == nullptr || (ms == nullptr && capacity > 0) || capacity < 0) return SQNGD_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  const int n = g_prof.used < capacity ? g_prof.used : capacity;
  for (int i = 0; i < n; ++i) {
    hipError_t err = hipEventSynchronize(g_prof.ev[2 * i + 1]);
    if (err != hipSuccess) return hip_fail(err);
    err = hipEventElapsedTime(&ms[i], g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
    if (err != hipSuccess) return hip_fail(err);
    ms[i] /= (float)g_prof.repeat;
  }
  *count = g_prof.used;
  return SQNGD_OK;
}

int sqngd_buffer_sizes(const sqngd_problem* probs, int32_t nprob, int64_t* z_floats, int64_t* wave_c64,
                       int64_t* adam_floats, int64_t* cube_c64) {
  int rc = validate_batch(probs, nprob);
  if (rc != SQNGD_OK) return rc;
  int64_t zf = 0, wc = 0, af = 0, cc = 0;
  for (int i = 0; i < nprob; ++i) {
    const sqngd_problem& p = probs[i];
    zf += (int64_t)p.M * p.N * p.L;
    wc += (int64_t)p.M * p.N;
    af += SQNGD_ADAM_FLOATS(p.M, p.N, p.L);
    cc += (int64_t)p.M * p.M * p.F * (2 * p.N - 1);
  }
  if (z_floats) *z_floats = zf;
  if (wave_c64) *wave_c64 = wc;
  if (adam_floats) *adam_floats = af;
  if (cube_c64) *cube_c64 = cc;
  return SQNGD_OK;
}

int sqngd_workspace_size(const sqngd_problem* probs, int32_t nprob, size_t* bytes) {
  int rc = validate_batch(probs, nprob);
  if (rc != SQNGD_OK) return rc;
  if (bytes == nullptr) return SQNGD_E_INVALID_ARG;
  *bytes = (size_t)build_plan(probs, nprob)->hdr.total;
  return SQNGD_OK;
}

int sqngd_set_roi_weights(const sqngd_problem* probs, int32_t nprob, const float* weights, void* ws,
                          size_t ws_bytes) {
  if (!aligned(weights, 4)) return SQNGD_E_ALIGN;
  const Plan* pl = nullptr;
  int rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  pl->roi_w = weights;
  return SQNGD_OK;
}

int sqngd_set_stop_mask(const sqngd_problem* probs, int32_t nprob, const int32_t* stopped, void* ws,
                        size_t ws_bytes) {
  if (!aligned(stopped, 4)) return SQNGD_E_ALIGN;
  const Plan* pl = nullptr;
  int rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  pl->frozen = stopped;
  return SQNGD_OK;
}

int sqngd_stop_update(int32_t nprob, const sqngd_stats* stats, float min_gain_db, int32_t patience,
                      const int32_t* step_counter, float* best_db, int32_t* stall, int32_t* stopped,
                      int32_t* stop_iter, void* stream) {
  if (nprob < 1 || nprob > (1 << 20) || patience < 1 || !finite(min_gain_db)) return SQNGD_E_INVALID_ARG;
  if (stats == nullptr || best_db == nullptr || stall == nullptr || stopped == nullptr || stop_iter == nullptr)
    return SQNGD_E_INVALID_ARG;
  if (!aligned(stats, 4) || !aligned(step_counter, 4) || !aligned(best_db, 4) || !aligned(stall, 4) ||
      !aligned(stopped, 4) || !aligned(stop_iter, 4))
    return SQNGD_E_ALIGN;
  hipLaunchKernelGGL(k_stop, dim3((nprob + 255) / 256), dim3(256), 0, (hipStream_t)stream, nprob, stats,
                     min_gain_db, patience, step_counter, best_db, stall, stopped, stop_iter);
  return check_launch();
}

int sqngd_workspace_init(const sqngd_problem* probs, int32_t nprob, void* ws, size_t ws_bytes, void* stream) {
  int rc = validate_batch(probs, nprob);
  if (rc != SQNGD_OK) return rc;
  if (ws == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(ws, kAlign)) return SQNGD_E_ALIGN;
  auto pl = build_plan(probs, nprob);
  if (ws_bytes < (size_t)pl->hdr.total) return SQNGD_E_WORKSPACE;
  rc = put_plan(*pl, ws, (hipStream_t)stream);
  if (rc != SQNGD_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  g_ws[ws] = std::move(pl);  // frees the plan this workspace held before
  return SQNGD_OK;
}

int sqngd_workspace_release(const void* ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ws.erase(ws) == 1 ? SQNGD_OK : SQNGD_E_INVALID_ARG;
}

int sqngd_af_forward(const sqngd_problem* probs, int32_t nprob, const float* z, int32_t wave_mode,
                     const sqngd_c64* s_given, const sqngd_c64* h, sqngd_stats* stats, sqngd_c64* af_cube,
                     void* ws, size_t ws_bytes, void* stream) {
  if (wave_mode < SQNGD_WAVE_SOFT || wave_mode > SQNGD_WAVE_GIVEN) return SQNGD_E_INVALID_ARG;
  if (wave_mode != SQNGD_WAVE_GIVEN && z == nullptr) return SQNGD_E_INVALID_ARG;
  if (wave_mode == SQNGD_WAVE_GIVEN && s_given == nullptr) return SQNGD_E_INVALID_ARG;
  if (h == nullptr || stats == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(s_given, 8) || !aligned(h, 8) || !aligned(stats, 4) || !aligned(af_cube, 8))
    return SQNGD_E_ALIGN;
  const Plan* pl = nullptr;
  int rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  Ptrs w = ptrs(*pl, ws);
  PrepArgs pa{};
  pa.mode = wave_mode == SQNGD_WAVE_SOFT ? PREP_B_SOFT : (wave_mode == SQNGD_WAVE_HARD ? PREP_B_HARD : PREP_B_GIVEN);
  pa.z = z;
  pa.s_given = (const float2*)s_given;
  pa.h = (const float2*)h;
  launch_prep(*pl, w, pa, s);
  PassArgs ka{};
  ka.orient = 0;
  ka.want_grad = 0;
  ka.self_w = w.wself;
  ka.cube = (float2*)af_cube;
  launch_pass(*pl, w, ka, s);
  FinArgs fa{};
  fa.orient = 0;
  fa.mode = FIN_STATS;
  fa.snrl = w.snrl;
  fa.stats = stats;
  launch_final(*pl, w, fa, s);
  return check_launch();
}

}  // extern "C"

namespace {

int check_backward_args(const float* z, int32_t wave_mode, const sqngd_c64* s_given, const sqngd_c64* h,
                        const float* grad_loss, const float* grad_z, const sqngd_c64* grad_h,
                        const sqngd_c64* grad_s, const sqngd_stats* stats) {
  if (wave_mode < SQNGD_WAVE_SOFT || wave_mode > SQNGD_WAVE_GIVEN) return SQNGD_E_INVALID_ARG;
  if (wave_mode != SQNGD_WAVE_GIVEN && z == nullptr) return SQNGD_E_INVALID_ARG;
  if (wave_mode == SQNGD_WAVE_GIVEN && (s_given == nullptr || grad_z != nullptr)) return SQNGD_E_INVALID_ARG;
  if (h == nullptr) return SQNGD_E_INVALID_ARG;
  if (grad_z == nullptr && grad_h == nullptr && grad_s == nullptr && stats == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(s_given, 8) || !aligned(h, 8) || !aligned(grad_loss, 4) || !aligned(grad_z, 4) ||
      !aligned(grad_h, 8) || !aligned(grad_s, 8) || !aligned(stats, 4))
    return SQNGD_E_ALIGN;
  return SQNGD_OK;
}

// The launch sequence of sqngd_af_backward on a workspace that holds `pl`.
int af_backward_launch(const Plan* pl, void* ws, const float* z, int32_t wave_mode, const sqngd_c64* s_given,
                       const sqngd_c64* h, const float* grad_loss, float* grad_z, sqngd_c64* grad_h,
                       sqngd_c64* grad_s, sqngd_stats* stats, hipStream_t s) {
  Ptrs w = ptrs(*pl, ws);
  float4* snrl0 = w.snrl;
  float4* snrl1 = w.snrl + pl->hdr.nrows;
  PrepArgs pa{};
  pa.mode = wave_mode == SQNGD_WAVE_SOFT ? PREP_B_SOFT : (wave_mode == SQNGD_WAVE_HARD ? PREP_B_HARD : PREP_B_GIVEN);
  pa.z = z;
  pa.s_given = (const float2*)s_given;
  pa.h = (const float2*)h;
  pa.snrl = snrl0;
  // The filter-side pass alone yields the statistics too (the same cells in
  // swapped roles), so a call that wants only grad_h (and stats) skips the
  // waveform side; with the waveforms given it also needs no copy of them.
  const bool wave_side = grad_z != nullptr || grad_s != nullptr || grad_h == nullptr;
  const bool given_only = !wave_side && wave_mode == SQNGD_WAVE_GIVEN;
  if (!given_only) launch_prep(*pl, w, pa, s);
  if (wave_side) {
  // waveform side (orientation 0)
  PassArgs ka{};
  ka.orient = 0;
  ka.want_grad = 1;
  ka.self_w = w.wself;
  launch_pass(*pl, w, ka, s);
  FinArgs fa{};
  fa.orient = 0;
  fa.mode = FIN_GRAD;
  fa.wave_mode = wave_mode;
  fa.self_w = w.wself;
  fa.part_w = (const float2*)h;
  fa.snrl = snrl0;
  fa.stats = stats;
  fa.grad_loss = grad_loss;
  fa.grad_w = (float2*)grad_s;
  fa.grad_z = grad_z;
  fa.z = const_cast<float*>(z);
  launch_final(*pl, w, fa, s);
  }
  if (grad_h != nullptr) {
    // filter side (orientation 1): self = h, partners = the waveforms of wself
    PrepArgs pb{};
    pb.mode = given_only ? PREP_A_GIVEN : PREP_A_SELF;
    pb.h = (const float2*)h;
    pb.s_given = (const float2*)s_given;
    pb.snrl = snrl1;
    launch_prep(*pl, w, pb, s);
    PassArgs kb{};
    kb.orient = 1;
    kb.want_grad = 1;
    kb.self_w = (const float2*)h;
    launch_pass(*pl, w, kb, s);
    FinArgs fb{};
    fb.orient = 1;
    fb.mode = FIN_GRAD;
    fb.wave_mode = SQNGD_WAVE_GIVEN;
    fb.self_w = (const float2*)h;
    fb.part_w = given_only ? (const float2*)s_given : w.wself;
    fb.snrl = snrl1;
    fb.stats = wave_side ? nullptr : stats;
    fb.grad_loss = grad_loss;
    fb.grad_w = (float2*)grad_h;
    launch_final(*pl, w, fb, s);
  }
  return check_launch();
}

}  // namespace

extern "C" {

int sqngd_af_backward(const sqngd_problem* probs, int32_t nprob, const float* z, int32_t wave_mode,
                      const sqngd_c64* s_given, const sqngd_c64* h, const float* grad_loss, float* grad_z,
                      sqngd_c64* grad_h, sqngd_c64* grad_s, sqngd_stats* stats, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = check_backward_args(z, wave_mode, s_given, h, grad_loss, grad_z, grad_h, grad_s, stats);
  if (rc != SQNGD_OK) return rc;
  const Plan* pl = nullptr;
  rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  return af_backward_launch(pl, ws, z, wave_mode, s_given, h, grad_loss, grad_z, grad_h, grad_s, stats,
                            (hipStream_t)stream);
}

static int validate_opt(const sqngd_opt* opt) {
  if (opt == nullptr) return SQNGD_E_INVALID_ARG;
  const sqngd_opt& o = *opt;
  if (!finite(o.lr_z) || !finite(o.lr_h) || o.lr_z < 0.f || o.lr_h < 0.f) return SQNGD_E_INVALID_ARG;
  if (!(o.beta1 >= 0.f && o.beta1 < 1.f && o.beta2 >= 0.f && o.beta2 < 1.f)) return SQNGD_E_INVALID_ARG;
  if (!finite(o.eps) || o.eps <= 0.f) return SQNGD_E_INVALID_ARG;
  if (o.n_h < 0 || o.n_x < 0 || o.n_h + o.n_x < 1 || o.n_h > 1000 || o.n_x > 1000) return SQNGD_E_INVALID_ARG;
  if (!finite(o.T0) || !finite(o.T1) || o.T0 <= 0.f || o.T1 <= 0.f || o.total_iters < 1) return SQNGD_E_INVALID_ARG;
  if ((o.flags & ~SQNGD_OPT_SGD) != 0) return SQNGD_E_INVALID_ARG;
  return SQNGD_OK;
}

int sqngd_run(const sqngd_problem* probs, int32_t nprob, const sqngd_opt* opt, int32_t n_iters, float* z,
              sqngd_c64* h, float* adam_state, int32_t* step_counter, sqngd_stats* stats, void* ws,
              size_t ws_bytes, void* stream) {
  int rc = validate_opt(opt);
  if (rc != SQNGD_OK) return rc;
  if (n_iters < 1 || n_iters > 100000) return SQNGD_E_INVALID_ARG;
  if (z == nullptr || h == nullptr || adam_state == nullptr || step_counter == nullptr) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(h, 8) || !aligned(adam_state, 4) || !aligned(step_counter, 4) ||
      !aligned(stats, 4))
    return SQNGD_E_ALIGN;
  const Plan* pl = nullptr;
  rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  const sqngd_opt& o = *opt;
  hipStream_t s = (hipStream_t)stream;
  Ptrs w = ptrs(*pl, ws);
  float4* snrl_buf[2] = {w.snrl, w.snrl + pl->hdr.nrows};
  int q = 0;  // pass index within the call: pass q reads snrl_buf[q & 1]
  // With k_step on every group, the finalize that ends an outer iteration
  // leaves the step counter to the first kernel of the next pass (which does
  // not read it), saving the last-block atomics; the last iteration of the
  // call advances it itself.
  int32_t* bump = nullptr;
  // inputs of the first pass
  PrepArgs pa{};
  pa.mode = o.n_h > 0 ? PREP_A_HARD : PREP_B_SOFT;
  pa.use_schedule = 1;
  pa.opt = o;
  pa.counter = step_counter;
  pa.z = z;
  pa.h = (const float2*)h;
  pa.snrl = snrl_buf[0];
  launch_prep(*pl, w, pa, s);
  for (int it = 0; it < n_iters; ++it) {
    const bool more = it + 1 < n_iters;
    for (int i = 0; i < o.n_h; ++i, ++q) {
      PassArgs ka{};
      ka.orient = 1;
      ka.want_grad = 1;
      ka.self_w = (const float2*)h;
      ka.bump = bump;
      bump = nullptr;
      launch_pass(*pl, w, ka, s);
      FinArgs fa{};
      fa.orient = 1;
      fa.mode = FIN_STEP_A;
      fa.inner = i;
      fa.count_step = (o.n_x == 0 && i == o.n_h - 1) ? 1 : 0;
      fa.next = i + 1 < o.n_h ? NEXT_A_SNRL : (o.n_x > 0 ? NEXT_B_FULL : (more ? NEXT_A_SNRL : NEXT_NONE));
      fa.self_w = (const float2*)h;
      fa.part_w = w.wpart;
      fa.snrl = snrl_buf[q & 1];
      fa.snrl_next = snrl_buf[(q + 1) & 1];
      fa.stats = stats;
      fa.z = z;
      fa.h = (float2*)h;
      fa.adam = adam_state;
      fa.counter = step_counter;
      fa.opt = o;
      if (fa.count_step && fa.next != NEXT_NONE && pl->all_step) {
        fa.count_step = 0;
        bump = step_counter;
      }
      launch_final(*pl, w, fa, s);
    }
    for (int j = 0; j < o.n_x; ++j, ++q) {
      PassArgs ka{};
      ka.orient = 0;
      ka.want_grad = 1;
      ka.self_w = w.wself;
      ka.bump = bump;
      bump = nullptr;
      launch_pass(*pl, w, ka, s);
      FinArgs fa{};
      fa.orient = 0;
      fa.mode = FIN_STEP_B;
      fa.inner = j;
      fa.count_step = (j == o.n_x - 1) ? 1 : 0;
      if (j + 1 < o.n_x) {
        fa.next = NEXT_B_SOFT;
      } else if (more) {
        fa.next = o.n_h > 0 ? NEXT_A_FULL : NEXT_B_SOFT;
        fa.next_t_offset = 1;
      }
      fa.self_w = w.wself;
      fa.part_w = (const float2*)h;
      fa.snrl = snrl_buf[q & 1];
      fa.snrl_next = snrl_buf[(q + 1) & 1];
      fa.stats = stats ? stats + nprob : nullptr;
      fa.z = z;
      fa.h = (float2*)h;
      fa.adam = adam_state;
      fa.counter = step_counter;
      fa.opt = o;
      if (fa.count_step && fa.next != NEXT_NONE && pl->all_step) {
        fa.count_step = 0;
        bump = step_counter;
      }
      launch_final(*pl, w, fa, s);
    }
  }
  return check_launch();
}

int sqngd_step(const sqngd_problem* probs, int32_t nprob, const sqngd_opt* opt, float* z, sqngd_c64* h,
               float* adam_state, int32_t* step_counter, sqngd_stats* stats, void* ws, size_t ws_bytes,
               void* stream) {
  return sqngd_run(probs, nprob, opt, 1, z, h, adam_state, step_counter, stats, ws, ws_bytes, stream);
}

int sqngd_hard_quantize(const sqngd_problem* probs, int32_t nprob, const float* z, int32_t* idx, sqngd_c64* x,
                        void* ws, size_t ws_bytes, void* stream) {
  if (z == nullptr || (idx == nullptr && x == nullptr)) return SQNGD_E_INVALID_ARG;
  if (!aligned(z, 4) || !aligned(idx, 4) || !aligned(x, 8)) return SQNGD_E_ALIGN;
  const Plan* pl = nullptr;
  int rc = lookup(probs, nprob, ws, ws_bytes, &pl);
  if (rc != SQNGD_OK) return rc;
  Ptrs w = ptrs(*pl, ws);
  HardArgs a{w.plans, w.row_prob, z, idx, (float2*)x};
  hipLaunchKernelGGL(k_hardq, dim3(pl->hdr.nrows), dim3(256), 0, (hipStream_t)stream, a);
  return check_launch();
}

}  // extern "C"

// ------------------------------------------------ entry point without a workspace

// The scratch of sqngd_af_backward_noalloc: one static array per GPU, held
// until the process ends. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it uses the
// device address hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[SQNGD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNoAllocScratch = (size_t)SQNGD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return SQNGD_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (ptr == nullptr || !aligned(ptr, kAlign)) return SQNGD_E_ALIGN;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return SQNGD_OK;
}

}  // namespace

extern "C" {

int sqngd_af_backward_noalloc(const sqngd_problem* probs, int32_t nprob, const float* z, int32_t wave_mode,
                              const sqngd_c64* s_given, const sqngd_c64* h, const float* grad_loss,
                              float* grad_z, sqngd_c64* grad_h, sqngd_c64* grad_s, sqngd_stats* stats,
                              void* stream) {
  int rc = check_backward_args(z, wave_mode, s_given, h, grad_loss, grad_z, grad_h, grad_s, stats);
  if (rc != SQNGD_OK) return rc;
  rc = validate_batch(probs, nprob);
  if (rc != SQNGD_OK) return rc;
  auto pl = build_plan(probs, nprob);
  if ((size_t)pl->hdr.total > kNoAllocScratch) return SQNGD_E_SCRATCH;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != SQNGD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = put_plan(*pl, ws, s);
  if (rc != SQNGD_OK) return rc;
  return af_backward_launch(pl.get(), ws, z, wave_mode, s_given, h, grad_loss, grad_z, grad_h, grad_s, stats, s);
}

}  // extern "C"

// the warm-start network (same translation unit: it uses the helpers above)
#include "net.hip"
// the paper's transmit parameterisation (same translation unit)
#include "sqn.hip"
