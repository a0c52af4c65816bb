// plan.hpp - device-side description of a batch, written into the caller's
// workspace by sqngd_workspace_init and read by every kernel.
#pragma once

#include <cstdint>

namespace sq {

constexpr int kNumPGroups = 6;  // FFT lengths 128, 256, 512, 1024, 2048, 4096
constexpr int kMinLogP = 7;

// One problem of the batch. Offsets are element offsets: off_z into z-sized
// arrays (floats), off_w into waveform-sized arrays (complex), off_state into
// the Adam state (floats), off_cube into the AF cube (complex); ws_* are
// offsets into the workspace regions of the same element type.
struct ProbPlan {
  int32_t M, N, L, F;
  int32_t P, logP, tau_lo, tau_hi;
  float p, p_tar;
  float w_psl, w_snrl, temperature, inv_NP;
  int32_t sq_mode, ph_log;  // ph_log = log2(p/2) when p/2 is a power of two <= 32, else -1
  int32_t units, row0;      // units = M*wpr statistics entries; row0 = first row in the batch
  int32_t wpr;              // fused-pass blocks per row (ceil(F / Doppler bins per block))
  int32_t spec_wave;        // 1: partner spectra stored in the one-wave FFT layout (the latency
                            // pass reads them), 0: in the throughput pass's layout
  int64_t off_z, off_w, off_state, off_cube;
  int64_t ws_spec;   // complex: [M][P] spectra
  int64_t ws_unit;   // UnitStat index and row index of upart ([units][N] complex, stride N)
  int64_t ws_upart;  // complex offset of this problem's unit partials
  int64_t off_rw;    // float offset of this problem's ROI weights [F][2N-1]
  // Doppler grid nu_f = nu_min + f dnu in FP64: wide spans put hundreds of
  // turns into the modulation phase n nu_f / N, whose fraction FP32 would lose
  double nu_min, dnu;
  // Doppler bins [cut_lo, cut_hi) whose auto-pair tau = 0 cell is outside the
  // region of interest: every bin (eq. 8), or the mainlobe bins |nu_f| < 1
  int32_t cut_lo, cut_hi;
};
static_assert(sizeof(ProbPlan) == 168, "ProbPlan layout");


// Per-unit partial statistics of one fused pass. Keys pack the squared raw
// magnitude (float bits, monotone for non-negative values) in the high word
// and the complement of the cell index in the low word, so a max over keys
// selects the largest cell and, among equal values, the lowest index.
struct UnitStat {
  float sigma;   // running scale: max raw |r| over the ROI cells of the unit
  float S;       // sum over the unit's ROI cells of (|r| / sigma)^p
  uint32_t pad0, pad1;
  unsigned long long key_auto, key_cross;
};
static_assert(sizeof(UnitStat) == 32, "UnitStat layout");

// Batch header at the start of the workspace.
struct WsHeader {
  uint32_t magic;
  int32_t nprob, nrows, pad0;
  int64_t plans;          // byte offset of ProbPlan[nprob]
  int64_t group_prob[kNumPGroups];   // byte offset of int32 problem ids of each FFT-length group
  int64_t group_wave[kNumPGroups];   // byte offset of int32 [n+1] wave prefix (fused pass)
  int64_t group_rwave[kNumPGroups];  // byte offset of int32 [n+1] wave prefix (one slot per row)
  int64_t group_rows[kNumPGroups];   // byte offset of int32 batch rows of each group
  int32_t group_n[kNumPGroups];
  int32_t group_waves[kNumPGroups];
  int32_t group_rwaves[kNumPGroups];
  int32_t group_nrows[kNumPGroups];
  int64_t row_prob;       // byte offset of int32 [nrows]: problem of each row
  int64_t spec, wself, wpart, ustat, upart, counters;  // region byte offsets
  int64_t snrl;  // float4 [2][rows]: mainlobe products, double-buffered by pass parity
  int64_t gbuf;   // float2 [sum M N]: gradient rows of an optimiser step (packed waveform layout)
  int64_t pflag;  // int32 [nprob]: non-finite loss of the step's evaluation
  int64_t rowsync;  // int32 [rows of FFT length 2048 or 4096]: k_step2's blocks done per row (in the zeroed table)
  int64_t rowpart;  // float4 [rows of FFT length 2048 or 4096][8]: k_step2's partial products per block
  int64_t total;
};

constexpr uint32_t kWsMagic = 0x53514e47u;  // "SQNG"

// Number of 32-bit device counters at WsHeader::counters.
constexpr int kNumCounters = 4;

}  // namespace sq
