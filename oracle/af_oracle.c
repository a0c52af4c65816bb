/*
 * af_oracle.c - FP64 CPU oracle of the SQNGD ambiguity function, sidelobe
 * loss, SNRL penalty and their gradients, written as the plain definitions.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the correctness reference for the
 * gfx950 kernels. Only the tests, the package smoke check and the CPU-baseline
 * leg of the benchmark may load it. It shares no code with the HIP path.
 *
 * Paper: arXiv 2604.25728 (SQNGD). Conventions (0-based indices, packed
 * complex gradients dL/dRe + j dL/dIm, Doppler grid including both end
 * points) are listed in the oracle's Python wrapper, sqngd_ref.py.
 *
 * Every routine below is a direct sum over the index sets the paper defines:
 * no FFT, no blocking, no reordering of terms beyond the loop nesting. The
 * cost is O(M^2 F N^2) complex multiply-adds per cube or gradient, split over
 * (m, l, f) with OpenMP.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Doppler bin f of a uniform grid that includes both end points; a single
   bin sits at nu_min. The paper leaves the grid implicit (Algorithm 1 takes a
   Doppler grid as input); this is the reading the library uses. */
double sqngd_ref_nu(int F, double nu_min, double nu_max, int f) {
  if (F <= 1) return nu_min;
  return nu_min + (double)f * (nu_max - nu_min) / (double)(F - 1);
}

/* Doppler-modulated waveform (Sec. III-B, eq. 33): xh(n) = x(n) e^{j 2 pi n nu / N}. */
static void modulate(int N, const cplx* x, double nu, cplx* xh) {
  for (int n = 0; n < N; ++n) xh[n] = x[n] * cexp(I * 2.0 * M_PI * (double)n * nu / (double)N);
}

/* One row of the AF (Sec. II-A, eq. 6, written on the modulated waveform as
   eq. 34): A(tau) = sum over n with 0 <= n < N and 0 <= n + tau < N of
   xh(n) conj(h(n + tau)), for tau = -(N-1) .. N-1, stored at tau + N - 1. */
static void af_row(int N, const cplx* xh, const cplx* h, cplx* row) {
  for (int tau = -(N - 1); tau <= N - 1; ++tau) {
    cplx acc = 0.0;
    for (int n = 0; n < N; ++n) {
      int k = n + tau;
      if (k < 0 || k >= N) continue;
      acc += xh[n] * conj(h[k]);
    }
    row[tau + N - 1] = acc;
  }
}

/* The full cube A[m][l][f][tau + N - 1] of every waveform s_m against every
   filter h_l (eq. 6; m = l gives the auto-AF, m != l the cross-AF). */
void sqngd_ref_af_cube(int M, int N, int F, double nu_min, double nu_max, const double* s_in,
                       const double* h_in, double* A_out) {
  const cplx* s = (const cplx*)s_in;
  const cplx* h = (const cplx*)h_in;
  cplx* A = (cplx*)A_out;
  const int T = 2 * N - 1;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int m = 0; m < M; ++m) {
    for (int f = 0; f < F; ++f) {
      cplx* xh = (cplx*)malloc(sizeof(cplx) * (size_t)N);
      modulate(N, s + (size_t)m * N, sqngd_ref_nu(F, nu_min, nu_max, f), xh);
      for (int l = 0; l < M; ++l)
        af_row(N, xh, h + (size_t)l * N, A + (((size_t)m * M + l) * F + f) * T);
      free(xh);
    }
  }
}

/* One row A_ml(., f) of the cube, for sampled checks at sizes where the whole
   cube is not wanted. */
void sqngd_ref_af_row(int M, int N, int F, double nu_min, double nu_max, const double* s_in,
                      const double* h_in, int m, int l, int f, double* row_out) {
  const cplx* s = (const cplx*)s_in;
  const cplx* h = (const cplx*)h_in;
  (void)M;
  cplx* xh = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  modulate(N, s + (size_t)m * N, sqngd_ref_nu(F, nu_min, nu_max, f), xh);
  af_row(N, xh, h + (size_t)l * N, (cplx*)row_out);
  free(xh);
}

/* Region of interest (eq. 7-9): a cell (m, l, tau, f) counts when
   tau_lo <= tau <= tau_hi, except the tau = 0 cut of an auto pair (eq. 8
   excludes tau = 0 for m1 = m2; eq. 9 keeps every tau for m1 != m2). With
   auto_mask = 1 (an option beside the paper's rule) only the cells of that cut
   inside the Doppler mainlobe, |nu_f| < 1, are excluded: A_mm(0, nu) of a
   matched unimodular pair is sum_n e^{j 2 pi n nu / N}, whose first nulls sit
   at nu = +-1. Inside the region a cell carries the weight w(tau, f) of eq.
   8-9: wt[f][tau + N - 1] when a table is given, else 1. */
static int in_roi(int m, int l, int tau, double nu, int tau_lo, int tau_hi, int auto_mask) {
  if (tau < tau_lo || tau > tau_hi) return 0;
  if (m == l && tau == 0 && (auto_mask == 0 || fabs(nu) < 1.0)) return 0;
  return 1;
}
static double roi_weight(const double* wt, int N, int f, int tau) {
  return wt ? wt[(size_t)f * (2 * N - 1) + tau + N - 1] : 1.0;
}

/* Loss and statistics from a cube (wt: the weights w(tau, f) of eq. 8-9 as
   [F][2N-1], or NULL for w = 1).
   out[0] loss = w_psl * lp + w_snrl * l_snrl             (eq. 42, p-norm for the max)
   out[1] lp = (sum over the ROI of a^p)^(1/p), a = w |A|/N (p-norm of eq. 37's max)
   out[2] l_snrl = (1/M) sum_m (p_m - p_tar)^2             (eq. 41)
   out[3] psl_auto = max w |A| over auto cells             (eq. 8)
   out[4] psl_cross = max w |A| over cross cells           (eq. 9)
   out[5] pslr_db = 20 log10(max(out[3], out[4]) / N)      (eq. 48)
   out[6] max over m of SNRL_m in dB                       (eq. 10)
   out[7] min over m of p_m = |h_m^H s_m| / N              (eq. 38)
   arg[0..3] = (m, l, tau, f) of the first cell, in m, l, f, tau order, holding
   the larger of the two PSLs. snrl_db and pm (length M, may be NULL) receive
   SNRL_m and p_m. lp is evaluated as amax (sum (a/amax)^p)^(1/p), which equals
   the definition and does not overflow. */
void sqngd_ref_loss(int M, int N, int F, double nu_min, double nu_max, const double* A_in,
                    const double* s_in, const double* h_in, int tau_lo, int tau_hi, int auto_mask,
                    const double* wt, double p, double mu_db, double w_psl,
                    double w_snrl, double* out, int* arg, double* snrl_db, double* pm) {
  const cplx* A = (const cplx*)A_in;
  const cplx* s = (const cplx*)s_in;
  const cplx* h = (const cplx*)h_in;
  const int T = 2 * N - 1;
  double psl_auto = 0.0, psl_cross = 0.0, amax = 0.0;
  int best[4] = {0, 0, 0, 0};
  double best_val = -1.0;
  for (int m = 0; m < M; ++m)
    for (int l = 0; l < M; ++l)
      for (int f = 0; f < F; ++f)
        for (int tau = -(N - 1); tau <= N - 1; ++tau) {
          if (!in_roi(m, l, tau, sqngd_ref_nu(F, nu_min, nu_max, f), tau_lo, tau_hi, auto_mask)) continue;
          double v = roi_weight(wt, N, f, tau) * cabs(A[(((size_t)m * M + l) * F + f) * T + tau + N - 1]);
          if (m == l) {
            if (v > psl_auto) psl_auto = v;
          } else if (v > psl_cross) {
            psl_cross = v;
          }
          if (v > best_val) {
            best_val = v;
            best[0] = m; best[1] = l; best[2] = tau; best[3] = f;
          }
          if (v / N > amax) amax = v / N;
        }
  double acc = 0.0;
  if (amax > 0.0) {
    for (int m = 0; m < M; ++m)
      for (int l = 0; l < M; ++l)
        for (int f = 0; f < F; ++f)
          for (int tau = -(N - 1); tau <= N - 1; ++tau) {
            if (!in_roi(m, l, tau, sqngd_ref_nu(F, nu_min, nu_max, f), tau_lo, tau_hi, auto_mask)) continue;
            double a = roi_weight(wt, N, f, tau) * cabs(A[(((size_t)m * M + l) * F + f) * T + tau + N - 1]) / N;
            acc += pow(a / amax, p);
          }
  }
  double lp = amax > 0.0 ? amax * pow(acc, 1.0 / p) : 0.0;
  /* eq. 38-41 and eq. 10 */
  double p_tar = pow(10.0, -mu_db / 20.0);
  double l_snrl = 0.0, snrl_max = -INFINITY, p_min = INFINITY;
  for (int m = 0; m < M; ++m) {
    cplx c = 0.0;
    double es = 0.0, eh = 0.0;
    for (int n = 0; n < N; ++n) {
      c += conj(h[(size_t)m * N + n]) * s[(size_t)m * N + n];
      es += creal(s[(size_t)m * N + n] * conj(s[(size_t)m * N + n]));
      eh += creal(h[(size_t)m * N + n] * conj(h[(size_t)m * N + n]));
    }
    double p_m = cabs(c) / N;
    double snrl = 10.0 * log10(es * eh / (cabs(c) * cabs(c)));
    l_snrl += (p_m - p_tar) * (p_m - p_tar) / M;
    if (snrl > snrl_max) snrl_max = snrl;
    if (p_m < p_min) p_min = p_m;
    if (snrl_db) snrl_db[m] = snrl;
    if (pm) pm[m] = p_m;
  }
  double psl = psl_auto > psl_cross ? psl_auto : psl_cross;
  out[0] = w_psl * lp + w_snrl * l_snrl;
  out[1] = lp;
  out[2] = l_snrl;
  out[3] = psl_auto;
  out[4] = psl_cross;
  out[5] = 20.0 * log10(psl / N);
  out[6] = snrl_max;
  out[7] = p_min;
  if (arg) memcpy(arg, best, sizeof(best));
}

/* Gradients of the loss of sqngd_ref_loss with respect to the waveforms and
   the filters, packed as dL/dRe + j dL/dIm.

   With a = w |A|/N on the ROI, dlp/da = lp^(1-p) a^(p-1) and the packed
   derivative of a with respect to A is w A / (N |A|), so the sidelobe term
   has packed gradient G = w_psl lp^(1-p) a^(p-2) w^2 A / N^2 on the ROI, 0
   elsewhere.
   A is linear in s_m and conjugate-linear in h_l (eq. 6), which gives
     grad_s_m(n) = sum_{l,f,tau} e^{-j 2 pi n nu_f / N} G_ml(tau,f) h_l(n + tau)
     grad_h_l(k) = sum_{m,f,tau} conj(G_ml(tau,f)) s_m(k - tau) e^{j 2 pi (k - tau) nu_f / N}.
   The SNRL term (eq. 38, 41) with c_m = h_m^H s_m adds
     G_S = w_snrl (2/M) (p_m - p_tar) c_m / (N |c_m|),
     grad_s_m += G_S h_m,  grad_h_m += conj(G_S) s_m.
   Requires the cube of sqngd_ref_af_cube for the same inputs. */
void sqngd_ref_grads(int M, int N, int F, double nu_min, double nu_max, const double* s_in,
                     const double* h_in, const double* A_in, int tau_lo, int tau_hi, int auto_mask,
                     const double* wt, double p, double mu_db, double w_psl, double w_snrl, double* gs_out,
                     double* gh_out) {
  const cplx* s = (const cplx*)s_in;
  const cplx* h = (const cplx*)h_in;
  const cplx* A = (const cplx*)A_in;
  cplx* gs = (cplx*)gs_out;
  cplx* gh = (cplx*)gh_out;
  const int T = 2 * N - 1;
  double stats[8];
  sqngd_ref_loss(M, N, F, nu_min, nu_max, A_in, s_in, h_in, tau_lo, tau_hi, auto_mask, wt, p, mu_db,
                 w_psl, w_snrl, stats, NULL, NULL, NULL);
  const double lp = stats[1];
  const size_t ncell = (size_t)M * M * F * T;
  cplx* G = (cplx*)calloc(ncell, sizeof(cplx));
  if (lp > 0.0) {
    for (int m = 0; m < M; ++m)
      for (int l = 0; l < M; ++l)
        for (int f = 0; f < F; ++f)
          for (int tau = -(N - 1); tau <= N - 1; ++tau) {
            if (!in_roi(m, l, tau, sqngd_ref_nu(F, nu_min, nu_max, f), tau_lo, tau_hi, auto_mask)) continue;
            size_t i = (((size_t)m * M + l) * F + f) * T + tau + N - 1;
            double w = roi_weight(wt, N, f, tau);
            double a = w * cabs(A[i]) / N;
            G[i] = w_psl * pow(lp, 1.0 - p) * pow(a, p - 2.0) * w * w * A[i] / ((double)N * N);
          }
  }
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      cplx acc = 0.0;
      for (int l = 0; l < M; ++l)
        for (int f = 0; f < F; ++f) {
          double nu = sqngd_ref_nu(F, nu_min, nu_max, f);
          cplx demod = cexp(-I * 2.0 * M_PI * (double)n * nu / (double)N);
          cplx inner = 0.0;
          for (int tau = -(N - 1); tau <= N - 1; ++tau) {
            int k = n + tau;
            if (k < 0 || k >= N) continue;
            inner += G[(((size_t)m * M + l) * F + f) * T + tau + N - 1] * h[(size_t)l * N + k];
          }
          acc += demod * inner;
        }
      gs[(size_t)m * N + n] = acc;
    }
  /* modulated waveforms xh[m][f][n] of eq. 33, computed once */
  cplx* XH = (cplx*)malloc(sizeof(cplx) * (size_t)M * F * N);
  for (int m = 0; m < M; ++m)
    for (int f = 0; f < F; ++f)
      modulate(N, s + (size_t)m * N, sqngd_ref_nu(F, nu_min, nu_max, f),
               XH + ((size_t)m * F + f) * N);
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int l = 0; l < M; ++l)
    for (int k = 0; k < N; ++k) {
      cplx acc = 0.0;
      for (int m = 0; m < M; ++m)
        for (int f = 0; f < F; ++f) {
          const cplx* xh = XH + ((size_t)m * F + f) * N;
          for (int tau = -(N - 1); tau <= N - 1; ++tau) {
            int n = k - tau;
            if (n < 0 || n >= N) continue;
            acc += conj(G[(((size_t)m * M + l) * F + f) * T + tau + N - 1]) * xh[n];
          }
        }
      gh[(size_t)l * N + k] = acc;
    }
  free(XH);
  free(G);
  /* SNRL penalty (eq. 38, 41) */
  double p_tar = pow(10.0, -mu_db / 20.0);
  for (int m = 0; m < M; ++m) {
    cplx c = 0.0;
    for (int n = 0; n < N; ++n) c += conj(h[(size_t)m * N + n]) * s[(size_t)m * N + n];
    double mag = cabs(c);
    if (mag == 0.0) continue;
    double p_m = mag / N;
    cplx gS = w_snrl * (2.0 / M) * (p_m - p_tar) * c / ((double)N * mag);
    for (int n = 0; n < N; ++n) {
      gs[(size_t)m * N + n] += gS * h[(size_t)m * N + n];
      gh[(size_t)m * N + n] += conj(gS) * s[(size_t)m * N + n];
    }
  }
}
