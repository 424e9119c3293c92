/*
 * gbsub_oracle.c -- plain FP64 CPU oracle of the iterative galactic-binary
 * subtraction.  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * It is written to be checked by eye against the paper: each function names
 * the passage it follows.  There is no blocking, fusion or reordering beyond
 * what the definitions state.  Sums run in ascending index order and the
 * build disables FMA contraction, so every result is a fixed sequence of
 * IEEE binary64 operations.  Parallelism (OpenMP) is only over independent
 * outputs (one median per bin, one SNR per source) and does not change any
 * result.
 */
#include "gbsub_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_C_LIGHT 299792458.0   /* m/s */

void orc_default_config(orc_config *c)
{
    memset(c, 0, sizeof(*c));
    c->window_bins   = 1001;
    c->snr_threshold = 7.0;                 /* rho_th = 7 */
    c->kappa         = 1.0 / 7.0;           /* kappa = 1/rho_th: keep sources with rho_0 >= 1 */
    c->median_scale  = 729.0 / 512.0;       /* C = (1 - 2/(9 nu))^-3 with nu = 2 */
    c->estimator     = ORC_MEDIAN;
    c->track_model   = ORC_TRACK_SWEEP;
    c->max_iter      = 0;
    c->oms_pm        = 15.0;                /* SciRDv1: P = 15 */
    c->tm_fm         = 3.0;                 /* SciRDv1: A = 3 */
    c->arm_m         = 2.5e9;               /* L = 2.5e6 km */
    c->noise_scale   = 1.0;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------- O1 grid
 * The subtraction output is a frequency series with resolution 1/T_obs
 * (Sec. "Coarse-graining of the data").  Grid points are the DFT
 * frequencies (k0 + k)/T; an input frequency maps to the nearest one. */
int orc_grid(double T, double fmin, double fmax, int64_t *k0, int64_t *n_bins)
{
    if (!(T > 0.0) || !(fmin > 0.0) || !(fmax > fmin) || !isfinite(T) || !isfinite(fmax))
        return ORC_E_INVALID;
    double a = floor(fmin * T + 0.5);
    double b = floor(fmax * T + 0.5);
    if (!(b - a + 1.0 >= 1.0) || b - a + 1.0 > 2147483647.0 || a > 9.0e15)
        return ORC_E_INVALID;
    *k0 = (int64_t)a;
    *n_bins = (int64_t)b - (int64_t)a + 1;
    return ORC_OK;
}

/* ---------------------------------------------------------------- O2 noise
 * Appendix "LISA instrumental noise": OMS and test-mass noise
 *   P_OMS = (P pm)^2 [1 + (2 mHz/f)^4] (2 pi f / c)^2
 *   P_TM  = (A fm)^2 [1 + (0.4 mHz/f)^2] [1 + (f / 8 mHz)^4] (2 pi f)^-4 (2 pi f / c)^2
 * (the printed "(f/8 mHz^4)" is read as (f / 8 mHz)^4), and for an equilateral
 * constellation the A-channel PSD
 *   S_AA = 8 sin^2(u) { 4 [1 + cos u + cos^2 u] P_TM + [2 + cos u] P_OMS },
 * with u = f/f*, f* = c / (2 pi L). */
double orc_s_aa(double f, double oms_pm, double tm_fm, double arm_m)
{
    const double fstar = ORC_C_LIGHT / (2.0 * ORC_PI * arm_m);
    const double u = f / fstar;
    const double w = 2.0 * ORC_PI * f;            /* 2 pi f */
    const double wc = w / ORC_C_LIGHT;            /* 2 pi f / c */
    const double oms = oms_pm * 1e-12;
    const double tm = tm_fm * 1e-15;
    const double r_oms = 2e-3 / f;
    const double r_tm1 = 4e-4 / f;
    const double r_tm2 = f / 8e-3;
    const double p_oms = (oms * oms) * (1.0 + r_oms * r_oms * r_oms * r_oms) * (wc * wc);
    const double p_tm = (tm * tm) * (1.0 + r_tm1 * r_tm1)
                        * (1.0 + r_tm2 * r_tm2 * r_tm2 * r_tm2)
                        / (w * w * w * w) * (wc * wc);
    const double s = sin(u), co = cos(u);
    return 8.0 * (s * s) * (4.0 * (1.0 + co + co * co) * p_tm + (2.0 + co) * p_oms);
}

/* Appendix "Characteristic strain", TDI-response equation:
 *   R_AA = 16 sin^2(u) u^2 * (9/20) / (1 + 0.7 u^2). */
double orc_r_aa(double f, double arm_m)
{
    const double fstar = ORC_C_LIGHT / (2.0 * ORC_PI * arm_m);
    const double u = f / fstar;
    const double s = sin(u);
    return 16.0 * (s * s) * (u * u) * (0.45 / (1.0 + 0.7 * (u * u)));
}

/* The same appendix rescales the noise by the response, S -> S / R: the
 * strain-equivalent instrumental PSD that the catalog's strain amplitudes
 * are compared with. */
double orc_sinstr(double f, double oms_pm, double tm_fm, double arm_m)
{
    return orc_s_aa(f, oms_pm, tm_fm, arm_m) / orc_r_aa(f, arm_m);
}

void orc_sinstr_table(const orc_config *c, int64_t k0, int64_t n_bins, double *out)
{
    for (int64_t k = 0; k < n_bins; ++k) {
        double f = (double)(k0 + k) / c->t_obs_s;
        out[k] = orc_sinstr(f, c->oms_pm, c->tm_fm, c->arm_m) * c->noise_scale;
    }
}

/* ---------------------------------------------------------------- O3 track
 * A monochromatic source of amplitude A observed for T puts power
 * P = A^2 T / 2 in one bin of the one-sided periodogram.  With the phase
 * expansion phi = phi0 + 2 pi f t + pi fdot t^2 (Sec. "Signal
 * parametrization") the frequency sweeps f .. f + fdot T, i.e. |fdot| T^2
 * bins; the power is spread uniformly over n = 1 + floor(|fdot| T^2) bins
 * centred on the mid-track frequency.  Bins outside the grid are dropped. */
int orc_track(const orc_config *c, int64_t k0, int64_t n_bins, float Af, float ff, float fdf,
              int64_t *lo, int64_t *n, double *q, int64_t *glo, int64_t *ghi)
{
    const double T = c->t_obs_s;
    const double A = (double)Af, f = (double)ff, fd = (double)fdf;
    if (!isfinite(A) || !(A >= 0.0) || !isfinite(f) || !(f > 0.0) || !isfinite(fd))
        return ORC_E_INVALID;
    const double P = ((A * A) * T) * 0.5;
    const double fbar = f + (fd * T) * 0.5;
    const double x = fbar * T + 0.5;
    const double s = (fabs(fd) * T) * T;
    if (!(fabs(x) < 4503599627370496.0) || !(s < 4503599627370496.0)) {
        /* 2^52 bins or more away, or long: at most 2^-52 of the power in
         * any bin; no power on the grid (as for a source off the grid) */
        *lo = 0;
        *n = 0;
        *q = 0.0;
        *glo = 1;
        *ghi = 0;
        return ORC_OK;
    }
    const int64_t cbin = (int64_t)floor(x) - k0;
    const int64_t nn = (c->track_model == ORC_TRACK_SINGLE) ? 1 : 1 + (int64_t)floor(s);
    const int64_t l = cbin - (nn - 1) / 2;
    const int64_t h = l + nn - 1;
    *lo = l;
    *n = nn;
    *q = P / (double)nn;
    *glo = l < 0 ? 0 : l;
    *ghi = h > n_bins - 1 ? n_bins - 1 : h;
    return ORC_OK;
}

/* ---------------------------------------------------------------- O4 SNR
 * Eqs. "SNR inner product" and "inner product": rho^2 = sum over channels of
 * 4 Re int |h|^2 / S df.  A source of per-bin power q contributes, per
 * channel and bin, <h|h> = 2 q / S (one-sided PSD, df = 1/T); the A and E
 * channels carry the same sky-averaged power and T is insensitive, so
 * rho^2 = 4 q sum_k 1/S[k]. */
double orc_snr2(double q, int64_t glo, int64_t ghi, const double *S)
{
    double sum = 0.0;
    for (int64_t k = glo; k <= ghi; ++k)
        sum += 1.0 / S[k];
    return (4.0 * q) * sum;
}

/* ---------------------------------------------------------------- O6 estimators
 * Eq. "running median": S(f_k) = C median{X_j, j in window(k)} + S_instr(f_k).
 * Window: W (odd) consecutive bins centred on k, shifted inward at the grid
 * edges so that it always holds W bins; the median is the ((W+1)/2)-th
 * smallest.  If the grid is shorter than W the window is the whole grid and
 * the median is the ceil(B/2)-th smallest. */

/* k-th smallest (0-based) of a[0..n-1] by quickselect with a three-way
 * partition; a[] is permuted. */
static double select_kth(double *a, int64_t n, int64_t k)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        double x = a[lo], y = a[mid], z = a[hi], p;
        if (x < y) p = (y < z) ? y : ((x < z) ? z : x);
        else       p = (x < z) ? x : ((y < z) ? z : y);
        int64_t lt = lo, i = lo, gt = hi;
        while (i <= gt) {
            if (a[i] < p)      { double t = a[lt]; a[lt] = a[i]; a[i] = t; ++lt; ++i; }
            else if (a[i] > p) { double t = a[gt]; a[gt] = a[i]; a[i] = t; --gt; }
            else               { ++i; }
        }
        if (k < lt)      hi = lt - 1;
        else if (k > gt) lo = gt + 1;
        else             return p;
    }
    return a[lo];
}

static void window_of(int64_t k, int64_t n_bins, int64_t W, int64_t *a, int64_t *len, int64_t *rank)
{
    if (n_bins < W) {
        *a = 0;
        *len = n_bins;
        *rank = (n_bins + 1) / 2 - 1;
        return;
    }
    int64_t h = (W - 1) / 2;
    int64_t s = k - h;
    if (s < 0) s = 0;
    if (s > n_bins - W) s = n_bins - W;
    *a = s;
    *len = W;
    *rank = h;
}

void orc_running_median(const double *X, int64_t n_bins, int64_t W, double *out)
{
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(W < n_bins ? W : n_bins));
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n_bins; ++k) {
            int64_t a, len, rank;
            window_of(k, n_bins, W, &a, &len, &rank);
            memcpy(buf, X + a, sizeof(double) * (size_t)len);
            out[k] = select_kth(buf, len, rank);
        }
        free(buf);
    }
}

/* Eq. "running mean": S(f_k) = (1/W) sum_{j in window(k)} (X_j + S_instr(f_j)),
 * with the same window as the median. */
void orc_running_mean_psd(const double *X, const double *Sx, int64_t n_bins, int64_t W, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n_bins; ++k) {
        int64_t a, len, rank;
        window_of(k, n_bins, W, &a, &len, &rank);
        double sum = 0.0;
        for (int64_t j = a; j < a + len; ++j)
            sum += X[j] + Sx[j];
        out[k] = sum / (double)len;
    }
}

/* Coarse-graining: Sec. "Coarse-graining of the data".  Every grid sample is
 * assigned to its logarithmic bin by comparing f_i with the edges; the
 * spectrum and the frequencies are averaged over each bin in ascending i. */
int orc_coarse(const double *S, int64_t k0, int64_t n_bins, double T, double f_lo, double f_hi,
               int64_t n_out, double *f_out, double *s_out, int64_t *count)
{
    if (!(f_lo > 0.0) || !(f_hi > f_lo) || n_out < 1 || !(T > 0.0)) return ORC_E_INVALID;
    double *edge = (double *)malloc((size_t)(n_out + 1) * sizeof(double));
    if (!edge) return ORC_E_INVALID;
    for (int64_t j = 0; j <= n_out; ++j) edge[j] = f_lo * pow(f_hi / f_lo, (double)j / (double)n_out);
    edge[n_out] = f_hi;
    for (int64_t k = 0; k < n_out; ++k) {
        f_out[k] = 0.0;
        s_out[k] = 0.0;
        count[k] = 0;
    }
    for (int64_t i = 0; i < n_bins; ++i) {
        const double fi = (double)(k0 + i) / T;
        if (fi < edge[0] || fi > edge[n_out]) continue;
        int64_t k = 0;
        while (k + 1 < n_out && fi >= edge[k + 1]) ++k;
        f_out[k] += fi;
        s_out[k] += S[i];
        count[k] += 1;
    }
    for (int64_t k = 0; k < n_out; ++k) {
        if (count[k] > 0) {
            f_out[k] /= (double)count[k];
            s_out[k] /= (double)count[k];
        }
    }
    free(edge);
    return ORC_OK;
}

/* ---------------------------------------------------------------- X^t and S^t
 * The data "h_AET minus subtracted templates" in the power model: the
 * per-bin power of every source not yet subtracted, summed in ascending
 * source index (appendix "Subtraction algorithm", the subtraction step). */
static void bin_unsubtracted(int64_t n, const int32_t *iter_of, const int64_t *glo, const int64_t *ghi,
                             const double *q, int64_t B, double *X)
{
    for (int64_t k = 0; k < B; ++k) X[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (iter_of[i] >= 0) continue;
        for (int64_t k = glo[i]; k <= ghi[i]; ++k) X[k] += q[i];
    }
}

/* The PSD estimate of the data X (Eqs. "running median" and "running
 * mean"); med is scratch of B entries. */
static void estimate_psd(const orc_config *c, const double *X, const double *Sx, int64_t B, double *med,
                         double *S)
{
    if (c->estimator == ORC_MEAN) {
        orc_running_mean_psd(X, Sx, B, c->window_bins, S);
    } else {
        orc_running_median(X, B, c->window_bins, med);
        for (int64_t k = 0; k < B; ++k) S[k] = c->median_scale * med[k] + Sx[k];
    }
}

int orc_spectra_after(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
                      const uint8_t *subtracted, double *X, double *S)
{
    int64_t k0, B;
    if (n < 0 || !(c->window_bins >= 1) || (c->window_bins % 2) == 0) return ORC_E_INVALID;
    if (orc_grid(c->t_obs_s, c->f_min_hz, c->f_max_hz, &k0, &B) != ORC_OK) return ORC_E_INVALID;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t *glo = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *ghi = (int64_t *)malloc(sizeof(int64_t) * nn);
    double *q = (double *)malloc(sizeof(double) * nn);
    int32_t *iter_of = (int32_t *)malloc(sizeof(int32_t) * nn);
    double *Sx = (double *)malloc(sizeof(double) * (size_t)B);
    double *med = (double *)malloc(sizeof(double) * (size_t)B);
    int rc = ORC_OK;
    for (int64_t i = 0; i < n && rc == ORC_OK; ++i) {
        int64_t lo, nb;
        if (orc_track(c, k0, B, A[i], f[i], fdot[i], &lo, &nb, &q[i], &glo[i], &ghi[i]) != ORC_OK)
            rc = ORC_E_INVALID;
        iter_of[i] = subtracted[i] ? 0 : -1;
    }
    if (rc == ORC_OK) {
        orc_sinstr_table(c, k0, B, Sx);
        bin_unsubtracted(n, iter_of, glo, ghi, q, B, X);
        estimate_psd(c, X, Sx, B, med, S);
    }
    free(glo); free(ghi); free(q); free(iter_of); free(Sx); free(med);
    return rc;
}

/* ---------------------------------------------------------------- the loop
 * Appendix "Subtraction algorithm":
 *   2. SNR of every source against S_instr;
 *   3. keep the sources with rho >= kappa rho_th (candidates);
 *   repeat:
 *   5. estimate S^(t) with the running median (or mean) of the data that
 *      still holds every unsubtracted source;
 *   6. SNR of every candidate against S^(t);
 *   7-9. subtract every source with rho > rho_th;
 *   until nothing is subtracted (then S^(t) is also stationary).
 * The data "h_AET minus subtracted templates" is, in the power model, the
 * per-bin power X^t[k] = sum of q_i over unsubtracted sources i whose track
 * covers k; it is summed afresh each iteration in ascending source index. */
int orc_run(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
            orc_io *io, orc_summary *sum)
{
    int64_t k0, B;
    memset(sum, 0, sizeof(*sum));
    if (!(c->window_bins >= 1) || (c->window_bins % 2) == 0 || !(c->snr_threshold > 0.0) ||
        !(c->kappa >= 0.0) || !(c->median_scale >= 0.0) || n < 0)
        return ORC_E_INVALID;
    if (orc_grid(c->t_obs_s, c->f_min_hz, c->f_max_hz, &k0, &B) != ORC_OK)
        return ORC_E_INVALID;
    /* S_AA / R_AA is 0/0 where sin(f/f*) = 0; the first zero is at f = c/(2L). */
    if (!(c->arm_m > 0.0) || !(c->f_max_hz < ORC_C_LIGHT / (2.0 * c->arm_m)))
        return ORC_E_INVALID;
    sum->n_bins = B;
    sum->k0 = k0;

    const double rth = c->snr_threshold;
    const double rth2 = rth * rth;
    const double cut = c->kappa * rth;
    const double cut2 = cut * cut;
    const double band = (io && io->near_band > 0.0) ? io->near_band : 1e-6;

    double *Sx = (double *)malloc(sizeof(double) * (size_t)B);
    double *X = (double *)malloc(sizeof(double) * (size_t)B);
    double *S = (double *)malloc(sizeof(double) * (size_t)B);
    double *med = (double *)malloc(sizeof(double) * (size_t)B);
    int64_t *glo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *ghi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t *iter_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *rho2 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int rc = ORC_OK;

    orc_sinstr_table(c, k0, B, Sx);

    /* O3 for every source, then O4/O5: rho_0^2 against S_instr and the cut. */
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo, nn;
        if (orc_track(c, k0, B, A[i], f[i], fdot[i], &lo, &nn, &q[i], &glo[i], &ghi[i]) != ORC_OK) {
            rc = ORC_E_INVALID;
            goto done;
        }
        iter_of[i] = -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        double r0 = orc_snr2(q[i], glo[i], ghi[i], Sx);
        if (io && io->rho0_sq) io->rho0_sq[i] = r0;
        int is_c = r0 >= cut2;
        if (io && io->is_candidate) io->is_candidate[i] = (uint8_t)is_c;
        if (is_c) cand[nc++] = i;
    }
    sum->n_candidates = nc;
    const int64_t max_iter = c->max_iter > 0 ? c->max_iter : nc + 1;
    sum->min_rel_margin = INFINITY;

    for (int64_t t = 0;; ++t) {
        /* X^t: every source not yet subtracted; S^t */
        bin_unsubtracted(n, iter_of, glo, ghi, q, B, X);
        estimate_psd(c, X, Sx, B, med, S);
        /* rho^2 of every unsubtracted candidate against S^t */
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nc; ++j) {
            int64_t i = cand[j];
            rho2[j] = (iter_of[i] >= 0) ? -1.0 : orc_snr2(q[i], glo[i], ghi[i], S);
        }
        if (io && io->trace) io->trace(io->trace_user, t, B, X, S, nc, cand, rho2);
        /* decisions */
        int64_t n_new = 0;
        for (int64_t j = 0; j < nc; ++j) {
            if (rho2[j] < 0.0) continue;
            int64_t i = cand[j];
            double rel = fabs(sqrt(rho2[j]) / rth - 1.0);
            if (rel < sum->min_rel_margin) sum->min_rel_margin = rel;
            if (rel <= band) {
                if (io && sum->n_near < io->near_cap && io->near_t && io->near_i) {
                    io->near_t[sum->n_near] = t;
                    io->near_i[sum->n_near] = i;
                }
                sum->n_near++;
            }
            int dec = rho2[j] > rth2;
            if (io && io->n_over > 0) {
                for (int64_t o = 0; o < io->n_over; ++o)
                    if (io->over_t[o] == t && io->over_i[o] == i) dec = io->over_dec[o] != 0;
            }
            if (dec) {
                iter_of[i] = (int32_t)t;   /* marks it; X for this t is already summed */
                ++n_new;
            }
        }
        if (n_new == 0) {
            sum->n_iter = t + 1;
            if (io && io->S_final) memcpy(io->S_final, S, sizeof(double) * (size_t)B);
            if (io && io->X_final) memcpy(io->X_final, X, sizeof(double) * (size_t)B);
            break;
        }
        sum->n_resolved += n_new;
        if (t + 1 >= max_iter) {
            sum->n_iter = t + 1;
            rc = ORC_E_MAXITER;
            break;
        }
    }
done:
    if (io && io->iter_of && n > 0) memcpy(io->iter_of, iter_of, sizeof(int32_t) * (size_t)n);
    free(Sx); free(X); free(S); free(med); free(glo); free(ghi); free(q);
    free(iter_of); free(cand); free(rho2);
    return rc;
}
