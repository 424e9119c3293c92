/*
 * template_oracle.c -- plain FP64 CPU oracle of the complex-template data
 * model.  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and
 * the benchmark's CPU-baseline leg, never by the product path.
 *
 * The data is one complex frequency series per TDI channel, h_A and h_E
 * (the T channel is insensitive to gravitational waves: Sec.
 * "Simulations"), holding the sum of the frequency-domain templates of all
 * injected sources (appendix "Subtraction algorithm": the starting point is
 * the sum of every source).  A template has N = 128 samples around the
 * source's central frequency (Sec. "Simulations"), and resolved sources are
 * taken out of h at their template's bins (Eq. "vectorized-subtraction").
 * The paper draws its templates from gbgpu, which is not available; the
 * waveform and response model below is a sky-averaged one of our own:
 *
 *   template   q = floor((f + fdot T/2) T + 1/2)        central DFT index
 *              delta = f T - q,  d = fdot T^2
 *              s_n = (A/2) exp(2 pi i theta_n),  theta_n = delta x_n + d x_n^2 / 2,
 *              x_n = n / N  (n = 0 .. N-1)
 *              U_j = (T/N) sum_n s_n exp(-2 pi i m n / N),  m = j mod N,
 *              j = -N/2 .. N/2-1, at DFT index q + j.
 *              s is the slowly varying factor of the analytic signal
 *              (A/2) exp(2 pi i (f t + fdot t^2 / 2)) once the carrier q/T
 *              is taken out, sampled N times over T; its N-point DFT gives
 *              the N bins around q (a fast/slow template).  A track wider
 *              than N bins wraps around inside the N bins.
 *   channels   H_c,j = exp(i phi_c) U_j, c in {A, E}: the same sky-averaged
 *              power in A and E, and a phase of each channel per source
 *              (catalog inputs).
 *   data       h_c[k] = sum over sources of H_c,j with k = q + j - k0 on the
 *              grid (bins off the grid are dropped).
 *   power      X_c[k] = (2/T) |h_c[k]|^2: the one-sided periodogram; a
 *              bin-centred monochromatic source gives A^2 T / 2, as in the
 *              power model.
 *   PSD        S_c = C median_W(X_c) + S_instr (Eq. "running median") or the
 *              running mean (Eq. "running mean"), channel by channel.
 *   SNR        rho^2 = sum_c (4/T) sum_j |H_c,j|^2 / S_c[q + j - k0] over the
 *              grid bins (Eqs. "SNR inner product" and "inner product" with
 *              df = 1/T).
 *
 * A source with |fdot| T^2 >= 2^20 or |(f + fdot T/2) T| >= 2^52 has no
 * template on the grid (its phases would lose their fractional part).
 *
 * Every sum runs in ascending index order (no FMA contraction), so each
 * result is a fixed sequence of binary64 operations.  OpenMP runs only over
 * independent outputs.
 */
#include "gbsub_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define T_PI 3.14159265358979323846

/* ---------------------------------------------------------------- template */
int orc_cx_template(const orc_config *c, float Af, float ff, float fdf, int64_t *q, double *U)
{
    const double T = c->t_obs_s;
    const double A = (double)Af, f = (double)ff, fd = (double)fdf;
    const int N = ORC_CX_NF;
    if (!isfinite(A) || !(A >= 0.0) || !isfinite(f) || !(f > 0.0) || !isfinite(fd))
        return ORC_E_INVALID;
    for (int k = 0; k < 2 * N; ++k) U[k] = 0.0;
    const double x = (f + (fd * T) * 0.5) * T + 0.5;
    const double d = (fd * T) * T;
    if (!(fabs(x) < 4503599627370496.0) || !(fabs(d) < 1048576.0)) {
        *q = INT64_MIN;              /* no template on the grid */
        return ORC_OK;
    }
    const double qd = floor(x);
    *q = (int64_t)qd;
    const double delta = f * T - qd;
    /* samples of the slowly varying factor */
    double sr[ORC_CX_NF], si[ORC_CX_NF];
    for (int n = 0; n < N; ++n) {
        const double xn = (double)n / (double)N;
        double th = delta * xn + (d * 0.5) * (xn * xn);
        th = th - floor(th);         /* whole turns removed (exact) */
        sr[n] = (A * 0.5) * cos(2.0 * T_PI * th);
        si[n] = (A * 0.5) * sin(2.0 * T_PI * th);
    }
    /* N-point DFT, term by term */
    for (int m = 0; m < N; ++m) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < N; ++n) {
            const double ang = 2.0 * T_PI * (double)((m * n) % N) / (double)N;
            const double cr = cos(ang), ci = -sin(ang);        /* exp(-i ang) */
            re += sr[n] * cr - si[n] * ci;
            im += sr[n] * ci + si[n] * cr;
        }
        const int j = m < N / 2 ? m : m - N;
        U[2 * (j + N / 2)] = (T / (double)N) * re;
        U[2 * (j + N / 2) + 1] = (T / (double)N) * im;
    }
    return ORC_OK;
}

/* H_c,j = exp(i phi) U_j */
static void channel_template(const double *U, double phi, double *H)
{
    const double cp = cos(phi), sp = sin(phi);
    for (int j = 0; j < ORC_CX_NF; ++j) {
        const double ur = U[2 * j], ui = U[2 * j + 1];
        H[2 * j] = cp * ur - sp * ui;
        H[2 * j + 1] = sp * ur + cp * ui;
    }
}

/* (4/T) sum_j |H_j|^2 / S[q + j - k0] over the grid bins */
static double channel_snr2(const double *H, int64_t q, int64_t k0, int64_t B, double T, const double *S)
{
    double sum = 0.0;
    for (int j = 0; j < ORC_CX_NF; ++j) {
        const int64_t k = q + (j - ORC_CX_NF / 2) - k0;
        if (k < 0 || k >= B) continue;
        const double p = H[2 * j] * H[2 * j] + H[2 * j + 1] * H[2 * j + 1];
        sum += p / S[k];
    }
    return (4.0 / T) * sum;
}

/* h_c = sum of the channel templates of the sources not subtracted, in
 * ascending source index; X_c = (2/T) |h_c|^2.  h is [2][B] complex
 * (re, im interleaved), X is [2][B]. */
static void data_of(int64_t n, const int32_t *iter_of, const int64_t *q, const double *H, int64_t k0,
                    int64_t B, double T, double *h, double *X)
{
    const int N = ORC_CX_NF;
    for (int64_t k = 0; k < 4 * B; ++k) h[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (iter_of[i] >= 0 || q[i] == INT64_MIN) continue;
        for (int ch = 0; ch < 2; ++ch) {
            const double *Hc = H + ((size_t)i * 2 + (size_t)ch) * 2 * N;
            double *hc = h + (size_t)ch * 2 * (size_t)B;
            for (int j = 0; j < N; ++j) {
                const int64_t k = q[i] + (j - N / 2) - k0;
                if (k < 0 || k >= B) continue;
                hc[2 * k] += Hc[2 * j];
                hc[2 * k + 1] += Hc[2 * j + 1];
            }
        }
    }
    for (int ch = 0; ch < 2; ++ch)
        for (int64_t k = 0; k < B; ++k) {
            const double re = h[(size_t)ch * 2 * B + 2 * k], im = h[(size_t)ch * 2 * B + 2 * k + 1];
            X[(size_t)ch * B + k] = (2.0 / T) * (re * re + im * im);
        }
}

static void psd_of(const orc_config *c, const double *X, const double *Sx, int64_t B, double *med, double *S)
{
    if (c->estimator == ORC_MEAN) {
        orc_running_mean_psd(X, Sx, B, c->window_bins, S);
    } else {
        orc_running_median(X, B, c->window_bins, med);
        for (int64_t k = 0; k < B; ++k) S[k] = c->median_scale * med[k] + Sx[k];
    }
}

/* ---------------------------------------------------------------- the loop
 * Appendix "Subtraction algorithm" on the complex data: rho_0 of every
 * source against S_instr in both channels, the candidate cut, then loop
 * bodies t = 0, 1, ... of {h_c^t = templates of the sources not yet
 * subtracted; S_c^t of each channel; rho^2 of every unsubtracted candidate;
 * subtract every source with rho > rho_th} until a body subtracts nothing. */
int orc_cx_run(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
               const float *phi_a, const float *phi_e, orc_cx_io *io, orc_summary *sum)
{
    int64_t k0, B;
    const int N = ORC_CX_NF;
    memset(sum, 0, sizeof(*sum));
    if (!(c->window_bins >= 1) || (c->window_bins % 2) == 0 || !(c->snr_threshold > 0.0) ||
        !(c->kappa >= 0.0) || !(c->median_scale >= 0.0) || n < 0)
        return ORC_E_INVALID;
    if (orc_grid(c->t_obs_s, c->f_min_hz, c->f_max_hz, &k0, &B) != ORC_OK) return ORC_E_INVALID;
    if (!(c->arm_m > 0.0) || !(c->f_max_hz < 299792458.0 / (2.0 * c->arm_m))) return ORC_E_INVALID;
    sum->n_bins = B;
    sum->k0 = k0;
    const double T = c->t_obs_s;
    const double rth = c->snr_threshold, rth2 = rth * rth;
    const double cut = c->kappa * rth, cut2 = cut * cut;
    const double band = (io && io->near_band > 0.0) ? io->near_band : 1e-6;
    const size_t nn = (size_t)(n > 0 ? n : 1);

    double *Sx = (double *)malloc(sizeof(double) * (size_t)B);
    double *h = (double *)malloc(sizeof(double) * 4 * (size_t)B);
    double *X = (double *)malloc(sizeof(double) * 2 * (size_t)B);
    double *S = (double *)malloc(sizeof(double) * 2 * (size_t)B);
    double *med = (double *)malloc(sizeof(double) * (size_t)B);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * nn);
    double *H = (double *)malloc(sizeof(double) * nn * 4 * (size_t)N);   /* [n][2 channels][N] complex */
    int32_t *iter_of = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * nn);
    double *rho2 = (double *)malloc(sizeof(double) * nn);
    int rc = ORC_OK;
    orc_sinstr_table(c, k0, B, Sx);

    for (int64_t i = 0; i < n; ++i) {
        double U[2 * ORC_CX_NF];
        if (!isfinite(phi_a[i]) || !isfinite(phi_e[i]) ||
            orc_cx_template(c, A[i], f[i], fdot[i], &q[i], U) != ORC_OK) {
            rc = ORC_E_INVALID;
            goto done;
        }
        channel_template(U, (double)phi_a[i], H + (size_t)i * 4 * N);
        channel_template(U, (double)phi_e[i], H + (size_t)i * 4 * N + 2 * N);
        iter_of[i] = -1;
    }
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        double r0 = 0.0;
        if (q[i] != INT64_MIN)
            r0 = channel_snr2(H + (size_t)i * 4 * N, q[i], k0, B, T, Sx) +
                 channel_snr2(H + (size_t)i * 4 * N + 2 * N, q[i], k0, B, T, Sx);
        if (io && io->rho0_sq) io->rho0_sq[i] = r0;
        const int is_c = r0 >= cut2;
        if (io && io->is_candidate) io->is_candidate[i] = (uint8_t)is_c;
        if (is_c) cand[nc++] = i;
    }
    sum->n_candidates = nc;
    const int64_t max_iter = c->max_iter > 0 ? c->max_iter : nc + 1;
    sum->min_rel_margin = INFINITY;

    for (int64_t t = 0;; ++t) {
        data_of(n, iter_of, q, H, k0, B, T, h, X);
        psd_of(c, X, Sx, B, med, S);
        psd_of(c, X + B, Sx, B, med, S + B);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nc; ++j) {
            const int64_t i = cand[j];
            rho2[j] = iter_of[i] >= 0 ? -1.0
                                      : channel_snr2(H + (size_t)i * 4 * N, q[i], k0, B, T, S) +
                                            channel_snr2(H + (size_t)i * 4 * N + 2 * N, q[i], k0, B, T, S + B);
        }
        int64_t n_new = 0;
        for (int64_t j = 0; j < nc; ++j) {
            if (rho2[j] < 0.0) continue;
            const double rel = fabs(sqrt(rho2[j]) / rth - 1.0);
            if (rel < sum->min_rel_margin) sum->min_rel_margin = rel;
            if (rel <= band) sum->n_near++;
            if (rho2[j] > rth2) {
                iter_of[cand[j]] = (int32_t)t;
                ++n_new;
            }
        }
        if (io && io->rho2_last) {
            for (int64_t j = 0; j < nc; ++j)
                if (rho2[j] >= 0.0) io->rho2_last[cand[j]] = rho2[j];
        }
        if (n_new == 0) {
            sum->n_iter = t + 1;
            if (io && io->S_final) memcpy(io->S_final, S, sizeof(double) * 2 * (size_t)B);
            if (io && io->X_final) memcpy(io->X_final, X, sizeof(double) * 2 * (size_t)B);
            if (io && io->h_final) memcpy(io->h_final, h, sizeof(double) * 4 * (size_t)B);
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
    if (io && io->q && rc != ORC_E_INVALID) {
        for (int64_t i = 0; i < n; ++i) io->q[i] = q[i];
    }
    free(Sx); free(h); free(X); free(S); free(med); free(q); free(H);
    free(iter_of); free(cand); free(rho2);
    return rc;
}
