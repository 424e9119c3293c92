/*
 * gbsub_oracle.h -- plain FP64 CPU oracle of the iterative galactic-binary
 * subtraction (TEST INFRASTRUCTURE ONLY).
 *
 * This is the reference that the HIP library is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * What it computes follows the paper (De Santi et al., "Inferring the
 * population properties of galactic binaries from LISA's stochastic
 * foreground"):
 *   - frequency grid with resolution 1/T_obs (Sec. "Coarse-graining of the
 *     data": the subtraction output has resolution 1/T_obs);
 *   - SciRDv1 instrumental noise S_AA (appendix "LISA instrumental noise")
 *     divided by the TDI response R_AA (appendix "Characteristic strain",
 *     TDI-response equation) to give a strain-equivalent PSD;
 *   - SNR^2 = sum over the A and E channels of <h|h> (Eqs. "SNR inner product"
 *     and "inner product") in the sky-averaged power form;
 *   - the subtraction algorithm of the appendix "Subtraction algorithm":
 *     initial SNR against S_instr, candidate cut rho >= kappa*rho_th, then
 *     repeat { running-median (or running-mean) PSD estimate, SNR against it,
 *     subtract every source with rho > rho_th } until nothing is subtracted.
 * Precision: IEEE binary64, round-to-nearest, no FMA contraction
 * (-ffp-contract=off), every sum in ascending index order.
 */
#ifndef GBSUB_ORACLE_H
#define GBSUB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_MAXITER = -6 };
enum { ORC_MEDIAN = 0, ORC_MEAN = 1 };
enum { ORC_TRACK_SWEEP = 0, ORC_TRACK_SINGLE = 1 };

typedef struct {
    double   t_obs_s, f_min_hz, f_max_hz;
    int64_t  window_bins;       /* odd, >= 1 */
    double   snr_threshold;     /* rho_th */
    double   kappa;             /* candidate cut rho_0 >= kappa*rho_th */
    double   median_scale;      /* C in S = C*median + S_instr */
    int32_t  estimator;         /* ORC_MEDIAN | ORC_MEAN */
    int32_t  track_model;       /* ORC_TRACK_SWEEP | ORC_TRACK_SINGLE */
    int64_t  max_iter;          /* 0 = n_candidates + 1 */
    double   oms_pm, tm_fm, arm_m;  /* SciRDv1: P = 15, A = 3, L = 2.5e9 m */
    double   noise_scale;       /* test hook: S_instr is multiplied by this (1.0 normally) */
} orc_config;

typedef struct {
    int64_t n_iter, n_bins, k0, n_candidates, n_resolved, n_near;
    double  min_rel_margin;     /* min over evaluated (t,i) of |rho/rho_th - 1| */
} orc_summary;

/* Per-iteration trace: called after S^t and the candidates' rho^2 at t are
 * known and before anything is subtracted.  X and S have n_bins entries;
 * cand[j] is the source index of candidate j, rho2[j] its rho^2 at t, or -1
 * if it was already resolved. */
typedef void (*orc_trace_fn)(void *user, int64_t t, int64_t n_bins,
                             const double *X, const double *S,
                             int64_t n_cand, const int64_t *cand, const double *rho2);

typedef struct {
    /* outputs (any may be NULL) */
    int32_t *iter_of;       /* [n] : t at which source i was resolved, -1 if never */
    uint8_t *is_candidate;  /* [n] */
    double  *rho0_sq;       /* [n] : rho^2 against S_instr */
    double  *S_final;       /* [n_bins] */
    double  *X_final;       /* [n_bins] */
    /* near-threshold log: (t, i) with |rho_i/rho_th - 1| <= near_band */
    double   near_band;     /* 1e-6 by default if <= 0 */
    int64_t  near_cap;
    int64_t *near_t, *near_i;
    /* guided replay: for these (t, i) the decision is taken from over_dec
     * (1 = resolve at t, 0 = do not) instead of from the comparison. */
    int64_t  n_over;
    const int64_t *over_t, *over_i;
    const uint8_t *over_dec;
    orc_trace_fn trace;
    void    *trace_user;
} orc_io;

void    orc_default_config(orc_config *c);
int     orc_set_threads(int n);           /* OpenMP threads; returns the count in use */

/* O1: grid.  k0 = floor(f_min*T + 1/2), k1 = floor(f_max*T + 1/2), B = k1-k0+1. */
int     orc_grid(double t_obs_s, double f_min_hz, double f_max_hz, int64_t *k0, int64_t *n_bins);

/* O2: strain-equivalent instrumental PSD S_AA(f)/R_AA(f), and its parts. */
double  orc_s_aa(double f, double oms_pm, double tm_fm, double arm_m);
double  orc_r_aa(double f, double arm_m);
double  orc_sinstr(double f, double oms_pm, double tm_fm, double arm_m);
void    orc_sinstr_table(const orc_config *c, int64_t k0, int64_t n_bins, double *out);

/* O3: power and track of one source.  Returns ORC_OK or ORC_E_INVALID. */
int     orc_track(const orc_config *c, int64_t k0, int64_t n_bins, float A, float f, float fdot,
                  int64_t *lo, int64_t *n, double *q, int64_t *glo, int64_t *ghi);

/* O4: rho^2 = 4 q sum_{k in [glo,ghi]} 1/S[k] (0 if the range is empty). */
double  orc_snr2(double q, int64_t glo, int64_t ghi, const double *S);

/* O6: running-median (clamped full window of odd width W) and running-mean
 * order statistics; out[k] = ((W+1)/2)-th smallest of the window of k. */
void    orc_running_median(const double *X, int64_t n_bins, int64_t W, double *out);
void    orc_running_mean_psd(const double *X, const double *Sx, int64_t n_bins, int64_t W, double *out);

/* Coarse-graining (Sec. "Coarse-graining of the data", Eqs. "coarse graining
 * spectrum" and "coarse graining frequencies"): n_out logarithmically spaced
 * bins with edges e_j = f_lo (f_hi/f_lo)^(j/n_out); grid sample i (f_i =
 * (k0+i)/T) belongs to bin k iff e_k <= f_i < e_{k+1} (the last bin also
 * takes f_i = f_hi).  f_out[k] and s_out[k] are the means of f_i and S[i]
 * over the bin; count[k] = N_k (means are 0 where N_k = 0).  Returns
 * ORC_E_INVALID for bad arguments. */
int     orc_coarse(const double *S, int64_t k0, int64_t n_bins, double T, double f_lo, double f_hi,
                   int64_t n_out, double *f_out, double *s_out, int64_t *count);

/* X^t and S^t of the loop once exactly the sources with subtracted[i] != 0
 * have been subtracted: the binned power of all others (ascending source
 * index) and the PSD estimate over it, the same operations as a loop body.
 * With the final resolved set this is the run's X_final and S_final.
 * X and S have n_bins entries.  Returns ORC_OK or ORC_E_INVALID. */
int     orc_spectra_after(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
                          const uint8_t *subtracted, double *X, double *S);

/* The whole subtraction.  Returns ORC_OK, ORC_E_INVALID or ORC_E_MAXITER. */
int     orc_run(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
                orc_io *io, orc_summary *sum);

/* Complex-template data model (template_oracle.c; Sec. "Simulations",
 * appendix "Subtraction algorithm", Eq. "vectorized-subtraction"): N-sample
 * templates U (re, im interleaved, j = -N/2 .. N/2-1 at DFT index q + j),
 * one complex series per channel A and E. */
#define ORC_CX_NF 128
typedef struct {
    int32_t *iter_of;       /* [n] */
    uint8_t *is_candidate;  /* [n] */
    double  *rho0_sq;       /* [n]  rho^2 against S_instr (both channels) */
    double  *rho2_last;     /* [n]  rho^2 at the last evaluation (candidates only) */
    int64_t *q;             /* [n]  central DFT index, INT64_MIN if no template */
    double  *S_final;       /* [2][n_bins]  S_A, S_E */
    double  *X_final;       /* [2][n_bins]  X_A, X_E */
    double  *h_final;       /* [2][n_bins][2]  h_A, h_E (re, im) */
    double   near_band;     /* 1e-6 by default if <= 0 */
} orc_cx_io;
/* U[2N] and *q of one source (INT64_MIN and U = 0 if it has no template on
 * the grid); ORC_E_INVALID for an invalid entry. */
int     orc_cx_template(const orc_config *c, float A, float f, float fdot, int64_t *q, double *U);
int     orc_cx_run(const orc_config *c, int64_t n, const float *A, const float *f, const float *fdot,
                   const float *phi_a, const float *phi_e, orc_cx_io *io, orc_summary *sum);

/* ---------------------------------------------------------------- population model
 * (population_oracle.c; Sec. "Population model", Table "priors", appendix
 * "Copulas") */
typedef struct {
    double alpha_pl;            /* power-law index of f, alpha_PL != -1 */
    double alpha_g, beta_g;     /* Gamma shape and rate of log10(fdot) - mu_Gamma */
    double mu_g;                /* mu_Gamma */
    double mu;                  /* mu of the rescaled log amplitude */
    double sigma;               /* log-normal shape of the rescaled log amplitude */
    double rho;                 /* Gaussian-copula correlation of (f, fdot), |rho| < 1 */
    double f_lo_hz, f_hi_hz;    /* support of the power law */
} orc_population;

/* Philox4x32-10: out = the 10-round bijection of ctr under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Regularized lower incomplete gamma P(a, x). */
double orc_gamma_p(double a, double x);
/* Quantile of Gamma(shape, rate): x with P(shape, rate x) = p. */
double orc_gamma_quantile(double shape, double rate, double p);
/* (u, v) copula uniforms and w ~ N(0,1) -> f, fdot, A. */
void orc_pop_transform(const orc_population *p, double u, double v, double w, double *f, double *fdot,
                       double *A);
/* Sources first .. first+n-1 of the catalog drawn with `seed` (fp32 A, f,
 * fdot; id = source index; id may be NULL).  ORC_E_INVALID on bad
 * parameters. */
int orc_pop_draw(const orc_population *p, uint64_t seed, uint64_t first, int64_t n, float *A, float *f,
                 float *fdot, uint32_t *id);

#ifdef __cplusplus
}
#endif
#endif
