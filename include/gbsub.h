/*
 * gbsub.h -- C ABI of the MI355X (gfx950) iterative galactic-binary
 * subtraction library ``libgbsub.so``.
 *
 * The library turns a catalog of galactic binaries (amplitude A, frequency f,
 * frequency derivative fdot) into the reconstructed total PSD
 * S_n = S_instr + S_gal on the 1/T_obs frequency grid, following the
 * subtraction algorithm of De Santi et al., "Inferring the population
 * properties of galactic binaries from LISA's stochastic foreground",
 * appendix "Subtraction algorithm" (initial SNR against S_instr, candidate
 * cut rho >= kappa*rho_th, then repeat {running-median PSD estimate, SNR
 * against it, subtract every source with rho > rho_th} until nothing is
 * subtracted).  Power model: each source puts A^2 T/2 of one-sided power,
 * spread uniformly over the 1 + floor(|fdot| T^2) bins of its linear
 * frequency drift (Sec. "Signal parametrization"); SNR^2 = 4 q sum 1/S over
 * those bins, the A and E channels of Eq. "SNR inner product"; S_instr is the
 * SciRDv1 A-channel noise of appendix "LISA instrumental noise" divided by the
 * TDI response of appendix "Characteristic strain".
 *
 * Conventions for every call:
 *  - All functions are thread-compatible: one context per host thread.
 *  - No call throws; every call returns a gbsub_status.  Outputs are valid
 *    only on GBSUB_OK.  After GBSUB_E_DEVICE the context must be destroyed;
 *    after GBSUB_E_INVALID, GBSUB_E_TRUNCATED or GBSUB_E_MAXITER it stays
 *    usable.
 *  - "Device pointer" means memory on the GPU the context was created on
 *    (e.g. a torch CUDA tensor's data_ptr()); "host pointer" means ordinary
 *    host memory.  The library allocates no device memory at run time: every
 *    device buffer (catalog, workspace, device-side outputs) belongs to the
 *    caller, except the fixed array behind gbsub_run_static.
 *  - ``stream`` is a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef GBSUB_H
#define GBSUB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gbsub_ctx gbsub_ctx;              /* opaque, one per host thread */

typedef enum {
    GBSUB_OK = 0,
    GBSUB_E_INVALID = -1,      /* bad argument, config or catalog entry */
    GBSUB_E_NOMEM = -2,        /* host allocation failed / workspace too small */
    GBSUB_E_DEVICE = -3,       /* HIP runtime or kernel error: destroy the context */
    GBSUB_E_STATE = -4,        /* call out of order (e.g. results before any run) */
    GBSUB_E_TRUNCATED = -5,    /* output capacity too small; *n holds the size needed */
    GBSUB_E_MAXITER = -6       /* max_iter loop bodies ran and sources were still resolving */
} gbsub_status;

enum { GBSUB_MEDIAN = 0, GBSUB_MEAN = 1 };                 /* PSD estimator */
enum { GBSUB_TRACK_SWEEP = 0, GBSUB_TRACK_SINGLE = 1 };    /* spectral support of a source */
enum { GBSUB_FP64 = 0, GBSUB_FP32_COMP = 1, GBSUB_FP32_NAIVE = 2 };  /* accumulation precision */
enum {                                                     /* gbsub_spectrum kinds */
    GBSUB_SPEC_SN = 0,          /* S_n = C*median(X) + S_instr at the fixed point */
    GBSUB_SPEC_X_RESIDUAL = 1,  /* X: per-bin power of the sources left unresolved */
    GBSUB_SPEC_S_GAL = 2,       /* S_n - S_instr */
    GBSUB_SPEC_S_INSTR = 3      /* S_instr on the grid */
};

/* Run parameters.  Grid: bins k = 0..B-1 at f_k = (k0+k)/T with
 * k0 = floor(f_min*T + 1/2), B = floor(f_max*T + 1/2) - k0 + 1 (Sec.
 * "Coarse-graining of the data": resolution 1/T_obs).  Window: window_bins
 * (odd) consecutive bins, shifted inward at the grid edges; the median is
 * the ((W+1)/2)-th smallest (Eq. "running median").  Candidate cut:
 * rho_0^2 >= (kappa*rho_th)^2; resolve: rho^2 > rho_th^2. */
typedef struct {
    double   t_obs_s;          /* T_obs in seconds, > 0 */
    double   f_min_hz;         /* grid start, > 0 */
    double   f_max_hz;         /* grid end, f_min < f_max < c/(2 arm_m) */
    uint32_t window_bins;      /* odd W, 1 <= W <= 2817 */
    uint32_t estimator;        /* GBSUB_MEDIAN: S = C med_W(X) + S_instr; GBSUB_MEAN:
                                  S = (1/W) sum_window (X + S_instr) (FP64 only) */
    double   snr_threshold;    /* rho_th, default 7 */
    double   kappa;            /* candidate cut, default 1/rho_th */
    double   median_scale;     /* C, default 729/512 = (1 - 2/18)^-3 */
    uint32_t track_model;      /* GBSUB_TRACK_SWEEP (default) | GBSUB_TRACK_SINGLE */
    uint32_t precision;        /* loop arithmetic: GBSUB_FP64 (default: exact 128-bit fixed-point bin
                                  sums, fp64 S and SNR sums) | GBSUB_FP32_COMP (double-fp32 bin sums,
                                  prefixes and SNR sums, fp32 S) | GBSUB_FP32_NAIVE (plain fp32 sums
                                  by float atomics); median estimator only for the FP32 modes */
    uint32_t max_iter;         /* maximum loop bodies; 0 = n_candidates + 1 */
    uint32_t reserved0;
    double   oms_pm;           /* SciRDv1 OMS level P, default 15 (pm/sqrt(Hz)) */
    double   tm_fm;            /* SciRDv1 test-mass level A, default 3 (fm/s^2/sqrt(Hz)) */
    double   arm_m;            /* arm length L, default 2.5e9 m */
    /* Schedule (results are the same up to the association of the fp64 sums
     * of 1/S, see the tuner in paper_2602_18560_amd/autotune.py): */
    uint32_t tile_bins;        /* bins per tile: a power of two in [256, 2048] with
                                  tile_bins + W - 1 <= 3072; 0 = the largest allowed */
    uint32_t split_blocks;     /* the median runs one block per 512-bin part while
                                  dirty tiles x parts per tile <= split_blocks (shared by
                                  the running catalogs of a batch); 0 = 512, 1 = never */
} gbsub_config;

/* A catalog in structure-of-arrays form.  A, f, fdot, id are DEVICE
 * pointers to n entries each, read-only, not retained after gbsub_run
 * returns.  Valid entries: finite A >= 0, finite f > 0, finite fdot,
 * a source with |fdot|*T^2 or |(f + fdot*T/2)*T| at 2^52 or beyond puts no
 * power on the grid (at most 2^-52 of it would fall in any bin).  ids are
 * opaque. */
typedef struct {
    uint64_t        n;
    const float    *A;
    const float    *f;
    const float    *fdot;
    const uint32_t *id;
} gbsub_catalog;

typedef struct {
    uint32_t n_iter;             /* loop bodies run, including the final one that resolved nothing */
    uint32_t reserved0;
    uint64_t n_bins;             /* B */
    uint64_t n_candidates;       /* sources with rho_0 >= kappa*rho_th */
    uint64_t n_resolved;         /* sources subtracted */
    uint64_t n_near_threshold;   /* evaluations (t, i) with |rho/rho_th - 1| <= 1e-6 */
    double   min_rel_margin;     /* min over evaluations of |rho/rho_th - 1| */
} gbsub_summary;

/* Fills *cfg with the paper's defaults (rho_th = 7, kappa = 1/7, C = 729/512,
 * SciRDv1 P = 15, A = 3, L = 2.5e9 m, median estimator, sweep tracks, FP64)
 * and T = 4 yr on [0.1, 30] mHz with W = 1001.  Never fails. */
void gbsub_default_config(gbsub_config *cfg);

/* Validates *cfg (host pointer) and creates a context bound to the current
 * HIP device.  *out receives the context (host pointer owned by the library,
 * freed by gbsub_destroy).  INVALID on a bad config, NOMEM if the host
 * allocation fails, DEVICE if no HIP device is usable. */
gbsub_status gbsub_create(const gbsub_config *cfg, gbsub_ctx **out);

/* Bytes of device workspace that gbsub_run needs for a catalog of n_sources
 * sources on this context's grid (written to *bytes, host pointer). */
gbsub_status gbsub_workspace_size(const gbsub_ctx *ctx, uint64_t n_sources, uint64_t *bytes);

/* Runs the whole subtraction on `cat` (host pointer to a struct holding
 * device pointers): appendix "Subtraction algorithm" end to end -- the
 * initial SNR against S_instr and the candidate cut (its steps 2-3), then
 * loop bodies t = 0, 1, ... of {running-median PSD estimate S^t (Eq.
 * "running median"), rho^2 of every unresolved candidate against S^t (Eq.
 * "SNR inner product"), subtraction of every source with rho > rho_th (steps
 * 6-9)} until a body subtracts nothing (step 10; n_iter counts the bodies,
 * the last one included).  `workspace` is a DEVICE pointer to at least
 * gbsub_workspace_size() bytes, 256-byte aligned, owned by the caller and
 * holding the results until the next run or destroy.  All work is enqueued
 * on `stream`; the call returns after it has completed.  While it runs, the
 * calling thread keeps a couple of loop bodies queued ahead of the GPU,
 * polling (and yielding) on a progress word that the loop writes to the
 * context's pinned host memory.  *out (host
 * pointer, may be NULL) receives the summary.  INVALID for a bad catalog
 * entry or too small a workspace, MAXITER if the loop did not settle within
 * max_iter bodies, DEVICE on a HIP error. */
gbsub_status gbsub_run(gbsub_ctx *ctx, const gbsub_catalog *cat, void *workspace,
                       uint64_t ws_bytes, void *stream, gbsub_summary *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as gbsub_run, with the workspace taken from an array of
 * GBSUB_STATIC_WORKSPACE_BYTES bytes that the library holds on each GPU it
 * runs on (from the first gbsub_create on that GPU until the process ends).
 * The call allocates nothing; the caller still passes the catalog (device
 * arrays, as for gbsub_run) and reads results with gbsub_spectrum /
 * gbsub_resolved / gbsub_candidates / gbsub_coarse as after gbsub_run.
 * Every context on one GPU shares that GPU's array: a context's results stay
 * valid only until the next gbsub_run_static call on the same GPU (by any
 * context), and calls that overlap in time on one GPU (several host threads
 * or streams) race and must be serialised by the caller.  The grid tables
 * are recomputed on every call.  Profiling is not applied to these runs.
 * Errors: NOMEM if gbsub_workspace_size(ctx, cat->n) exceeds
 * GBSUB_STATIC_WORKSPACE_BYTES (e.g. the 1-yr [0.3, 10] mHz grid fits up to
 * ~5e5 sources, the 4-yr [0.1, 30] mHz grid does not fit); STATE while the
 * context holds a batch slot; otherwise as gbsub_run. */
#define GBSUB_STATIC_WORKSPACE_BYTES (64u << 20)
gbsub_status gbsub_run_static(gbsub_ctx *ctx, const gbsub_catalog *cat, void *stream, gbsub_summary *out);

/* Copies spectrum `kind` (GBSUB_SPEC_*) of the last successful run, B fp64
 * values in grid order, to `out` (host pointer if out_on_device == 0, device
 * pointer otherwise): S_n, the frequency series of the estimated PSD on the
 * 1/T_obs grid that the paper's statement of the problem returns (Sec.
 * "Coarse-graining of the data"), at the loop's fixed point; X, the binned
 * power of the sources left in the data; S_gal = S_n - S_instr (computed on
 * the device); S_instr (appendices "LISA instrumental noise" and
 * "Characteristic strain").  *n_bins (host) receives B.  TRUNCATED if cap < B,
 * STATE if no run has completed. */
gbsub_status gbsub_spectrum(const gbsub_ctx *ctx, uint32_t kind, double *out, uint64_t cap,
                            uint64_t *n_bins, int out_on_device);

/* Copies the resolved sources of the last successful run (the sources the
 * appendix "Subtraction algorithm" takes out of the data, step 9, with the
 * loop body of each): ids[j] (uint32) in ascending id order, and iter_of[j]
 * (int32, may be NULL) = the loop body t in which ids[j] was subtracted.
 * Built on the device (compaction of the candidate records, radix sort by
 * id) in the run's workspace; the run's spectra are untouched.  Host pointers if out_on_device == 0,
 * device pointers otherwise.  *n (host) receives the count; TRUNCATED if
 * cap is smaller.  STATE if no run has completed. */
gbsub_status gbsub_resolved(const gbsub_ctx *ctx, uint32_t *ids, int32_t *iter_of, uint64_t cap,
                            uint64_t *n, int out_on_device);

/* Coarse-graining of a spectrum of the last successful run (Sec.
 * "Coarse-graining of the data"): n_out (1..256) logarithmic bins with edges
 * e_j = f_lo (f_hi/f_lo)^(j/n_out); grid sample f_i = (k0+i)/T belongs to bin
 * k iff e_k <= f_i < e_{k+1} (the last bin also takes f_i = f_hi).  Writes,
 * to HOST arrays of n_out entries, the mean frequency f_k and the mean
 * spectrum of each bin (kind as in gbsub_spectrum), the characteristic
 * strain sqrt(f_k S_k) (Eq. "characteristic strain"; S_n is already the
 * response-rescaled PSD) to hc_out (may be NULL) and N_k to count (may be
 * NULL); empty bins get 0.  The paper's setting is f_lo = 0.1 mHz,
 * f_hi = 10 mHz, n_out = 100.  STATE if no run has completed. */
gbsub_status gbsub_coarse(const gbsub_ctx *ctx, uint32_t kind, double f_lo, double f_hi, uint32_t n_out,
                          double *f_out, double *s_out, double *hc_out, uint32_t *count);

/* Every candidate of the last successful run (the sources with rho_0 >=
 * kappa rho_th), in ascending id: ids[], the loop body that resolved it in
 * iter_of[] (-1 if never; may be NULL) and rho^2 in rho2[] (may be NULL):
 * at the body that resolved it, else against the final spectrum (as last
 * evaluated, in the latest body whose spectrum changed on its track).
 * All pointers are HOST memory of `cap` entries; *n (host) receives the
 * candidate count; TRUNCATED if cap is smaller; STATE if no run has
 * completed.  The rho^2 values are those of the run's precision mode. */
gbsub_status gbsub_candidates(const gbsub_ctx *ctx, uint32_t *ids, int32_t *iter_of, double *rho2,
                              uint64_t cap, uint64_t *n);

/* ---------------------------------------------------------------- catalogs
 * Population model of Sec. "Population model" (Table "priors", appendix
 * "Copulas"): f ~ f^alpha_PL on [f_lo, f_hi]; log10(fdot) - mu_Gamma ~
 * Gamma(alpha_Gamma, rate beta_Gamma); log10(f^(-2/3) A) - mu ~ log-normal
 * with log-scale 0 and shape sigma; (f, fdot) joined by a Gaussian copula
 * with correlation rho. */
typedef struct {
    double alpha_pl;     /* power-law index of f; != -1 (prior U(-4, -2)) */
    double alpha_g;      /* Gamma shape, > 0 (prior U(1, 3)) */
    double beta_g;       /* Gamma rate, > 0 (prior U(1, 3)) */
    double mu_g;         /* mu_Gamma (prior U(-22, -20)) */
    double mu;           /* amplitude offset mu (prior U(-23, -21)) */
    double sigma;        /* log-normal shape, >= 0 (prior U(0.1, 0.3)) */
    double rho;          /* copula correlation, |rho| < 1 (prior U(0, 1)) */
    double f_lo_hz;      /* power-law support, 0 < f_lo < f_hi (the paper: 1e-4 .. 1e-2 Hz) */
    double f_hi_hz;
} gbsub_population;

/* Draws sources first .. first+n-1 of the catalog defined by (pop, seed)
 * into DEVICE arrays A, f, fdot (fp32, n entries each, caller-owned) and, if
 * id is non-null, id[i] = first + i (uint32).  Source i is a function of
 * (pop, seed, first + i) only: Philox4x32-10 with key = seed and counter =
 * (index, block) gives its random numbers, so a catalog can be drawn in
 * pieces, and the same catalog results on any launch shape.  Enqueued on
 * `stream` (hipStream_t; NULL = default stream) on the current device;
 * returns without waiting.  Allocates nothing.  Errors: INVALID for bad
 * parameters or a NULL output with n > 0, DEVICE for a launch failure. */
gbsub_status gbsub_generate(const gbsub_population *pop, uint64_t seed, uint64_t first, uint64_t n, float *A,
                            float *f, float *fdot, uint32_t *id, void *stream);

/* Kernel families of the profiling mode (bit k of the mask selects family k). */
enum {
    GBSUB_KF_TABLES = 0,         /* S_instr and its prefix tables (first run on a workspace) */
    GBSUB_KF_RESET = 1,          /* per-run state */
    GBSUB_KF_PREP = 2,           /* candidate cut, binning, fixed-point accumulation */
    GBSUB_KF_XUPDATE = 3,        /* X from the fixed-point accumulators */
    GBSUB_KF_MEDIAN = 4,         /* running median, S = C med + S_instr, in-part prefix of 1/S */
    GBSUB_KF_SNR = 5,            /* rho^2 (the part sums of 1/S under each track), decisions,
                                    subtraction, dirty tiles, settle test */
    GBSUB_KF_OUTPUT = 6,         /* candidate ids */
    GBSUB_KF_COUNT = 7
};
#define GBSUB_PROFILE_ALL 0x7Fu

/* Per-kernel timing of the runs made while profiling is enabled. */
typedef struct {
    char     name[24];           /* kernel family: "tables", "reset", "prep", "xupdate",
                                    "median", "snr", "output" */
    uint64_t launches;           /* launches that did work (bodies past the settled one excluded) */
    double   total_ms;           /* sum of HIP-event durations on the run's stream */
    double   units;              /* work units processed by those launches */
    char     unit[16];           /* "bins", "sources", "candidates" */
} gbsub_kernel_stat;

/* Selects the kernel families to time (a mask of 1u << GBSUB_KF_*, 0 = off,
 * GBSUB_PROFILE_ALL = every family) and clears the accumulated stats.  While
 * a family is selected, gbsub_run times each of its launches with HIP
 * events (host-side events only; no device memory): the loop-body kernels
 * (xupdate, median, snr) carry the events on their dispatches, the
 * once-per-run families are bracketed by events recorded on the stream.
 * Either way an event costs some microseconds of idle time between
 * launches, so time a run with only the families of interest selected.
 * Batched runs are not timed. */
gbsub_status gbsub_set_profiling(gbsub_ctx *ctx, uint32_t families);

/* Copies up to `cap` accumulated kernel stats into out[] (host pointer);
 * *n (host) receives the number of kernel families (GBSUB_KF_COUNT).
 * TRUNCATED if cap < GBSUB_KF_COUNT. */
gbsub_status gbsub_kernel_stats(const gbsub_ctx *ctx, gbsub_kernel_stat *out, uint32_t cap,
                                uint32_t *n);

/* ---------------------------------------------------------------- batches
 * Many catalogs, possibly on different grids, share every kernel launch of
 * the loop: one launch covers all running slots (one slot per catalog; the
 * launches are sized for the running slots only, and a slot whose loop
 * settles inside a step does nothing until the next poll drops it from the
 * launches).  Catalogs are admitted and retired
 * between steps (continuous batching).  Each admitted slot uses its own
 * context (configuration, results) and its own workspace; the results of a
 * retired slot are read with gbsub_spectrum / gbsub_resolved on that context.
 * Results are identical to gbsub_run on the same context and catalog. */
typedef struct gbsub_batch gbsub_batch;

enum {                                   /* slot states reported by gbsub_batch_poll */
    GBSUB_SLOT_RUNNING = 0,
    GBSUB_SLOT_SETTLED = 1,              /* the resolved set stopped changing */
    GBSUB_SLOT_MAXITER = 2,              /* max_iter bodies ran, sources still resolving */
    GBSUB_SLOT_INVALID = 3,              /* an input entry failed validation */
    GBSUB_SLOT_FREE = 255
};

/* Bytes of DEVICE memory for the descriptor tables of max_slots slots (one
 * entry per slot and a compacted copy of the running ones). */
gbsub_status gbsub_batch_table_size(uint32_t max_slots, uint64_t *bytes);

/* Creates a batch of up to max_slots (1..4096) slots on the current device.
 * `table` is a DEVICE pointer to gbsub_batch_table_size() bytes, 256-byte
 * aligned, owned by the caller and kept until gbsub_batch_destroy. */
gbsub_status gbsub_batch_create(uint32_t max_slots, void *table, uint64_t table_bytes,
                                gbsub_batch **out);

/* Admits `cat` (device arrays, read until the slot is retired) into a free
 * slot with context `ctx` and its DEVICE workspace (gbsub_workspace_size()
 * bytes for cat->n, owned by the caller until retirement).  Enqueues the
 * grid tables, reset and prep on `stream` and returns at once; *slot (host)
 * receives the slot index.  INVALID for bad arguments or a context that
 * already holds a slot, NOMEM if no slot is free. */
gbsub_status gbsub_batch_admit(gbsub_batch *b, gbsub_ctx *ctx, const gbsub_catalog *cat,
                               void *workspace, uint64_t ws_bytes, void *stream, uint32_t *slot);

/* Enqueues n_bodies loop bodies for every running slot on `stream`
 * (captured in a HIP graph, replayed until the set of running slots changes,
 * when `stream` is not the null stream); returns at once, except that after
 * an admission or a poll that saw slots settle it first waits for `stream`
 * to rewrite the compacted table. */
gbsub_status gbsub_batch_step(gbsub_batch *b, uint32_t n_bodies, void *stream);

/* Waits for `stream`, then writes the state of slot i to state[i] (host,
 * cap >= max_slots entries) and the number of slots still running to
 * *n_running (host, may be NULL). */
gbsub_status gbsub_batch_poll(gbsub_batch *b, void *stream, uint8_t *state, uint32_t cap,
                              uint32_t *n_running);

/* Retires a slot that is no longer running: its results become the last
 * run of its context, *out (host, may be NULL) receives the summary, and the
 * slot is freed.  Returns the slot's outcome: OK, MAXITER or INVALID;
 * STATE if the slot is free or still running. */
gbsub_status gbsub_batch_retire(gbsub_batch *b, uint32_t slot, void *stream, gbsub_summary *out);

/* Releases the batch (NULL is ignored); caller memory is not touched. */
void gbsub_batch_destroy(gbsub_batch *b);

/* ---------------------------------------------------------------- complex-template data model
 * The data as the paper holds it (Sec. "Simulations"; appendix "Subtraction
 * algorithm", Eq. "vectorized-subtraction"): one complex frequency series
 * per TDI channel A and E (T is insensitive), the sum of every source's
 * frequency-domain template of GBSUB_CX_NF = 128 samples around its central
 * frequency; resolved sources are scattered out of it.  The paper's
 * templates come from gbgpu; this library uses a sky-averaged fast/slow
 * template of its own: with q = floor((f + fdot T/2) T + 1/2),
 * delta = f T - q and d = fdot T^2, U_j = (T/128) sum_n s_n e^{-2 pi i m n/128}
 * (m = j mod 128, j = -64..63, at grid bin q + j - k0) of the samples
 * s_n = (A/2) e^{2 pi i (delta x + d x^2/2)}, x = n/128; channel c carries
 * e^{i phi_c} U.  Per channel, X_c = (2/T)|h_c|^2 and S_c = C median_W(X_c)
 * + S_instr (or the running mean); rho^2 = (4/T) sum_c sum_j |U_j|^2 / S_c.
 * A source with |fdot| T^2 >= 2^20 or |(f + fdot T/2) T| >= 2^52 has no
 * template.  Runs use the context's configuration (grid, window, estimator,
 * thresholds, max_iter; FP64 only: the data are exact 64-bit fixed point,
 * so a subtracted template cancels to the last bit); grids of at most
 * 8192 x 1024 bins. */
#define GBSUB_CX_NF 128
enum { GBSUB_SPEC_H_RESIDUAL = 4 };   /* gbsub_cx_spectrum: h_c, 2B fp64 (re, im interleaved) */

typedef struct {
    uint64_t        n;
    const float    *A;        /* device pointers to n entries each, as gbsub_catalog */
    const float    *f;
    const float    *fdot;
    const float    *phi_a;    /* phase of the A channel (rad), finite */
    const float    *phi_e;    /* phase of the E channel (rad), finite */
    const uint32_t *id;
} gbsub_cx_catalog;

/* Bytes of device workspace gbsub_cx_run needs for n_sources on this
 * context's grid (*bytes, host).  INVALID if the grid has more than
 * 8192 x 1024 bins or the context is not FP64. */
gbsub_status gbsub_cx_workspace_size(const gbsub_ctx *ctx, uint64_t n_sources, uint64_t *bytes);

/* The subtraction of the appendix "Subtraction algorithm" on the complex
 * data: every template injected into h_A, h_E; rho_0^2 against S_instr in
 * both channels and the candidate cut; then loop bodies {X_c and S_c of each
 * channel, rho^2 of every unresolved candidate, the templates of every
 * source with rho > rho_th scattered out of h (Eq. "vectorized-subtraction")}
 * until a body subtracts nothing.  Arguments, workspace ownership, stream
 * use and errors as gbsub_run (the workspace from gbsub_cx_workspace_size);
 * results are read with gbsub_cx_spectrum, gbsub_cx_resolved and
 * gbsub_cx_candidates and stay in the workspace until the next
 * complex-template run of this context or until the caller reuses that
 * memory (a power-model run in the same buffer overwrites them). */
gbsub_status gbsub_cx_run(gbsub_ctx *ctx, const gbsub_cx_catalog *cat, void *workspace, uint64_t ws_bytes,
                          void *stream, gbsub_summary *out);

/* Spectrum `kind` of channel `channel` (0 = A, 1 = E) of the last
 * complex-template run: GBSUB_SPEC_SN, _X_RESIDUAL, _S_GAL, _S_INSTR (B fp64
 * values) or GBSUB_SPEC_H_RESIDUAL (the data left after the subtraction,
 * 2B fp64 values: re, im of each bin).  Pointers and errors as
 * gbsub_spectrum; cap counts fp64 values. */
gbsub_status gbsub_cx_spectrum(const gbsub_ctx *ctx, uint32_t channel, uint32_t kind, double *out, uint64_t cap,
                               uint64_t *n_bins, int out_on_device);

/* The resolved sources of the last complex-template run (ids ascending,
 * with their loop body), as gbsub_resolved. */
gbsub_status gbsub_cx_resolved(const gbsub_ctx *ctx, uint32_t *ids, int32_t *iter_of, uint64_t cap, uint64_t *n,
                               int out_on_device);

/* Every candidate of the last complex-template run, in ascending id, as
 * gbsub_candidates: ids[], the loop body that resolved it (iter_of, -1 if
 * never; may be NULL) and rho^2 at its last evaluation (rho2; may be NULL).
 * HOST pointers of `cap` entries; TRUNCATED if cap is smaller; STATE if no
 * complex-template run has completed. */
gbsub_status gbsub_cx_candidates(const gbsub_ctx *ctx, uint32_t *ids, int32_t *iter_of, double *rho2, uint64_t cap,
                                 uint64_t *n);

/* Templates of n sources on the device (Sec. "Simulations", the model above):
 * q[i] (int64, central DFT index; INT64_MIN if the source has no template)
 * and U[i][128][2] (fp64 re, im of U_j, j = -64..63).  A, f, fdot, q, U are
 * device pointers; enqueued on `stream`, which the call synchronizes.
 * INVALID for null pointers with n > 0. */
gbsub_status gbsub_cx_templates(const gbsub_ctx *ctx, uint64_t n, const float *A, const float *f,
                                const float *fdot, int64_t *q, double *U, void *stream);

/* Releases the context (NULL is ignored).  Does not touch caller memory.
 * A context that holds a batch slot must be retired from the batch first. */
void gbsub_destroy(gbsub_ctx *ctx);

/* Static description of a status code; never NULL. */
const char *gbsub_status_str(gbsub_status s);

#ifdef __cplusplus
}
#endif
#endif /* GBSUB_H */
