// gbsub_internal.h -- shared definitions of the HIP kernels and the host
// runtime of libgbsub (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbs {

constexpr int WG = 256;            // threads per workgroup for every tiled kernel
constexpr int MMAX = 3072;         // median tile: outputs + W - 1 must fit
constexpr int TILE_MAX = 2048;     // bins per tile (also the binning bucket)
constexpr int NBK_MAX = 8192;      // tiles the prep histogram can hold (B <= 8192 tiles)
constexpr int NARROW = 16;         // tracks of <= NARROW bins: SNR summed bin by bin
constexpr int SNR_BLOCKS = 1024;   // fixed grid of the per-candidate kernels
constexpr int COOP_PARTS = 8;      // tracks over more parts: the part sums are added by the whole wave
constexpr int PREP_SRC = 4096;     // sources per block of the prep passes (count and scatter)
constexpr int SEG_BINS = 128;      // bins per segment of the 1/S_instr bounds of the candidate test
constexpr int CS_WG = 1024;        // threads of a column-pass block (64 tiles, 16 waves over the blocks)
constexpr int ACC_EV = 65536;      // binning events per accumulation block
constexpr int RED_BINS = 256;      // bins per reduction block of the hot buckets
constexpr int NEW_CAP = 1 << 16;   // per-iteration counters kept (iterations beyond: not recorded)
constexpr int KEYBITS = 20;        // bits of the per-tile order key of the median sort
constexpr int POSBITS = 12;        // sort word = key << 12 | position (MMAX <= 4096)
enum Prec { PREC_FP64 = 0, PREC_COMP = 1, PREC_NAIVE = 2 };   // Grid::prec (= gbsub_config precision)
constexpr int COARSE_MAX = 256;    // coarse-graining bins at most
constexpr int PART_MAX = 512;      // outputs of a median block in split mode (prefix-of-1/S granule)
constexpr int SPLIT_BLOCKS = 512;  // split the median into parts while dirty tiles x parts fit this
constexpr int MED_GRID = 2048;     // blocks of a median launch (per slot); they stride over the dirty list

// Signed 128-bit fixed-point accumulator (two's complement: hi*2^64 + lo).
// Every power is accumulated as an exact integer multiple of 2^L, so sums
// and differences are exact and independent of the order of the atomics.
struct alignas(16) I128 {
    uint64_t lo;
    int64_t hi;
};

// Signed 128-bit sum kept as h 2^32 + l in two 64-bit words, so that adds
// need no carry between the words: non-returning atomics, exact while fewer
// than 2^32 terms have been added.
struct alignas(16) SplitSum {
    int64_t h;
    uint64_t l;
};

// Double-fp32 value hi + lo (|lo| at most half an ulp of hi once
// normalised): the arithmetic of the compensated FP32 precision mode.
struct alignas(8) FF {
    float hi;
    float lo;
};

// Device control block (lives in the workspace).
struct Ctl {
    uint32_t amax_bits;      // max over sources of the fp32 bits of A (A >= 0)
    uint32_t bad;            // nonzero: an input entry failed validation
    uint32_t n_cand;         // candidates
    uint32_t done;           // the loop has settled
    uint32_t n_iter;         // loop bodies run (valid when done)
    uint32_t n_resolved;     // sources subtracted so far
    uint32_t n_chunks;       // accumulation blocks of the binning
    uint32_t cand_cursor;    // candidate slots handed out
    uint32_t n_events;       // binning events
    uint32_t iter;           // index t of the next loop body
    uint64_t n_near;         // evaluations within 1e-6 of the threshold
    uint64_t min_margin;     // bits of min |rho/rho_th - 1| (non-negative double)
    uint64_t units_x;        // bins converted by k_xupdate
    uint64_t units_med;      // median outputs computed by k_median
    uint64_t units_snr;      // candidate evaluations by k_snr
    uint32_t status;         // 0 running/settled, 6 = max_iter reached with sources still resolving
    uint32_t med_split;      // next median launch: one block per part (1) or per tile (0)
    uint32_t xupd;           // stamp of the tiles the next k_xupdate converts
    uint32_t tail_due;       // k_snr has run; its partials await the tail
    uint32_t n_new_body;     // complex-template model: sources subtracted by the running body
    uint32_t n_sdl;          // tiles listed in sdl for the next median launch
};

// Per-block partial results of k_snr (combined by the tail: the last block
// of the next k_xupdate, or k_snr_tail in the naive FP32 mode).
struct SnrPart {
    uint32_t n_new;          // sources subtracted
    uint32_t pad;
    uint64_t near;           // evaluations within 1e-6 of the threshold
    uint64_t evals;          // candidate evaluations
    double minm;             // min |rho/rho_th - 1|
};

// Kernels that the profiling mode times separately.
enum KernelId { K_TABLES = 0, K_RESET, K_PREP, K_XUPDATE, K_MEDIAN, K_SNR, K_OUTPUT, K_COUNT };

struct Grid {
    int32_t B;               // bins
    int32_t W;               // window (odd)
    int32_t h;               // (W-1)/2
    int32_t tile;            // bins per tile (power of two, 256 .. TILE_MAX)
    int32_t nt;              // tiles = ceil(B / tile)
    int32_t part;            // bins per part: min(tile, PART_MAX)
    int32_t np;              // parts per tile
    int32_t nparts;          // parts = ceil(B / part)
    uint32_t split_tiles;    // median in split mode while at most this many tiles are dirty
    uint32_t split_blocks;   // the budget behind split_tiles (shared by a batch's running slots)
    int32_t track_single;    // 1: every source occupies one bin
    int32_t prec;            // 0 FP64, 1 FP32 with compensated sums, 2 naive FP32 (loop arithmetic)
    int32_t est;             // 0 running median, 1 running mean
    int32_t pad1;
    int64_t k0;              // first grid index
    double T;                // observation time
    double C;                // median scale
    double rth2;             // rho_th^2
    double cut2;             // (kappa rho_th)^2
    double rth;              // rho_th
    double oms_pm, tm_fm, arm_m;
    uint32_t max_iter;       // loop bodies allowed; 0 = candidates + 1
    uint32_t pad;
};

// Pointers into the caller's workspace.
struct Dev {
    // grid tables (kept across runs with the same workspace and grid)
    double *sx;              // [B]    S_instr
    double *isx;             // [B]    1 / S_instr
    double *isx_pre;         // [B]    inclusive prefix of 1/S_instr inside each tile
    double *isx_tsum;        // [nt]   tile sums of 1/S_instr
    double *isx_tile;        // [nt+1] exclusive prefix of the tile sums
    double2 *isx_seg;        // [ceil(B/SEG_BINS)] (min, max) of 1/S_instr over each segment
    // binned power: X = Xn + prefix(D), all exact 128-bit fixed point
    I128 *Xn;                // [B]    sources whose clipped track is one bin
    I128 *D;                 // [B+1]  difference array of the wider tracks
    I128 *Dtile;             // [nt+1] per-tile sums of D (binning)
    I128 *Dcarry;            // [nt+1] sum of D before each tile, as binned
    SplitSum *Dadj;          // [nt]   change of that sum by the subtractions so far
    // naive FP32 mode only: the binned power accumulated in fp32
    float *Xf;               // [B]    one-bin tracks
    float *Df;               // [B+1]  difference array of the wider tracks
    float *Dtf;              // [nt+1] per-tile sums of Df (binning and subtractions)
    float *Dcf;              // [nt+1] exclusive prefix of Dtf (rescanned every body)
    // compensated FP32 mode only: the binned power as double-fp32 sums
    FF *Xc;                  // [B]    one-bin tracks
    FF *Dc;                  // [B+1]  difference array of the wider tracks
    FF *Dtc;                 // [nt+1] per-tile sums of Dc (binning and subtractions)
    double *X;               // [B]    X^t
    double *S;               // [B]    S^t
    double *is_pre;          // [B]    inclusive prefix of 1/S^t inside each part (an FF in the
                             //        compensated FP32 mode, a float in the naive one)
    double *is_psum;         // [nparts] part sums of 1/S^t
    // dirty tiles: a tile is converted (X) / filtered (S) in body t iff its
    // stamp equals t; k_snr stamps t + 1 where a subtraction changes them
    uint32_t *xstamp;        // [nt]
    uint32_t *sstamp;        // [nt]
    uint32_t *sdl;           // [nt] the tiles the next median launch filters, in tile order
    // binning by tile (multisplit): events sorted by tile
    uint32_t *btot;          // [nt]   events per tile
    uint32_t *bhist;         // [prep blocks][(nt+1)/2] events per (block, tile), two 16-bit counts a word
    uint32_t *boff;          // [prep blocks][nt] events of the blocks before, per tile
    uint32_t *bbase;         // [nt+1] first event of each tile
    uint32_t *nch;           // [nt]   accumulation blocks per tile
    uint32_t *chunk_base;    // [nt+1]
    uint32_t *slot_base;     // [nt]   partial-sum slots of tiles with several blocks
    uint32_t *ev_key;        // [2n]   bin | (1<<31 for difference events)
    int64_t *ev_val;         // [2n]   signed fixed-point power
    I128 *partial;           // [slots][2][tile] partial sums of the hot tiles
    uint64_t *cbits;         // [ceil(n/64)] candidate flags of the sources (count pass)
    uint32_t *rs_hist;       // [resolved_scratch_words(n)] block counts of the resolved-list kernels
    uint32_t *blk_cand;      // [count blocks + 1] candidates per count block, then their exclusive prefix
    uint32_t *blk_amax;      // [count blocks] max fp32 bits of A per count block
    // candidates (capacity: all sources)
    uint32_t *c_src;         // source index
    uint32_t *c_id;          // its id (written at the end of a run)
    int32_t *c_glo, *c_ghi;  // clipped track
    int32_t *c_iter;         // loop body that subtracted it, -1 while unresolved
    double *c_q;             // per-bin power
    uint64_t *c_qfx;         // per-bin power in fixed point
    double *c_rho2;          // rho^2 at the last evaluation
    SnrPart *b_part;         // [SNR_BLOCKS] per-block partials of k_snr
    uint32_t *n_new;         // [NEW_CAP] sources subtracted per loop body
    double *coarse;          // [3 * COARSE_MAX] coarse-graining sums (f, value, count)
    Ctl *ctl;
    uint32_t max_slots;      // capacity of `partial`
    uint32_t max_chunks;     // grid of the accumulation kernel
};

// One catalog of a launch: its grid, workspace, catalog.  Kernels read the
// descriptor of slot blockIdx.y from a device array, so one launch serves a
// whole batch of catalogs with different grids; inactive slots exit at once.
struct Slot {
    Grid g;
    Dev d;
    const float *A, *F, *FD;
    const uint32_t *ids;
    uint64_t n;
    uint32_t active;
    uint32_t pad;
    uint32_t *prog;          // host-mapped word of a single run: bodies finished << 1 | settled (null in batches)
};

// Launch extents: the largest per-slot block counts of a set of slots.
struct Dims {
    int ns;                  // slots (gridDim.y)
    int maxB, maxnt, maxtile, maxparts;
    uint32_t est_mask;       // bit e: some slot uses estimator e
    uint32_t naive;          // some slot runs in naive FP32
    uint32_t prep_blocks, accum_blocks;
};

// Kernel launchers (gbsub_kernels.hip); all enqueue on `st` and return the
// launch status.  `ds` is the device array of `dm.ns` slot descriptors.
hipError_t launch_grid_tables(const Slot *ds, const Dims &dm, hipStream_t st);
hipError_t launch_reset(const Slot *ds, const Dims &dm, hipStream_t st);
hipError_t launch_prep(const Slot *ds, const Dims &dm, hipStream_t st);
// The loop body's launchers take optional events that the dispatch itself
// stamps with its start and end (nullptr: none).
hipError_t launch_xupdate(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea = nullptr,
                          hipEvent_t eb = nullptr);
hipError_t launch_median(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea = nullptr,
                         hipEvent_t eb = nullptr);
hipError_t launch_snr(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea = nullptr,
                      hipEvent_t eb = nullptr);
hipError_t launch_outputs(const Slot *ds, const Dims &dm, hipStream_t st);

// Output kernels (gbsub_output.hip).  The resolved list: the (id, loop body)
// pairs of the m candidates with iter >= 0 among nc, compacted and sorted by
// id into kA / vA (kB / vB: the same sizes, scratch); `hist` holds
// resolved_scratch_words(n) words for catalogs of up to n sources.
uint64_t resolved_scratch_words(uint64_t n_max);
hipError_t launch_resolved(const int32_t *iter, const uint32_t *id, uint32_t nc, uint32_t m, uint32_t *hist,
                           uint32_t *kA, int32_t *vA, uint32_t *kB, int32_t *vB, hipStream_t st);
// out[k] = S[k] - sx[k] for k < B.
hipError_t launch_sgal(const double *S, const double *sx, int B, double *out, hipStream_t st);
// out[i] = the control block of slot i of the device table, i < n (one launch).
hipError_t launch_gather_ctl(const Slot *table, uint32_t n, Ctl *out, hipStream_t st);

// ---- complex-template data model (gbsub_cx.hip)
constexpr int CX_NF = 128;          // samples per template
constexpr int CX_TILE = 1024;       // bins per binning tile of the injection
constexpr int CX_NTC_MAX = 8192;    // binning tiles at most (B <= CX_NTC_MAX * CX_TILE)

// Pointers into the workspace of a complex-template run.
struct CxDev {
    Slot *slots;             // [2] median descriptors of the A and E channels
    Ctl *ctl;                // shared by both channels
    double *sx;              // [B] S_instr
    double *isx;             // [B] 1 / S_instr
    double *isx_max;         // [ceil(B/128)] largest 1/S_instr of each 128-bin segment
    double *X;               // [2][B] periodograms (2/T)|h_c|^2
    double *S;               // [2][B] PSD estimates
    double *is_pre;          // [2][B] in-part prefixes of 1/S (written by the median kernel)
    double *is_psum;         // [2][nparts] part sums of 1/S
    int64_t *h;              // [4][B] re h_A, im h_A, re h_E, im h_E in fixed point (unit 2^-E)
    uint32_t *xstamp;        // [nt] tiles whose X is recomputed in body t
    uint32_t *sstamp;        // [nt] tiles whose S is recomputed in body t
    uint32_t *sdl;           // [nt] the tiles of the next PSD launch, in tile order
    uint32_t *tcnt;          // [ntc+1] sources per binning tile, then their exclusive prefix
    uint32_t *tcur;          // [ntc] scatter cursors
    uint32_t *cbase;         // [ntc+1] first injection chunk of each binning tile
    uint32_t *order;         // [n] source indices grouped by binning tile
    uint32_t *c_src;         // [n] candidates (slot order of discovery)
    int32_t *c_iter;         // [n] loop body that subtracted it, -1 while unresolved
    uint32_t *c_id;          // [n] its id (written at the end of a run)
    double *c_rho2;          // [n] rho^2 at the last evaluation
    int32_t *c_qb;           // [n] its template's centre bin (the SNR pass's dirty-tile test)
    uint32_t *rs_hist;       // resolved-list scratch
    uint32_t *kA, *kB;       // [n] each: resolved-list keys
    int32_t *vA, *vB;        // [n] each: resolved-list values
    int32_t ntc;             // binning tiles
    int32_t pad;
};

// Bytes of the workspace of a complex-template run of n sources on grid g
// (with base: the layout is written to *d).
uint64_t cx_carve(const Grid &g, uint64_t n, char *base, CxDev *d);
// The run's kernels (all enqueue on st).  `prog`: host-mapped progress word.
struct CxIn {
    const float *A, *F, *FD, *PA, *PE;
    const uint32_t *ids;
    uint32_t n;
    uint32_t *prog;
};
hipError_t cx_launch_prep(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st);
// A loop body: X update, the PSD of both channels (the median or mean
// kernels; optional events stamped by the dispatch), SNR + subtraction and
// the tail.
hipError_t cx_launch_power(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st);
hipError_t cx_launch_psd(const Grid &g, const CxDev &d, hipStream_t st, hipEvent_t ea = nullptr,
                         hipEvent_t eb = nullptr);
hipError_t cx_launch_snr(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st);
hipError_t cx_launch_outputs(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st);
// h_ch in fp64, re and im of bin k at out[2k], out[2k + 1].
hipError_t cx_launch_h(const Grid &g, const CxDev &d, uint32_t n, int ch, double *out, hipStream_t st);
// Templates of n sources: q[i] (INT64_MIN: none) and U[i][CX_NF] (re, im).
hipError_t cx_launch_templates(const Grid &g, const float *A, const float *F, const float *FD, uint32_t n,
                               int64_t *q, double *U, hipStream_t st);

struct CoarseEdges { double e[COARSE_MAX + 1]; };

// Population hyperparameters of a generator launch (gbsub_population).
struct PopParams {
    double alpha_pl, alpha_g, beta_g, mu_g, mu, sigma, rho, f_lo_hz, f_hi_hz;
};
// Sources first .. first+n-1 of the catalog drawn with `seed` into the fp32
// columns A, F, FD and (if non-null) the ids (gbsub_population.hip).
hipError_t launch_generate(const PopParams &pp, uint64_t seed, uint64_t first, uint64_t n, float *A, float *F,
                           float *FD, uint32_t *id, hipStream_t st);
// Sums of f_i and of the chosen spectrum over each logarithmic bin
// [e_k, e_{k+1}) (the last bin closed) into out[3k .. 3k+2] = (sum f, sum v, count).
hipError_t launch_coarse(const double *S, const double *sx, const double *X, int kind, int64_t k0, int B,
                         double T, const CoarseEdges &ed, int n_out, double *out, hipStream_t st);

}  // namespace gbs
