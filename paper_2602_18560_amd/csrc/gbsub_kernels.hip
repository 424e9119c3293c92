// gbsub_kernels.hip -- HIP kernels (gfx950) of the iterative galactic-binary
// subtraction.
//
// Data layout in HBM (all structure-of-arrays, see gbsub_internal.h):
//   catalog     A, f, fdot fp32 [n]            read by the two prep passes
//   S_instr     sx, 1/sx fp64 [B] + 1/S_instr prefix tables (per grid, cached)
//   binned power Xn (one-bin tracks) and D (difference array of wider
//               tracks): 128-bit fixed point [B], [B+1]; X = Xn + prefix(D)
//   X, S, in-part prefix of 1/S: fp64 [B]; tile- and part-level tables
//   candidates  SoA records (source, clipped track, q, q in fixed point, iter)
//
// Every per-bin power sum is exact integer arithmetic on multiples of 2^L
// (L from the largest amplitude), so the binned spectrum does not depend on
// the order in which atomics land and subtracting a source is exact.  The
// SNR and the median read fp64 values converted from it with one rounding.

#include "gbsub_internal.h"
#include "gbsub_device.h"
#include <hip/hip_ext.h>

#include <math.h>

namespace gbs {

#define DEVI __device__ __forceinline__

// ------------------------------------------------------------------ helpers

DEVI I128 i128_add(I128 a, I128 b)
{
    I128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (int64_t)(r.lo < a.lo);
    return r;
}

DEVI I128 i128_from(int64_t v)
{
    I128 r;
    r.lo = (uint64_t)v;
    r.hi = v < 0 ? -1 : 0;
    return r;
}

// Exact, order-independent: adds v into the 128-bit accumulator *p.
DEVI void atomic_add_i128(I128 *p, int64_t v)
{
    const uint64_t vlo = (uint64_t)v;
    const int64_t vhi = v < 0 ? -1 : 0;
    const uint64_t old = atomicAdd((unsigned long long *)&p->lo, (unsigned long long)vlo);
    const int64_t add_hi = vhi + (int64_t)((uint64_t)(old + vlo) < old);
    if (add_hi != 0) atomicAdd((unsigned long long *)&p->hi, (unsigned long long)add_hi);
}

// Correctly rounded conversion of a non-negative 128-bit integer to fp64.
DEVI double i128_to_double(I128 v)
{
    if (v.hi < 0) return 0.0;   // cannot happen for a sum of non-negative powers
    if (v.hi == 0) return (double)v.lo;
    const uint64_t hi = (uint64_t)v.hi;
    const int lz = __clzll(hi);
    uint64_t top = lz ? ((hi << lz) | (v.lo >> (64 - lz))) : hi;
    const uint64_t rest = v.lo << lz;
    top |= (uint64_t)(rest != 0);       // sticky bit keeps round-to-nearest exact
    return ldexp((double)top, 64 - lz);
}

DEVI void split_sum_add(SplitSum *p, int64_t v)
{
    atomicAdd((unsigned long long *)&p->h, (unsigned long long)(v >> 32));   // floor(v / 2^32)
    atomicAdd((unsigned long long *)&p->l, (unsigned long long)((uint64_t)v & 0xFFFFFFFFull));
}

DEVI I128 split_sum_value(SplitSum s)
{
    I128 x;
    x.lo = (uint64_t)s.h << 32;
    x.hi = s.h >> 32;
    I128 y;
    y.lo = s.l;
    y.hi = 0;
    return i128_add(x, y);
}

// ---- double-fp32 (compensated FP32 mode)
//
// TwoSum (Knuth): s + e == a + b exactly, s = fl(a + b).  An FF add keeps the
// rounding error of the high parts and adds the low parts (the "sloppy"
// double-float addition, error O(2^-44) relative); FastTwoSum normalises.
DEVI FF ff_two_sum(float a, float b)
{
    FF r;
    r.hi = a + b;
    const float bb = r.hi - a;
    r.lo = (a - (r.hi - bb)) + (b - bb);
    return r;
}

DEVI FF ff_norm(float s, float e)                 // |s| >= |e|
{
    FF r;
    r.hi = s + e;
    r.lo = e - (r.hi - s);
    return r;
}

DEVI FF ff_add(FF a, FF b)
{
    const FF s = ff_two_sum(a.hi, b.hi);
    return ff_norm(s.hi, s.lo + (a.lo + b.lo));
}

DEVI FF ff_neg(FF a)
{
    FF r;
    r.hi = -a.hi;
    r.lo = -a.lo;
    return r;
}

DEVI FF ff_of(float x)
{
    FF r;
    r.hi = x;
    r.lo = 0.0f;
    return r;
}

DEVI float ff_float(FF a) { return a.hi + a.lo; }

// Compensated accumulation by atomics: the atomic add on hi returns the
// value it added v to; TwoSum of that value and v gives the exact rounding
// error of the sum it stored, which goes to lo.  hi + lo is then the sum up
// to the roundings of lo (second order), whatever the order of the atomics.
DEVI void ff_atomic_add(FF *p, float v)
{
    const float old = atomicAdd(&p->hi, v);
    const float e = ff_two_sum(old, v).lo;
    if (e != 0.0f) atomicAdd(&p->lo, e);
}

// Fixed-point unit 2^L: every per-bin power q <= A_max^2 T / 2 maps to an
// integer below 2^62, so 2^65 sources fit in one 128-bit accumulator.
DEVI int fx_exp(uint32_t amax_bits, double T)
{
    const double a = (double)__uint_as_float(amax_bits);
    const double pmax = ((a * a) * T) * 0.5;
    if (!(pmax > 0.0)) return 0;
    return ilogb(pmax) - 61;
}

DEVI uint64_t to_fx(double q, int L) { return (uint64_t)rint(ldexp(q, -L)); }

// The FP32 modes hold powers and PSDs scaled by 2^sc (exact): the largest
// one-bin power becomes ~2^20, so S_instr (~1e-40 in SI units, below the
// fp32 normal range) and its reciprocal stay representable; rho^2 is
// unchanged by the scale.
DEVI int f32_scale(uint32_t amax_bits, double T)
{
    const double a = (double)__uint_as_float(amax_bits);
    const double pmax = ((a * a) * T) * 0.5;
    if (!(pmax > 0.0)) return 128;
    return 20 - ilogb(pmax);
}

DEVI int lane_id() { return __lane_id(); }


// Makes the compiler produce v here (an empty asm that reads it): loads
// issued together stay together instead of being sunk into the branches
// that use them, each with its own wait.
DEVI void pin(float v) { asm volatile("" ::"v"(v)); }
DEVI void pin(double v) { asm volatile("" ::"v"(v)); }
DEVI void pin(uint64_t v) { asm volatile("" ::"v"(v)); }

template <typename T>
DEVI T shfl_up_t(T x, int d) { return __shfl_up(x, d, 64); }

DEVI I128 shfl_up_t(I128 x, int d)
{
    I128 r;
    r.lo = (uint64_t)__shfl_up((unsigned long long)x.lo, d, 64);
    r.hi = (int64_t)__shfl_up((long long)x.hi, d, 64);
    return r;
}

DEVI FF shfl_up_t(FF x, int d)
{
    FF r;
    r.hi = __shfl_up(x.hi, d, 64);
    r.lo = __shfl_up(x.lo, d, 64);
    return r;
}

DEVI double add_t(double a, double b) { return a + b; }
DEVI FF add_t(FF a, FF b) { return ff_add(a, b); }
DEVI float add_t(float a, float b) { return a + b; }
DEVI I128 add_t(I128 a, I128 b) { return i128_add(a, b); }
DEVI uint32_t add_t(uint32_t a, uint32_t b) { return a + b; }

template <typename T> DEVI T zero_t();
template <> DEVI double zero_t<double>() { return 0.0; }
template <> DEVI float zero_t<float>() { return 0.0f; }
template <> DEVI uint32_t zero_t<uint32_t>() { return 0u; }
template <> DEVI I128 zero_t<I128>() { I128 z; z.lo = 0; z.hi = 0; return z; }
template <> DEVI FF zero_t<FF>() { return ff_of(0.0f); }

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
DEVI T wave_incl_scan(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = shfl_up_t(x, d);
        if (lane >= d) x = add_t(x, y);
    }
    return x;
}

// Exclusive scan across the WG threads of a block; *total gets the block sum.
// `sh` must hold WG/64 elements.  Contains __syncthreads().
template <typename T, int NT = WG>
DEVI T block_excl_scan(T x, T *sh, T *total)
{
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T inc = wave_incl_scan(x);
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    T pre = zero_t<T>(), tot = zero_t<T>();
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wave) pre = add_t(pre, sh[w]);
        tot = add_t(tot, sh[w]);
    }
    __syncthreads();
    T ex = shfl_up_t(inc, 1);
    if (lane == 0) ex = zero_t<T>();
    *total = tot;
    return add_t(pre, ex);
}

DEVI double wave_sum(double x)
{
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}


// sum_{k=lo..hi} 1/v[k] from the tile tables (inclusive in-tile prefix `pre`,
// exclusive tile prefix `tl`); short ranges are summed bin by bin in
// ascending order.
DEVI double range_inv_sum(const double *v, const double *pre, const double *tl, int lo, int hi,
                          int tile)
{
    if (hi - lo + 1 <= NARROW) {
        double s = 0.0;
        for (int k = lo; k <= hi; ++k) s += 1.0 / v[k];
        return s;
    }
    const int tlo = div_p2(lo, tile), thi = div_p2(hi, tile);
    const double below = mod_p2(lo, tile) == 0 ? 0.0 : pre[lo - 1];
    if (tlo == thi) return pre[hi] - below;
    return ((tl[thi] - tl[tlo]) - below) + pre[hi];
}

// ------------------------------------------------------------------ grid tables


__global__ __launch_bounds__(WG) void k_sinstr(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const int k = blockIdx.x * WG + threadIdx.x;
    if (k >= g.B) return;
    const double f = (double)(g.k0 + k) / g.T;
    const double v = sinstr_dev(f, g.oms_pm, g.tm_fm, g.arm_m);
    d.sx[k] = v;
    d.isx[k] = 1.0 / v;
}

// In-tile inclusive prefix of 1/v and the tile sums (one block per tile).
__global__ __launch_bounds__(WG) void k_inv_prefix(const Slot *S)
{
    __shared__ double sh[WG / 64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const double *v = d.sx;
    double *pre = d.isx_pre, *tsum = d.isx_tsum;
    const int tile = blockIdx.x, R = g.tile / WG;
    if (tile >= g.nt) return;
    const int base = tile * g.tile + threadIdx.x * R;
    double loc[8];
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int k = base + r;
        if (r < R) s += (k < g.B) ? 1.0 / v[k] : 0.0;
        loc[r] = s;
    }
    double tot;
    const double ex = block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int k = base + r;
        if (r < R && k < g.B) pre[k] = ex + loc[r];
    }
    if (threadIdx.x == 0) tsum[tile] = tot;
}

// Exclusive prefix over the tile sums (single block).  Each thread owns a
// contiguous run of ceil(n / WG) entries: its loads are all issued at once
// (no chain of per-chunk scans waiting on memory), one block scan combines
// the run totals, and a second pass over the (cached) run writes the prefix.
template <typename T, int NT = WG, typename A = T>
DEVI void block_scan_array(const T *in, T *out, int n)
{
    __shared__ A sh[NT / 64];
    constexpr int RUN = 8;                 // runs this short stay in registers
    const int per = (n + NT - 1) / NT;
    const int b = min((int)threadIdx.x * per, n), e = min(b + per, n);
    if (per <= RUN) {
        // every load of the run issued before the first use (clamped
        // indices, no branches around the loads)
        A v[RUN];
#pragma unroll
        for (int r = 0; r < RUN; ++r) v[r] = (A)in[min(b + r, n - 1 < 0 ? 0 : n - 1)];
        A s = zero_t<A>();
#pragma unroll
        for (int r = 0; r < RUN; ++r)
            if (b + r < e) s = add_t(s, v[r]);
        A tot;
        A run = block_excl_scan<A, NT>(s, sh, &tot);
#pragma unroll
        for (int r = 0; r < RUN; ++r) {
            if (b + r < e) {
                out[b + r] = (T)run;
                run = add_t(run, v[r]);
            }
        }
        if (threadIdx.x == 0) out[n] = (T)tot;
        return;
    }
    A s = zero_t<A>();
#pragma unroll 8
    for (int i = b; i < e; ++i) s = add_t(s, (A)in[i]);
    A tot;
    A run = block_excl_scan<A, NT>(s, sh, &tot);
#pragma unroll 8
    for (int i = b; i < e; ++i) {
        const A x = (A)in[i];
        out[i] = (T)run;
        run = add_t(run, x);
    }
    if (threadIdx.x == 0) out[n] = (T)tot;
}

__global__ __launch_bounds__(WG) void k_sx_scan(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    block_scan_array<double>(d.isx_tsum, d.isx_tile, g.nt);
}

// (min, max) of 1/S_instr over each segment of SEG_BINS bins (one wave per
// segment): bounds that decide most one-bin candidate tests without the
// table value of the source's bin.
__global__ __launch_bounds__(WG) void k_isx_seg(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const int seg = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const int nseg = (g.B + SEG_BINS - 1) / SEG_BINS;
    if (seg >= nseg) return;
    double mn = INFINITY, mx = -INFINITY;
    for (int k = seg * SEG_BINS + lane_id(); k < min((seg + 1) * SEG_BINS, g.B); k += 64) {
        const double x = d.isx[k];
        mn = fmin(mn, x);
        mx = fmax(mx, x);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if (lane_id() == 0) d.isx_seg[seg] = make_double2(mn, mx);
}

// ------------------------------------------------------------------ reset

// Clears the per-run state of a slot: control block, tile counters, dirty
// stamps (every tile is dirty for the first loop body, t = 0).
__global__ __launch_bounds__(WG) void k_reset(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl *c = d.ctl;
        c->amax_bits = 0;
        c->bad = 0;
        c->n_cand = 0;
        c->done = 0;
        c->n_iter = 0;
        c->n_resolved = 0;
        c->n_chunks = 0;
        c->cand_cursor = 0;
        c->n_events = 0;
        c->iter = 0;
        c->n_near = 0;
        c->min_margin = 0x7FF0000000000000ull;   // +inf
        c->units_x = (uint64_t)g.B;              // the first body converts and filters every bin
        c->units_med = (uint64_t)g.B;
        c->units_snr = 0;
        c->status = 0;
        c->med_split = (uint32_t)g.nt <= g.split_tiles;   // every tile is dirty
        c->n_sdl = (uint32_t)g.nt;
        c->xupd = 0;
        c->tail_due = 0;
    }
    for (int i = blockIdx.x * WG + threadIdx.x; i < g.nt; i += gridDim.x * WG) {
        d.xstamp[i] = 0;          // body 0 converts and filters every tile
        d.sstamp[i] = 0;
        d.sdl[i] = (uint32_t)i;
        d.Dadj[i].h = 0;
        d.Dadj[i].l = 0;
    }
}

// ------------------------------------------------------------------ prep
//
// Per source (Sec. "Signal parametrization"; appendix "Subtraction
// algorithm", steps 2-3): power P = A^2 T / 2, mid-track frequency
// f + fdot T/2, centre bin floor(fbar T + 1/2) - k0, n = 1 + floor(|fdot| T^2)
// bins, per-bin power q = P/n, track clipped to the grid; rho_0^2 against
// S_instr; candidate iff rho_0^2 >= (kappa rho_th)^2.
//
// Binning without global atomics: a count pass tallies the binning events
// of each block of PREP_SRC sources per tile in LDS and writes that row of
// counts; a column pass gives every (block, tile) its first slot among the
// tile's events (the counts of the blocks before it) and the tile totals;
// after a scan of the totals, a scatter pass writes every event to its
// tile's contiguous segment; accumulation blocks then sum up to ACC_EV
// events of one tile in LDS (exact 128-bit integers) and write the tile's
// bins, hot tiles through partial sums reduced by a last pass.

struct Trk {
    bool ok, live;
    int glo, ghi;
    double q;
};

// Track and per-bin power of one source (no candidate test).
DEVI Trk track_geom(const Grid &g, float Af, float Ff, float FDf)
{
    Trk t;
    t.ok = false;
    t.live = false;
    t.glo = 0;
    t.ghi = -1;
    t.q = 0.0;
    const double a = (double)Af, f = (double)Ff, fd = (double)FDf;
    bool ok = isfinite(a) && a >= 0.0 && isfinite(f) && f > 0.0 && isfinite(fd);
    const double P = ((a * a) * g.T) * 0.5;
    const double fbar = f + (fd * g.T) * 0.5;
    const double x = fbar * g.T + 0.5;
    const double s = (fabs(fd) * g.T) * g.T;
    if (!ok) return t;
    t.ok = true;
    // 2^52 bins or more away, or long (beyond exact integers): at most 2^-52
    // of the power in any bin; no power on the grid
    if (!(fabs(x) < 4503599627370496.0 && s < 4503599627370496.0)) return t;
    // integer-valued fp64 throughout (|values| < 2^53: exact)
    const double c = floor(x) - (double)g.k0;
    const double nn = g.track_single ? 1.0 : 1.0 + floor(s);
    const double lo = c - floor((nn - 1.0) * 0.5);
    const double hi = lo + (nn - 1.0);
    t.q = nn == 1.0 ? P : P / nn;
    const double gl = fmax(lo, 0.0);
    const double gh = fmin(hi, (double)(g.B - 1));
    if (gl > gh) return t;
    t.live = true;
    t.glo = (int)gl;
    t.ghi = (int)gh;
    return t;
}

// rho_0^2 >= (kappa rho_th)^2 against S_instr.  Short tracks sum the stored
// reciprocals 1/S_instr bin by bin in ascending order (the same values and
// order as summing 1/S_instr directly), longer ones use the prefix tables.
// x0 = 1/S_instr of the track's first bin, loaded by the caller.
DEVI bool cand_test(const Grid &g, const Dev &d, const Trk &t, double x0)
{
    if (!t.live) return false;
    double sum;
    if (t.glo == t.ghi) {
        sum = x0;
    } else if (t.ghi - t.glo + 1 <= NARROW) {
        sum = x0;
        for (int k = t.glo + 1; k <= t.ghi; ++k) sum += d.isx[k];
    } else {
        sum = range_inv_sum(d.sx, d.isx_pre, d.isx_tile, t.glo, t.ghi, g.tile);
    }
    return (4.0 * t.q) * sum >= g.cut2;
}

DEVI int tile_of(int bin, int tile) { return div_p2(bin, tile); }

// Count pass: events per tile and candidates of this block.  The per-tile
// counts are 16-bit halves of LDS words (at most 2 PREP_SRC < 2^16 events
// of a block fall in one tile), which keeps the block's LDS at 16 KB; the
// packed words are the block's row of bhist.
DEVI void k_prep_count_body(Grid g, Dev d, const float *A, const float *F, const float *FD, uint64_t n)
{
    __shared__ uint32_t hist[NBK_MAX / 2];
    __shared__ uint32_t scand, samax;
    auto hadd = [&](int b) { atomicAdd(&hist[b >> 1], 1u << (16 * (b & 1))); };
    for (int b = threadIdx.x; b < (g.nt + 1) / 2; b += WG) hist[b] = 0;
    if (threadIdx.x == 0) {
        scand = 0;
        samax = 0;
    }
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * PREP_SRC;
    uint32_t cc = 0, bad = 0, amax = 0;
    constexpr int CB = 8;
    // CB sources per thread in flight: loads first, then the tracks and
    // the S_instr gathers of the candidate tests
    for (int r0 = 0; r0 < PREP_SRC / WG; r0 += CB) {
        float a[CB], f[CB], fd[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const uint64_t i = base + (uint64_t)(r0 + q) * WG + threadIdx.x;
            const bool in = i < n;
            const uint64_t ic = in ? i : n - 1;        // unconditional loads: all in flight at once
            const float av = A[ic], fv = F[ic], fdv = FD[ic];
            a[q] = in ? av : 0.0f;
            f[q] = in ? fv : 1.0f;
            fd[q] = in ? fdv : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            pin(a[q]);
            pin(f[q]);
            pin(fd[q]);
        }
        Trk t[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) t[q] = track_geom(g, a[q], f[q], fd[q]);
        // Bounds from the (min, max) of 1/S_instr over the segments under the
        // track decide most tests without the table values.  One bin:
        // rho_0^2 = (4q) (1/S_instr) lies between (4q) min and (4q) max (the
        // product is monotone).  2 .. NARROW bins (at most two segments): the
        // fp64 sum of the n values lies within n min (1 - n 2^-53) and
        // n max (1 + n 2^-53), so a margin of 1e-12 on n min and n max is
        // safe.  Otherwise, or if the cut falls between the bounds, the table
        // values decide (their gathers all in flight).
        double2 sb[CB], se[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            sb[q] = d.isx_seg[t[q].live ? t[q].glo / SEG_BINS : 0];
            se[q] = d.isx_seg[t[q].live ? t[q].ghi / SEG_BINS : 0];
        }
        bool cand[CB], exact[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const double q4 = 4.0 * t[q].q;
            const int nb = t[q].ghi - t[q].glo + 1;
            const bool one = t[q].live && nb == 1;
            const bool few = t[q].live && nb > 1 && nb <= NARROW;
            const double mn = fmin(sb[q].x, se[q].x), mx = fmax(sb[q].y, se[q].y);
            const double lo = few ? q4 * ((double)nb * mn) * (1.0 - 1e-12) : q4 * mn;
            const double hi = few ? q4 * ((double)nb * mx) * (1.0 + 1e-12) : q4 * mx;
            const bool yes = (one || few) && lo >= g.cut2;
            const bool no = (one || few) && hi < g.cut2;
            cand[q] = yes;
            exact[q] = t[q].live && !yes && !no;
        }
        double x0[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) x0[q] = exact[q] ? d.isx[t[q].glo] : 0.0;
#pragma unroll
        for (int q = 0; q < CB; ++q)
            if (exact[q]) cand[q] = cand_test(g, d, t[q], x0[q]);
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const uint64_t i = base + (uint64_t)(r0 + q) * WG + threadIdx.x;
            const bool in = i < n;
            const bool c = in && t[q].ok && cand[q];
            const uint64_t m = (uint64_t)__ballot(c);
            const uint64_t w0 = i - (uint64_t)lane_id();       // first source of this wave
            if (lane_id() == 0 && w0 < n) d.cbits[w0 >> 6] = m;
            if (!in) continue;
            if (!t[q].ok) {
                bad = 1;
                continue;
            }
            amax = max(amax, __float_as_uint(a[q]));      // A >= 0: bit patterns in value order
            if (t[q].live) {
                hadd(tile_of(t[q].glo, g.tile));
                if (t[q].glo != t[q].ghi && t[q].ghi + 1 < g.B) hadd(tile_of(t[q].ghi + 1, g.tile));
            }
            cc += c;
        }
    }
    for (int s = 32; s >= 1; s >>= 1) {
        cc += (uint32_t)__shfl_xor((int)cc, s, 64);
        amax = max(amax, (uint32_t)__shfl_xor((int)amax, s, 64));
    }
    if (lane_id() == 0 && cc) atomicAdd(&scand, cc);
    if (lane_id() == 0 && amax) atomicMax(&samax, amax);
    __syncthreads();
    // per-block results (k_prep_plan combines them: no atomics on one address)
    if (threadIdx.x == 0) {
        d.blk_cand[blockIdx.x] = scand;
        d.blk_amax[blockIdx.x] = samax;
    }
    const int hw = (g.nt + 1) / 2;
    for (int b = threadIdx.x; b < hw; b += WG) d.bhist[(size_t)blockIdx.x * hw + b] = hist[b];
    if (bad) atomicOr(&d.ctl->bad, 1u);
}

__global__ __launch_bounds__(WG) void k_prep_count(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || (uint64_t)blockIdx.x * PREP_SRC >= sl.n) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const float *A = sl.A, *F = sl.F, *FD = sl.FD;
    const uint64_t n = sl.n;
    k_prep_count_body(g, d, A, F, FD, n);
}


// Column pass: for each tile, the exclusive prefix over the prep blocks of
// its event counts (where each block's events start inside the tile's
// segment) and the tile's total.  A block takes 64 tiles (one per lane; the
// loads and stores of consecutive tiles are coalesced) and its 16 waves
// split the prep blocks into ranges: each wave sums its range, a prefix
// over the waves gives each range its start, and each wave walks its range
// again writing the offsets.
__global__ __launch_bounds__(CS_WG) void k_prep_colscan(const Slot *S)
{
    constexpr int NV = CS_WG / 64;
    __shared__ uint32_t part[NV][64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int tile = blockIdx.x * 64 + lane;
    const bool ok = tile < g.nt;
    const int col = ok ? tile : g.nt - 1;                      // a valid column; results dropped
    const int nb = (int)((sl.n + PREP_SRC - 1) / PREP_SRC);
    const int per = (nb + NV - 1) / NV;
    const int b0 = min(w * per, nb), b1 = min(b0 + per, nb);
    const size_t row = 2 * (size_t)((g.nt + 1) / 2);          // 16-bit counts per bhist row
    const uint16_t *h16 = reinterpret_cast<const uint16_t *>(d.bhist);
    constexpr int U = 16;
    uint32_t sum = 0;
    for (int bb = b0; bb < b1; bb += U) {
        uint32_t c[U];
#pragma unroll
        for (int q = 0; q < U; ++q) c[q] = h16[(size_t)min(bb + q, b1 - 1) * row + col];
#pragma unroll
        for (int q = 0; q < U; ++q) sum += bb + q < b1 ? c[q] : 0u;
    }
    part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const uint32_t x = part[v][lane];
        run += v < w ? x : 0u;
        tot += x;
    }
    if (w == 0 && ok) d.btot[tile] = tot;
    for (int bb = b0; bb < b1; bb += U) {
        uint32_t c[U];
#pragma unroll
        for (int q = 0; q < U; ++q) c[q] = h16[(size_t)min(bb + q, b1 - 1) * row + col];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (bb + q < b1) {
                if (ok) d.boff[(size_t)(bb + q) * g.nt + tile] = run;
                run += c[q];
            }
        }
    }
}

// Plan (one block): tile bases, accumulation blocks and partial-sum slots;
// clears the tile sums of D.
__global__ __launch_bounds__(WG) void k_prep_plan(const Slot *S)
{
    __shared__ uint32_t sh[WG / 64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;

    // largest A and the candidates of the count blocks: their exclusive
    // prefix is each scatter block's first candidate slot
    {
        const int nb = (int)((sl.n + PREP_SRC - 1) / PREP_SRC);
        uint32_t am = 0;
        for (int b = threadIdx.x; b < nb; b += WG) am = max(am, d.blk_amax[b]);
        for (int s = 32; s >= 1; s >>= 1) am = max(am, (uint32_t)__shfl_xor((int)am, s, 64));
        if (lane_id() == 0) sh[threadIdx.x >> 6] = am;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < WG / 64; ++w) am = max(am, sh[w]);
            d.ctl->amax_bits = am;
        }
        __syncthreads();
        block_scan_array<uint32_t>(d.blk_cand, d.blk_cand, nb);   // in place: each thread rereads its own run
        if (threadIdx.x == 0) d.ctl->n_cand = d.blk_cand[nb];
        __syncthreads();
    }

    uint32_t carry_e = 0, carry_c = 0, carry_s = 0;
    for (int base = 0; base < g.nt; base += WG) {
        const int b = base + threadIdx.x;
        const uint32_t cnt = b < g.nt ? d.btot[b] : 0u;
        const uint32_t nc = b < g.nt ? max(1u, (cnt + ACC_EV - 1) / ACC_EV) : 0u;
        const uint32_t ns = nc > 1 ? nc : 0u;
        uint32_t te, tc, ts;
        const uint32_t ee = block_excl_scan(cnt, sh, &te);
        const uint32_t ec = block_excl_scan(nc, sh, &tc);
        const uint32_t es = block_excl_scan(ns, sh, &ts);
        if (b < g.nt) {
            d.bbase[b] = carry_e + ee;
            d.nch[b] = nc;
            d.chunk_base[b] = carry_c + ec;
            d.slot_base[b] = carry_s + es;
            d.Dtile[b].lo = 0;
            d.Dtile[b].hi = 0;
            if (g.prec == PREC_COMP) d.Dtc[b] = ff_of(0.0f);
        }
        carry_e += te;
        carry_c += tc;
        carry_s += ts;
    }
    if (threadIdx.x == 0) {
        d.bbase[g.nt] = carry_e;
        d.chunk_base[g.nt] = carry_c;
        d.Dtile[g.nt].lo = 0;
        d.Dtile[g.nt].hi = 0;
        d.ctl->n_events = carry_e;
        d.ctl->n_chunks = carry_c;
        if (carry_s > d.max_slots || carry_c > d.max_chunks) d.ctl->bad |= 2u;   // cannot happen: sized for the worst case
    }
}

// Scatter pass: the block's events start, inside each tile's segment, at
// the slot the column pass gave it; it writes the events and the candidate
// records.
DEVI void k_prep_scatter_body(Grid g, Dev d, const float *A, const float *F, const float *FD, uint64_t n)
{
    __shared__ uint32_t cur[NBK_MAX];
    __shared__ uint32_t scand, cbase;
    for (int b = threadIdx.x; b < g.nt; b += WG) cur[b] = d.bbase[b] + d.boff[(size_t)blockIdx.x * g.nt + b];
    if (threadIdx.x == 0) {
        cbase = d.blk_cand[blockIdx.x];
        scand = 0;
    }
    __syncthreads();
    const int L = fx_exp(d.ctl->amax_bits, g.T);
    const uint64_t base = (uint64_t)blockIdx.x * PREP_SRC;
    constexpr int SB = 8;                    // sources per thread in flight
    for (int r0 = 0; r0 < PREP_SRC / WG; r0 += SB) {
        float a[SB], f[SB], fd[SB];
        uint64_t cw[SB];                         // candidate-flag words of the sources
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            const uint64_t i = base + (uint64_t)(r0 + q) * WG + threadIdx.x;
            const bool in = i < n;
            const uint64_t ic = in ? i : n - 1;        // unconditional loads: all in flight at once
            const float av = A[ic], fv = F[ic], fdv = FD[ic];
            a[q] = in ? av : 0.0f;
            f[q] = in ? fv : 1.0f;
            fd[q] = in ? fdv : 0.0f;
            cw[q] = d.cbits[ic >> 6];
        }
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            pin(a[q]);
            pin(f[q]);
            pin(fd[q]);
            pin(cw[q]);
        }
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            const uint64_t i = base + (uint64_t)(r0 + q) * WG + threadIdx.x;
            if (i >= n) continue;
            const Trk t = track_geom(g, a[q], f[q], fd[q]);
            if (!t.ok) continue;
            const uint64_t qfx = to_fx(t.q, L);
            if (t.live) {                  // every live source, so the counts match
                if (t.glo == t.ghi) {
                    const uint32_t p = atomicAdd(&cur[tile_of(t.glo, g.tile)], 1u);
                    d.ev_key[p] = (uint32_t)t.glo;
                    d.ev_val[p] = (int64_t)qfx;
                } else {
                    uint32_t p = atomicAdd(&cur[tile_of(t.glo, g.tile)], 1u);
                    d.ev_key[p] = (uint32_t)t.glo | 0x80000000u;
                    d.ev_val[p] = (int64_t)qfx;
                    if (t.ghi + 1 < g.B) {
                        p = atomicAdd(&cur[tile_of(t.ghi + 1, g.tile)], 1u);
                        d.ev_key[p] = (uint32_t)(t.ghi + 1) | 0x80000000u;
                        d.ev_val[p] = -(int64_t)qfx;
                    }
                }
            }
            if ((cw[q] >> (i & 63)) & 1ull) {
                const uint32_t j = cbase + atomicAdd(&scand, 1u);
                d.c_src[j] = (uint32_t)i;
                d.c_glo[j] = t.glo;
                d.c_ghi[j] = t.ghi;
                d.c_q[j] = t.q;
                d.c_qfx[j] = qfx;
                d.c_iter[j] = -1;
            }
        }
    }
}

__global__ __launch_bounds__(WG) void k_prep_scatter(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || (uint64_t)blockIdx.x * PREP_SRC >= sl.n) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const float *A = sl.A, *F = sl.F, *FD = sl.FD;
    const uint64_t n = sl.n;
    k_prep_scatter_body(g, d, A, F, FD, n);
}


DEVI void lds_add_i128(I128 *p, int64_t v)
{
    const uint64_t vlo = (uint64_t)v;
    const int64_t vhi = v < 0 ? -1 : 0;
    const uint64_t old = atomicAdd((unsigned long long *)&p->lo, (unsigned long long)vlo);
    const int64_t add_hi = vhi + (int64_t)((uint64_t)(old + vlo) < old);
    if (add_hi != 0) atomicAdd((unsigned long long *)&p->hi, (unsigned long long)add_hi);
}

DEVI void atomic_add_i128_full(I128 *p, I128 v)
{
    const uint64_t old = atomicAdd((unsigned long long *)&p->lo, (unsigned long long)v.lo);
    const int64_t add_hi = v.hi + (int64_t)((uint64_t)(old + v.lo) < old);
    if (add_hi != 0) atomicAdd((unsigned long long *)&p->hi, (unsigned long long)add_hi);
}

// Accumulation: block c sums up to ACC_EV events of one tile in LDS.  Each
// 64-bit event value v = vh 2^32 + vl (vl in [0, 2^32)) goes into two 64-bit
// LDS sums with non-returning atomics (no carry to propagate: at most ACC_EV
// events per block, so |sum vh| < 2^47 and sum vl < 2^48); the exact
// 128-bit total is sum_vh 2^32 + sum_vl.
struct SplitAcc {
    int64_t h[TILE_MAX];
    uint64_t l[TILE_MAX];
};

DEVI void split_add(SplitAcc &a, int k, int64_t v)
{
    atomicAdd((unsigned long long *)&a.h[k], (unsigned long long)(v >> 32));
    atomicAdd((unsigned long long *)&a.l[k], (unsigned long long)((uint64_t)v & 0xFFFFFFFFull));
}

DEVI I128 split_total(const SplitAcc &a, int k)
{
    const int64_t h = a.h[k];
    I128 x;
    x.lo = (uint64_t)h << 32;
    x.hi = h >> 32;
    I128 y;
    y.lo = a.l[k];
    y.hi = 0;
    return i128_add(x, y);
}

// The compensated FP32 mode's binning of events e0 .. e1 of tile b (chunk
// ci): every event's power rounded to fp32 (scaled by 2^sc), summed per bin
// in LDS by compensated atomics (xc: one-bin tracks, dc: difference array;
// TILE_MAX entries each); written to Xc, Dc and the tile sum of Dc, or to
// the chunk's partial-sum slot of a hot tile.
DEVI void accum_comp(const Grid &g, const Dev &d, int b, uint32_t ci, uint32_t e0, uint32_t e1, FF *xc, FF *dc)
{
    __shared__ FF shf[WG / 64];
    const int k0 = b * g.tile;
    const int L = fx_exp(d.ctl->amax_bits, g.T);
    const int sc = f32_scale(d.ctl->amax_bits, g.T);
    for (int k = threadIdx.x; k < g.tile; k += WG) {
        xc[k] = ff_of(0.0f);
        dc[k] = ff_of(0.0f);
    }
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += WG) {
        const uint32_t key = d.ev_key[e];
        const float v = (float)ldexp((double)d.ev_val[e], L + sc);
        const int k = (int)(key & 0x7FFFFFFFu) - k0;
        ff_atomic_add((key >> 31) ? &dc[k] : &xc[k], v);
    }
    __syncthreads();
    const int nbin = min(g.tile, g.B - k0);
    if (d.nch[b] == 1) {
        FF s = ff_of(0.0f);
        for (int k = threadIdx.x; k < g.tile; k += WG) {
            if (k < nbin) {
                const FF x = ff_norm(xc[k].hi, xc[k].lo), y = ff_norm(dc[k].hi, dc[k].lo);
                d.Xc[k0 + k] = x;
                d.Dc[k0 + k] = y;
                s = ff_add(s, y);
            }
        }
        FF tot;
        block_excl_scan(s, shf, &tot);
        if (threadIdx.x == 0) d.Dtc[b] = tot;
    } else {
        FF *slot = reinterpret_cast<FF *>(d.partial + (size_t)(d.slot_base[b] + ci) * 2 * g.tile);
        for (int k = threadIdx.x; k < g.tile; k += WG) {
            slot[k] = ff_norm(xc[k].hi, xc[k].lo);
            slot[g.tile + k] = ff_norm(dc[k].hi, dc[k].lo);
        }
    }
}

__global__ __launch_bounds__(WG) void k_accum(const Slot *S)
{
    __shared__ SplitAcc xn, dd;
    __shared__ I128 sh[WG / 64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;

    const uint32_t c = blockIdx.x;
    if (c >= d.ctl->n_chunks) return;
    // tile b: the last with chunk_base[b] <= c
    int lo = 0, hi = g.nt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.chunk_base[mid] <= c) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const uint32_t ci = c - d.chunk_base[b];
    const uint32_t e0 = d.bbase[b] + ci * ACC_EV;
    const uint32_t e1 = min(e0 + (uint32_t)ACC_EV, d.bbase[b + 1]);
    const int k0 = b * g.tile;
    if (g.prec == PREC_COMP) {
        accum_comp(g, d, b, ci, e0, e1, reinterpret_cast<FF *>(xn.h), reinterpret_cast<FF *>(dd.h));
        return;
    }
    for (int k = threadIdx.x; k < g.tile; k += WG) {
        xn.h[k] = 0; xn.l[k] = 0;
        dd.h[k] = 0; dd.l[k] = 0;
    }
    __syncthreads();
    // four events per thread in flight
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += 4 * WG) {
        uint32_t key[4];
        int64_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t ee = e + (uint32_t)(q * WG);
            key[q] = ee < e1 ? d.ev_key[ee] : 0u;
            v[q] = ee < e1 ? d.ev_val[ee] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (e + (uint32_t)(q * WG) >= e1) continue;
            const int k = (int)(key[q] & 0x7FFFFFFFu) - k0;
            split_add((key[q] >> 31) ? dd : xn, k, v[q]);
        }
    }
    __syncthreads();
    const int nbin = min(g.tile, g.B - k0);
    if (d.nch[b] == 1) {
        I128 s = zero_t<I128>();
        for (int k = threadIdx.x; k < g.tile; k += WG) {
            if (k < nbin) {
                const I128 dk = split_total(dd, k);
                d.Xn[k0 + k] = split_total(xn, k);
                d.D[k0 + k] = dk;
                s = i128_add(s, dk);
            }
        }
        I128 tot;
        block_excl_scan(s, sh, &tot);
        if (threadIdx.x == 0) d.Dtile[b] = tot;
    } else {
        I128 *slot = d.partial + (size_t)(d.slot_base[b] + ci) * 2 * g.tile;
        for (int k = threadIdx.x; k < g.tile; k += WG) {
            slot[k] = split_total(xn, k);
            slot[g.tile + k] = split_total(dd, k);
        }
    }
}

// Hot tiles (several accumulation blocks): sum the partials, RED_BINS bins
// per block.
__global__ __launch_bounds__(RED_BINS) void k_accum_reduce(const Slot *S)
{
    __shared__ I128 sh[RED_BINS / 64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const int per = g.tile / RED_BINS;
    const int b = blockIdx.x / per, part = blockIdx.x % per;
    if (b >= g.nt) return;
    const uint32_t nc = d.nch[b];
    if (nc <= 1) return;
    const int k = part * RED_BINS + threadIdx.x;
    const int k0 = b * g.tile;
    const int nbin = min(g.tile, g.B - k0);
    if (g.prec == PREC_COMP) {
        // the chunks' double-fp32 partials in chunk order; the block's sum
        // of Dc goes to the tile sum by a compensated atomic
        __shared__ FF shc[RED_BINS / 64];
        const FF *slot = reinterpret_cast<const FF *>(d.partial + (size_t)d.slot_base[b] * 2 * g.tile);
        FF xs = ff_of(0.0f), ys = ff_of(0.0f);
        for (uint32_t c = 0; c < nc; ++c) {
            xs = ff_add(xs, slot[(size_t)c * 4 * g.tile + k]);
            ys = ff_add(ys, slot[(size_t)c * 4 * g.tile + g.tile + k]);
        }
        if (k < nbin) {
            d.Xc[k0 + k] = xs;
            d.Dc[k0 + k] = ys;
        } else {
            ys = ff_of(0.0f);
        }
        FF tot;
        block_excl_scan<FF, RED_BINS>(ys, shc, &tot);
        if (threadIdx.x == 0) {
            ff_atomic_add(&d.Dtc[b], tot.hi);
            ff_atomic_add(&d.Dtc[b], tot.lo);
        }
        return;
    }
    I128 x = zero_t<I128>(), y = zero_t<I128>();
    const I128 *slot = d.partial + (size_t)d.slot_base[b] * 2 * g.tile;
    for (uint32_t s = 0; s < nc; ++s) {
        x = i128_add(x, slot[(size_t)s * 2 * g.tile + k]);
        y = i128_add(y, slot[(size_t)s * 2 * g.tile + g.tile + k]);
    }
    I128 dsum = zero_t<I128>();
    if (k < nbin) {
        d.Xn[k0 + k] = x;
        d.D[k0 + k] = y;
        dsum = y;
    }
    // block sum of D into the tile sum (one exact 128-bit atomic per block)
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    I128 inc = wave_incl_scan(dsum);
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        I128 t = zero_t<I128>();
        for (int w = 0; w < RED_BINS / 64; ++w) t = i128_add(t, sh[w]);
        atomic_add_i128_full(&d.Dtile[b], t);
    }
}

__global__ __launch_bounds__(WG) void k_dscan(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;

    block_scan_array<I128>(d.Dtile, d.Dcarry, g.nt);
    if (g.prec == PREC_NAIVE) {
        __syncthreads();
        block_scan_array<float>(d.Dtf, d.Dcf, g.nt);
    }
}

// Naive FP32 mode: the same events summed again in fp32, in whatever order
// the atomics land (the accumulation the paper's float scatter performs).
__global__ __launch_bounds__(WG) void k_zero_f32(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.prec != PREC_NAIVE) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    for (int i = blockIdx.x * WG + threadIdx.x; i <= g.B; i += gridDim.x * WG) {
        if (i < g.B) d.Xf[i] = 0.0f;
        d.Df[i] = 0.0f;
        if (i <= g.nt) d.Dtf[i] = 0.0f;
    }
}

__global__ __launch_bounds__(WG) void k_accum_f32(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.prec != PREC_NAIVE) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    const int L = fx_exp(d.ctl->amax_bits, g.T);
    const int sc = f32_scale(d.ctl->amax_bits, g.T);
    const uint32_t ne = d.ctl->n_events;
    for (uint32_t e = blockIdx.x * WG + threadIdx.x; e < ne; e += gridDim.x * WG) {
        const uint32_t key = d.ev_key[e];
        const float v = (float)ldexp((double)d.ev_val[e], L + sc);
        const int k = (int)(key & 0x7FFFFFFFu);
        if (key >> 31) {
            atomicAdd(&d.Df[k], v);
            atomicAdd(&d.Dtf[div_p2(k, g.tile)], v);
        } else {
            atomicAdd(&d.Xf[k], v);
        }
    }
}

// ------------------------------------------------------------------ X update

// X[k] = 2^L * (Xn[k] + prefix(D)[k]) for the tiles whose X changed.  D and
// Xn are read and X written in coalesced order; the in-tile prefix runs over
// thread-contiguous runs staged in LDS (one pad entry per 8 against bank
// conflicts).
DEVI int xpad(int i) { return i + (i >> 3); }

template <int NT> DEVI void snr_tail(const Slot &sl);

// The compensated FP32 mode's X of one tile: X = Xc + (carry + in-tile
// prefix of Dc), every sum double-fp32, rounded once to fp32 at the end.
// The carry is the sum of the tile sums of Dc before the tile (kept current
// by the subtractions), added up here in a fixed order.  `st` is LDS for the
// tile (xpad layout).
DEVI void xupdate_comp(const Grid &g, const Dev &d, int tile, int t0, int n, int R, int b, FF *st)
{
    __shared__ FF shc[WG / 64];
    const int sc = f32_scale(d.ctl->amax_bits, g.T);
    FF c = ff_of(0.0f);
    for (int j = threadIdx.x; j < tile; j += WG) c = ff_add(c, d.Dtc[j]);
    FF carry;
    block_excl_scan(c, shc, &carry);
    for (int i = threadIdx.x; i < n; i += WG) st[xpad(i)] = d.Dc[t0 + i];
    __syncthreads();
    FF s = ff_of(0.0f);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (r < R && b + r < n) {
            s = ff_add(s, st[xpad(b + r)]);
            st[xpad(b + r)] = s;
        }
    }
    FF tot;
    const FF ex = ff_add(block_excl_scan(s, shc, &tot), carry);
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (r < R && b + r < n) st[xpad(b + r)] = ff_add(st[xpad(b + r)], ex);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += WG)
        d.X[t0 + i] = ldexp((double)ff_float(ff_add(st[xpad(i)], d.Xc[t0 + i])), -sc);
}

// The last block of the grid is the tail of the previous k_snr; the other
// blocks convert the tiles stamped with the value k_snr published.  They
// touch disjoint data: the tail reads the partials and the stamps and
// writes the control block's counters and flags, while the converting
// blocks read the accumulators, the stamps and the control fields set
// before this launch (bad, xupd, amax_bits), never the settled flag.  Past the
// settled body no k_snr runs and the accumulators stay as they are: a body
// that settles the loop subtracted nothing and stamped nothing, and after a
// max_iter stop the tiles of the last stamp are only converted again to the
// same values.
__global__ __launch_bounds__(WG) void k_xupdate(const Slot *S)
{
    __shared__ I128 sh[WG / 64];
    __shared__ I128 stage[TILE_MAX + TILE_MAX / 8];
    __shared__ float shf[WG / 64];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    if (blockIdx.x == gridDim.x - 1) {
        snr_tail<WG>(sl);
        return;
    }
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->bad) return;
    const int tile = blockIdx.x;
    if (tile >= g.nt || d.xstamp[tile] != d.ctl->xupd) return;
    const int L = fx_exp(d.ctl->amax_bits, g.T);
    const int t0 = tile * g.tile;
    const int n = min(g.tile, g.B - t0);
    const int R = g.tile / WG;
    const int b = (int)threadIdx.x * R;
    if (g.prec == PREC_COMP) {
        xupdate_comp(g, d, tile, t0, n, R, b, reinterpret_cast<FF *>(stage));
        return;
    }
    for (int i = threadIdx.x; i < n; i += WG) stage[xpad(i)] = d.D[t0 + i];
    __syncthreads();
    I128 s = zero_t<I128>();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (r < R && b + r < n) {
            s = i128_add(s, stage[xpad(b + r)]);
            stage[xpad(b + r)] = s;
        }
    }
    I128 tot;
    I128 ex = block_excl_scan(s, sh, &tot);
    ex = i128_add(ex, i128_add(d.Dcarry[tile], split_sum_value(d.Dadj[tile])));
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (r < R && b + r < n) stage[xpad(b + r)] = i128_add(stage[xpad(b + r)], ex);
    __syncthreads();
    if (g.prec == PREC_FP64) {
        for (int i = threadIdx.x; i < n; i += WG)
            d.X[t0 + i] = ldexp(i128_to_double(i128_add(stage[xpad(i)], d.Xn[t0 + i])), L);
        return;
    }
    const int sc = f32_scale(d.ctl->amax_bits, g.T);
    // naive fp32: X = Xf + prefix of Df, all in fp32
    __syncthreads();
    float *fst = reinterpret_cast<float *>(stage);
    for (int i = threadIdx.x; i < n; i += WG) fst[xpad(i)] = d.Df[t0 + i];
    __syncthreads();
    float fs = 0.0f;
    float floc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (r < R && b + r < n) fs += fst[xpad(b + r)];
        floc[r] = fs;
    }
    float ftot;
    const float fex = block_excl_scan<float>(fs, shf, &ftot) + d.Dcf[tile];
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (r < R && b + r < n) fst[xpad(b + r)] = fex + floc[r];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += WG) d.X[t0 + i] = ldexp((double)(d.Xf[t0 + i] + fst[xpad(i)]), -sc);
}

// ------------------------------------------------------------------ running median
//
// S[k] = C * median{X[a_k .. a_k+W-1]} + S_instr[k]   (Eq. "running median").
//
// One block per tile of `tile` outputs.  The union of the tile's windows
// (tile + W - 1 bins) is loaded once into LDS and sorted there: a stable LSD
// radix sort on a per-tile 20-bit order key (the fp64 bit pattern minus the
// tile minimum, shifted), then an exact repair that orders equal keys by
// the full fp64 value.  The sorted index (rank) of every union position
// then goes into a wavelet matrix: one stable partition of the rank
// sequence per rank bit, most significant first, down to buckets of 32
// consecutive ranks, with the bit words and a zero count per 64 positions
// kept in LDS.  The median of a window is the h-th smallest rank among its
// W positions: descending the levels (two rank queries per level) gives its
// bucket and its index there, and the bucket's 32 sorted elements are
// tested against the window.  Each of the 512 threads answers its
// R = tile/512 (at most 4) windows independently.  Selection is exact: no
// arithmetic touches X.

constexpr int MWG = 512;                    // threads of a median block
constexpr int RMAX = TILE_MAX / MWG;        // outputs per thread, at most
constexpr int MCH = MMAX / MWG;             // union elements per thread in the sort
constexpr int REPAIR_ROUNDS = 16;           // tie-repair rounds after which the sort is refined
constexpr int WLB = 12;                     // wavelet levels, at most: ranks < MMAX <= 2^12
constexpr int WWD = MMAX / 64 + 1;          // 64-position words per level (+1: the end position)

// One 64-position word of a wavelet level: its bits and the zeros before it.
struct alignas(16) WWord {
    uint64_t bits;
    uint32_t zpre;
    uint32_t pad;
};

struct MedianSmem {
    double xv[MMAX];                       // X over the union, position order
    uint32_t kp[2][MMAX];                  // sort words: key << POSBITS | position
    uint16_t rank[MMAX];                   // sorted index of each position
    union {
        uint16_t off[16 * MWG];             // radix: per-thread digit offsets
        struct {
            WWord w[WLB][WWD];             // bits of the positions, level by level
            uint32_t zt[WLB];              // zeros of the level
            uint32_t zc[MCH * (MWG / 64)]; // zeros per (element chunk, wave)
        } wm;                              // wavelet matrix of the ranks
        double stage[TILE_MAX];            // outputs, for coalesced stores
    } u;
    uint32_t wsc[(MWG / 64 + 1) * 8];       // cross-wave scan exchange of the radix sort
    uint64_t red[2 * (MWG / 64)];
    double dsh[MWG / 64];
    int flag;
};

// Inclusive scan of a u32 across the 64 lanes of a wave (DPP row shifts and
// row broadcasts; every lane must be active).
DEVI uint32_t wave_scan_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

// Block-wide exclusive scan of NW words per thread (fields must not
// overflow); tot[] receives the block totals.  The per-wave totals are
// combined by NW threads (one word each), so a thread keeps only its own
// words in registers.  Contains two barriers; `wsc` holds (MWG/64 + 1) * NW
// words and may be rewritten only after a further barrier.
template <int NW>
DEVI void block_scan_words(const uint32_t (&w)[NW], uint32_t (&ex)[NW], uint32_t (&tot)[NW],
                           uint32_t *wsc)
{
    constexpr int NV = MWG / 64;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) inc[j] = wave_scan_u32(w[j]);
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < NW; ++j) wsc[wave * NW + j] = inc[j];
    }
    __syncthreads();
    if ((int)threadIdx.x < NW) {
        const int j = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const uint32_t x = wsc[v * NW + j];
            wsc[v * NW + j] = run;
            run += x;
        }
        wsc[NV * NW + j] = run;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        ex[j] = wsc[wave * NW + j] + inc[j] - w[j];
        tot[j] = wsc[NV * NW + j];
    }
}

// Stable LSD radix sort of the M words in sm.kp[0] by bits [POSBITS,
// POSBITS + 4*passes), 4 bits per pass; returns the buffer holding the
// result.  Thread chunks are contiguous in the current order; within-chunk
// ranks are kept in registers.
DEVI int radix_sort_tile(MedianSmem &sm, int M, int passes)
{
    const int tid = threadIdx.x;
    const int CH = (M + MWG - 1) / MWG;
    const int beg = tid * CH;
    int in = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int sh = POSBITS + 4 * ps;
        const uint32_t *kin = sm.kp[in];
        uint32_t *kout = sm.kp[in ^ 1];
        uint32_t e[MCH];
        uint32_t lr[MCH];
        uint64_t c = 0;
#pragma unroll
        for (int i = 0; i < MCH; ++i) e[i] = (i < CH && beg + i < M) ? kin[beg + i] : 0u;
#pragma unroll
        for (int i = 0; i < MCH; ++i) {
            if (i < CH && beg + i < M) {
                const uint32_t dg = (e[i] >> sh) & 15u;
                lr[i] = (uint32_t)(c >> (4 * dg)) & 15u;
                c += 1ull << (4 * dg);
            }
        }
        uint32_t w[8], ex[8], tot[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            w[j] = (uint32_t)((c >> (8 * j)) & 15u) | ((uint32_t)((c >> (8 * j + 4)) & 15u) << 16);
        block_scan_words<8>(w, ex, tot, sm.wsc);
        uint32_t run = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sm.u.off[(2 * j) * MWG + tid] = (uint16_t)(run + (ex[j] & 0xFFFFu));
            run += tot[j] & 0xFFFFu;
            sm.u.off[(2 * j + 1) * MWG + tid] = (uint16_t)(run + (ex[j] >> 16));
            run += tot[j] >> 16;
        }
        // offsets are private to the thread: no barrier before reading them
#pragma unroll
        for (int i = 0; i < MCH; ++i) {
            if (i < CH && beg + i < M) {
                const uint32_t dg = (e[i] >> sh) & 15u;
                kout[sm.u.off[dg * MWG + tid] + lr[i]] = e[i];
            }
        }
        __syncthreads();
        in ^= 1;
    }
    return in;
}

// In-part inclusive prefix of the values st[0 .. t1-t0) of a median block
// (thread-contiguous runs of R outputs; a part is part/R threads, whole
// waves), accumulated in type A; writes the prefix back into st and the part
// sums to is_psum.  Contains one barrier.
template <typename A>
DEVI void part_prefix(double *dsh, double *st, const Grid &g, const Dev &d, int kb, int ke, int t0,
                      int t1, int R)
{
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    A loc[RMAX], s = zero_t<A>();
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        if (kb + r < ke) s += (A)st[kb + r - t0];
        loc[r] = s;
    }
    const int segw = (g.part / R) >> 6;
    const A inc = wave_incl_scan(s);
    A exw = shfl_up_t(inc, 1);
    if (lane == 0) exw = zero_t<A>();
    A *xch = reinterpret_cast<A *>(dsh);
    if (lane == 63) xch[wave] = inc;
    __syncthreads();
    const int ws0 = (wave / segw) * segw;
    A pre = zero_t<A>(), tot = zero_t<A>();
#pragma unroll
    for (int w = 0; w < MWG / 64; ++w) {
        const A x = xch[w];
        if (w >= ws0 && w < wave) pre += x;
        if (w >= ws0 && w < ws0 + segw) tot += x;
    }
    const A ex = pre + exw;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
        if (kb + r < ke) st[kb + r - t0] = (double)(ex + loc[r]);
    if ((tid & (segw * 64 - 1)) == 0) {
        const int p0 = t0 + (tid / (segw * 64)) * g.part;
        if (p0 < t1) d.is_psum[div_p2(p0, g.part)] = (double)tot;
    }
}

// part_prefix in double-fp32 (compensated FP32 mode): st[] holds fp32
// reciprocals on entry; on exit each slot holds the FF prefix (its 8 bytes),
// and is_psum the FF part sums.  Contains one barrier.
DEVI void part_prefix_ff(double *dsh, double *st, const Grid &g, const Dev &d, int kb, int ke, int t0, int t1,
                         int R)
{
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    FF loc[RMAX], s = ff_of(0.0f);
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        if (kb + r < ke) s = ff_add(s, ff_of((float)st[kb + r - t0]));
        loc[r] = s;
    }
    const int segw = (g.part / R) >> 6;
    const FF inc = wave_incl_scan(s);
    FF exw = shfl_up_t(inc, 1);
    if (lane == 0) exw = ff_of(0.0f);
    FF *xch = reinterpret_cast<FF *>(dsh);
    if (lane == 63) xch[wave] = inc;
    __syncthreads();
    const int ws0 = (wave / segw) * segw;
    FF pre = ff_of(0.0f), tot = ff_of(0.0f);
#pragma unroll
    for (int w = 0; w < MWG / 64; ++w) {
        const FF x = xch[w];
        if (w >= ws0 && w < wave) pre = ff_add(pre, x);
        if (w >= ws0 && w < ws0 + segw) tot = ff_add(tot, x);
    }
    const FF ex = ff_add(pre, exw);
    FF *stf = reinterpret_cast<FF *>(st);
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
        if (kb + r < ke) stf[kb + r - t0] = ff_add(ex, loc[r]);
    if ((tid & (segw * 64 - 1)) == 0) {
        const int p0 = t0 + (tid / (segw * 64)) * g.part;
        if (p0 < t1) reinterpret_cast<FF *>(d.is_psum)[div_p2(p0, g.part)] = tot;
    }
}

// The work of one tile (or part) of a PSD launch.
DEVI void median_work(MedianSmem &sm, const Slot *slp, int blk, int span)
{
    const Grid g = slp->g;
    const Dev d = slp->d;
    const int tid = threadIdx.x;
    const int B = g.B, W = g.W, h = g.h;
    const int t0 = blk * span;
    const int t1 = min(t0 + span, B);
    const bool whole = B < W;
    const int u0 = whole ? 0 : win_start(t0, B, W, h);
    const int u1 = whole ? B - 1 : win_start(t1 - 1, B, W, h) + W - 1;
    const int M = u1 - u0 + 1;

    // ---- load the union (all loads in flight together); tile min / max
    double xr[MCH];
#pragma unroll
    for (int i = 0; i < MCH; ++i) {
        const int p = tid + i * MWG;
        xr[i] = p < M ? d.X[u0 + p] : 0.0;
    }
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int i = 0; i < MCH; ++i) {
        const int p = tid + i * MWG;
        if (p < M) {
            sm.xv[p] = xr[i];
            const uint64_t b = (uint64_t)__double_as_longlong(xr[i]);
            mn = (b != 0 && b < mn) ? b : mn;          // smallest positive value
            mx = b > mx ? b : mx;
        }
    }
    for (int s = 32; s >= 1; s >>= 1) {
        const uint64_t a = (uint64_t)__shfl_xor((long long)mn, s, 64);
        const uint64_t b = (uint64_t)__shfl_xor((long long)mx, s, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (lane_id() == 0) {
        sm.red[tid >> 6] = mn;
        sm.red[(MWG / 64) + (tid >> 6)] = mx;
    }
    __syncthreads();
    mn = sm.red[0];
    mx = sm.red[MWG / 64];
    for (int w = 1; w < MWG / 64; ++w) {
        mn = sm.red[w] < mn ? sm.red[w] : mn;
        mx = sm.red[MWG / 64 + w] > mx ? sm.red[MWG / 64 + w] : mx;
    }
    // order key: 0 for an empty bin, 1 + (bits - smallest positive bits) >> shift
    // otherwise (X >= 0, so the fp64 bit patterns are in value order); empty
    // bins do not stretch the key range of the occupied ones
    const uint64_t vspan = mx > mn ? mx - mn : 0;
    const int span_bits = vspan ? 64 - __clzll(vspan) : 0;
    const int shift = span_bits > KEYBITS - 1 ? span_bits - (KEYBITS - 1) : 0;
    const uint32_t kmax = mx ? 1u + (uint32_t)(vspan >> shift) : 0u;
    const int passes = ((kmax ? 32 - __clz(kmax) : 0) + 3) / 4;
#pragma unroll
    for (int i = 0; i < MCH; ++i) {
        const int p = tid + i * MWG;
        if (p < M) {
            const uint64_t b = (uint64_t)__double_as_longlong(xr[i]);
            const uint32_t key = b ? 1u + (uint32_t)((b - mn) >> shift) : 0u;
            sm.kp[0][p] = (key << POSBITS) | (uint32_t)p;
        }
    }
    __syncthreads();

    // ---- sort
    int rb = radix_sort_tile(sm, M, passes);
    uint32_t *sw = sm.kp[rb];

    // ---- repair key ties: order equal keys by (fp64 value, position), by
    // odd-even transposition inside runs of equal keys.  A run needs about
    // as many rounds as its elements must travel; an outlier can stretch
    // the key range until long runs of distinct values share a key, so past
    // REPAIR_ROUNDS rounds the tile is sorted again by the KEYBITS bits below
    // the key and then stably by the key, which leaves only short runs.
    if (shift > 0) {
        bool refined = false;
        for (int round = 0;; ++round) {
            if (round == REPAIR_ROUNDS && !refined) {
                refined = true;
                const int sh2 = shift > KEYBITS ? shift - KEYBITS : 0;
                const uint64_t lmask = (1ull << (shift - sh2)) - 1ull;
                for (int p = tid; p < M; p += MWG) {
                    const uint64_t bp = (uint64_t)__double_as_longlong(sm.xv[p]);
                    const uint32_t lk = bp ? (uint32_t)(((bp - mn) >> sh2) & lmask) : 0u;
                    sm.kp[0][p] = (lk << POSBITS) | (uint32_t)p;
                }
                __syncthreads();
                const int r2 = radix_sort_tile(sm, M, (shift - sh2 + 3) / 4);
                for (int i = tid; i < M; i += MWG) {       // the key again, in the low-key order
                    const uint32_t p = sm.kp[r2][i] & 0xFFFu;
                    const uint64_t bp = (uint64_t)__double_as_longlong(sm.xv[p]);
                    const uint32_t key = bp ? 1u + (uint32_t)((bp - mn) >> shift) : 0u;
                    sm.kp[0][i] = (key << POSBITS) | p;
                }
                __syncthreads();
                rb = radix_sort_tile(sm, M, passes);
                sw = sm.kp[rb];
            }
            if (tid == 0) sm.flag = 0;
            __syncthreads();
            int swapped = 0;
            for (int par = 0; par < 2; ++par) {
                for (int i = par + 2 * tid; i + 1 < M; i += 2 * MWG) {
                    const uint32_t a = sw[i], b = sw[i + 1];
                    if ((a >> POSBITS) != (b >> POSBITS)) continue;
                    const uint32_t pa = a & 0xFFFu, pb = b & 0xFFFu;
                    const uint64_t ba = (uint64_t)__double_as_longlong(sm.xv[pa]);
                    const uint64_t bb = (uint64_t)__double_as_longlong(sm.xv[pb]);
                    if (ba > bb || (ba == bb && pa > pb)) {
                        sw[i] = b;
                        sw[i + 1] = a;
                        swapped = 1;
                    }
                }
                __syncthreads();
            }
            if (swapped) sm.flag = 1;
            __syncthreads();
            const int any = sm.flag;
            __syncthreads();
            if (!any) break;
        }
    }
    for (int i = tid; i < M; i += MWG) sm.rank[sw[i] & 0xFFFu] = (uint16_t)i;
    __syncthreads();

    const int R = (span + MWG - 1) / MWG;
    const int kb = t0 + tid * R;
    const int ke = min(kb + R, t1);
    double med[RMAX];
    if (whole) {
        const double m = sm.xv[sw[(B + 1) / 2 - 1] & 0xFFFu];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) med[r] = m;
    } else {
        // ---- wavelet matrix of the rank sequence, levels LB-1 .. WB (the
        // rank bits above the 32-rank buckets).  Element i of a level is
        // handled by thread i % MWG (chunk j = i / MWG), so a wave's ballot
        // is one 64-position word.
        constexpr int NV = MWG / 64;
        constexpr int WB = 5;                           // bucket: 2^WB consecutive ranks
        const int lane = lane_id();
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int NJ = (M + MWG - 1) / MWG;
        const int LB = M > 1 ? 32 - __clz((uint32_t)(M - 1)) : 1;
        const uint64_t below = (1ull << lane) - 1ull;
        uint16_t *src = sm.rank;
        uint16_t *dst = reinterpret_cast<uint16_t *>(sm.kp[rb ^ 1]);   // free after the sort
        uint64_t in[MCH];
#pragma unroll
        for (int j = 0; j < MCH; ++j) in[j] = __ballot(j < NJ && j * MWG + tid < M);
        for (int lvl = LB - 1; lvl >= WB; --lvl) {
            uint32_t v[MCH];
            uint64_t one[MCH];
#pragma unroll
            for (int j = 0; j < MCH; ++j) {
                const int i = j * MWG + tid;
                const bool ok = j < NJ && i < M;
                v[j] = ok ? (uint32_t)src[i] : 0u;
                one[j] = __ballot(ok && ((v[j] >> lvl) & 1u));
                if (lane == 0 && j < NJ) sm.u.wm.zc[j * NV + wave] = (uint32_t)__popcll(in[j] & ~one[j]);
            }
            __syncthreads();
            // exclusive prefix of the zero counts in element order
            const uint32_t zv = lane < NJ * NV ? sm.u.wm.zc[lane] : 0u;
            const uint32_t zinc = wave_scan_u32(zv);
            const uint32_t zex = zinc - zv;
            const uint32_t ztot = (uint32_t)__builtin_amdgcn_readlane((int)zinc, NJ * NV - 1);
#pragma unroll
            for (int j = 0; j < MCH; ++j) {
                const uint32_t zw = (uint32_t)__builtin_amdgcn_readlane((int)zex, min(j, NJ - 1) * NV + wave);
                const int i = j * MWG + tid;
                if (j < NJ && i < M) {
                    const uint32_t zb = zw + (uint32_t)__popcll(in[j] & ~one[j] & below);
                    const bool bit = (v[j] >> lvl) & 1u;
                    dst[bit ? ztot + (uint32_t)i - zb : zb] = (uint16_t)v[j];
                    if (lane == 0) {
                        WWord e;
                        e.bits = one[j];
                        e.zpre = zw;
                        e.pad = 0;
                        sm.u.wm.w[lvl][i >> 6] = e;
                    }
                }
            }
            if (tid == 0) {
                sm.u.wm.zt[lvl] = ztot;
                if ((M & 63) == 0) {
                    WWord e;
                    e.bits = 0;
                    e.zpre = ztot;
                    e.pad = 0;
                    sm.u.wm.w[lvl][M >> 6] = e;
                }
            }
            __syncthreads();
            uint16_t *tmp = src;
            src = dst;
            dst = tmp;
        }

        // ---- median of each window: the h-th smallest rank (0-based) among
        // positions [a, a + W) of the union.  A thread's first window: the
        // levels give its bucket and its index among the window's elements
        // in the bucket; the bucket's 32 sorted elements are then tested
        // against the window.  Each next window of the thread is the
        // previous one moved by one position (or the same one, at a grid
        // edge): one element leaves, one enters, and the median stays or
        // becomes the nearest element above or below it in sorted order
        // whose position lies in the new window, found by walking the
        // sorted words (at most SLIDE_MAX steps, else the levels again).
        // The sorted order is (fp64 value, position) in lexicographic
        // order, so comparisons with the median need no ranks.
        auto rank0 = [&](int lvl, int x) -> int {      // zeros among positions < x
            const WWord e = sm.u.wm.w[lvl][x >> 6];
            const uint64_t m = ~e.bits & ((1ull << (x & 63)) - 1ull);
            return (int)e.zpre + __popcll(m);
        };
        auto query = [&](int a) -> int {               // sorted index of the median of [a, a + W)
            int lo = a, hi = a + W, kk = h, base = 0;
            for (int lvl = LB - 1; lvl >= WB; --lvl) {
                const int Z = (int)sm.u.wm.zt[lvl];
                const int zl = rank0(lvl, lo), zh = rank0(lvl, hi);
                const int zeros = zh - zl;
                if (kk < zeros) {
                    lo = zl;
                    hi = zh;
                } else {
                    kk -= zeros;
                    lo = Z + lo - zl;
                    hi = Z + hi - zh;
                    base |= 1 << lvl;
                }
            }
            // base: first rank of the bucket (MMAX is a multiple of 32)
            uint32_t mask = 0;
#pragma unroll
            for (int i0 = 0; i0 < 32; i0 += 4) {
                const uint4 q4 = *reinterpret_cast<const uint4 *>(&sw[base + i0]);
                const uint32_t qq[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bool act = base + i0 + c < M && (qq[c] & 0xFFFu) - (uint32_t)a < (uint32_t)W;
                    mask |= (uint32_t)act << (i0 + c);
                }
            }
            // position of the (kk+1)-th set bit
            int pos = 0;
#pragma unroll
            for (int wdt = 16; wdt >= 1; wdt >>= 1) {
                const int c = __popc(mask & ((1u << wdt) - 1u));
                if (kk >= c) {
                    kk -= c;
                    mask >>= wdt;
                    pos += wdt;
                }
            }
            return base + pos;
        };
        // (value bits, position) of union position p before that of q
        auto before = [&](int p, int q) -> bool {
            const uint64_t bp = (uint64_t)__double_as_longlong(sm.xv[p]);
            const uint64_t bq = (uint64_t)__double_as_longlong(sm.xv[q]);
            return bp < bq || (bp == bq && p < q);
        };
        constexpr int SLIDE_MAX = 32;
        int qm[RMAX];
        int ap = kb < ke ? win_start(min(kb, ke - 1), B, W, h) - u0 : 0;
        qm[0] = query(ap);
#pragma unroll
        for (int r = 1; r < RMAX; ++r) {
            if (r >= R) break;                          // R is the same for the whole block
            const int k = min(kb + r, ke - 1);          // past the run: repeat its last window
            const int a = kb < ke ? win_start(k, B, W, h) - u0 : 0;
            int m = qm[r - 1];
            if (a != ap) {                              // a == ap + 1: ap leaves, ap + W enters
                const int pm = (int)(sw[m] & 0xFFFu);
                const int po = ap, pi = ap + W;
                int dir = 0;                            // +1: the next element above; -1: below
                if (po == pm) {
                    dir = before(pi, pm) ? -1 : 1;
                } else {
                    const bool ob = before(po, pm), ib = before(pi, pm);
                    if (ob != ib) dir = ob ? 1 : -1;
                }
                if (dir != 0) {
                    // an element on that side lies in the new window (the one
                    // that entered, or the one below or above that took the
                    // median's place), so the walk stays inside [0, M)
                    int c = m, found = -1;
                    for (int st = 0; st < SLIDE_MAX; ++st) {
                        c += dir;
                        if ((sw[c] & 0xFFFu) - (uint32_t)a < (uint32_t)W) {
                            found = c;
                            break;
                        }
                    }
                    m = found >= 0 ? found : query(a);
                }
            }
            qm[r] = m;
            ap = a;
        }
#pragma unroll
        for (int r = 0; r < RMAX; ++r) med[r] = (kb + r < ke && r < R) ? sm.xv[sw[qm[r]] & 0xFFFu] : 0.0;
    }

    // ---- S = C med + S_instr; in-tile prefix of 1/S and the tile sum.  The
    // outputs pass through LDS so that global loads and stores are coalesced.
    __syncthreads();                       // the wavelet matrix is dead: reuse it
    double *st = sm.u.stage;
    const int sc = g.prec == PREC_FP64 ? 0 : f32_scale(d.ctl->amax_bits, g.T);
    const int n = t1 - t0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
        if (kb + r < ke) st[kb + r - t0] = med[r];
    __syncthreads();
    for (int i = tid; i < n; i += MWG) {
        double Sk, inv;
        if (g.prec == PREC_FP64) {
            Sk = g.C * st[i] + d.sx[t0 + i];
            inv = 1.0 / Sk;
        } else {                           // S and 1/S in fp32, scaled by 2^sc
            const float sf = (float)g.C * (float)ldexp(st[i], sc) + (float)ldexp(d.sx[t0 + i], sc);
            Sk = ldexp((double)sf, -sc);
            inv = (double)(1.0f / sf);
        }
        d.S[t0 + i] = Sk;
        st[i] = inv;
    }
    __syncthreads();
    // prefix of 1/S restarted at every part: fp64 sums, double-fp32 sums in
    // the compensated FP32 mode, plain fp32 sums in the naive one
    if (g.prec == PREC_NAIVE)
        part_prefix<float>(sm.dsh, st, g, d, kb, ke, t0, t1, R);
    else if (g.prec == PREC_COMP)
        part_prefix_ff(sm.dsh, st, g, d, kb, ke, t0, t1, R);
    else
        part_prefix<double>(sm.dsh, st, g, d, kb, ke, t0, t1, R);
    __syncthreads();
    for (int i = tid; i < n; i += MWG) d.is_pre[t0 + i] = st[i];
}

// One block per tile, or (split mode, chosen by the previous body's SNR
// launch when few tiles are dirty) one block per part: more, shorter
// blocks; a block whose tile is clean exits.  The launch of one slot.
__global__ __launch_bounds__(MWG, 2) void k_median(const Slot *S)
{
    __shared__ MedianSmem sm;
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.est != 0) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->done || d.ctl->bad) return;
    const bool split = d.ctl->med_split != 0;
    const int span = split ? g.part : g.tile;
    const int blk = blockIdx.x;
    const int tile = split ? blk / g.np : blk;
    if (tile >= g.nt || blk * span >= g.B || d.sstamp[tile] != d.ctl->iter) return;
    median_work(sm, &sl, blk, span);
}

// Not inlined: the listed launch loops over the tiles, and the loop must
// not change the registers the work gets.
__device__ __noinline__ void median_entry(MedianSmem &sm, const Slot *slp, int blk, int span)
{
    median_work(sm, slp, blk, span);
}

__global__ __launch_bounds__(MWG, 4) void k_median_listed(const Slot *S)
{
    __shared__ MedianSmem sm;
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.est != 0) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->done || d.ctl->bad) return;
    // The launch of several slots (batches, the template model's two
    // channels): the dirty tiles come listed in tile order by the previous
    // body's tail (every tile for the first body), and a grid of at most
    // MED_GRID blocks per slot strides over the list, so the working blocks
    // are dispatched first and a slot's clean tiles cost no blocks.
    const bool split = d.ctl->med_split != 0;
    const int span = split ? g.part : g.tile;
    const uint32_t n_ent = d.ctl->n_sdl * (split ? (uint32_t)g.np : 1u);
    for (uint32_t e = blockIdx.x; e < n_ent; e += gridDim.x) {
        const int tile = (int)d.sdl[split ? e / (uint32_t)g.np : e];
        const int blk = split ? tile * g.np + (int)(e % (uint32_t)g.np) : tile;
        if (blk * span >= g.B) continue;
        median_entry(sm, &sl, blk, span);
        __syncthreads();                   // LDS is reused by the next entry
    }
}

// ------------------------------------------------------------------ running mean
//
// S[k] = (1/W) sum_{j in window(k)} (X[j] + S_instr[j])   (the mean form of the
// PSD estimate, as printed: S_instr inside the sum).  Same tiles, parts,
// dirty stamps and outputs as the median; the window sums are differences of
// an in-LDS prefix over the block's union, so no sum runs across the grid.

struct MeanSmem {
    double v[MMAX];                        // X + S_instr over the union, then its inclusive prefix
    double stage[TILE_MAX];                // outputs, for coalesced stores
    double dsh[MWG / 64];
};

// The work of one tile (or part) of a PSD launch.
DEVI void mean_work(MeanSmem &sm, const Slot *slp, int blk, int span)
{
    const Grid g = slp->g;
    const Dev d = slp->d;
    const int tid = threadIdx.x;
    const int B = g.B, W = g.W, h = g.h;
    const int t0 = blk * span;
    const int t1 = min(t0 + span, B);
    const bool whole = B < W;
    const int u0 = whole ? 0 : win_start(t0, B, W, h);
    const int u1 = whole ? B - 1 : win_start(t1 - 1, B, W, h) + W - 1;
    const int M = u1 - u0 + 1;

    for (int p = tid; p < M; p += MWG) sm.v[p] = d.X[u0 + p] + d.sx[u0 + p];
    __syncthreads();
    // inclusive prefix over the union: thread-contiguous runs
    const int ch = (M + MWG - 1) / MWG;
    const int pb = tid * ch;
    double loc[MCH], s = 0.0;
#pragma unroll
    for (int i = 0; i < MCH; ++i) {
        if (i < ch && pb + i < M) s += sm.v[pb + i];
        loc[i] = s;
    }
    double tot;
    const double ex = block_excl_scan<double, MWG>(s, sm.dsh, &tot);
#pragma unroll
    for (int i = 0; i < MCH; ++i)
        if (i < ch && pb + i < M) sm.v[pb + i] = ex + loc[i];
    __syncthreads();
    const int n = t1 - t0;
    for (int i = tid; i < n; i += MWG) {
        const int k = t0 + i;
        double sum, len;
        if (whole) {
            sum = sm.v[M - 1];
            len = (double)B;
        } else {
            const int a = win_start(k, B, W, h) - u0;
            sum = sm.v[a + W - 1] - (a > 0 ? sm.v[a - 1] : 0.0);
            len = (double)W;
        }
        const double Sk = sum / len;
        d.S[k] = Sk;
        sm.stage[i] = 1.0 / Sk;
    }
    __syncthreads();
    const int R = (span + MWG - 1) / MWG;
    const int kb = t0 + tid * R;
    const int ke = min(kb + R, t1);
    part_prefix<double>(sm.dsh, sm.stage, g, d, kb, ke, t0, t1, R);
    __syncthreads();
    for (int i = tid; i < n; i += MWG) d.is_pre[t0 + i] = sm.stage[i];
}

// One block per tile, or (split mode, chosen by the previous body's SNR
// launch when few tiles are dirty) one block per part: more, shorter
// blocks; a block whose tile is clean exits.  The launch of one slot.
__global__ __launch_bounds__(MWG) void k_mean(const Slot *S)
{
    __shared__ MeanSmem sm;
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.est != 1) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->done || d.ctl->bad) return;
    const bool split = d.ctl->med_split != 0;
    const int span = split ? g.part : g.tile;
    const int blk = blockIdx.x;
    const int tile = split ? blk / g.np : blk;
    if (tile >= g.nt || blk * span >= g.B || d.sstamp[tile] != d.ctl->iter) return;
    mean_work(sm, &sl, blk, span);
}

// Not inlined: the listed launch loops over the tiles, and the loop must
// not change the registers the work gets.
__device__ __noinline__ void mean_entry(MeanSmem &sm, const Slot *slp, int blk, int span)
{
    mean_work(sm, slp, blk, span);
}

__global__ __launch_bounds__(MWG) void k_mean_listed(const Slot *S)
{
    __shared__ MeanSmem sm;
    const Slot &sl = S[blockIdx.y];
    if (!sl.active || sl.g.est != 1) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->done || d.ctl->bad) return;
    // The launch of several slots (batches, the template model's two
    // channels): the dirty tiles come listed in tile order by the previous
    // body's tail (every tile for the first body), and a grid of at most
    // MED_GRID blocks per slot strides over the list, so the working blocks
    // are dispatched first and a slot's clean tiles cost no blocks.
    const bool split = d.ctl->med_split != 0;
    const int span = split ? g.part : g.tile;
    const uint32_t n_ent = d.ctl->n_sdl * (split ? (uint32_t)g.np : 1u);
    for (uint32_t e = blockIdx.x; e < n_ent; e += gridDim.x) {
        const int tile = (int)d.sdl[split ? e / (uint32_t)g.np : e];
        const int blk = split ? tile * g.np + (int)(e % (uint32_t)g.np) : tile;
        if (blk * span >= g.B) continue;
        mean_entry(sm, &sl, blk, span);
        __syncthreads();                   // LDS is reused by the next entry
    }
}

// ------------------------------------------------------------------ SNR, decisions, subtraction

// Sum of 1/S over bins lo..hi from the in-part prefixes of 1/S and `mid`,
// the sum of the part sums of the parts plo .. phi-1 (plo, phi: the parts
// of lo and hi); short tracks are summed bin by bin in ascending order.
DEVI double track_inv_sum(const double *v, const double *pre, int lo, int hi, int part, double mid)
{
    if (hi - lo + 1 <= NARROW) {
        double s = 0.0;
        for (int k = lo; k <= hi; ++k) s += 1.0 / v[k];
        return s;
    }
    const double below = mod_p2(lo, part) == 0 ? 0.0 : pre[lo - 1];
    if (div_p2(lo, part) == div_p2(hi, part)) return pre[hi] - below;
    return (mid - below) + pre[hi];
}

// rho^2 in fp32 (the FP32 precision modes): 4 q sum 1/S with the sum in
// fp32.  Compensated: Kahan over short tracks, and for longer ones
// double-fp32 differences of the double-fp32 in-part prefixes plus midc, the
// double-fp32 sum of the part sums in between.  Naive: plain fp32 (bin by
// bin, or the fp32 in-part prefixes and the fp32 sum `mid` of the part sums).
DEVI double snr2_f32(const Grid &g, const Dev &d, double qd, int lo, int hi, double mid, FF midc)
{
    // q and S scaled by 2^sc; the prefix tables already hold 1/(2^sc S)
    const int sc = f32_scale(d.ctl->amax_bits, g.T);
    const float q = (float)ldexp(qd, sc);
    float sum;
    if (hi - lo + 1 <= NARROW) {
        float s = 0.0f, c = 0.0f;
        for (int k = lo; k <= hi; ++k) {
            const float x = 1.0f / (float)ldexp(d.S[k], sc);
            if (g.prec == PREC_COMP) {         // Kahan
                const float y = x - c;
                const float t = s + y;
                c = (t - s) - y;
                s = t;
            } else {
                s += x;
            }
        }
        sum = s;
    } else if (g.prec == PREC_COMP) {
        const FF *pre = reinterpret_cast<const FF *>(d.is_pre);
        const FF below = mod_p2(lo, g.part) == 0 ? ff_of(0.0f) : pre[lo - 1];
        const FF top = pre[hi];
        const FF r = div_p2(lo, g.part) == div_p2(hi, g.part) ? ff_add(top, ff_neg(below))
                                                              : ff_add(ff_add(midc, ff_neg(below)), top);
        sum = ff_float(r);
    } else {
        const float below = mod_p2(lo, g.part) == 0 ? 0.0f : (float)d.is_pre[lo - 1];
        sum = div_p2(lo, g.part) == div_p2(hi, g.part) ? (float)d.is_pre[hi] - below
                                                         : ((float)mid - below) + (float)d.is_pre[hi];
    }
    return (double)((4.0f * q) * sum);
}

// Removes a resolved source's power from the exact accumulators: its one
// bin of Xn, or the two entries of the difference array D plus the carries
// into the tiles that start inside (glo, ghi + 1] (X = Xn + prefix of D,
// with the prefix split into a carry per tile and a sum inside the tile).
DEVI void subtract_track(const Grid &g, const Dev &d, int glo, int ghi, int64_t v)
{
    if (glo == ghi) {
        atomic_add_i128(&d.Xn[glo], -v);
        return;
    }
    atomic_add_i128(&d.D[glo], -v);
    if (ghi + 1 < g.B) atomic_add_i128(&d.D[ghi + 1], v);
    const int te = min(div_p2(ghi + 1, g.tile), g.nt - 1);
    for (int tl = div_p2(glo, g.tile) + 1; tl <= te; ++tl) split_sum_add(&d.Dadj[tl], -v);
}

// The same subtraction in fp32 (naive FP32 mode), vf = the power as a float:
// the fp32 difference array and its per-tile sums (k_snr_tail rescans the
// tile sums into the carries in fp32 every body).
DEVI void subtract_track_f32(const Grid &g, const Dev &d, int glo, int ghi, float vf)
{
    if (glo == ghi) {
        atomicAdd(&d.Xf[glo], -vf);
        return;
    }
    atomicAdd(&d.Df[glo], -vf);
    atomicAdd(&d.Dtf[div_p2(glo, g.tile)], -vf);
    if (ghi + 1 < g.B) {
        atomicAdd(&d.Df[ghi + 1], vf);
        atomicAdd(&d.Dtf[div_p2(ghi + 1, g.tile)], vf);
    }
}

// The same subtraction in the compensated FP32 mode (double-fp32
// accumulators, compensated atomics), vf = the power as a float.
DEVI void subtract_track_comp(const Grid &g, const Dev &d, int glo, int ghi, float vf)
{
    if (glo == ghi) {
        ff_atomic_add(&d.Xc[glo], -vf);
        return;
    }
    ff_atomic_add(&d.Dc[glo], -vf);
    ff_atomic_add(&d.Dtc[div_p2(glo, g.tile)], -vf);
    if (ghi + 1 < g.B) {
        ff_atomic_add(&d.Dc[ghi + 1], vf);
        ff_atomic_add(&d.Dtc[div_p2(ghi + 1, g.tile)], vf);
    }
}

// Stamps tiles lo/tile .. hi/tile for body `nxt` (every writer stores the
// same value, read after the launch ends; the tail counts the stamped
// tiles).


// True when S^t may differ from S^{t-1} somewhere on tiles lo/tile ..
// hi/tile: one of them was refiltered in body t (stamp t), or was stamped
// for body t + 1 by a writer of this same launch, which may have replaced a
// stamp t (every stamp is at most t + 1).  Tracks over more than SKIP_TILES
// tiles count as changed without looking.
constexpr int SKIP_TILES = 4;
DEVI bool track_refiltered(const uint32_t *stamp, const Grid &g, int lo, int hi, uint32_t t)
{
    const int a = div_p2(lo, g.tile), b = div_p2(hi, g.tile);
    if (b - a >= SKIP_TILES) return true;
    bool r = false;
    for (int tl = a; tl <= b; ++tl) {
        const uint32_t s = stamp[tl];
        r |= s == t || s == t + 1;
    }
    return r;
}

// rho^2 = 4 q sum_{k in track} 1/S^t[k] for every unsubtracted candidate
// (Eq. "SNR inner product" in the sky-averaged power form); rho^2 >
// rho_th^2 subtracts the source from the binned power at once (appendix
// "Subtraction algorithm", steps 6-9: the data X^{t+1} no longer holds it)
// and stamps the tiles the next body must convert (the track) and filter
// (every output whose window holds a bin of the track, window_reach).  A candidate whose track lies in
// tiles the median left alone this body sees the same S as at its last
// evaluation, so its stored rho^2 stands (it was not above threshold then,
// or it would have been subtracted); body 0 filters every tile.  Per-block
// counts go to b_part for the tail (snr_tail).
__global__ __launch_bounds__(WG) void k_snr(const Slot *S)
{
    constexpr int NW = WG / 64;
    __shared__ uint64_t s_red[3][NW];     // new, near, evals
    __shared__ double s_min[NW];
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Grid g = sl.g;
    const Dev d = sl.d;
    if (d.ctl->done || d.ctl->bad) return;
    const int t = (int)d.ctl->iter;
    const uint32_t nxt = (uint32_t)t + 1;
    const uint32_t nc = d.ctl->n_cand;
    const bool naive = g.prec == PREC_NAIVE;
    const bool comp = g.prec == PREC_COMP;
    const FF *psum_ff = reinterpret_cast<const FF *>(d.is_psum);
    const int lane = lane_id();
    uint32_t my_new = 0;
    uint64_t near = 0, evals = 0;
    double minm = INFINITY;
    // the wave walks its candidates together (uniform trip count), so that
    // all its lanes can sum the part sums under a wide track
    const uint32_t stride = gridDim.x * WG;
    for (uint32_t jb = blockIdx.x * WG + (threadIdx.x & ~63u); jb < nc; jb += stride) {
        const uint32_t j = jb + (uint32_t)lane;
        const bool live = j < nc && d.c_iter[j] < 0;
        int glo = 0, ghi = 0;
        bool eval = false;
        double r2 = 0.0;
        if (live) {
            glo = d.c_glo[j];
            ghi = d.c_ghi[j];
            eval = t == 0 || track_refiltered(d.sstamp, g, glo, ghi, (uint32_t)t);
            if (!eval) r2 = d.c_rho2[j];
        }
        // sum of the part sums of 1/S over the parts strictly before the
        // track's last part: a loop for tracks over a few parts, all lanes
        // of the wave together for wider ones, one track at a time
        const int plo = div_p2(glo, g.part), phi = div_p2(ghi, g.part);
        const bool need = eval && ghi - glo + 1 > NARROW && phi > plo;
        const bool wide = need && phi - plo > COOP_PARTS;
        double mid = 0.0;
        FF midc = ff_of(0.0f);
        if (need && !wide) {
            if (naive) {
                float m = 0.0f;
                for (int pp = plo; pp < phi; ++pp) m += (float)d.is_psum[pp];
                mid = (double)m;
            } else if (comp) {
                for (int pp = plo; pp < phi; ++pp) midc = ff_add(midc, psum_ff[pp]);
            } else {
                for (int pp = plo; pp < phi; ++pp) mid += d.is_psum[pp];
            }
        }
        for (uint64_t wm = (uint64_t)__ballot(wide); wm; wm &= wm - 1) {
            const int L = __builtin_ctzll(wm);
            const int a = __builtin_amdgcn_readlane(plo, L), b = __builtin_amdgcn_readlane(phi, L);
            double sum = 0.0;
            FF sumc = ff_of(0.0f);
            if (naive) {
                float m = 0.0f;
                for (int pp = a + lane; pp < b; pp += 64) m += (float)d.is_psum[pp];
                for (int o = 32; o >= 1; o >>= 1) m += __shfl_xor(m, o, 64);
                sum = (double)m;
            } else if (comp) {
                FF m = ff_of(0.0f);
                for (int pp = a + lane; pp < b; pp += 64) m = ff_add(m, psum_ff[pp]);
                for (int o = 32; o >= 1; o >>= 1) {
                    FF y;
                    y.hi = __shfl_xor(m.hi, o, 64);
                    y.lo = __shfl_xor(m.lo, o, 64);
                    m = ff_add(m, y);
                }
                sumc = m;
            } else {
                double m = 0.0;
                for (int pp = a + lane; pp < b; pp += 64) m += d.is_psum[pp];
                sum = wave_sum(m);
            }
            if (lane == L) {
                mid = sum;
                midc = sumc;
            }
        }
        if (eval) {
            ++evals;
            const double q = d.c_q[j];
            r2 = g.prec == PREC_FP64 ? (4.0 * q) * track_inv_sum(d.S, d.is_pre, glo, ghi, g.part, mid)
                                     : snr2_f32(g, d, q, glo, ghi, mid, midc);
            d.c_rho2[j] = r2;
        }
        if (!live) continue;
        const double rel = fabs(sqrt(r2) / g.rth - 1.0);
        minm = fmin(minm, rel);
        near += rel <= 1e-6;
        if (r2 > g.rth2) {
            d.c_iter[j] = t;
            ++my_new;
            const int64_t v = (int64_t)d.c_qfx[j];
            if (v) {
                const float vf = (float)ldexp((double)v, fx_exp(d.ctl->amax_bits, g.T) +
                                                             f32_scale(d.ctl->amax_bits, g.T));
                if (comp) {
                    subtract_track_comp(g, d, glo, ghi, vf);
                } else {
                    subtract_track(g, d, glo, ghi, v);
                    if (naive) subtract_track_f32(g, d, glo, ghi, vf);
                }
            }
            stamp_tiles(d.xstamp, g, glo, ghi, nxt);
            int sa, sb;
            window_reach(g, glo, ghi, &sa, &sb);
            stamp_tiles(d.sstamp, g, sa, sb, nxt);
        }
    }
    for (int s = 32; s >= 1; s >>= 1) {
        my_new += (uint32_t)__shfl_xor((int)my_new, s, 64);
        near += (uint64_t)__shfl_xor((long long)near, s, 64);
        evals += (uint64_t)__shfl_xor((long long)evals, s, 64);
        minm = fmin(minm, __shfl_xor(minm, s, 64));
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_red[0][w] = my_new;
        s_red[1][w] = near;
        s_red[2][w] = evals;
        s_min[w] = minm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) {
            d.ctl->xupd = nxt;
            d.ctl->tail_due = 1;
        }
        for (int v = 1; v < NW; ++v) {
            for (int r = 0; r < 3; ++r) s_red[r][0] += s_red[r][v];
            s_min[0] = fmin(s_min[0], s_min[v]);
        }
        SnrPart p;
        p.n_new = (uint32_t)s_red[0][0];
        p.pad = 0;
        p.near = s_red[1][0];
        p.evals = s_red[2][0];
        p.minm = s_min[0];
        d.b_part[blockIdx.x] = p;
    }
}

// The tail of a loop body, run by one block of NT threads once k_snr has
// ended: combines the per-block partials, counts the tiles stamped for the
// next body, takes the stop decision (nothing new subtracted, or max_iter)
// and whether the next median runs in split mode.  It runs at most once per
// k_snr (tail_due).
template <int NT> DEVI void snr_tail(const Slot &sl)
{
    constexpr int NW = NT / 64;
    __shared__ uint64_t s_red[5][NW];     // new, near, evals, ux, us
    __shared__ uint32_t s_nds[NW];
    __shared__ uint32_t s_wl[NW];
    __shared__ double s_min[NW];
    const Grid g = sl.g;
    const Dev d = sl.d;
    Ctl *c = d.ctl;
    if (!c->tail_due || c->done || c->bad) return;
    if (g.prec == PREC_NAIVE) block_scan_array<float, NT>(d.Dtf, d.Dcf, g.nt);
    const uint32_t nxt = c->iter + 1;
    uint64_t nw = 0, near = 0, evals = 0, ux = 0, us = 0;
    uint32_t nds = 0;
    double minm = INFINITY;
    for (int i = threadIdx.x; i < SNR_BLOCKS; i += NT) {
        const SnrPart p = d.b_part[i];
        nw += p.n_new;
        near += p.near;
        evals += p.evals;
        minm = fmin(minm, p.minm);
    }
    // stamped-tile counts, and the list of the tiles to filter in the next
    // body in tile order (per round of NT tiles: a ballot and a prefix over
    // the waves)
    uint32_t listed = 0;                  // block-uniform
    for (int base = 0; base < g.nt; base += NT) {
        const int tl = base + (int)threadIdx.x;
        bool sd = false;
        if (tl < g.nt) {
            const uint64_t width = (uint64_t)min(g.tile, g.B - tl * g.tile);
            if (d.xstamp[tl] == nxt) ux += width;
            sd = d.sstamp[tl] == nxt;
            if (sd) {
                us += width;
                ++nds;
            }
        }
        const uint64_t m = (uint64_t)__ballot(sd);
        if (lane_id() == 0) s_wl[threadIdx.x >> 6] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const uint32_t x = s_wl[v];
            pre += v < (int)(threadIdx.x >> 6) ? x : 0u;
            tot += x;
        }
        if (sd) d.sdl[listed + pre + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull))] = (uint32_t)tl;
        listed += tot;
        __syncthreads();
    }
    for (int s = 32; s >= 1; s >>= 1) {
        nw += (uint64_t)__shfl_xor((long long)nw, s, 64);
        near += (uint64_t)__shfl_xor((long long)near, s, 64);
        evals += (uint64_t)__shfl_xor((long long)evals, s, 64);
        ux += (uint64_t)__shfl_xor((long long)ux, s, 64);
        us += (uint64_t)__shfl_xor((long long)us, s, 64);
        nds += (uint32_t)__shfl_xor((int)nds, s, 64);
        minm = fmin(minm, __shfl_xor(minm, s, 64));
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_red[0][w] = nw;
        s_red[1][w] = near;
        s_red[2][w] = evals;
        s_red[3][w] = ux;
        s_red[4][w] = us;
        s_nds[w] = nds;
        s_min[w] = minm;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int v = 1; v < NW; ++v) {
        for (int r = 0; r < 5; ++r) s_red[r][0] += s_red[r][v];
        s_nds[0] += s_nds[v];
        s_min[0] = fmin(s_min[0], s_min[v]);
    }
    const int t = (int)c->iter;
    const uint32_t n_new = (uint32_t)s_red[0][0];
    c->tail_due = 0;
    c->med_split = s_nds[0] <= g.split_tiles;
    c->n_sdl = s_nds[0];
    if (t < NEW_CAP) d.n_new[t] = n_new;
    c->n_resolved += n_new;
    c->n_near += s_red[1][0];
    c->units_snr += s_red[2][0];
    if (s_min[0] < __longlong_as_double((long long)c->min_margin))
        c->min_margin = (uint64_t)__double_as_longlong(s_min[0]);
    const uint32_t mi = g.max_iter ? g.max_iter : c->n_cand + 1;
    uint32_t done = 0;
    if (n_new == 0) {
        done = 1;
        c->n_iter = (uint32_t)t + 1;
    } else if ((uint32_t)t + 1 >= mi) {
        done = 1;                    // the loop did not settle within max_iter bodies
        c->status = 6;
        c->n_iter = (uint32_t)t + 1;
    } else {
        c->iter = (uint32_t)t + 1;
        c->units_x += s_red[3][0];
        c->units_med += s_red[4][0];
    }
    c->done = done;
    // progress for the host that paces the launches: bodies finished and the
    // settled flag in one word, so that the host never sees one without the other
    if (sl.prog)
        __hip_atomic_store(sl.prog, ((uint32_t)t + 1) << 1 | done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The tail as a kernel of its own, ahead of k_xupdate: the naive FP32 mode
// rescans the fp32 tile sums into the carries that k_xupdate reads.
__global__ __launch_bounds__(SNR_BLOCKS) void k_snr_tail(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    snr_tail<SNR_BLOCKS>(sl);
}

// ------------------------------------------------------------------ outputs

// ids of the candidates (the catalog is not retained after the run).
__global__ __launch_bounds__(WG) void k_cand_ids(const Slot *S)
{
    const Slot &sl = S[blockIdx.y];
    if (!sl.active) return;
    const Dev d = sl.d;
    const uint32_t *ids = sl.ids;
    const uint32_t nc = d.ctl->n_cand;
    for (uint32_t j = blockIdx.x * WG + threadIdx.x; j < nc; j += gridDim.x * WG)
        d.c_id[j] = ids[d.c_src[j]];
}

// ------------------------------------------------------------------ launchers

hipError_t launch_grid_tables(const Slot *ds, const Dims &dm, hipStream_t st)
{
    k_sinstr<<<dim3((dm.maxB + WG - 1) / WG, dm.ns), WG, 0, st>>>(ds);
    k_inv_prefix<<<dim3(dm.maxnt, dm.ns), WG, 0, st>>>(ds);
    k_sx_scan<<<dim3(1, dm.ns), WG, 0, st>>>(ds);
    const int nseg = (dm.maxB + SEG_BINS - 1) / SEG_BINS;
    k_isx_seg<<<dim3((nseg + WG / 64 - 1) / (WG / 64), dm.ns), WG, 0, st>>>(ds);
    return hipGetLastError();
}

hipError_t launch_reset(const Slot *ds, const Dims &dm, hipStream_t st)
{
    const unsigned nb = (unsigned)((dm.maxnt + WG - 1) / WG);
    k_reset<<<dim3(nb, dm.ns), WG, 0, st>>>(ds);
    if (dm.naive) k_zero_f32<<<dim3(1024, dm.ns), WG, 0, st>>>(ds);
    return hipGetLastError();
}

hipError_t launch_prep(const Slot *ds, const Dims &dm, hipStream_t st)
{
    if (dm.prep_blocks > 0) k_prep_count<<<dim3(dm.prep_blocks, dm.ns), WG, 0, st>>>(ds);
    k_prep_colscan<<<dim3((dm.maxnt + 63) / 64, dm.ns), CS_WG, 0, st>>>(ds);
    k_prep_plan<<<dim3(1, dm.ns), WG, 0, st>>>(ds);
    if (dm.prep_blocks > 0) k_prep_scatter<<<dim3(dm.prep_blocks, dm.ns), WG, 0, st>>>(ds);
    k_accum<<<dim3(dm.accum_blocks, dm.ns), WG, 0, st>>>(ds);
    k_accum_reduce<<<dim3(dm.maxnt * (dm.maxtile / RED_BINS), dm.ns), RED_BINS, 0, st>>>(ds);
    if (dm.naive) k_accum_f32<<<dim3(2048, dm.ns), WG, 0, st>>>(ds);
    k_dscan<<<dim3(1, dm.ns), WG, 0, st>>>(ds);
    return hipGetLastError();
}

// One kernel of the loop body; with events, the dispatch itself records its
// start (ea) and end (eb), which adds no work to the stream.
hipError_t go(const void *kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t ea, hipEvent_t eb,
              const Slot *ds)
{
    void *args[] = {(void *)&ds};
    if (!ea && !eb) return hipLaunchKernel(kernel, grid, block, args, 0, st);
    return hipExtLaunchKernel(kernel, grid, block, args, 0, st, ea, eb, 0);
}

hipError_t launch_xupdate(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea, hipEvent_t eb)
{
    return go((const void *)k_xupdate, dim3(dm.maxnt + 1, dm.ns), dim3(WG), st, ea, eb, ds);
}

hipError_t launch_median(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea, hipEvent_t eb)
{
    const bool med = dm.est_mask & 1u, mean = dm.est_mask & 2u;
    hipError_t e = hipSuccess;
    // one slot: a block per part; several: the listed launch (its blocks stride
    // over each slot's dirty tiles)
    const bool listed = dm.ns > 1;
    const unsigned gx = (unsigned)(listed ? min(dm.maxparts, MED_GRID) : dm.maxparts);
    const void *km = listed ? (const void *)k_median_listed : (const void *)k_median;
    const void *kn = listed ? (const void *)k_mean_listed : (const void *)k_mean;
    if (med) e = go(km, dim3(gx, dm.ns), dim3(MWG), st, ea, mean ? nullptr : eb, ds);
    if (mean && e == hipSuccess) e = go(kn, dim3(gx, dm.ns), dim3(MWG), st, med ? nullptr : ea, eb, ds);
    return e;
}

hipError_t launch_snr(const Slot *ds, const Dims &dm, hipStream_t st, hipEvent_t ea, hipEvent_t eb)
{
    if (!dm.naive) return go((const void *)k_snr, dim3(SNR_BLOCKS, dm.ns), dim3(WG), st, ea, eb, ds);
    hipError_t e = go((const void *)k_snr, dim3(SNR_BLOCKS, dm.ns), dim3(WG), st, ea, nullptr, ds);
    if (e != hipSuccess) return e;
    return go((const void *)k_snr_tail, dim3(1, dm.ns), dim3(SNR_BLOCKS), st, nullptr, eb, ds);
}

// ------------------------------------------------------------------ coarse-graining
//
// Sec. "Coarse-graining of the data": the spectrum averaged over logarithmic
// frequency bins, and the mean frequency of each bin.  One block per bin; the
// bin is a contiguous range of grid samples, found by binary search on f_i.

__global__ __launch_bounds__(WG) void k_coarse(const double *S, const double *sx, const double *X, int kind,
                                               int64_t k0, int B, double T, CoarseEdges ed, int n_out,
                                               double *out)
{
    __shared__ double sf[WG], sv[WG];
    const int kb = blockIdx.x;
    if (kb >= n_out) return;
    auto first = [&](double x, bool strict) -> int {   // first i with f_i >= x (> x if strict)
        int lo = 0, hi = B;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const double f = (double)(k0 + mid) / T;
            if (strict ? f > x : f >= x) hi = mid; else lo = mid + 1;
        }
        return lo;
    };
    const int i0 = first(ed.e[kb], false);
    const int i1 = kb == n_out - 1 ? first(ed.e[n_out], true) : first(ed.e[kb + 1], false);
    double af = 0.0, av = 0.0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += WG) {
        af += (double)(k0 + i) / T;
        av += kind == 0 ? S[i] : kind == 1 ? X[i] : kind == 2 ? S[i] - sx[i] : sx[i];
    }
    sf[threadIdx.x] = af;
    sv[threadIdx.x] = av;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sf[threadIdx.x] += sf[threadIdx.x + w];
            sv[threadIdx.x] += sv[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[3 * kb] = sf[0];
        out[3 * kb + 1] = sv[0];
        out[3 * kb + 2] = (double)(i1 > i0 ? i1 - i0 : 0);
    }
}

hipError_t launch_coarse(const double *S, const double *sx, const double *X, int kind, int64_t k0, int B,
                         double T, const CoarseEdges &ed, int n_out, double *out, hipStream_t st)
{
    k_coarse<<<n_out, WG, 0, st>>>(S, sx, X, kind, k0, B, T, ed, n_out, out);
    return hipGetLastError();
}

hipError_t launch_outputs(const Slot *ds, const Dims &dm, hipStream_t st)
{
    k_cand_ids<<<dim3(SNR_BLOCKS, dm.ns), WG, 0, st>>>(ds);
    return hipGetLastError();
}

}  // namespace gbs
