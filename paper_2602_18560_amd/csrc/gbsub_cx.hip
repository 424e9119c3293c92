// gbsub_cx.hip -- the complex-template data model of libgbsub.
//
// The data is one complex frequency series per TDI channel, h_A and h_E (the
// T channel is insensitive: Sec. "Simulations"), holding the sum of the
// 128-sample frequency-domain templates of every source (Sec. "Simulations";
// appendix "Subtraction algorithm").  Resolved sources are scattered out of
// h at their template's bins (Eq. "vectorized-subtraction").  The template
// of a source (A, f, fdot) and its channel phases (phi_A, phi_E) is
//
//   q = floor((f + fdot T/2) T + 1/2), delta = f T - q, d = fdot T^2,
//   s_n = (A/2) exp(2 pi i (delta x + d x^2 / 2)), x = n/128,
//   U_j = (T/128) DFT_128(s)_m, m = j mod 128, j = -64 .. 63, at bin q + j - k0,
//   H_c,j = exp(i phi_c) U_j,
//
// the slowly varying factor of the signal once the carrier q/T is taken
// out, sampled 128 times over T (a fast/slow template of our own
// sky-averaged model; the paper's templates come from gbgpu).  Then per
// channel X_c = (2/T)|h_c|^2, S_c = C median_W(X_c) + S_instr (or the running
// mean), and rho^2 = (4/T) sum_j |U_j|^2 (1/S_A + 1/S_E) over the grid bins.
//
// Design for gfx950:
//  * A template is one wave's work: two samples per lane, the first radix-2
//    stage inside the lane, then two 64-point FFTs across the lanes by
//    xor-shuffles; twiddles from a 128-entry table in LDS.  Templates are
//    recomputed wherever they are needed (injection, every SNR evaluation,
//    subtraction) instead of stored (2 KB per candidate, 20 GB for 1e7
//    sources): about 350 VALU instructions of one wave per template.
//  * h is exact fixed point (int64, unit 2^-E with E from the largest
//    amplitude and the source count), so injection and subtraction are
//    order-independent integer adds and a subtracted template cancels to the
//    last bit: h always equals the sum of the (rounded) templates of the
//    sources left.
//  * Injection is binned: sources are grouped by 1024-bin tile (LDS
//    histograms, one scan, a scatter with per-block range reservations);
//    each block accumulates up to CH sources of one tile into an LDS window
//    of the tile plus the template reach on each side, then adds the window
//    to h with one global atomic per touched word.  Each wave takes 64
//    sources at a time: their constants are computed one per lane and
//    broadcast by readlane while the wave synthesises one template after
//    the other.
//  * The per-channel PSD is the power model's median (or mean) kernel, run
//    over a two-slot descriptor table (A and E), with the same dirty-tile
//    stamps; a body is X update, PSD, SNR + subtraction, and a one-block tail.

#include "gbsub_internal.h"
#include "gbsub_device.h"

#include <climits>
#include <math.h>

namespace gbs {

namespace {

constexpr int NF = CX_NF;
constexpr int HALO = NF / 2;                  // template reach on each side of its centre
constexpr int CXW = CX_TILE + NF;             // LDS window of an injection block
constexpr int SRC_PB = 4096;                  // sources per block of the count and scatter passes
constexpr int CH = 4096;                      // sources per injection block at most
constexpr int SNR_GRID = 2048;                // blocks of the SNR launch
constexpr int PLAN_T = 1024;                  // threads of the one-block plan

struct KArgs {
    Grid g;
    CxDev d;
    CxIn in;
};

__device__ __forceinline__ int lane() { return __lane_id(); }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 shfl_xor2(double2 v, int m)
{
    return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

// Sum over the wave, the same value on every lane (lane 0's).
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return __shfl(v, 0, 64);
}

// Fixed-point exponent E: every template component is at most A T / 2, so
// the sum over all n sources of |component| 2^E stays below 2^62.
__device__ __forceinline__ int cx_exp(uint32_t amax_bits, uint32_t n, double T)
{
    const double v = (double)n * (double)__uint_as_float(amax_bits) * (T * 0.5);
    if (!(v > 0.0)) return 0;
    return 61 - ilogb(v);
}

__device__ __forceinline__ long long fx(double v, int E) { return __double2ll_rn(ldexp(v, E)); }

// Central DFT index q, delta = f T - q and d = fdot T^2 (the operations of
// the definition, in this order); false if the source has no template
// (|d| >= 2^20 or |q| >= 2^52: its phases would lose their fraction).
__device__ __forceinline__ bool cx_centre(double f, double fd, double T, double *qd, double *delta, double *d)
{
    const double x = (f + (fd * T) * 0.5) * T + 0.5;
    const double dd = (fd * T) * T;
    if (!(fabs(x) < 4503599627370496.0) || !(fabs(dd) < 1048576.0)) return false;
    *qd = floor(x);
    *delta = f * T - *qd;
    *d = dd;
    return true;
}

// Twiddles tw[r] = exp(-2 pi i r / 128), set by the block's first 128 threads.
__device__ __forceinline__ void set_twiddles(double2 *tw)
{
    if (threadIdx.x < NF) {
        double s, c;
        sincospi((double)threadIdx.x / (NF / 2), &s, &c);
        tw[threadIdx.x] = make_double2(c, -s);
    }
}

// The template of one source, by the whole wave: on return lane l holds
// ue = U at m = 2 r and uo = U at m = 2 r + 1, r = bitrev6(l).  Samples n = l
// and l + 64; the first decimation-in-frequency stage (n, n + 64) inside the
// lane gives the even and odd outputs as two 64-point DFTs, each finished
// across the lanes in six stages.
__device__ __forceinline__ void wave_template(double A, double delta, double d, double T, const double2 *tw,
                                              double2 *ue, double2 *uo)
{
    const int l = lane();
    const double x0 = (double)l / NF, x1 = (double)(l + NF / 2) / NF;
    double t0 = delta * x0 + (d * 0.5) * (x0 * x0);
    double t1 = delta * x1 + (d * 0.5) * (x1 * x1);
    t0 = t0 - floor(t0);
    t1 = t1 - floor(t1);
    double s0, c0, s1, c1;
    sincospi(2.0 * t0, &s0, &c0);
    sincospi(2.0 * t1, &s1, &c1);
    const double hA = A * 0.5;
    const double2 a = make_double2(hA * c0, hA * s0), b = make_double2(hA * c1, hA * s1);
    double2 y0 = cadd(a, b);
    double2 y1 = cmul(csub(a, b), tw[l]);
    // Butterflies without branches: top lanes take v + p (twiddle 1, which
    // leaves the sum exact), bottom lanes (p - v) w; both as p + sgn v.
#pragma unroll
    for (int span = 32; span >= 4; span >>= 1) {
        const double2 p0 = shfl_xor2(y0, span), p1 = shfl_xor2(y1, span);
        const bool bottom = (l & span) != 0;
        const double sg = bottom ? -1.0 : 1.0;
        const double2 w = bottom ? tw[(l & (span - 1)) * (64 / span)] : make_double2(1.0, 0.0);
        y0 = cmul(make_double2(fma(sg, y0.x, p0.x), fma(sg, y0.y, p0.y)), w);
        y1 = cmul(make_double2(fma(sg, y1.x, p1.x), fma(sg, y1.y, p1.y)), w);
    }
    // span 2: twiddles 1 and -i (a swap and a sign); span 1: twiddle 1
    {
        const double2 p0 = shfl_xor2(y0, 2), p1 = shfl_xor2(y1, 2);
        const double sg = (l & 2) ? -1.0 : 1.0;
        const double2 d0 = make_double2(fma(sg, y0.x, p0.x), fma(sg, y0.y, p0.y));
        const double2 d1 = make_double2(fma(sg, y1.x, p1.x), fma(sg, y1.y, p1.y));
        const bool rot = (l & 3) == 3;
        y0 = rot ? make_double2(d0.y, -d0.x) : d0;
        y1 = rot ? make_double2(d1.y, -d1.x) : d1;
    }
    {
        const double2 p0 = shfl_xor2(y0, 1), p1 = shfl_xor2(y1, 1);
        const double sg = (l & 1) ? -1.0 : 1.0;
        y0 = make_double2(fma(sg, y0.x, p0.x), fma(sg, y0.y, p0.y));
        y1 = make_double2(fma(sg, y1.x, p1.x), fma(sg, y1.y, p1.y));
    }
    const double sc = T / NF;
    *ue = make_double2(y0.x * sc, y0.y * sc);
    *uo = make_double2(y1.x * sc, y1.y * sc);
}

// Template offsets j (in -64 .. 63) of a lane's two values.
__device__ __forceinline__ void lane_offsets(int *je, int *jo)
{
    const int r = (int)(__brev((unsigned)lane()) >> 26);
    const int me = 2 * r, mo = 2 * r + 1;
    *je = me < NF / 2 ? me : me - NF;
    *jo = mo < NF / 2 ? mo : mo - NF;
}

// A source's entry: valid (finite A >= 0, f > 0, finite fdot and phases).
__device__ __forceinline__ bool entry_ok(float A, float f, float fd, float pa, float pe)
{
    return isfinite(A) && A >= 0.0f && isfinite(f) && f > 0.0f && isfinite(fd) && isfinite(pa) && isfinite(pe);
}

// Grid bin of the centre, or INT_MIN when no bin of the template is on the grid.
__device__ __forceinline__ int centre_bin(const Grid &g, float f, float fd, double *delta, double *d)
{
    double qd;
    if (!cx_centre((double)f, (double)fd, g.T, &qd, delta, d)) return INT_MIN;
    const double qb = qd - (double)g.k0;
    if (qb + (HALO - 1) < 0.0 || qb - HALO > (double)(g.B - 1)) return INT_MIN;
    return (int)qb;
}

// Binning tile of a source centred at grid bin qb (clamped to the grid).
__device__ __forceinline__ int bin_tile(const Grid &g, int qb)
{
    const int k = qb < 0 ? 0 : (qb > g.B - 1 ? g.B - 1 : qb);
    return k / CX_TILE;
}

// ------------------------------------------------------------------ prep

__global__ __launch_bounds__(WG) void k_cx_reset(KArgs a)
{
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const size_t stride = (size_t)gridDim.x * WG;
    const size_t i0 = (size_t)blockIdx.x * WG + threadIdx.x;
    for (size_t k = i0; k < 4 * (size_t)g.B; k += stride) d.h[k] = 0;
    for (size_t k = i0; k <= (size_t)d.ntc; k += stride) d.tcnt[k] = 0;
    for (size_t k = i0; k < (size_t)g.nt; k += stride) {
        d.xstamp[k] = 0;
        d.sstamp[k] = 0;
        d.sdl[k] = (uint32_t)k;
    }
    if (i0 == 0) {
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
        c->units_x = (uint64_t)g.B;
        c->units_med = (uint64_t)g.B;
        c->units_snr = 0;
        c->status = 0;
        c->med_split = (uint32_t)g.nt <= g.split_tiles;
        c->n_sdl = (uint32_t)g.nt;
        c->xupd = 0;
        c->tail_due = 0;
        c->n_new_body = 0;
    }
}

__global__ __launch_bounds__(WG) void k_cx_sinstr(KArgs a)
{
    const int k = blockIdx.x * WG + threadIdx.x;
    if (k >= a.g.B) return;
    const double v = sinstr_dev((double)(a.g.k0 + k) / a.g.T, a.g.oms_pm, a.g.tm_fm, a.g.arm_m);
    a.d.sx[k] = v;
    a.d.isx[k] = 1.0 / v;
}

// Largest 1/S_instr of each 128-bin segment (one wave per segment).
__global__ __launch_bounds__(WG) void k_cx_isxmax(KArgs a)
{
    const int seg = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const int nseg = (a.g.B + NF - 1) / NF;
    if (seg >= nseg) return;
    const int k0 = seg * NF + lane(), k1 = k0 + 64;
    double m = k0 < a.g.B ? a.d.isx[k0] : 0.0;
    if (k1 < a.g.B) m = fmax(m, a.d.isx[k1]);
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane() == 0) a.d.isx_max[seg] = m;
}

// Sources per binning tile (LDS histogram per block), the largest amplitude
// of the valid entries (it sets the fixed-point unit, a function of the
// catalog's size and amplitudes only), and the validity of every entry.
__global__ __launch_bounds__(WG) void k_cx_count(KArgs a)
{
    __shared__ uint32_t hist[CX_NTC_MAX];
    __shared__ uint32_t s_amax;
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const CxIn &in = a.in;
    for (int t = threadIdx.x; t < d.ntc; t += WG) hist[t] = 0;
    if (threadIdx.x == 0) s_amax = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * (uint32_t)SRC_PB;
    uint32_t amax = 0, bad = 0;
    for (int r = 0; r < SRC_PB / WG; ++r) {
        const uint32_t i = b0 + (uint32_t)(r * WG) + threadIdx.x;
        if (i >= in.n) break;
        const float A = in.A[i], f = in.F[i], fd = in.FD[i];
        if (!entry_ok(A, f, fd, in.PA[i], in.PE[i])) {
            bad = 1;
            continue;
        }
        amax = max(amax, __float_as_uint(A));
        double delta, dd;
        const int qb = centre_bin(g, f, fd, &delta, &dd);
        if (qb == INT_MIN) continue;
        atomicAdd(&hist[bin_tile(g, qb)], 1u);
    }
    if (bad) atomicOr(&d.ctl->bad, 1u);
    atomicMax(&s_amax, amax);
    __syncthreads();
    for (int t = threadIdx.x; t < d.ntc; t += WG)
        if (hist[t]) atomicAdd(&d.tcnt[t], hist[t]);
    if (threadIdx.x == 0 && s_amax) atomicMax(&d.ctl->amax_bits, s_amax);
}

// One block: tile offsets (tcnt becomes its exclusive prefix, tcnt[ntc] the
// total), scatter cursors, and the injection chunks of each tile (cbase).
__global__ __launch_bounds__(PLAN_T) void k_cx_plan(KArgs a)
{
    __shared__ uint32_t sw[2][PLAN_T / 64];
    __shared__ uint32_t carry[2];
    const CxDev &d = a.d;
    const int ntc = d.ntc;
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    const int l = lane(), w = threadIdx.x >> 6;
    for (int base = 0; base < ntc; base += PLAN_T) {
        const int t = base + (int)threadIdx.x;
        const uint32_t cnt = t < ntc ? d.tcnt[t] : 0u;
        const uint32_t nch = (cnt + CH - 1) / CH;
        uint32_t ic = cnt, ih = nch;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t yc = (uint32_t)__shfl_up((int)ic, o, 64);
            const uint32_t yh = (uint32_t)__shfl_up((int)ih, o, 64);
            if (l >= o) {
                ic += yc;
                ih += yh;
            }
        }
        if (l == 63) {
            sw[0][w] = ic;
            sw[1][w] = ih;
        }
        __syncthreads();
        uint32_t pc = carry[0], ph = carry[1], tc = 0, th = 0;
        for (int v = 0; v < PLAN_T / 64; ++v) {
            pc += v < w ? sw[0][v] : 0u;
            ph += v < w ? sw[1][v] : 0u;
            tc += sw[0][v];
            th += sw[1][v];
        }
        if (t < ntc) {
            d.tcnt[t] = pc + ic - cnt;
            d.tcur[t] = pc + ic - cnt;
            d.cbase[t] = ph + ih - nch;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry[0] += tc;
            carry[1] += th;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.tcnt[ntc] = carry[0];
        d.cbase[ntc] = carry[1];
    }
}

// Groups the sources by binning tile: per block, an LDS count per tile, one
// global reservation of each tile's range, then LDS ranks inside it.
__global__ __launch_bounds__(WG) void k_cx_scatter(KArgs a)
{
    __shared__ uint32_t cnt[CX_NTC_MAX];
    __shared__ uint32_t rank[CX_NTC_MAX];
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const CxIn &in = a.in;
    for (int t = threadIdx.x; t < d.ntc; t += WG) {
        cnt[t] = 0;
        rank[t] = 0;
    }
    __syncthreads();
    const uint32_t b0 = blockIdx.x * (uint32_t)SRC_PB;
    int key[SRC_PB / WG];
#pragma unroll
    for (int r = 0; r < SRC_PB / WG; ++r) {
        const uint32_t i = b0 + (uint32_t)(r * WG) + threadIdx.x;
        key[r] = -1;
        if (i < in.n) {
            const float A = in.A[i], f = in.F[i], fd = in.FD[i];
            if (entry_ok(A, f, fd, in.PA[i], in.PE[i])) {
                double delta, dd;
                const int qb = centre_bin(g, f, fd, &delta, &dd);
                if (qb != INT_MIN) key[r] = bin_tile(g, qb);
            }
        }
        if (key[r] >= 0) atomicAdd(&cnt[key[r]], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < d.ntc; t += WG)
        if (cnt[t]) cnt[t] = atomicAdd(&d.tcur[t], cnt[t]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SRC_PB / WG; ++r) {
        if (key[r] < 0) continue;
        const uint32_t i = b0 + (uint32_t)(r * WG) + threadIdx.x;
        d.order[cnt[key[r]] + atomicAdd(&rank[key[r]], 1u)] = i;
    }
}

// Per-source constants of a template, one source per lane: index, centre
// bin, delta, d, A and the channel rotations (cos, sin of phi_A and phi_E).
struct SrcConsts {
    uint32_t i;
    int qb;
    double delta, d, A, ca, sa, ce, se;
};

__device__ __forceinline__ SrcConsts src_consts(const Grid &g, const CxIn &in, uint32_t i, bool rot)
{
    SrcConsts c;
    c.i = i;
    c.qb = centre_bin(g, in.F[i], in.FD[i], &c.delta, &c.d);
    c.A = (double)in.A[i];
    c.ca = c.sa = c.ce = c.se = 0.0;
    if (rot) {
        sincos((double)in.PA[i], &c.sa, &c.ca);
        sincos((double)in.PE[i], &c.se, &c.ce);
    }
    return c;
}

// Lane k's constants (k wave-uniform), on every lane.
__device__ __forceinline__ double rl(double v, int k)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ SrcConsts bcast(const SrcConsts &c, int k)
{
    SrcConsts r;
    r.i = (uint32_t)__builtin_amdgcn_readlane((int)c.i, k);
    r.qb = __builtin_amdgcn_readlane(c.qb, k);
    r.delta = rl(c.delta, k);
    r.d = rl(c.d, k);
    r.A = rl(c.A, k);
    r.ca = rl(c.ca, k);
    r.sa = rl(c.sa, k);
    r.ce = rl(c.ce, k);
    r.se = rl(c.se, k);
    return r;
}

// Injection: h += every template (both channels), and the candidate cut
// rho_0^2 = (8/T) sum_j |U_j|^2 / S_instr >= (kappa rho_th)^2.  One block per
// chunk of at most CH sources of one binning tile; each wave takes 64
// sources at a time, their constants computed one per lane, then one
// template after the other by the whole wave.
__global__ __launch_bounds__(WG) void k_cx_inject(KArgs a)
{
    __shared__ long long acc[4][CXW];
    __shared__ double2 tw[NF];
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const CxIn &in = a.in;
    const uint32_t b = blockIdx.x;
    if (b >= d.cbase[d.ntc]) return;
    // the tile of this chunk: the last t with cbase[t] <= b
    int lo = 0, hi = d.ntc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.cbase[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const int tile = lo;
    const uint32_t s0 = d.tcnt[tile] + (b - d.cbase[tile]) * (uint32_t)CH;
    const uint32_t s1 = min(s0 + (uint32_t)CH, d.tcnt[tile + 1]);
    for (int k = threadIdx.x; k < 4 * CXW; k += WG) (&acc[0][0])[k] = 0;
    set_twiddles(tw);
    __syncthreads();
    const int E = cx_exp(d.ctl->amax_bits, in.n, g.T);
    const int w0 = tile * CX_TILE - HALO;        // grid bin of acc[.][0]
    int je, jo;
    lane_offsets(&je, &jo);
    const double cut2 = g.cut2, T = g.T;
    const int wave = threadIdx.x >> 6;
    for (uint32_t base = s0 + 64u * (uint32_t)wave; base < s1; base += 64u * (WG / 64)) {
        const uint32_t s = base + (uint32_t)lane();
        const SrcConsts mine = src_consts(g, in, d.order[s < s1 ? s : s0], true);
        const int cnt = (int)min(64u, s1 - base);
        for (int k = 0; k < cnt; ++k) {
            const SrcConsts c = bcast(mine, k);
            double2 ue, uo;
            wave_template(c.A, c.delta, c.d, T, tw, &ue, &uo);
            const int be = c.qb + je, bo = c.qb + jo;
            const bool ine = be >= 0 && be < g.B, ino = bo >= 0 && bo < g.B;
            // the candidate cut: sum_j |U_j|^2 = T^2 A^2 / 4 (Parseval), so
            // rho_0^2 <= 2 T A^2 max 1/S_instr over the template's (at most
            // two) segments; below the cut by that bound, no exact sum
            const int s0 = max(c.qb - HALO, 0) / NF, s1 = min(c.qb + HALO - 1, g.B - 1) / NF;
            const double bound = 2.0 * T * (c.A * c.A) * fmax(d.isx_max[s0], d.isx_max[s1]);
            double r0 = 0.0;
            if (bound * (1.0 + 1e-9) >= cut2) {
                const double pe = ue.x * ue.x + ue.y * ue.y, po = uo.x * uo.x + uo.y * uo.y;
                r0 = (ine ? pe * d.isx[be] : 0.0) + (ino ? po * d.isx[bo] : 0.0);
                r0 = (8.0 / T) * wave_sum(r0);
            }
            if (r0 >= cut2 && lane() == 0) {
                const uint32_t slot = atomicAdd(&d.ctl->cand_cursor, 1u);
                d.c_src[slot] = c.i;
                d.c_iter[slot] = -1;
                d.c_rho2[slot] = r0;
            }
            if (ine) {
                unsigned long long *p = (unsigned long long *)&acc[0][be - w0];
                atomicAdd(p, (unsigned long long)fx(c.ca * ue.x - c.sa * ue.y, E));
                atomicAdd(p + CXW, (unsigned long long)fx(c.sa * ue.x + c.ca * ue.y, E));
                atomicAdd(p + 2 * CXW, (unsigned long long)fx(c.ce * ue.x - c.se * ue.y, E));
                atomicAdd(p + 3 * CXW, (unsigned long long)fx(c.se * ue.x + c.ce * ue.y, E));
            }
            if (ino) {
                unsigned long long *p = (unsigned long long *)&acc[0][bo - w0];
                atomicAdd(p, (unsigned long long)fx(c.ca * uo.x - c.sa * uo.y, E));
                atomicAdd(p + CXW, (unsigned long long)fx(c.sa * uo.x + c.ca * uo.y, E));
                atomicAdd(p + 2 * CXW, (unsigned long long)fx(c.ce * uo.x - c.se * uo.y, E));
                atomicAdd(p + 3 * CXW, (unsigned long long)fx(c.se * uo.x + c.ce * uo.y, E));
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < CXW; k += WG) {
        const int bin = w0 + k;
        if (bin < 0 || bin >= g.B) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const long long v = acc[c][k];
            if (v) atomicAdd((unsigned long long *)&d.h[(size_t)c * g.B + bin], (unsigned long long)v);
        }
    }
}

// ------------------------------------------------------------------ loop body

// X_c = (2/T) |h_c|^2 on the tiles stamped for this body.
__global__ __launch_bounds__(WG) void k_cx_power(KArgs a)
{
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const Ctl *c = d.ctl;
    if (c->done || c->bad) return;
    const int tile = blockIdx.x;
    if (tile >= g.nt || d.xstamp[tile] != c->iter) return;
    const int E = cx_exp(c->amax_bits, a.in.n, g.T);
    const double s2 = 2.0 / g.T;
    const int t0 = tile * g.tile, t1 = min(t0 + g.tile, g.B);
    const size_t B = (size_t)g.B;
    for (int k = t0 + (int)threadIdx.x; k < t1; k += WG) {
        const double ra = ldexp((double)d.h[k], -E), ia = ldexp((double)d.h[B + k], -E);
        const double re = ldexp((double)d.h[2 * B + k], -E), ie = ldexp((double)d.h[3 * B + k], -E);
        d.X[k] = s2 * (ra * ra + ia * ia);
        d.X[B + k] = s2 * (re * re + ie * ie);
    }
}

// rho^2 of every unsubtracted candidate whose template meets a tile
// refiltered in this body (or stamped for the next one by a subtraction of
// this launch: re-evaluating against an unchanged S gives the same value);
// rho^2 > rho_th^2 subtracts its templates from h at once and stamps the
// tiles whose X and S change.  Each wave takes 64 candidates at a time: the
// lanes find which need an evaluation and their constants, then the wave
// evaluates them one after the other.
__global__ __launch_bounds__(WG) void k_cx_snr(KArgs a)
{
    __shared__ double2 tw[NF];
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const CxIn &in = a.in;
    Ctl *c = d.ctl;
    set_twiddles(tw);
    __syncthreads();
    if (c->done || c->bad) return;
    const uint32_t t = c->iter, nxt = t + 1;
    const uint32_t nc = c->cand_cursor;
    const int E = cx_exp(c->amax_bits, in.n, g.T);
    const double T = g.T;
    const size_t B = (size_t)g.B;
    int je, jo;
    lane_offsets(&je, &jo);
    const uint32_t waves = gridDim.x * (WG / 64);
    uint32_t my_new = 0, my_near = 0, evals = 0;
    double minm = INFINITY;
    for (uint32_t base = (blockIdx.x * (WG / 64) + (threadIdx.x >> 6)) * 64u; base < nc; base += waves * 64u) {
        const uint32_t j = base + (uint32_t)lane();
        bool need = j < nc && d.c_iter[j] < 0;
        SrcConsts mine{};
        if (need) {
            mine = src_consts(g, in, d.c_src[j], false);
            if (t > 0) {
                const int lo = max(mine.qb - HALO, 0), hi = min(mine.qb + HALO - 1, g.B - 1);
                bool changed = false;
                for (int tl = div_p2(lo, g.tile); tl <= div_p2(hi, g.tile); ++tl) changed |= d.sstamp[tl] >= t;
                need = changed;
            }
        }
        uint64_t todo = (uint64_t)__ballot(need);
        while (todo) {
            const int k = (int)__builtin_ctzll(todo);
            todo &= todo - 1;
            const SrcConsts cs = bcast(mine, k);
            const uint32_t jk = base + (uint32_t)k;
            ++evals;
            double2 ue, uo;
            wave_template(cs.A, cs.delta, cs.d, T, tw, &ue, &uo);
            const int be = cs.qb + je, bo = cs.qb + jo;
            const bool ine = be >= 0 && be < g.B, ino = bo >= 0 && bo < g.B;
            const double pe = ue.x * ue.x + ue.y * ue.y, po = uo.x * uo.x + uo.y * uo.y;
            double r = 0.0;
            if (ine) {
                const double sA = d.S[be], sE = d.S[B + be];
                r += pe * ((sA + sE) / (sA * sE));
            }
            if (ino) {
                const double sA = d.S[bo], sE = d.S[B + bo];
                r += po * ((sA + sE) / (sA * sE));
            }
            const double r2 = (4.0 / T) * wave_sum(r);
            const double rel = fabs(sqrt(r2) / g.rth - 1.0);
            minm = fmin(minm, rel);
            my_near += rel <= 1e-6;
            if (lane() == 0) d.c_rho2[jk] = r2;
            if (!(r2 > g.rth2)) continue;
            ++my_new;
            if (lane() == 0) d.c_iter[jk] = (int32_t)t;
            double sa, ca, se, ce;
            sincos((double)in.PA[cs.i], &sa, &ca);
            sincos((double)in.PE[cs.i], &se, &ce);
            if (ine) {
                unsigned long long *p = (unsigned long long *)&d.h[be];
                atomicAdd(p, (unsigned long long)-fx(ca * ue.x - sa * ue.y, E));
                atomicAdd(p + B, (unsigned long long)-fx(sa * ue.x + ca * ue.y, E));
                atomicAdd(p + 2 * B, (unsigned long long)-fx(ce * ue.x - se * ue.y, E));
                atomicAdd(p + 3 * B, (unsigned long long)-fx(se * ue.x + ce * ue.y, E));
            }
            if (ino) {
                unsigned long long *p = (unsigned long long *)&d.h[bo];
                atomicAdd(p, (unsigned long long)-fx(ca * uo.x - sa * uo.y, E));
                atomicAdd(p + B, (unsigned long long)-fx(sa * uo.x + ca * uo.y, E));
                atomicAdd(p + 2 * B, (unsigned long long)-fx(ce * uo.x - se * uo.y, E));
                atomicAdd(p + 3 * B, (unsigned long long)-fx(se * uo.x + ce * uo.y, E));
            }
            if (lane() == 0) {
                const int lo = max(cs.qb - HALO, 0), hi = min(cs.qb + HALO - 1, g.B - 1);
                stamp_tiles(d.xstamp, g, lo, hi, nxt);
                int sa_, sb_;
                window_reach(g, lo, hi, &sa_, &sb_);
                stamp_tiles(d.sstamp, g, sa_, sb_, nxt);
            }
        }
    }
    if (lane() == 0) {
        if (my_new) atomicAdd(&c->n_new_body, my_new);
        if (my_near) atomicAdd((unsigned long long *)&c->n_near, (unsigned long long)my_near);
        if (evals) atomicAdd((unsigned long long *)&c->units_snr, (unsigned long long)evals);
        if (minm < INFINITY)
            atomicMin((unsigned long long *)&c->min_margin, (unsigned long long)__double_as_longlong(minm));
    }
}

// The body's end (one block): the stop decision, the split mode of the next
// median launch, and the progress word for the host.
__global__ __launch_bounds__(WG) void k_cx_tail(KArgs a)
{
    __shared__ uint32_t s_nds[WG / 64];
    const Grid &g = a.g;
    const CxDev &d = a.d;
    Ctl *c = d.ctl;
    if (c->done) return;
    __shared__ uint32_t s_wl[WG / 64];
    const uint32_t t = c->iter, nxt = t + 1;
    uint32_t nds = 0;
    uint64_t units = 0;
    // the tiles the next PSD launch filters, listed in tile order
    uint32_t listed = 0;
    for (int base = 0; base < g.nt; base += WG) {
        const int tl = base + (int)threadIdx.x;
        bool sd = false;
        if (tl < g.nt) {
            sd = d.sstamp[tl] == nxt;
            nds += sd;
            if (d.xstamp[tl] == nxt) units += (uint64_t)min(g.tile, g.B - tl * g.tile);
        }
        const uint64_t m = (uint64_t)__ballot(sd);
        if (lane() == 0) s_wl[threadIdx.x >> 6] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int v = 0; v < WG / 64; ++v) {
            pre += v < (int)(threadIdx.x >> 6) ? s_wl[v] : 0u;
            tot += s_wl[v];
        }
        if (sd) d.sdl[listed + pre + (uint32_t)__popcll(m & ((1ull << lane()) - 1ull))] = (uint32_t)tl;
        listed += tot;
        __syncthreads();
    }
    for (int o = 32; o >= 1; o >>= 1) {
        nds += (uint32_t)__shfl_xor((int)nds, o, 64);
        units += (uint64_t)__shfl_xor((long long)units, o, 64);
    }
    __shared__ uint64_t s_units[WG / 64];
    if (lane() == 0) {
        s_nds[threadIdx.x >> 6] = nds;
        s_units[threadIdx.x >> 6] = units;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t done = 0;
    if (c->bad) {
        done = 1;
        c->n_iter = t;
    } else {
        for (int v = 1; v < WG / 64; ++v) {
            s_nds[0] += s_nds[v];
            s_units[0] += s_units[v];
        }
        const uint32_t n_new = c->n_new_body;
        c->n_new_body = 0;
        c->n_resolved += n_new;
        const uint32_t mi = g.max_iter ? g.max_iter : c->cand_cursor + 1;
        if (n_new == 0) {
            done = 1;
            c->n_iter = nxt;
        } else if (nxt >= mi) {
            done = 1;
            c->status = 6;
            c->n_iter = nxt;
        } else {
            c->iter = nxt;
            c->med_split = s_nds[0] <= g.split_tiles;
            c->n_sdl = s_nds[0];
            c->units_x += s_units[0];
            c->units_med += s_units[0];
        }
    }
    c->n_cand = c->cand_cursor;
    c->done = done;
    if (a.in.prog)
        __hip_atomic_store(a.in.prog, (nxt << 1) | done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------ outputs

__global__ __launch_bounds__(WG) void k_cx_ids(KArgs a)
{
    const CxDev &d = a.d;
    const uint32_t nc = d.ctl->cand_cursor;
    for (uint32_t j = blockIdx.x * WG + threadIdx.x; j < nc; j += gridDim.x * WG)
        d.c_id[j] = a.in.ids[d.c_src[j]];
}

__global__ __launch_bounds__(WG) void k_cx_hout(KArgs a, int ch, double *out)
{
    const CxDev &d = a.d;
    const size_t B = (size_t)a.g.B;
    const int E = cx_exp(d.ctl->amax_bits, a.in.n, a.g.T);
    const int64_t *re = d.h + (size_t)(2 * ch) * B, *im = re + B;
    for (size_t k = (size_t)blockIdx.x * WG + threadIdx.x; k < B; k += (size_t)gridDim.x * WG) {
        out[2 * k] = ldexp((double)re[k], -E);
        out[2 * k + 1] = ldexp((double)im[k], -E);
    }
}

// Templates of n sources (one wave each): q (INT64_MIN if none) and U in
// offset order j = -64 .. 63.
__global__ __launch_bounds__(WG) void k_cx_templates(Grid g, const float *A, const float *F, const float *FD,
                                                     uint32_t n, int64_t *q, double *U)
{
    __shared__ double2 tw[NF];
    set_twiddles(tw);
    __syncthreads();
    int je, jo;
    lane_offsets(&je, &jo);
    const uint32_t waves = gridDim.x * (WG / 64);
    for (uint32_t i = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); i < n; i += waves) {
        double qd, delta, dd;
        const bool ok = cx_centre((double)F[i], (double)FD[i], g.T, &qd, &delta, &dd);
        double2 ue = make_double2(0.0, 0.0), uo = ue;
        if (ok) wave_template((double)A[i], delta, dd, g.T, tw, &ue, &uo);
        if (lane() == 0) q[i] = ok ? (int64_t)qd : INT64_MIN;
        double *u = U + (size_t)i * 2 * NF;
        u[2 * (je + HALO)] = ue.x;
        u[2 * (je + HALO) + 1] = ue.y;
        u[2 * (jo + HALO)] = uo.x;
        u[2 * (jo + HALO) + 1] = uo.y;
    }
}

KArgs args_of(const Grid &g, const CxDev &d, const CxIn &in) { return KArgs{g, d, in}; }

}  // namespace

uint64_t cx_carve(const Grid &g, uint64_t n, char *base, CxDev *out)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = (off + (bytes ? bytes : 1) + 255) & ~uint64_t(255);
        return p;
    };
    const uint64_t B = (uint64_t)g.B, nt = (uint64_t)g.nt, nn = n ? n : 1;
    CxDev d{};
    d.ntc = (int32_t)((B + CX_TILE - 1) / CX_TILE);
    d.slots = (Slot *)take(2 * sizeof(Slot));
    d.ctl = (Ctl *)take(sizeof(Ctl));
    d.sx = (double *)take(B * 8);
    d.isx = (double *)take(B * 8);
    d.isx_max = (double *)take(((B + CX_NF - 1) / CX_NF) * 8);
    d.X = (double *)take(2 * B * 8);
    d.S = (double *)take(2 * B * 8);
    d.is_pre = (double *)take(2 * B * 8);
    d.is_psum = (double *)take(2 * (uint64_t)g.nparts * 8);
    d.h = (int64_t *)take(4 * B * 8);
    d.xstamp = (uint32_t *)take(nt * 4);
    d.sstamp = (uint32_t *)take(nt * 4);
    d.sdl = (uint32_t *)take(nt * 4);
    d.tcnt = (uint32_t *)take(((uint64_t)d.ntc + 1) * 4);
    d.tcur = (uint32_t *)take((uint64_t)d.ntc * 4);
    d.cbase = (uint32_t *)take(((uint64_t)d.ntc + 1) * 4);
    d.order = (uint32_t *)take(nn * 4);
    d.c_src = (uint32_t *)take(nn * 4);
    d.c_iter = (int32_t *)take(nn * 4);
    d.c_id = (uint32_t *)take(nn * 4);
    d.c_rho2 = (double *)take(nn * 8);
    d.rs_hist = (uint32_t *)take(resolved_scratch_words(nn) * 4);
    d.kA = (uint32_t *)take(nn * 4);
    d.vA = (int32_t *)take(nn * 4);
    d.kB = (uint32_t *)take(nn * 4);
    d.vB = (int32_t *)take(nn * 4);
    if (out) *out = d;
    return off;
}

hipError_t cx_launch_prep(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st)
{
    const KArgs a = args_of(g, d, in);
    k_cx_reset<<<1024, WG, 0, st>>>(a);
    k_cx_sinstr<<<(g.B + WG - 1) / WG, WG, 0, st>>>(a);
    const int nseg = (g.B + NF - 1) / NF;
    k_cx_isxmax<<<(nseg + WG / 64 - 1) / (WG / 64), WG, 0, st>>>(a);
    const uint32_t nb = (in.n + SRC_PB - 1) / SRC_PB;
    if (nb) k_cx_count<<<nb, WG, 0, st>>>(a);
    k_cx_plan<<<1, PLAN_T, 0, st>>>(a);
    if (nb) k_cx_scatter<<<nb, WG, 0, st>>>(a);
    // chunks: at most one partial chunk per tile beyond n / CH full ones
    const uint32_t chunks = in.n / CH + (uint32_t)d.ntc;
    if (in.n) k_cx_inject<<<chunks, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t cx_launch_power(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st)
{
    k_cx_power<<<g.nt, WG, 0, st>>>(args_of(g, d, in));
    return hipGetLastError();
}

hipError_t cx_launch_psd(const Grid &g, const CxDev &d, hipStream_t st, hipEvent_t ea, hipEvent_t eb)
{
    Dims dm{};
    dm.ns = 2;
    dm.maxB = g.B;
    dm.maxnt = g.nt;
    dm.maxtile = g.tile;
    dm.maxparts = g.nparts;
    dm.est_mask = 1u << g.est;
    return launch_median(d.slots, dm, st, ea, eb);
}

hipError_t cx_launch_snr(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st)
{
    const KArgs a = args_of(g, d, in);
    k_cx_snr<<<SNR_GRID, WG, 0, st>>>(a);
    k_cx_tail<<<1, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t cx_launch_outputs(const Grid &g, const CxDev &d, const CxIn &in, hipStream_t st)
{
    k_cx_ids<<<256, WG, 0, st>>>(args_of(g, d, in));
    return hipGetLastError();
}

hipError_t cx_launch_h(const Grid &g, const CxDev &d, uint32_t n, int ch, double *out, hipStream_t st)
{
    CxIn in{};
    in.n = n;
    k_cx_hout<<<1024, WG, 0, st>>>(args_of(g, d, in), ch, out);
    return hipGetLastError();
}

hipError_t cx_launch_templates(const Grid &g, const float *A, const float *F, const float *FD, uint32_t n,
                               int64_t *q, double *U, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint32_t blocks = min((n + WG / 64 - 1) / (WG / 64), 4096u);
    k_cx_templates<<<blocks, WG, 0, st>>>(g, A, F, FD, n, q, U);
    return hipGetLastError();
}

}  // namespace gbs
