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
//    stage inside the lane, then two 64-point FFTs across the lanes.  The
//    exchanges run on the VALU, not through the LDS crossbar: row swaps
//    (v_permlane32_swap, v_permlane16_swap) of the two FFTs' registers for
//    spans 32 and 16, after which each lane computes whole butterflies, and
//    DPP moves for spans 8 .. 1 (the lanes hold their positions permuted so
//    that span 4 is one half-row mirror).  exp(2 pi i t) is a 16-entry LDS
//    table (one bank row: no conflicts) times short Taylor polynomials;
//    twiddles and signs are lane constants in registers.  Templates are
//    recomputed wherever they are needed (injection, every SNR evaluation,
//    subtraction) instead of stored (2 KB per candidate, 20 GB for 1e7
//    sources): about 240 VALU instructions of one wave per template.
//  * h is exact fixed point (int64, unit 2^-E with E from the largest
//    amplitude and the source count), so injection and subtraction are
//    order-independent integer adds and a subtracted template cancels to the
//    last bit: h always equals the sum of the (rounded) templates of the
//    sources left.
//  * Injection is binned: sources are grouped by 1024-bin tile (LDS
//    histograms, one scan, a scatter with per-block range reservations);
//    each block accumulates up to CH sources of one tile into an LDS window
//    of the tile plus the template reach on each side (even and odd bins
//    apart: the lanes of one atomic add hit pairs of neighbouring words), then
//    adds the window to h with one global atomic per touched word.  Each
//    wave takes an equal share of the chunk, 64 sources at a time: their
//    constants are computed one per lane and broadcast by readlane while
//    the wave synthesises one template after the other.
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
constexpr int CH = 8192;                      // sources per injection block at most
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
// Exchanges between lanes without the LDS crossbar.
//  * Row swaps (gfx950): v_permlane32_swap(P, Q) leaves P = [P lanes 0-31,
//    Q lanes 0-31] and Q = [P lanes 32-63, Q lanes 32-63];
//    v_permlane16_swap(P, Q) does the same on rows of 16 lanes, P = [P row 0,
//    Q row 0, P row 2, Q row 2] and Q = [P row 1, Q row 1, P row 3, Q row 3].
//  * DPP moves within rows of 16 lanes: lane l reads lane l ^ 8 (row rotate
//    by 8), l ^ 7 (half-row mirror), l ^ 2 and l ^ 1 (quad permutes).
template <int SPAN> __device__ __forceinline__ void row_swap(double *P, double *Q)
{
    static_assert(SPAN == 32 || SPAN == 16, "row-swap spans");
    const long long bp = __double_as_longlong(*P), bq = __double_as_longlong(*Q);
    const unsigned plo = (unsigned)(bp & 0xffffffffll), phi = (unsigned)(bp >> 32);
    const unsigned qlo = (unsigned)(bq & 0xffffffffll), qhi = (unsigned)(bq >> 32);
    unsigned p0, q0, p1, q1;
    if constexpr (SPAN == 32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(plo, qlo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(phi, qhi, false, false);
        p0 = rl[0]; q0 = rl[1]; p1 = rh[0]; q1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(plo, qlo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(phi, qhi, false, false);
        p0 = rl[0]; q0 = rl[1]; p1 = rh[0]; q1 = rh[1];
    }
    *P = __longlong_as_double(((long long)p1 << 32) | p0);
    *Q = __longlong_as_double(((long long)q1 << 32) | q0);
}

// DPP patterns: 8 = l ^ 8, 7 = l ^ 7, 2 = l ^ 2, 1 = l ^ 1.  Every lane of
// the wave is active and every source lane is in range: the moves need no
// old value (bound_ctrl).
template <int PAT> __device__ __forceinline__ int dpp_move(int v)
{
    static_assert(PAT == 8 || PAT == 7 || PAT == 2 || PAT == 1, "DPP patterns");
    if constexpr (PAT == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, true);   // row_ror:8
    else if constexpr (PAT == 7) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, true); // row_half_mirror
    else if constexpr (PAT == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, true);  // quad_perm [2,3,0,1]
    else return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, true);                        // quad_perm [1,0,3,2]
}

template <int PAT> __device__ __forceinline__ double partner(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_move<PAT>((int)(b & 0xffffffffll)), hi = dpp_move<PAT>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int PAT> __device__ __forceinline__ double2 partner2(double2 v)
{
    return make_double2(partner<PAT>(v.x), partner<PAT>(v.y));
}

// Sum over the wave, the same value on every lane: a butterfly over lane
// pairs that differ in bit 5, bit 4, bit 3, bits 0-2, bit 1 and bit 0 (both
// lanes of a pair add the same two values).
__device__ __forceinline__ double wave_sum(double v)
{
    double w = v;
    row_swap<32>(&v, &w);
    v += w;
    w = v;
    row_swap<16>(&v, &w);
    v += w;
    v += partner<8>(v);
    v += partner<7>(v);
    v += partner<2>(v);
    v += partner<1>(v);
    return v;
}

// Fixed-point exponent E: every template component is at most A T / 2, so
// with m = max(n, 4096) sources the sum of the n components of one word
// stays below 2^62 and a single component below 2^50 (which the rounding
// of fxm needs).
__device__ __forceinline__ int cx_exp(uint32_t amax_bits, uint32_t n, double T)
{
    const double v = (double)max(n, 4096u) * (double)__uint_as_float(amax_bits) * (T * 0.5);
    if (!(v > 0.0)) return 0;
    return 61 - ilogb(v);
}

// v (already in units of 2^-E, |v| < 2^51) rounded to the nearest integer,
// ties to even: v + 1.5 2^52 lies in [2^52, 2^53), where the spacing of
// doubles is 1, so the addition rounds v and its low mantissa bits hold the
// integer plus 2^51.
__device__ __forceinline__ long long fxm(double v)
{
    return __double_as_longlong(v + 6755399441055744.0) - 0x4338000000000000ll;
}

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

constexpr int NEX = 16;                        // entries of the exp(2 pi i k / NEX) table

// ex[k] = exp(2 pi i k / 16), set by the block's first threads.  The 16
// entries fill one row of LDS banks: the lanes of a wave read them without
// bank conflicts.
__device__ __forceinline__ void set_cis_table(double2 *ex)
{
    if (threadIdx.x < NEX) {
        double s, c;
        sincospi((double)threadIdx.x / (NEX / 2), &s, &c);
        ex[threadIdx.x] = make_double2(c, s);
    }
}

// exp(2 pi i t) for |t| < 2^26 turns: t = k/16 + r with k = rint(16 t) and
// |r| <= 1/32 (both exact), the table entry of k mod 16 times the Taylor
// polynomials of cos and sin at x = 2 pi r (|x| <= pi/16; the first omitted
// terms are below 2e-19).
__device__ __forceinline__ double2 cis_turns(double t, const double2 *ex)
{
    const double kd = rint(t * (double)NEX);
    const double r = fma(kd, -1.0 / NEX, t);
    const double2 e = ex[(int)kd & (NEX - 1)];
    const double x = r * 6.283185307179586;
    const double z = x * x;
    double c = fma(z, 1.0 / 479001600.0, -1.0 / 3628800.0);
    c = fma(z, c, 1.0 / 40320.0);
    c = fma(z, c, -1.0 / 720.0);
    c = fma(z, c, 1.0 / 24.0);
    c = fma(z, c, -0.5);
    c = fma(z, c, 1.0);
    double p = fma(z, -1.0 / 39916800.0, 1.0 / 362880.0);
    p = fma(z, p, -1.0 / 5040.0);
    p = fma(z, p, 1.0 / 120.0);
    p = fma(z, p, -1.0 / 6.0);
    const double sn = fma(x * z, p, x);
    return make_double2(fma(c, e.x, -(sn * e.y)), fma(c, e.y, sn * e.x));
}

__device__ __forceinline__ double2 cmulf(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}

// The wave FFT.  Lane l holds the samples n = ell and ell + 64, where ell is
// l with its low three bits b mapped to b ^ 3 when b >= 4 (an involution):
// then the lanes that hold the positions ell and ell ^ 4 are l and l ^ 7,
// one DPP move apart, while positions ell ^ 8, ell ^ 2 and ell ^ 1 stay at
// l ^ 8, l ^ 2 and l ^ 1.
__device__ __forceinline__ int lane_pos(int l) { return l ^ ((l & 4) ? 3 : 0); }

// A lane's constants: its sample times x = n/128 with their squares, the
// twiddles of the in-lane stage (128 points), of the two row-swap stages
// (64 and 32 points, full butterflies in every lane) and of the spans 8
// and 4 (1 on the lane of the pair's first element), and the signs of the
// spans 8 .. 1 (+1 on the first element's lane, -1 on the other).
struct LaneFft {
    double x0, x0q, x1, x1q;
    double2 w1, wa, wb, w8, w4;
    double sg8, sg4, sg2, sg1;
};

__device__ __forceinline__ double2 twiddle(int m)   // exp(-2 pi i m / 128)
{
    double s, c;
    sincospi((double)m / (NF / 2), &s, &c);
    return make_double2(c, -s);
}

__device__ __forceinline__ LaneFft lane_fft()
{
    LaneFft L;
    const int e = lane_pos(lane()), u = e & 15;
    L.x0 = (double)e / NF;
    L.x1 = (double)(e + NF / 2) / NF;
    L.x0q = L.x0 * L.x0;
    L.x1q = L.x1 * L.x1;
    L.w1 = twiddle(e);                       // W_128^e
    L.wa = twiddle(2 * (e & 31));            // W_64^(e mod 32)
    L.wb = twiddle(4 * u);                   // W_32^(e mod 16)
    L.w8 = (u & 8) ? twiddle(8 * (u & 7)) : make_double2(1.0, 0.0);    // W_16
    L.w4 = (u & 4) ? twiddle(16 * (u & 3)) : make_double2(1.0, 0.0);   // W_8
    L.sg8 = (u & 8) ? -1.0 : 1.0;
    L.sg4 = (u & 4) ? -1.0 : 1.0;
    L.sg2 = (u & 2) ? -1.0 : 1.0;
    L.sg1 = (u & 1) ? -1.0 : 1.0;
    return L;
}

// Per-source constants of a template: index, centre bin, the phase
// delta x + dh x^2 in turns (dh = d/2), the scale sc = (A/2) (T/128) 2^E of
// the samples, and the channel rotations exp(i phi_A) = (ca, sa) and
// exp(i phi_E) = (ce, se); need: the template may reach the candidate cut
// (injection).
struct SrcConsts {
    uint32_t i;
    int qb;
    int need;
    double delta, dh, sc, ca, sa, ce, se;
};

// The template of one source, by the whole wave: on return each lane holds
// two values of 2^E U (U itself when sc = (A/2)(T/128)), at the offsets
// lane_offsets gives.  The phase is the definition's operations in their
// order (delta x, (d/2) x^2, their sum), so it is the same double as in a
// plain evaluation.  Decimation in frequency: the first stage (n, n + 64)
// inside the lane gives the even and odd outputs as two 64-point DFTs a and
// b (registers P = a, Q = b).  The spans 32 and 16 are row swaps of P with
// Q, after which every lane holds both elements of one butterfly (of a or
// of b) and computes both outputs; the spans 8 .. 1 exchange within each
// register (the partner's value p and the own v give p + sg v, times the
// twiddle, so the first lane gets the sum and the second the difference).
__device__ __forceinline__ void wave_template(const SrcConsts &c, const LaneFft &L, const double2 *ex,
                                              double2 *ue, double2 *uo)
{
    const double2 e0 = cis_turns(c.delta * L.x0 + c.dh * L.x0q, ex);
    const double2 e1 = cis_turns(c.delta * L.x1 + c.dh * L.x1q, ex);
    const double2 a = make_double2(c.sc * e0.x, c.sc * e0.y), b = make_double2(c.sc * e1.x, c.sc * e1.y);
    double2 P = cadd(a, b);
    double2 Q = cmulf(csub(a, b), L.w1);
    // span 32, then 16: full butterflies (twiddle 1 on the sum)
    row_swap<32>(&P.x, &Q.x);
    row_swap<32>(&P.y, &Q.y);
    {
        const double2 t = cadd(P, Q);
        Q = cmulf(csub(P, Q), L.wa);
        P = t;
    }
    row_swap<16>(&P.x, &Q.x);
    row_swap<16>(&P.y, &Q.y);
    {
        const double2 t = cadd(P, Q);
        Q = cmulf(csub(P, Q), L.wb);
        P = t;
    }
    // spans 8 and 4 (the latter between lanes l and l ^ 7)
    {
        const double2 p0 = partner2<8>(P), p1 = partner2<8>(Q);
        const double sg = L.sg8;
        P = cmulf(make_double2(fma(sg, P.x, p0.x), fma(sg, P.y, p0.y)), L.w8);
        Q = cmulf(make_double2(fma(sg, Q.x, p1.x), fma(sg, Q.y, p1.y)), L.w8);
    }
    {
        const double2 p0 = partner2<7>(P), p1 = partner2<7>(Q);
        const double sg = L.sg4;
        P = cmulf(make_double2(fma(sg, P.x, p0.x), fma(sg, P.y, p0.y)), L.w4);
        Q = cmulf(make_double2(fma(sg, Q.x, p1.x), fma(sg, Q.y, p1.y)), L.w4);
    }
    // span 2: twiddles 1 and -i (a swap and a sign); span 1: twiddle 1
    {
        const double2 p0 = partner2<2>(P), p1 = partner2<2>(Q);
        const double sg = L.sg2;
        const double2 d0 = make_double2(fma(sg, P.x, p0.x), fma(sg, P.y, p0.y));
        const double2 d1 = make_double2(fma(sg, Q.x, p1.x), fma(sg, Q.y, p1.y));
        const bool rot = (lane_pos(lane()) & 3) == 3;
        P = rot ? make_double2(d0.y, -d0.x) : d0;
        Q = rot ? make_double2(d1.y, -d1.x) : d1;
    }
    {
        const double2 p0 = partner2<1>(P), p1 = partner2<1>(Q);
        const double sg = L.sg1;
        *ue = make_double2(fma(sg, P.x, p0.x), fma(sg, P.y, p0.y));
        *uo = make_double2(fma(sg, Q.x, p1.x), fma(sg, Q.y, p1.y));
    }
}

// The value of a channel with rotation (c, s) = exp(i phi_c): exp(i phi_c) v.
__device__ __forceinline__ double2 rot(double2 v, double c, double s)
{
    return cmulf(v, make_double2(c, s));
}

// Template offsets j (in -64 .. 63) of a lane's two values.  After the
// FFT, register P of lane l (row r = l / 16) holds DFT a (rows 0, 1) or b
// (rows 2, 3) at position i = 32 (r mod 2) + (ell mod 16), and Q the same DFT
// at i + 16; position i of a 64-point decimation-in-frequency output is
// frequency bitrev6(i), and a and b are the even and odd outputs.
__device__ __forceinline__ void lane_offsets(int *je, int *jo)
{
    const int l = lane(), r = l >> 4;
    const int ip = 32 * (r & 1) + (lane_pos(l) & 15), iq = ip + 16;
    const int odd = r >= 2 ? 1 : 0;
    const int mp = 2 * (int)(__brev((unsigned)ip) >> 26) + odd, mq = 2 * (int)(__brev((unsigned)iq) >> 26) + odd;
    *je = mp < NF / 2 ? mp : mp - NF;
    *jo = mq < NF / 2 ? mq : mq - NF;
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

// The channel rotations of source i.
__device__ __forceinline__ void rotations(const CxIn &in, uint32_t i, SrcConsts *c)
{
    sincos((double)in.PA[i], &c->sa, &c->ca);
    sincos((double)in.PE[i], &c->se, &c->ce);
}

// The constants of source i (one source per lane) with fixed-point
// exponent E; the channel rotations only when rot.
__device__ __forceinline__ SrcConsts src_consts(const Grid &g, const CxIn &in, uint32_t i, int E, bool rot)
{
    SrcConsts c;
    double d;
    c.i = i;
    c.need = 1;
    c.qb = centre_bin(g, in.F[i], in.FD[i], &c.delta, &d);
    c.dh = d * 0.5;
    c.sc = ldexp(((double)in.A[i] * 0.5) * (g.T / NF), E);
    c.ca = c.sa = c.ce = c.se = 0.0;
    if (rot) rotations(in, i, &c);
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
    r.need = __builtin_amdgcn_readlane(c.need, k);
    r.delta = rl(c.delta, k);
    r.dh = rl(c.dh, k);
    r.sc = rl(c.sc, k);
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
    // per channel word, the window's even bins then its odd bins (w0 is
    // even): the lanes of one atomic add hit pairs of neighbouring words
    __shared__ long long acc[4][2][CXW / 2];
    __shared__ double2 ex[NEX];
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
    for (int k = threadIdx.x; k < 4 * CXW; k += WG) (&acc[0][0][0])[k] = 0;
    set_cis_table(ex);
    const LaneFft L = lane_fft();
    __syncthreads();
    const int E = cx_exp(d.ctl->amax_bits, in.n, g.T);
    const int w0 = tile * CX_TILE - HALO;        // grid bin of the window's first bin
    int je, jo;
    lane_offsets(&je, &jo);
    const double cut2 = g.cut2, T = g.T;
    // rho_0^2 of the 2^E-scaled values: (8/T) 2^-2E sum
    const double r0s = ldexp(8.0 / T, -2 * E);
    // each wave takes an equal share of the chunk, 64 sources at a time
    const uint32_t wave = threadIdx.x >> 6, share = (s1 - s0 + WG / 64 - 1) / (WG / 64);
    const uint32_t v0 = s0 + wave * share, v1 = min(v0 + share, s1);
    for (uint32_t base = v0; base < v1; base += 64u) {
        const uint32_t s = base + (uint32_t)lane();
        SrcConsts mine = src_consts(g, in, d.order[s < v1 ? s : v0], E, true);
        {
            // the candidate cut: sum_j |U_j|^2 = T^2 A^2 / 4 (Parseval), so
            // rho_0^2 <= 2 T A^2 max 1/S_instr over the template's (at most
            // two) segments; below the cut by that bound, no exact sum
            const double A = (double)in.A[mine.i];
            const int g0 = max(mine.qb - HALO, 0) / NF, g1 = min(mine.qb + HALO - 1, g.B - 1) / NF;
            const double bound = 2.0 * T * (A * A) * fmax(d.isx_max[g0], d.isx_max[g1]);
            mine.need = bound * (1.0 + 1e-9) >= cut2;
        }
        // the candidate cut and the template's values into the window
        auto add = [&](const SrcConsts &c, const double2 &ue, const double2 &uo) {
            const int be = c.qb + je, bo = c.qb + jo;
            const bool ine = be >= 0 && be < g.B, ino = bo >= 0 && bo < g.B;
            if (c.need) {
                const double pe = ue.x * ue.x + ue.y * ue.y, po = uo.x * uo.x + uo.y * uo.y;
                double r = (ine ? pe * d.isx[be] : 0.0) + (ino ? po * d.isx[bo] : 0.0);
                const double r0 = r0s * wave_sum(r);
                if (r0 >= cut2 && lane() == 0) {
                    const uint32_t slot = atomicAdd(&d.ctl->cand_cursor, 1u);
                    d.c_src[slot] = c.i;
                    d.c_iter[slot] = -1;
                    d.c_rho2[slot] = r0;
                    d.c_qb[slot] = c.qb;
                }
            }
            if (ine) {
                const double2 va = rot(ue, c.ca, c.sa), ve = rot(ue, c.ce, c.se);
                unsigned long long *p = (unsigned long long *)&acc[0][(be - w0) & 1][(be - w0) >> 1];
                atomicAdd(p, (unsigned long long)fxm(va.x));
                atomicAdd(p + CXW, (unsigned long long)fxm(va.y));
                atomicAdd(p + 2 * CXW, (unsigned long long)fxm(ve.x));
                atomicAdd(p + 3 * CXW, (unsigned long long)fxm(ve.y));
            }
            if (ino) {
                const double2 va = rot(uo, c.ca, c.sa), ve = rot(uo, c.ce, c.se);
                unsigned long long *p = (unsigned long long *)&acc[0][(bo - w0) & 1][(bo - w0) >> 1];
                atomicAdd(p, (unsigned long long)fxm(va.x));
                atomicAdd(p + CXW, (unsigned long long)fxm(va.y));
                atomicAdd(p + 2 * CXW, (unsigned long long)fxm(ve.x));
                atomicAdd(p + 3 * CXW, (unsigned long long)fxm(ve.y));
            }
        };
        const int cnt = (int)min(64u, v1 - base);
        for (int k = 0; k < cnt; ++k) {
            const SrcConsts c = bcast(mine, k);
            double2 ue, uo;
            wave_template(c, L, ex, &ue, &uo);
            add(c, ue, uo);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < CXW; k += WG) {
        const int bin = w0 + k;
        if (bin < 0 || bin >= g.B) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const long long v = acc[c][k & 1][k >> 1];
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
    __shared__ double2 ex[NEX];
    const Grid &g = a.g;
    const CxDev &d = a.d;
    const CxIn &in = a.in;
    Ctl *c = d.ctl;
    set_cis_table(ex);
    __syncthreads();
    if (c->done || c->bad) return;
    const uint32_t t = c->iter, nxt = t + 1;
    const uint32_t nc = c->cand_cursor;
    const int E = cx_exp(c->amax_bits, in.n, g.T);
    const double T = g.T;
    // rho^2 of the 2^E-scaled values: (4/T) 2^-2E sum
    const double rs = ldexp(4.0 / T, -2 * E);
    const size_t B = (size_t)g.B;
    int je, jo;
    lane_offsets(&je, &jo);
    const uint32_t waves = gridDim.x * (WG / 64);
    uint32_t my_new = 0, my_near = 0, evals = 0;
    double minm = INFINITY;
    for (uint32_t base = (blockIdx.x * (WG / 64) + (threadIdx.x >> 6)) * 64u; base < nc; base += waves * 64u) {
        const uint32_t j = base + (uint32_t)lane();
        bool need = j < nc && d.c_iter[j] < 0;
        if (need && t > 0) {
            const int qb = d.c_qb[j];
            const int lo = max(qb - HALO, 0), hi = min(qb + HALO - 1, g.B - 1);
            bool changed = false;
            for (int tl = div_p2(lo, g.tile); tl <= div_p2(hi, g.tile); ++tl) changed |= d.sstamp[tl] >= t;
            need = changed;
        }
        // the constants only of the candidates evaluated
        SrcConsts mine{};
        if (need) mine = src_consts(g, in, d.c_src[j], E, false);
        uint64_t todo = (uint64_t)__ballot(need);
        if (!todo) continue;
        // the FFT's lane constants only for waves with evaluations (in late
        // bodies most have none)
        const LaneFft L = lane_fft();
        while (todo) {
            const int k = (int)__builtin_ctzll(todo);
            todo &= todo - 1;
            const SrcConsts cs = bcast(mine, k);
            const uint32_t jk = base + (uint32_t)k;
            ++evals;
            const int be = cs.qb + je, bo = cs.qb + jo;
            const bool ine = be >= 0 && be < g.B, ino = bo >= 0 && bo < g.B;
            // the PSD under the template, loaded before the synthesis hides
            // their latency (off-grid lanes read bin 0 and drop it)
            const int bec = ine ? be : 0, boc = ino ? bo : 0;
            const double sAe = d.S[bec], sEe = d.S[B + bec], sAo = d.S[boc], sEo = d.S[B + boc];
            double2 ue, uo;
            wave_template(cs, L, ex, &ue, &uo);
            const double pe = ue.x * ue.x + ue.y * ue.y, po = uo.x * uo.x + uo.y * uo.y;
            double r = 0.0;
            if (ine) r += pe * ((sAe + sEe) / (sAe * sEe));
            if (ino) r += po * ((sAo + sEo) / (sAo * sEo));
            const double r2 = rs * wave_sum(r);
            const double rel = fabs(sqrt(r2) / g.rth - 1.0);
            minm = fmin(minm, rel);
            my_near += rel <= 1e-6;
            if (lane() == 0) d.c_rho2[jk] = r2;
            if (!(r2 > g.rth2)) continue;
            ++my_new;
            if (lane() == 0) d.c_iter[jk] = (int32_t)t;
            SrcConsts rc;
            rotations(in, cs.i, &rc);
            if (ine) {
                const double2 va = rot(ue, rc.ca, rc.sa), ve = rot(ue, rc.ce, rc.se);
                unsigned long long *p = (unsigned long long *)&d.h[be];
                atomicAdd(p, (unsigned long long)-fxm(va.x));
                atomicAdd(p + B, (unsigned long long)-fxm(va.y));
                atomicAdd(p + 2 * B, (unsigned long long)-fxm(ve.x));
                atomicAdd(p + 3 * B, (unsigned long long)-fxm(ve.y));
            }
            if (ino) {
                const double2 va = rot(uo, rc.ca, rc.sa), ve = rot(uo, rc.ce, rc.se);
                unsigned long long *p = (unsigned long long *)&d.h[bo];
                atomicAdd(p, (unsigned long long)-fxm(va.x));
                atomicAdd(p + B, (unsigned long long)-fxm(va.y));
                atomicAdd(p + 2 * B, (unsigned long long)-fxm(ve.x));
                atomicAdd(p + 3 * B, (unsigned long long)-fxm(ve.y));
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
    __shared__ double2 ex[NEX];
    set_cis_table(ex);
    const LaneFft L = lane_fft();
    __syncthreads();
    int je, jo;
    lane_offsets(&je, &jo);
    const uint32_t waves = gridDim.x * (WG / 64);
    for (uint32_t i = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); i < n; i += waves) {
        double qd, dd;
        SrcConsts c{};
        const bool ok = cx_centre((double)F[i], (double)FD[i], g.T, &qd, &c.delta, &dd);
        double2 ue = make_double2(0.0, 0.0), uo = ue;
        if (ok) {
            c.dh = dd * 0.5;
            c.sc = ((double)A[i] * 0.5) * (g.T / NF);
            wave_template(c, L, ex, &ue, &uo);
        }
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
    d.c_qb = (int32_t *)take(nn * 4);
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
