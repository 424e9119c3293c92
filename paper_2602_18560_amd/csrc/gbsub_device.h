// gbsub_device.h -- device helpers shared by the kernel files of libgbsub
// (grid tables, windows and dirty-tile stamps); not part of the public ABI.
#pragma once

#include "gbsub_internal.h"

namespace gbs {

#ifndef DEVI
#define DEVI __device__ __forceinline__
#endif

// x / p and x % p for x >= 0 and p a power of two (tile and part sizes).
DEVI int div_p2(int x, int p) { return x >> __builtin_ctz((unsigned)p); }
DEVI int mod_p2(int x, int p) { return x & (p - 1); }

// Window start of output k (clamped full window), grid of B >= W bins.
DEVI int win_start(int k, int B, int W, int h)
{
    int a = k - h;
    a = a < 0 ? 0 : a;
    return a > B - W ? B - W : a;
}

// Strain-equivalent SciRDv1 A-channel noise: S_AA(f) / R_AA(f) with
//   P_OMS = (P pm)^2 [1 + (2 mHz/f)^4] (2 pi f/c)^2,
//   P_TM  = (A fm)^2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4] (2 pi f)^-4 (2 pi f/c)^2,
//   S_AA  = 8 sin^2 u {4 [1 + cos u + cos^2 u] P_TM + [2 + cos u] P_OMS},
//   R_AA  = 16 sin^2 u u^2 (9/20) / (1 + 0.7 u^2),  u = f/f*, f* = c/(2 pi L)
// (appendices "LISA instrumental noise" and "Characteristic strain").
DEVI double sinstr_dev(double f, double oms_pm, double tm_fm, double arm_m)
{
    const double c = 299792458.0;
    const double two_pi = 6.283185307179586;
    const double u = f / (c / (two_pi * arm_m));
    const double w = two_pi * f;
    const double wc = w / c;
    const double oms = oms_pm * 1e-12, tm = tm_fm * 1e-15;
    const double a = 2e-3 / f, b = 4e-4 / f, e = f / 8e-3;
    const double p_oms = (oms * oms) * (1.0 + a * a * a * a) * (wc * wc);
    const double p_tm = (tm * tm) * (1.0 + b * b) * (1.0 + e * e * e * e) / (w * w * w * w) * (wc * wc);
    double s, co;
    sincos(u, &s, &co);
    const double saa = 8.0 * (s * s) * (4.0 * (1.0 + co + co * co) * p_tm + (2.0 + co) * p_oms);
    const double raa = 16.0 * (s * s) * (u * u) * (0.45 / (1.0 + 0.7 * (u * u)));
    return saa / raa;
}

DEVI void stamp_tiles(uint32_t *stamp, const Grid &g, int lo, int hi, uint32_t nxt)
{
    for (int tl = div_p2(lo, g.tile); tl <= div_p2(hi, g.tile); ++tl) stamp[tl] = nxt;
}

// Outputs whose window holds a bin of [lo, hi] (Eq. "running median" with the
// window shifted inward at the grid edges): [lo - h, hi + h] in the interior;
// every output of the lower edge (window [0, W-1]) once lo <= W-1, every
// output of the upper edge (window [B-W, B-1]) once hi >= B-W, and the whole
// grid when it is shorter than the window.
DEVI void window_reach(const Grid &g, int lo, int hi, int *a, int *b)
{
    const bool whole = g.B < g.W;
    *a = (whole || lo <= g.W - 1) ? 0 : lo - g.h;
    *b = (whole || hi >= g.B - g.W) ? g.B - 1 : hi + g.h;
}

}  // namespace gbs
