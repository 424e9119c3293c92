// gbsub_api.hip -- host runtime and C ABI of libgbsub (see include/gbsub.h).
//
// The runtime validates the configuration, carves the caller's workspace,
// enqueues the kernels of gbsub_kernels.hip and drives the loop: loop bodies
// are enqueued in growing chunks without waiting, every kernel of a body
// exits at once after the device-side "settled" flag is set, and the host
// reads the 64-byte control block once per chunk.

#include "gbsub_internal.h"
#include "gbsub.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace gbs;

struct gbsub_ctx {
    gbsub_config cfg;
    Grid g;
    int device;
    // results of the last successful run
    bool have_result;
    Dev dev;
    void *ws;
    gbsub_summary summ;
    uint32_t n_cand;
    // the S_instr tables in `tables_ws` were computed for this grid
    void *tables_ws;
    Ctl *host_ctl;     // pinned
    // profiling
    bool profiling;
    struct Rec { int kid; int64_t t; hipEvent_t a, b; };
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<Rec> recs;
    uint64_t k_launches[K_COUNT];
    double k_ms[K_COUNT];
    double k_units[K_COUNT];

    hipEvent_t next_event()
    {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }

    // Launches through `fn`, bracketed by events when profiling.
    template <typename F>
    hipError_t timed(int kid, int64_t t, hipStream_t st, F fn)
    {
        if (!profiling) return fn();
        hipEvent_t a = next_event(), b = next_event();
        if (!a || !b) return hipErrorOutOfMemory;
        hipError_t e = hipEventRecord(a, st);
        if (e == hipSuccess) e = fn();
        if (e == hipSuccess) e = hipEventRecord(b, st);
        recs.push_back({kid, t, a, b});
        return e;
    }

    void clear_stats()
    {
        for (int k = 0; k < K_COUNT; ++k) {
            k_launches[k] = 0;
            k_ms[k] = 0.0;
            k_units[k] = 0.0;
        }
    }
};

namespace {

constexpr double C_LIGHT = 299792458.0;

uint64_t align_up(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Lays the workspace out; with base == nullptr only the size is computed.
uint64_t carve(const Grid &g, uint64_t n, char *base, Dev *d)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + (bytes ? bytes : 1));
        return p;
    };
    const uint64_t B = (uint64_t)g.B, nt = (uint64_t)g.nt, nn = n ? n : 1;
    const uint64_t max_events = 2 * n;
    const uint64_t ev_chunks = (max_events + ACC_EV - 1) / ACC_EV;
    Dev t{};
    t.max_chunks = (uint32_t)(ev_chunks + nt);
    t.max_slots = (uint32_t)(2 * ev_chunks + 2);
    t.sx = (double *)take(B * 8);
    t.isx_pre = (double *)take(B * 8);
    t.isx_tsum = (double *)take(nt * 8);
    t.isx_tile = (double *)take((nt + 1) * 8);
    t.Xn = (I128 *)take(B * 16);
    t.D = (I128 *)take((B + 1) * 16);
    t.Dtile = (I128 *)take((nt + 1) * 16);
    t.Dcarry = (I128 *)take((nt + 1) * 16);
    t.X = (double *)take(B * 8);
    t.S = (double *)take(B * 8);
    t.is_pre = (double *)take(B * 8);
    t.is_tsum = (double *)take(nt * 8);
    t.is_tile = (double *)take((nt + 1) * 8);
    t.chgx = (int32_t *)take((nt + 1) * 4);
    t.chgs = (int32_t *)take((nt + 1) * 4);
    t.xdirty = (uint8_t *)take(align_up(nt));
    t.sdirty = (uint8_t *)take(align_up(nt));
    t.btot = (uint32_t *)take(nt * 4);
    t.bbase = (uint32_t *)take((nt + 1) * 4);
    t.cursor = (uint32_t *)take(nt * 4);
    t.nch = (uint32_t *)take(nt * 4);
    t.chunk_base = (uint32_t *)take((nt + 1) * 4);
    t.slot_base = (uint32_t *)take(nt * 4);
    t.ev_key = (uint32_t *)take((max_events ? max_events : 1) * 4);
    t.ev_val = (int64_t *)take((max_events ? max_events : 1) * 8);
    t.partial = (I128 *)take((uint64_t)t.max_slots * 2 * (uint64_t)g.tile * 16);
    t.amax_part = (uint32_t *)take((uint64_t)AMAX_BLOCKS * 4);
    t.c_src = (uint32_t *)take(nn * 4);
    t.c_id = (uint32_t *)take(nn * 4);
    t.c_glo = (int32_t *)take(nn * 4);
    t.c_ghi = (int32_t *)take(nn * 4);
    t.c_iter = (int32_t *)take(nn * 4);
    t.c_q = (double *)take(nn * 8);
    t.c_qfx = (uint64_t *)take(nn * 8);
    t.c_rho2 = (double *)take(nn * 8);
    t.b_new = (uint32_t *)take((uint64_t)SNR_BLOCKS * 4);
    t.b_near = (uint64_t *)take((uint64_t)SNR_BLOCKS * 8);
    t.b_evals = (uint64_t *)take((uint64_t)SNR_BLOCKS * 8);
    t.b_minm = (double *)take((uint64_t)SNR_BLOCKS * 8);
    t.n_new = (uint32_t *)take((uint64_t)NEW_CAP * 4);
    t.ctl = (Ctl *)take(sizeof(Ctl));
    if (d) *d = t;
    return off;
}

gbsub_status dev_err(hipError_t e) { return e == hipSuccess ? GBSUB_OK : GBSUB_E_DEVICE; }

gbsub_status validate(const gbsub_config *c, Grid *g)
{
    if (!c) return GBSUB_E_INVALID;
    if (!(c->t_obs_s > 0.0) || !std::isfinite(c->t_obs_s) || !(c->f_min_hz > 0.0) ||
        !(c->f_max_hz > c->f_min_hz) || !std::isfinite(c->f_max_hz))
        return GBSUB_E_INVALID;
    if (!(c->arm_m > 0.0) || !(c->f_max_hz < C_LIGHT / (2.0 * c->arm_m))) return GBSUB_E_INVALID;
    if (c->window_bins < 1 || (c->window_bins % 2) == 0 || c->window_bins > (uint32_t)(MMAX - WG + 1))
        return GBSUB_E_INVALID;
    if (c->estimator != GBSUB_MEDIAN) return GBSUB_E_INVALID;
    if (c->track_model > GBSUB_TRACK_SINGLE) return GBSUB_E_INVALID;
    if (c->precision != GBSUB_FP64) return GBSUB_E_INVALID;
    if (!(c->snr_threshold > 0.0) || !(c->kappa >= 0.0) || !(c->median_scale >= 0.0) ||
        !std::isfinite(c->snr_threshold) || !std::isfinite(c->kappa) || !std::isfinite(c->median_scale))
        return GBSUB_E_INVALID;
    if (!(c->oms_pm > 0.0) || !(c->tm_fm > 0.0)) return GBSUB_E_INVALID;
    const double a = std::floor(c->f_min_hz * c->t_obs_s + 0.5);
    const double b = std::floor(c->f_max_hz * c->t_obs_s + 0.5);
    if (!(b - a + 1.0 >= 1.0) || b - a + 1.0 > 268435456.0 || a > 9.0e15) return GBSUB_E_INVALID;
    Grid r{};
    r.k0 = (int64_t)a;
    r.B = (int32_t)((int64_t)b - (int64_t)a + 1);
    r.W = (int32_t)c->window_bins;
    r.h = (r.W - 1) / 2;
    // tile: outputs + W - 1 must fit the median kernel's LDS union
    int tile = ((MMAX - (r.W - 1)) / WG) * WG;
    if (tile > TILE_MAX) tile = TILE_MAX;
    if (tile < WG) return GBSUB_E_INVALID;
    r.tile = tile;
    r.nt = (r.B + tile - 1) / tile;
    if (r.nt > NBK_MAX) return GBSUB_E_INVALID;
    r.track_single = c->track_model == GBSUB_TRACK_SINGLE;
    r.T = c->t_obs_s;
    r.C = c->median_scale;
    r.rth = c->snr_threshold;
    r.rth2 = c->snr_threshold * c->snr_threshold;
    const double cut = c->kappa * c->snr_threshold;
    r.cut2 = cut * cut;
    r.oms_pm = c->oms_pm;
    r.tm_fm = c->tm_fm;
    r.arm_m = c->arm_m;
    *g = r;
    return GBSUB_OK;
}

}  // namespace

extern "C" {

void gbsub_default_config(gbsub_config *c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->t_obs_s = 4.0 * 31557600.0;
    c->f_min_hz = 1e-4;
    c->f_max_hz = 3e-2;
    c->window_bins = 1001;
    c->estimator = GBSUB_MEDIAN;
    c->snr_threshold = 7.0;
    c->kappa = 1.0 / 7.0;
    c->median_scale = 729.0 / 512.0;
    c->track_model = GBSUB_TRACK_SWEEP;
    c->precision = GBSUB_FP64;
    c->max_iter = 0;
    c->oms_pm = 15.0;
    c->tm_fm = 3.0;
    c->arm_m = 2.5e9;
}

const char *gbsub_status_str(gbsub_status s)
{
    switch (s) {
    case GBSUB_OK: return "ok";
    case GBSUB_E_INVALID: return "invalid argument";
    case GBSUB_E_NOMEM: return "out of memory";
    case GBSUB_E_DEVICE: return "device error";
    case GBSUB_E_STATE: return "bad call order";
    case GBSUB_E_TRUNCATED: return "output truncated";
    case GBSUB_E_MAXITER: return "iteration limit reached";
    }
    return "unknown status";
}

gbsub_status gbsub_create(const gbsub_config *cfg, gbsub_ctx **out)
{
    if (!out) return GBSUB_E_INVALID;
    *out = nullptr;
    Grid g;
    gbsub_status st = validate(cfg, &g);
    if (st != GBSUB_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GBSUB_E_DEVICE;
    gbsub_ctx *c = new (std::nothrow) gbsub_ctx();
    if (!c) return GBSUB_E_NOMEM;
    c->cfg = *cfg;
    c->g = g;
    c->device = dev;
    c->have_result = false;
    c->ws = nullptr;
    c->tables_ws = nullptr;
    c->host_ctl = nullptr;
    c->profiling = false;
    c->ev_used = 0;
    c->clear_stats();
    if (hipHostMalloc((void **)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return GBSUB_E_DEVICE;
    }
    *out = c;
    return GBSUB_OK;
}

void gbsub_destroy(gbsub_ctx *c)
{
    if (!c) return;
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

gbsub_status gbsub_workspace_size(const gbsub_ctx *c, uint64_t n, uint64_t *bytes)
{
    if (!c || !bytes || n >= (1ull << 31)) return GBSUB_E_INVALID;
    *bytes = carve(c->g, n, nullptr, nullptr);
    return GBSUB_OK;
}

gbsub_status gbsub_run(gbsub_ctx *c, const gbsub_catalog *cat, void *ws, uint64_t ws_bytes,
                       void *stream, gbsub_summary *out)
{
    if (!c || !cat || !ws) return GBSUB_E_INVALID;
    if (cat->n >= (1ull << 31)) return GBSUB_E_INVALID;
    if (cat->n > 0 && (!cat->A || !cat->f || !cat->fdot || !cat->id)) return GBSUB_E_INVALID;
    if (((uintptr_t)ws & 255u) != 0) return GBSUB_E_INVALID;
    const uint64_t need = carve(c->g, cat->n, nullptr, nullptr);
    if (ws_bytes < need) return GBSUB_E_INVALID;
    c->have_result = false;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return GBSUB_E_DEVICE;
    if (cur != c->device && hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    Dev d;
    carve(c->g, cat->n, (char *)ws, &d);
    const Grid &g = c->g;

    c->ev_used = 0;
    c->recs.clear();
    hipError_t e = hipSuccess;
    if (c->tables_ws != ws) {
        e = c->timed(K_TABLES, -1, st, [&] { return launch_grid_tables(g, d, st); });
        if (e != hipSuccess) return GBSUB_E_DEVICE;
        c->tables_ws = ws;
    }
    e = c->timed(K_RESET, -1, st, [&] { return launch_reset(g, d, cat->n, st); });
    if (e == hipSuccess)
        e = c->timed(K_PREP, -1, st, [&] { return launch_prep(g, d, cat->A, cat->f, cat->fdot, cat->n, st); });
    if (e == hipSuccess) e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        c->tables_ws = nullptr;
        return GBSUB_E_DEVICE;
    }
    if (c->host_ctl->bad) return GBSUB_E_INVALID;
    const uint64_t n_cand = c->host_ctl->n_cand;
    const uint64_t max_iter = c->cfg.max_iter ? c->cfg.max_iter : n_cand + 1;

    gbsub_status status = GBSUB_OK;
    uint64_t t = 0;
    uint64_t chunk = 4;
    for (;;) {
        const uint64_t k = std::min(chunk, max_iter - t);
        for (uint64_t i = 0; i < k && e == hipSuccess; ++i) {
            const int ti = (int)(t + i);
            e = c->timed(K_XUPDATE, ti, st, [&] { return launch_xupdate(g, d, st); });
            if (e == hipSuccess) e = c->timed(K_MEDIAN, ti, st, [&] { return launch_median(g, d, st); });
            if (e == hipSuccess) e = c->timed(K_SNR, ti, st, [&] { return launch_snr(g, d, ti, st); });
        }
        t += k;
        if (e == hipSuccess) e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return GBSUB_E_DEVICE;
        if (c->host_ctl->done) break;
        if (t >= max_iter) {
            status = GBSUB_E_MAXITER;
            break;
        }
        chunk = std::min<uint64_t>(chunk * 2, 32);
    }
    e = c->timed(K_OUTPUT, -1, st, [&] { return launch_outputs(g, d, cat->id, st); });
    if (e == hipSuccess) e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return GBSUB_E_DEVICE;

    const Ctl &h = *c->host_ctl;
    if (c->profiling) {
        const int64_t n_body = status == GBSUB_OK ? (int64_t)h.n_iter : (int64_t)t;
        for (const auto &r : c->recs) {
            if (r.t >= n_body) continue;        // bodies enqueued past the settled one
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GBSUB_E_DEVICE;
            c->k_ms[r.kid] += ms;
            c->k_launches[r.kid] += 1;
        }
        c->k_units[K_PREP] += (double)cat->n;
        c->k_units[K_RESET] += (double)g.B;
        c->k_units[K_XUPDATE] += (double)h.units_x;
        c->k_units[K_MEDIAN] += (double)h.units_med;
        c->k_units[K_SNR] += (double)h.units_snr;
        c->k_units[K_OUTPUT] += (double)h.n_cand;
        for (const auto &r : c->recs)
            if (r.kid == K_TABLES) c->k_units[K_TABLES] += (double)g.B;
    }
    gbsub_summary s{};
    s.n_iter = status == GBSUB_OK ? h.n_iter : (uint32_t)t;
    s.n_bins = (uint64_t)g.B;
    s.n_candidates = h.n_cand;
    s.n_resolved = h.n_resolved;
    s.n_near_threshold = h.n_near;
    double mm;
    std::memcpy(&mm, &h.min_margin, 8);
    s.min_rel_margin = mm;
    if (out) *out = s;
    if (status != GBSUB_OK) return status;
    c->summ = s;
    c->dev = d;
    c->ws = ws;
    c->n_cand = h.n_cand;
    c->have_result = true;
    return GBSUB_OK;
}

gbsub_status gbsub_spectrum(const gbsub_ctx *c, uint32_t kind, double *out, uint64_t cap,
                            uint64_t *n_bins, int out_on_device)
{
    if (!c || !n_bins) return GBSUB_E_INVALID;
    if (!c->have_result) return GBSUB_E_STATE;
    const uint64_t B = (uint64_t)c->g.B;
    *n_bins = B;
    if (kind > GBSUB_SPEC_S_INSTR) return GBSUB_E_INVALID;
    if (cap < B) return GBSUB_E_TRUNCATED;
    if (!out) return GBSUB_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const double *src = kind == GBSUB_SPEC_SN ? c->dev.S
                      : kind == GBSUB_SPEC_X_RESIDUAL ? c->dev.X
                      : kind == GBSUB_SPEC_S_INSTR ? c->dev.sx : c->dev.S;
    if (kind != GBSUB_SPEC_S_GAL) {
        return dev_err(hipMemcpy(out, src, B * 8,
                                 out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
    std::vector<double> s(B), x(B);
    hipError_t e = hipMemcpy(s.data(), c->dev.S, B * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(x.data(), c->dev.sx, B * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    for (uint64_t k = 0; k < B; ++k) s[k] -= x[k];
    return dev_err(hipMemcpy(out, s.data(), B * 8,
                             out_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
}

gbsub_status gbsub_resolved(const gbsub_ctx *c, uint32_t *ids, int32_t *iter_of, uint64_t cap,
                            uint64_t *n, int out_on_device)
{
    if (!c || !n) return GBSUB_E_INVALID;
    if (!c->have_result) return GBSUB_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const uint64_t nc = c->n_cand;
    std::vector<uint32_t> id(nc);
    std::vector<int32_t> it(nc);
    hipError_t e = hipSuccess;
    if (nc) {
        e = hipMemcpy(id.data(), c->dev.c_id, nc * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(it.data(), c->dev.c_iter, nc * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return GBSUB_E_DEVICE;
    }
    std::vector<uint64_t> key;
    key.reserve(c->summ.n_resolved);
    for (uint64_t j = 0; j < nc; ++j)
        if (it[j] >= 0) key.push_back(((uint64_t)id[j] << 32) | (uint32_t)it[j]);
    std::sort(key.begin(), key.end());
    const uint64_t m = key.size();
    *n = m;
    if (cap < m) return GBSUB_E_TRUNCATED;
    if (m == 0) return GBSUB_OK;
    if (!ids) return GBSUB_E_INVALID;
    id.resize(m);
    it.resize(m);
    for (uint64_t j = 0; j < m; ++j) {
        id[j] = (uint32_t)(key[j] >> 32);
        it[j] = (int32_t)(uint32_t)key[j];
    }
    const hipMemcpyKind kd = out_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    e = hipMemcpy(ids, id.data(), m * 4, kd);
    if (e == hipSuccess && iter_of) e = hipMemcpy(iter_of, it.data(), m * 4, kd);
    return dev_err(e);
}

gbsub_status gbsub_set_profiling(gbsub_ctx *c, int enable)
{
    if (!c) return GBSUB_E_INVALID;
    c->profiling = enable != 0;
    c->clear_stats();
    return GBSUB_OK;
}

gbsub_status gbsub_kernel_stats(const gbsub_ctx *c, gbsub_kernel_stat *out, uint32_t cap, uint32_t *n)
{
    if (!c || !n) return GBSUB_E_INVALID;
    static const char *names[K_COUNT] = {"tables", "reset", "prep", "xupdate", "median", "snr", "output"};
    static const char *units[K_COUNT] = {"bins", "bins", "sources", "bins", "bins", "candidates",
                                         "candidates"};
    *n = K_COUNT;
    if (cap < (uint32_t)K_COUNT) return GBSUB_E_TRUNCATED;
    if (!out) return GBSUB_E_INVALID;
    for (int k = 0; k < K_COUNT; ++k) {
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, names[k], sizeof(out[k].name) - 1);
        std::strncpy(out[k].unit, units[k], sizeof(out[k].unit) - 1);
        out[k].launches = c->k_launches[k];
        out[k].total_ms = c->k_ms[k];
        out[k].units = c->k_units[k];
    }
    return GBSUB_OK;
}

}  // extern "C"
