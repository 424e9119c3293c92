// gbsub_api.hip -- host runtime and C ABI of libgbsub (see include/gbsub.h).
//
// The runtime validates the configuration, carves the caller's workspace,
// writes slot descriptors (grid, workspace pointers, catalog) to device
// memory and enqueues the kernels of gbsub_kernels.hip.  Kernels read the
// descriptor of slot blockIdx.y, so a single catalog (gbsub_run, a one-slot
// table inside its workspace) and a batch of catalogs (gbsub_batch_*, a table
// in a caller buffer) use the same launches.  gbsub_run keeps a couple of
// loop bodies queued ahead of the GPU, paced by a progress word that the loop
// writes to pinned host memory; a batch step enqueues its bodies at once and
// the host reads the control blocks at each poll.  Every kernel of a body
// exits at once after the slot's device-side "settled" flag is set.

#include "gbsub_internal.h"
#include "gbsub.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
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
    Slot *host_slot;   // pinned staging of the one-slot table
    uint32_t *host_prog;   // pinned, device-mapped: bodies finished << 1 | settled, written by the tail
    uint32_t *dev_prog;    // the same word as the kernels address it
    int batch_slot;    // slot held in a batch, -1 if none
    // results of the last complex-template run
    bool cx_have_result;
    CxDev cx;
    gbsub_summary cx_summ;
    uint32_t cx_n;
    Slot *host_cx_slots;   // pinned staging of the two channel descriptors
    // profiling: bit k of `profiling` selects kernel family k
    uint32_t profiling;
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

    // Launches through `fn`, bracketed by events when profiling: the
    // events are recorded on the stream around fn().
    template <typename F>
    hipError_t timed(int kid, int64_t t, hipStream_t st, F fn)
    {
        return timed_ext(kid, t, [&](hipEvent_t a, hipEvent_t b) {
            hipError_t e = a ? hipEventRecord(a, st) : hipSuccess;
            if (e == hipSuccess) e = fn();
            if (e == hipSuccess && b) e = hipEventRecord(b, st);
            return e;
        });
    }

    // Launches through fn(start, end); a loop-body launcher hands the
    // events to its dispatch, which stamps them itself (no stream work).
    template <typename F>
    hipError_t timed_ext(int kid, int64_t t, F fn)
    {
        if (!(profiling >> kid & 1u)) return fn(nullptr, nullptr);
        hipEvent_t a = next_event(), b = next_event();
        if (!a || !b) return hipErrorOutOfMemory;
        const hipError_t e = fn(a, b);
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
    take(sizeof(Slot));                      // the one-slot table of gbsub_run
    t.max_chunks = (uint32_t)(ev_chunks + nt);
    t.max_slots = (uint32_t)(2 * ev_chunks + 2);
    t.sx = (double *)take(B * 8);
    t.isx = (double *)take(B * 8);
    t.isx_pre = (double *)take(B * 8);
    t.isx_tsum = (double *)take(nt * 8);
    t.isx_tile = (double *)take((nt + 1) * 8);
    t.isx_seg = (double2 *)take(((B + SEG_BINS - 1) / SEG_BINS) * 16);
    t.Xn = (I128 *)take(B * 16);
    t.D = (I128 *)take((B + 1) * 16);
    t.Dtile = (I128 *)take((nt + 1) * 16);
    t.Dcarry = (I128 *)take((nt + 1) * 16);
    t.Dadj = (SplitSum *)take(nt * 16);
    const bool naive = g.prec == GBSUB_FP32_NAIVE;
    t.Xf = (float *)take(naive ? B * 4 : 0);
    t.Df = (float *)take(naive ? (B + 1) * 4 : 0);
    t.Dtf = (float *)take(naive ? (nt + 1) * 4 : 0);
    t.Dcf = (float *)take(naive ? (nt + 1) * 4 : 0);
    const bool comp = g.prec == GBSUB_FP32_COMP;
    t.Xc = (FF *)take(comp ? B * 8 : 0);
    t.Dc = (FF *)take(comp ? (B + 1) * 8 : 0);
    t.Dtc = (FF *)take(comp ? (nt + 1) * 8 : 0);
    t.X = (double *)take(B * 8);
    t.S = (double *)take(B * 8);
    t.is_pre = (double *)take(B * 8);
    t.is_psum = (double *)take((uint64_t)g.nparts * 8);
    t.xstamp = (uint32_t *)take(nt * 4);
    t.sstamp = (uint32_t *)take(nt * 4);
    t.sdl = (uint32_t *)take(nt * 4);
    t.btot = (uint32_t *)take(nt * 4);
    const uint64_t npb = (nn + PREP_SRC - 1) / PREP_SRC;
    t.bhist = (uint32_t *)take(npb * ((nt + 1) / 2) * 4);
    t.boff = (uint32_t *)take(npb * nt * 4);
    t.bbase = (uint32_t *)take((nt + 1) * 4);
    t.nch = (uint32_t *)take(nt * 4);
    t.chunk_base = (uint32_t *)take((nt + 1) * 4);
    t.slot_base = (uint32_t *)take(nt * 4);
    t.ev_key = (uint32_t *)take((max_events ? max_events : 1) * 4);
    t.ev_val = (int64_t *)take((max_events ? max_events : 1) * 8);
    t.partial = (I128 *)take((uint64_t)t.max_slots * 2 * (uint64_t)g.tile * 16);
    t.cbits = (uint64_t *)take(((nn + 63) / 64) * 8);
    t.rs_hist = (uint32_t *)take(resolved_scratch_words(nn) * 4);
    const uint64_t ncb = npb;
    t.blk_cand = (uint32_t *)take((ncb + 1) * 4);
    t.blk_amax = (uint32_t *)take(ncb * 4);
    t.c_src = (uint32_t *)take(nn * 4);
    t.c_id = (uint32_t *)take(nn * 4);
    t.c_glo = (int32_t *)take(nn * 4);
    t.c_ghi = (int32_t *)take(nn * 4);
    t.c_iter = (int32_t *)take(nn * 4);
    t.c_q = (double *)take(nn * 8);
    t.c_qfx = (uint64_t *)take(nn * 8);
    t.c_rho2 = (double *)take(nn * 8);
    t.b_part = (SnrPart *)take((uint64_t)SNR_BLOCKS * sizeof(SnrPart));
    t.n_new = (uint32_t *)take((uint64_t)NEW_CAP * 4);
    t.coarse = (double *)take(3 * COARSE_MAX * 8);
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
    if (c->estimator > GBSUB_MEAN) return GBSUB_E_INVALID;
    if (c->estimator == GBSUB_MEAN && c->precision != GBSUB_FP64) return GBSUB_E_INVALID;
    if (c->track_model > GBSUB_TRACK_SINGLE) return GBSUB_E_INVALID;
    if (c->precision > GBSUB_FP32_NAIVE) return GBSUB_E_INVALID;
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
    // tile: a power of two (256 .. TILE_MAX) with outputs + W - 1 inside the
    // median kernel's LDS union (the largest such by default); parts of at
    // most PART_MAX bins
    const int room = MMAX - (r.W - 1);
    if (room < WG) return GBSUB_E_INVALID;
    int tile = TILE_MAX;
    while (tile > room) tile >>= 1;
    if (c->tile_bins) {
        const uint32_t tb = c->tile_bins;
        if (tb < (uint32_t)WG || tb > (uint32_t)tile || (tb & (tb - 1)) != 0) return GBSUB_E_INVALID;
        tile = (int)tb;
    }
    r.tile = tile;
    r.nt = (r.B + tile - 1) / tile;
    if (r.nt > NBK_MAX) return GBSUB_E_INVALID;
    r.part = tile < PART_MAX ? tile : PART_MAX;
    r.np = tile / r.part;
    r.nparts = (r.B + r.part - 1) / r.part;
    r.split_blocks = c->split_blocks ? c->split_blocks : (uint32_t)SPLIT_BLOCKS;
    r.split_tiles = r.split_blocks / (uint32_t)r.np;
    r.track_single = c->track_model == GBSUB_TRACK_SINGLE;
    r.prec = (int32_t)c->precision;
    r.est = (int32_t)c->estimator;
    r.T = c->t_obs_s;
    r.C = c->median_scale;
    r.rth = c->snr_threshold;
    r.rth2 = c->snr_threshold * c->snr_threshold;
    const double cut = c->kappa * c->snr_threshold;
    r.cut2 = cut * cut;
    r.oms_pm = c->oms_pm;
    r.tm_fm = c->tm_fm;
    r.arm_m = c->arm_m;
    r.max_iter = c->max_iter;
    *g = r;
    return GBSUB_OK;
}

Slot make_slot(const Grid &g, const Dev &d, const gbsub_catalog *cat)
{
    Slot sl{};
    sl.g = g;
    sl.d = d;
    sl.A = cat->A;
    sl.F = cat->f;
    sl.FD = cat->fdot;
    sl.ids = cat->id;
    sl.n = cat->n;
    sl.active = 1;
    return sl;
}

// Launch extents covering one slot.
Dims dims_of(const Slot &sl)
{
    Dims dm{};
    dm.ns = 1;
    dm.maxB = sl.g.B;
    dm.maxnt = sl.g.nt;
    dm.maxtile = sl.g.tile;
    dm.maxparts = sl.g.nparts;
    dm.est_mask = 1u << sl.g.est;
    dm.naive = sl.g.prec == PREC_NAIVE;
    dm.prep_blocks = (uint32_t)((sl.n + PREP_SRC - 1) / PREP_SRC);
    dm.accum_blocks = sl.d.max_chunks;
    return dm;
}

void widen(Dims &a, const Dims &b)
{
    a.maxB = std::max(a.maxB, b.maxB);
    a.maxnt = std::max(a.maxnt, b.maxnt);
    a.maxtile = std::max(a.maxtile, b.maxtile);
    a.maxparts = std::max(a.maxparts, b.maxparts);
    a.est_mask |= b.est_mask;
    a.naive |= b.naive;
    a.prep_blocks = std::max(a.prep_blocks, b.prep_blocks);
    a.accum_blocks = std::max(a.accum_blocks, b.accum_blocks);
}

gbsub_status check_catalog(const gbsub_ctx *c, const gbsub_catalog *cat, void *ws, uint64_t ws_bytes)
{
    if (!c || !cat || !ws) return GBSUB_E_INVALID;
    if (cat->n >= (1ull << 31)) return GBSUB_E_INVALID;
    if (cat->n > 0 && (!cat->A || !cat->f || !cat->fdot || !cat->id)) return GBSUB_E_INVALID;
    if (((uintptr_t)ws & 255u) != 0) return GBSUB_E_INVALID;
    if (ws_bytes < carve(c->g, cat->n, nullptr, nullptr)) return GBSUB_E_INVALID;
    return GBSUB_OK;
}

gbsub_status use_device(int dev)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return GBSUB_E_DEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return GBSUB_E_DEVICE;
    return GBSUB_OK;
}

// Summary of a settled slot from its control block.
gbsub_summary summary_of(const Grid &g, const Ctl &h)
{
    gbsub_summary s{};
    s.n_iter = h.n_iter;
    s.n_bins = (uint64_t)g.B;
    s.n_candidates = h.n_cand;
    s.n_resolved = h.n_resolved;
    s.n_near_threshold = h.n_near;
    double mm;
    std::memcpy(&mm, &h.min_margin, 8);
    s.min_rel_margin = mm;
    return s;
}

}  // namespace

// Workspace of gbsub_run_static, for callers that cannot allocate device
// memory: one array per GPU the library runs on, held until the process
// ends.  Host code never passes `scratch` itself (in host code the name is
// a host-side stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns on each device, cached by static_scratch().
static __device__ __align__(256) unsigned char scratch[GBSUB_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on device `dev`, which must be current.  The
// lookup runs once per device (at the first gbsub_create on it).
gbsub_status static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return GBSUB_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GBSUB_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
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
    c->host_slot = nullptr;
    c->host_prog = nullptr;
    c->dev_prog = nullptr;
    c->batch_slot = -1;
    c->cx_have_result = false;
    c->cx_n = 0;
    c->host_cx_slots = nullptr;
    c->profiling = 0;
    c->ev_used = 0;
    c->clear_stats();
    if (hipHostMalloc((void **)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_slot, sizeof(Slot), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_cx_slots, 2 * sizeof(Slot), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_prog, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->dev_prog, c->host_prog, 0) != hipSuccess) {
        if (c->host_ctl) (void)hipHostFree(c->host_ctl);
        if (c->host_slot) (void)hipHostFree(c->host_slot);
        if (c->host_cx_slots) (void)hipHostFree(c->host_cx_slots);
        if (c->host_prog) (void)hipHostFree(c->host_prog);
        delete c;
        return GBSUB_E_DEVICE;
    }
    void *scr = nullptr;
    if (static_scratch(dev, &scr) != GBSUB_OK) {
        gbsub_destroy(c);
        return GBSUB_E_DEVICE;
    }
    *out = c;
    return GBSUB_OK;
}

void gbsub_destroy(gbsub_ctx *c)
{
    if (!c) return;
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    if (c->host_slot) (void)hipHostFree(c->host_slot);
    if (c->host_cx_slots) (void)hipHostFree(c->host_cx_slots);
    if (c->host_prog) (void)hipHostFree(c->host_prog);
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
    gbsub_status st0 = check_catalog(c, cat, ws, ws_bytes);
    if (st0 != GBSUB_OK) return st0;
    if (c->batch_slot >= 0) return GBSUB_E_STATE;
    c->have_result = false;
    if (use_device(c->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    Dev d;
    carve(c->g, cat->n, (char *)ws, &d);
    const Grid &g = c->g;
    Slot *ds = reinterpret_cast<Slot *>(ws);    // one-slot table at the start of the workspace
    *c->host_slot = make_slot(g, d, cat);
    c->host_slot->prog = c->dev_prog;
    const Dims dm = dims_of(*c->host_slot);
    // every kernel of an earlier run has ended (each return below follows a
    // synchronization once loop bodies are in flight)
    volatile uint32_t *prog = c->host_prog;
    *prog = 0;

    c->ev_used = 0;
    c->recs.clear();
    hipError_t e = hipMemcpyAsync(ds, c->host_slot, sizeof(Slot), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && c->tables_ws != ws) {
        e = c->timed(K_TABLES, -1, st, [&] { return launch_grid_tables(ds, dm, st); });
        if (e == hipSuccess) c->tables_ws = ws;
    }
    if (e == hipSuccess) e = c->timed(K_RESET, -1, st, [&] { return launch_reset(ds, dm, st); });
    if (e == hipSuccess) e = c->timed(K_PREP, -1, st, [&] { return launch_prep(ds, dm, st); });
    if (e == hipSuccess)
        e = c->timed_ext(K_XUPDATE, -1, [&](hipEvent_t a, hipEvent_t b) { return launch_xupdate(ds, dm, st, a, b); });
    if (e != hipSuccess) {
        c->tables_ws = nullptr;
        return GBSUB_E_DEVICE;
    }
    // Loop bodies, paced by the progress word the tail writes to host
    // memory: the host keeps AHEAD bodies queued beyond the last finished
    // one and stops enqueuing once a body settles the loop, so the GPU never
    // waits for the host and at most AHEAD bodies run past the settled one
    // (their kernels exit at once).  The device enforces max_iter.  A body is
    // median, SNR, then the X update of the next body, whose last block
    // takes this body's stop decision.  Whenever the stream runs dry without
    // a settled flag in sight, the control block in device memory decides.
    constexpr uint64_t AHEAD = 2;
    const uint64_t guard = (uint64_t)cat->n + 2 + (c->cfg.max_iter ? c->cfg.max_iter : 0);
    auto fail = [&](gbsub_status s) {
        (void)hipStreamSynchronize(st);
        return s;
    };
    auto body = [&](int64_t ti) {
        hipError_t r = c->timed_ext(K_MEDIAN, ti, [&](hipEvent_t a, hipEvent_t b) {
            return launch_median(ds, dm, st, a, b);
        });
        if (r == hipSuccess)
            r = c->timed_ext(K_SNR, ti, [&](hipEvent_t a, hipEvent_t b) { return launch_snr(ds, dm, st, a, b); });
        if (r == hipSuccess)
            r = c->timed_ext(K_XUPDATE, ti, [&](hipEvent_t a, hipEvent_t b) {
                return launch_xupdate(ds, dm, st, a, b);
            });
        return r;
    };
    uint64_t t = 0;                  // bodies enqueued
    uint32_t seen_prev = 0;
    auto quiet_since = std::chrono::steady_clock::now();
    for (;;) {
        const uint32_t w = *prog;
        if (w & 1u) break;
        const uint32_t seen = w >> 1;
        if (t < (uint64_t)seen + AHEAD) {
            if (t > guard) return fail(GBSUB_E_DEVICE);   // the loop must settle within n + 1 bodies
            if (body((int64_t)t) != hipSuccess) return fail(GBSUB_E_DEVICE);
            ++t;
            continue;
        }
        const auto now = std::chrono::steady_clock::now();
        if (seen != seen_prev) {
            seen_prev = seen;
            quiet_since = now;
            continue;
        }
        if (now - quiet_since < std::chrono::microseconds(200)) {
            std::this_thread::yield();
            continue;
        }
        quiet_since = now;
        const hipError_t q = hipStreamQuery(st);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(GBSUB_E_DEVICE);
        // nothing in flight: read the control block itself
        e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(GBSUB_E_DEVICE);
        if (c->host_ctl->bad) return GBSUB_E_INVALID;
        if (c->host_ctl->done) break;
        if (t > guard) return GBSUB_E_DEVICE;
        if (body((int64_t)t) != hipSuccess) return fail(GBSUB_E_DEVICE);
        ++t;
    }
    e = c->timed(K_OUTPUT, -1, st, [&] { return launch_outputs(ds, dm, st); });
    if (e == hipSuccess) e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GBSUB_E_DEVICE);

    const Ctl &h = *c->host_ctl;
    const gbsub_status status = h.status == 6 ? GBSUB_E_MAXITER : GBSUB_OK;
    if (c->profiling) {
        const int64_t n_body = (int64_t)h.n_iter;
        for (const auto &r : c->recs) {
            if (r.t >= n_body) continue;        // bodies enqueued past the settled one
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GBSUB_E_DEVICE;
            c->k_ms[r.kid] += ms;
            c->k_launches[r.kid] += 1;
            if (r.kid == K_TABLES) c->k_units[K_TABLES] += (double)g.B;
        }
        const uint32_t m = c->profiling;
        if (m >> K_PREP & 1u) c->k_units[K_PREP] += (double)cat->n;
        if (m >> K_RESET & 1u) c->k_units[K_RESET] += (double)g.B;
        if (m >> K_XUPDATE & 1u) c->k_units[K_XUPDATE] += (double)h.units_x;
        if (m >> K_MEDIAN & 1u) c->k_units[K_MEDIAN] += (double)h.units_med;
        if (m >> K_SNR & 1u) c->k_units[K_SNR] += (double)h.units_snr;
        if (m >> K_OUTPUT & 1u) c->k_units[K_OUTPUT] += (double)h.n_cand;
    }
    const gbsub_summary s = summary_of(g, h);
    if (out) *out = s;
    if (status != GBSUB_OK) return status;
    c->summ = s;
    c->dev = d;
    c->ws = ws;
    c->n_cand = h.n_cand;
    c->have_result = true;
    return GBSUB_OK;
}

gbsub_status gbsub_run_static(gbsub_ctx *c, const gbsub_catalog *cat, void *stream, gbsub_summary *out)
{
    if (!c || !cat) return GBSUB_E_INVALID;
    if (c->batch_slot >= 0) return GBSUB_E_STATE;
    uint64_t need = 0;
    if (cat->n >= (1ull << 31)) return GBSUB_E_INVALID;
    need = carve(c->g, cat->n, nullptr, nullptr);
    if (need > (uint64_t)GBSUB_STATIC_WORKSPACE_BYTES) return GBSUB_E_NOMEM;
    if (use_device(c->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    void *ws = nullptr;
    if (static_scratch(c->device, &ws) != GBSUB_OK) return GBSUB_E_DEVICE;
    // Another context may have used the array since: the grid tables are
    // always recomputed, and every other buffer is rewritten by the run
    // (k_reset and prep start from arbitrary contents, as in a fresh
    // caller workspace).  No timing: the profiling mode creates events and
    // grows host-side records.
    const uint32_t prof = c->profiling;
    c->profiling = 0;
    c->tables_ws = nullptr;
    const gbsub_status st = gbsub_run(c, cat, ws, (uint64_t)GBSUB_STATIC_WORKSPACE_BYTES, stream, out);
    c->tables_ws = nullptr;
    c->profiling = prof;
    return st;
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
    // S - S_instr on the device, into `out` or (host output) into the
    // workspace's in-part 1/S prefix, which is dead once a run has settled
    double *dst = out_on_device ? out : c->dev.is_pre;
    hipError_t e = launch_sgal(c->dev.S, c->dev.sx, (int)B, dst, nullptr);
    if (e == hipSuccess) e = out_on_device ? hipDeviceSynchronize() : hipMemcpy(out, dst, B * 8, hipMemcpyDeviceToHost);
    return dev_err(e);
}

gbsub_status gbsub_coarse(const gbsub_ctx *c, uint32_t kind, double f_lo, double f_hi, uint32_t n_out,
                          double *f_out, double *s_out, double *hc_out, uint32_t *count)
{
    if (!c || !f_out || !s_out) return GBSUB_E_INVALID;
    if (!c->have_result) return GBSUB_E_STATE;
    if (kind > GBSUB_SPEC_S_INSTR || n_out < 1 || n_out > (uint32_t)COARSE_MAX || !(f_lo > 0.0) ||
        !(f_hi > f_lo) || !std::isfinite(f_hi))
        return GBSUB_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    CoarseEdges ed;
    for (uint32_t j = 0; j <= n_out; ++j) ed.e[j] = f_lo * std::pow(f_hi / f_lo, (double)j / (double)n_out);
    ed.e[n_out] = f_hi;
    const Grid &g = c->g;
    hipError_t e = launch_coarse(c->dev.S, c->dev.sx, c->dev.X, (int)kind, g.k0, g.B, g.T, ed, (int)n_out,
                                 c->dev.coarse, nullptr);
    std::vector<double> h(3 * (size_t)n_out);
    if (e == hipSuccess) e = hipMemcpy(h.data(), c->dev.coarse, h.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    for (uint32_t k = 0; k < n_out; ++k) {
        const double cnt = h[3 * k + 2];
        const double fm = cnt > 0 ? h[3 * k] / cnt : 0.0;
        const double sm = cnt > 0 ? h[3 * k + 1] / cnt : 0.0;
        f_out[k] = fm;
        s_out[k] = sm;
        if (hc_out) hc_out[k] = std::sqrt(fm * sm);
        if (count) count[k] = (uint32_t)cnt;
    }
    return GBSUB_OK;
}

gbsub_status gbsub_generate(const gbsub_population *pop, uint64_t seed, uint64_t first, uint64_t n, float *A,
                            float *f, float *fdot, uint32_t *id, void *stream)
{
    if (!pop) return GBSUB_E_INVALID;
    const gbsub_population &p = *pop;
    const double v[9] = {p.alpha_pl, p.alpha_g, p.beta_g, p.mu_g, p.mu, p.sigma, p.rho, p.f_lo_hz, p.f_hi_hz};
    for (double x : v)
        if (!std::isfinite(x)) return GBSUB_E_INVALID;
    if (p.alpha_pl == -1.0 || !(p.alpha_g > 0.0) || !(p.beta_g > 0.0) || !(p.sigma >= 0.0) || !(p.rho > -1.0) ||
        !(p.rho < 1.0) || !(p.f_lo_hz > 0.0) || !(p.f_hi_hz > p.f_lo_hz))
        return GBSUB_E_INVALID;
    if (n > 0 && (!A || !f || !fdot)) return GBSUB_E_INVALID;
    const PopParams pp{p.alpha_pl, p.alpha_g, p.beta_g, p.mu_g, p.mu, p.sigma, p.rho, p.f_lo_hz, p.f_hi_hz};
    return dev_err(launch_generate(pp, seed, first, n, A, f, fdot, id, (hipStream_t)stream));
}

gbsub_status gbsub_resolved(const gbsub_ctx *c, uint32_t *ids, int32_t *iter_of, uint64_t cap,
                            uint64_t *n, int out_on_device)
{
    if (!c || !n) return GBSUB_E_INVALID;
    if (!c->have_result) return GBSUB_E_STATE;
    const uint64_t m = c->summ.n_resolved;
    *n = m;
    if (cap < m) return GBSUB_E_TRUNCATED;
    if (m == 0) return GBSUB_OK;
    if (!ids) return GBSUB_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    // compaction and sort on the device, in the workspace's event buffer
    // (free once the binning is done: 16 bytes per source, m <= sources)
    const Dev &d = c->dev;
    uint32_t *kA = reinterpret_cast<uint32_t *>(d.ev_val);
    int32_t *vA = reinterpret_cast<int32_t *>(kA + m);
    uint32_t *kB = reinterpret_cast<uint32_t *>(vA + m);
    int32_t *vB = reinterpret_cast<int32_t *>(kB + m);
    hipError_t e = launch_resolved(d.c_iter, d.c_id, c->n_cand, (uint32_t)m, d.rs_hist, kA, vA, kB, vB, nullptr);
    const hipMemcpyKind kd = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (e == hipSuccess) e = hipMemcpy(ids, kA, m * 4, kd);
    if (e == hipSuccess && iter_of) e = hipMemcpy(iter_of, vA, m * 4, kd);
    return dev_err(e);
}

gbsub_status gbsub_candidates(const gbsub_ctx *c, uint32_t *ids, int32_t *iter_of, double *rho2,
                              uint64_t cap, uint64_t *n)
{
    if (!c || !n) return GBSUB_E_INVALID;
    if (!c->have_result) return GBSUB_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const uint64_t nc = c->n_cand;
    *n = nc;
    if (cap < nc) return GBSUB_E_TRUNCATED;
    if (nc == 0) return GBSUB_OK;
    if (!ids) return GBSUB_E_INVALID;
    std::vector<uint32_t> id(nc);
    std::vector<int32_t> it(nc);
    std::vector<double> r2(nc);
    hipError_t e = hipMemcpy(id.data(), c->dev.c_id, nc * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(it.data(), c->dev.c_iter, nc * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(r2.data(), c->dev.c_rho2, nc * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    std::vector<uint64_t> order(nc);
    for (uint64_t j = 0; j < nc; ++j) order[j] = ((uint64_t)id[j] << 32) | (uint32_t)j;
    std::sort(order.begin(), order.end());
    for (uint64_t q = 0; q < nc; ++q) {
        const uint32_t j = (uint32_t)order[q];
        ids[q] = id[j];
        if (iter_of) iter_of[q] = it[j];
        if (rho2) rho2[q] = r2[j];
    }
    return GBSUB_OK;
}

// ---------------------------------------------------------------- complex-template data model

namespace {

gbsub_status cx_grid_ok(const gbsub_ctx *c)
{
    if (c->g.prec != PREC_FP64) return GBSUB_E_INVALID;
    if ((uint64_t)c->g.B > (uint64_t)CX_NTC_MAX * CX_TILE) return GBSUB_E_INVALID;
    return GBSUB_OK;
}

}  // namespace

gbsub_status gbsub_cx_workspace_size(const gbsub_ctx *c, uint64_t n, uint64_t *bytes)
{
    if (!c || !bytes || n >= (1ull << 31)) return GBSUB_E_INVALID;
    if (cx_grid_ok(c) != GBSUB_OK) return GBSUB_E_INVALID;
    *bytes = cx_carve(c->g, n, nullptr, nullptr);
    return GBSUB_OK;
}

gbsub_status gbsub_cx_run(gbsub_ctx *c, const gbsub_cx_catalog *cat, void *ws, uint64_t ws_bytes, void *stream,
                          gbsub_summary *out)
{
    if (!c || !cat || !ws) return GBSUB_E_INVALID;
    if (cx_grid_ok(c) != GBSUB_OK) return GBSUB_E_INVALID;
    if (cat->n >= (1ull << 31)) return GBSUB_E_INVALID;
    if (cat->n > 0 && (!cat->A || !cat->f || !cat->fdot || !cat->phi_a || !cat->phi_e || !cat->id))
        return GBSUB_E_INVALID;
    if (((uintptr_t)ws & 255u) != 0 || ws_bytes < cx_carve(c->g, cat->n, nullptr, nullptr)) return GBSUB_E_INVALID;
    if (c->batch_slot >= 0) return GBSUB_E_STATE;
    c->cx_have_result = false;
    if (use_device(c->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    const Grid &g = c->g;
    CxDev d;
    cx_carve(g, cat->n, (char *)ws, &d);
    // the A and E channels as two descriptors of the median kernels
    for (int ch = 0; ch < 2; ++ch) {
        Slot sl{};
        sl.g = g;
        sl.d.sx = d.sx;
        sl.d.X = d.X + (size_t)ch * g.B;
        sl.d.S = d.S + (size_t)ch * g.B;
        sl.d.is_pre = d.is_pre + (size_t)ch * g.B;
        sl.d.is_psum = d.is_psum + (size_t)ch * g.nparts;
        sl.d.xstamp = d.xstamp;
        sl.d.sstamp = d.sstamp;
        sl.d.sdl = d.sdl;
        sl.d.ctl = d.ctl;
        sl.n = cat->n;
        sl.active = 1;
        c->host_cx_slots[ch] = sl;
    }
    CxIn in{cat->A, cat->f, cat->fdot, cat->phi_a, cat->phi_e, cat->id, (uint32_t)cat->n, c->dev_prog};
    volatile uint32_t *prog = c->host_prog;
    *prog = 0;
    auto fail = [&](gbsub_status s) {
        (void)hipStreamSynchronize(st);
        return s;
    };
    c->ev_used = 0;
    c->recs.clear();
    hipError_t e = hipMemcpyAsync(d.slots, c->host_cx_slots, 2 * sizeof(Slot), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = c->timed(K_PREP, -1, st, [&] { return cx_launch_prep(g, d, in, st); });
    if (e != hipSuccess) return fail(GBSUB_E_DEVICE);
    auto body = [&](int64_t ti) {
        hipError_t r = c->timed(K_XUPDATE, ti, st, [&] { return cx_launch_power(g, d, in, st); });
        if (r == hipSuccess)
            r = c->timed_ext(K_MEDIAN, ti, [&](hipEvent_t a, hipEvent_t b) { return cx_launch_psd(g, d, st, a, b); });
        if (r == hipSuccess) r = c->timed(K_SNR, ti, st, [&] { return cx_launch_snr(g, d, in, st); });
        return r;
    };
    // loop bodies paced by the progress word, as in gbsub_run
    constexpr uint64_t AHEAD = 2;
    const uint64_t guard = (uint64_t)cat->n + 2 + (c->cfg.max_iter ? c->cfg.max_iter : 0);
    uint64_t t = 0;
    uint32_t seen_prev = 0;
    auto quiet_since = std::chrono::steady_clock::now();
    for (;;) {
        const uint32_t w = *prog;
        if (w & 1u) break;
        const uint32_t seen = w >> 1;
        if (t < (uint64_t)seen + AHEAD) {
            if (t > guard) return fail(GBSUB_E_DEVICE);
            if (body((int64_t)t) != hipSuccess) return fail(GBSUB_E_DEVICE);
            ++t;
            continue;
        }
        const auto now = std::chrono::steady_clock::now();
        if (seen != seen_prev) {
            seen_prev = seen;
            quiet_since = now;
            continue;
        }
        if (now - quiet_since < std::chrono::microseconds(200)) {
            std::this_thread::yield();
            continue;
        }
        quiet_since = now;
        const hipError_t q = hipStreamQuery(st);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(GBSUB_E_DEVICE);
        e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(GBSUB_E_DEVICE);
        if (c->host_ctl->done) break;
        if (t > guard) return GBSUB_E_DEVICE;
        if (body((int64_t)t) != hipSuccess) return fail(GBSUB_E_DEVICE);
        ++t;
    }
    e = cx_launch_outputs(g, d, in, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->host_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GBSUB_E_DEVICE);
    const Ctl &h = *c->host_ctl;
    if (h.bad) return GBSUB_E_INVALID;
    if (c->profiling) {
        for (const auto &r : c->recs) {
            if (r.t >= (int64_t)h.n_iter) continue;        // bodies enqueued past the settled one
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GBSUB_E_DEVICE;
            c->k_ms[r.kid] += ms;
            c->k_launches[r.kid] += 1;
        }
        const uint32_t m = c->profiling;
        if (m >> K_PREP & 1u) c->k_units[K_PREP] += (double)cat->n;
        if (m >> K_XUPDATE & 1u) c->k_units[K_XUPDATE] += (double)h.units_x;
        if (m >> K_MEDIAN & 1u) c->k_units[K_MEDIAN] += 2.0 * (double)h.units_med;   // both channels
        if (m >> K_SNR & 1u) c->k_units[K_SNR] += (double)h.units_snr;
    }
    gbsub_summary s = summary_of(g, h);
    s.n_candidates = h.cand_cursor;
    if (out) *out = s;
    if (h.status == 6) return GBSUB_E_MAXITER;
    c->cx = d;
    c->cx_summ = s;
    c->cx_n = (uint32_t)cat->n;
    c->cx_have_result = true;
    return GBSUB_OK;
}

gbsub_status gbsub_cx_spectrum(const gbsub_ctx *c, uint32_t channel, uint32_t kind, double *out, uint64_t cap,
                               uint64_t *n_bins, int out_on_device)
{
    if (!c || !n_bins || channel > 1) return GBSUB_E_INVALID;
    if (!c->cx_have_result) return GBSUB_E_STATE;
    const uint64_t B = (uint64_t)c->g.B;
    *n_bins = B;
    if (kind > GBSUB_SPEC_H_RESIDUAL) return GBSUB_E_INVALID;
    const uint64_t need = kind == GBSUB_SPEC_H_RESIDUAL ? 2 * B : B;
    if (cap < need) return GBSUB_E_TRUNCATED;
    if (!out) return GBSUB_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const CxDev &d = c->cx;
    const hipMemcpyKind kd = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t off = (size_t)channel * B;
    if (kind == GBSUB_SPEC_SN) return dev_err(hipMemcpy(out, d.S + off, B * 8, kd));
    if (kind == GBSUB_SPEC_X_RESIDUAL) return dev_err(hipMemcpy(out, d.X + off, B * 8, kd));
    if (kind == GBSUB_SPEC_S_INSTR) return dev_err(hipMemcpy(out, d.sx, B * 8, kd));
    // device-computed kinds, into `out` or (host output) into the workspace's
    // in-part 1/S prefixes, dead once a run has settled (2B doubles)
    double *tmp = d.is_pre;
    hipError_t e;
    if (kind == GBSUB_SPEC_S_GAL) {
        double *dst = out_on_device ? out : tmp;
        e = launch_sgal(d.S + off, d.sx, (int)B, dst, nullptr);
        if (e == hipSuccess) e = out_on_device ? hipDeviceSynchronize() : hipMemcpy(out, dst, B * 8, kd);
        return dev_err(e);
    }
    // h of the channel: 2B doubles, through the prefix scratch (2B doubles)
    double *dst = out_on_device ? out : tmp;
    e = cx_launch_h(c->g, d, c->cx_n, (int)channel, dst, nullptr);
    if (e == hipSuccess) e = out_on_device ? hipDeviceSynchronize() : hipMemcpy(out, dst, 2 * B * 8, kd);
    return dev_err(e);
}

gbsub_status gbsub_cx_resolved(const gbsub_ctx *c, uint32_t *ids, int32_t *iter_of, uint64_t cap, uint64_t *n,
                               int out_on_device)
{
    if (!c || !n) return GBSUB_E_INVALID;
    if (!c->cx_have_result) return GBSUB_E_STATE;
    const uint64_t m = c->cx_summ.n_resolved;
    *n = m;
    if (cap < m) return GBSUB_E_TRUNCATED;
    if (m == 0) return GBSUB_OK;
    if (!ids) return GBSUB_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const CxDev &d = c->cx;
    hipError_t e = launch_resolved(d.c_iter, d.c_id, (uint32_t)c->cx_summ.n_candidates, (uint32_t)m, d.rs_hist, d.kA,
                                   d.vA, d.kB, d.vB, nullptr);
    const hipMemcpyKind kd = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (e == hipSuccess) e = hipMemcpy(ids, d.kA, m * 4, kd);
    if (e == hipSuccess && iter_of) e = hipMemcpy(iter_of, d.vA, m * 4, kd);
    return dev_err(e);
}

gbsub_status gbsub_cx_candidates(const gbsub_ctx *c, uint32_t *ids, int32_t *iter_of, double *rho2, uint64_t cap,
                                 uint64_t *n)
{
    if (!c || !n) return GBSUB_E_INVALID;
    if (!c->cx_have_result) return GBSUB_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return GBSUB_E_DEVICE;
    const uint64_t nc = c->cx_summ.n_candidates;
    *n = nc;
    if (cap < nc) return GBSUB_E_TRUNCATED;
    if (nc == 0) return GBSUB_OK;
    if (!ids) return GBSUB_E_INVALID;
    std::vector<uint32_t> id(nc);
    std::vector<int32_t> it(nc);
    std::vector<double> r2(nc);
    hipError_t e = hipMemcpy(id.data(), c->cx.c_id, nc * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(it.data(), c->cx.c_iter, nc * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(r2.data(), c->cx.c_rho2, nc * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    // candidate slots are handed out in order of discovery: order them by id
    std::vector<uint64_t> order(nc);
    for (uint64_t j = 0; j < nc; ++j) order[j] = ((uint64_t)id[j] << 32) | (uint32_t)j;
    std::sort(order.begin(), order.end());
    for (uint64_t q = 0; q < nc; ++q) {
        const uint32_t j = (uint32_t)order[q];
        ids[q] = id[j];
        if (iter_of) iter_of[q] = it[j];
        if (rho2) rho2[q] = r2[j];
    }
    return GBSUB_OK;
}

gbsub_status gbsub_cx_templates(const gbsub_ctx *c, uint64_t n, const float *A, const float *f, const float *fdot,
                                int64_t *q, double *U, void *stream)
{
    if (!c || n >= (1ull << 31)) return GBSUB_E_INVALID;
    if (n > 0 && (!A || !f || !fdot || !q || !U)) return GBSUB_E_INVALID;
    if (use_device(c->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = cx_launch_templates(c->g, A, f, fdot, (uint32_t)n, q, U, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return dev_err(e);
}

gbsub_status gbsub_set_profiling(gbsub_ctx *c, uint32_t families)
{
    if (!c) return GBSUB_E_INVALID;
    c->profiling = families & ((1u << K_COUNT) - 1u);
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


// ---------------------------------------------------------------- batches

struct gbsub_batch {
    uint32_t max_slots;
    int device;
    Slot *table;                       // device
    Slot *host_table;                  // pinned staging, one entry per slot
    Slot *run_table;                   // device: the running slots, compacted (loop launches)
    Slot *host_run;                    // pinned staging of run_table
    uint32_t n_run;                    // entries of run_table
    bool run_dirty;                    // the running set changed since run_table was written
    Dims run_dims;                     // launch extents of run_table
    Ctl *host_ctls;                    // pinned, one per slot
    Ctl *host_run_ctls;                // pinned, one per entry of run_table
    Ctl *ctl_stage;                    // device: the control blocks of run_table, gathered
    std::vector<uint32_t> run_slot;    // slot of each entry of run_table
    std::vector<gbsub_ctx *> owner;
    std::vector<void *> ws;            // each slot's workspace
    std::vector<uint8_t> state;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint32_t graph_bodies;
    Dims graph_dims;
    hipStream_t graph_stream;
};

namespace {
bool same_dims(const Dims &a, const Dims &b)
{
    return a.ns == b.ns && a.maxB == b.maxB && a.maxnt == b.maxnt && a.maxtile == b.maxtile &&
           a.maxparts == b.maxparts && a.est_mask == b.est_mask && a.naive == b.naive;
}

void drop_graph(gbsub_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

hipError_t enqueue_bodies(const Slot *ds, const Dims &dm, uint32_t n, hipStream_t st)
{
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < n && e == hipSuccess; ++i) {
        e = launch_median(ds, dm, st);
        if (e == hipSuccess) e = launch_snr(ds, dm, st);
        if (e == hipSuccess) e = launch_xupdate(ds, dm, st);
    }
    return e;
}
}  // namespace

gbsub_status gbsub_batch_table_size(uint32_t max_slots, uint64_t *bytes)
{
    if (!bytes || max_slots < 1 || max_slots > 4096) return GBSUB_E_INVALID;
    // all slots, then the running ones, then a staging copy of the running
    // slots' control blocks for the polls
    *bytes = align_up(2 * (uint64_t)max_slots * sizeof(Slot) + (uint64_t)max_slots * sizeof(Ctl));
    return GBSUB_OK;
}

gbsub_status gbsub_batch_create(uint32_t max_slots, void *table, uint64_t table_bytes, gbsub_batch **out)
{
    if (!out) return GBSUB_E_INVALID;
    *out = nullptr;
    uint64_t need = 0;
    if (gbsub_batch_table_size(max_slots, &need) != GBSUB_OK || !table || table_bytes < need ||
        ((uintptr_t)table & 255u) != 0)
        return GBSUB_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GBSUB_E_DEVICE;
    gbsub_batch *b = new (std::nothrow) gbsub_batch();
    if (!b) return GBSUB_E_NOMEM;
    b->max_slots = max_slots;
    b->device = dev;
    b->table = (Slot *)table;
    b->run_table = (Slot *)table + max_slots;
    b->ctl_stage = reinterpret_cast<Ctl *>((Slot *)table + 2 * (size_t)max_slots);
    b->host_run_ctls = nullptr;
    b->run_slot.assign(max_slots, 0u);
    b->host_table = nullptr;
    b->host_run = nullptr;
    b->n_run = 0;
    b->run_dirty = false;
    b->run_dims = Dims{};
    b->host_ctls = nullptr;
    b->owner.assign(max_slots, nullptr);
    b->ws.assign(max_slots, nullptr);
    b->state.assign(max_slots, (uint8_t)GBSUB_SLOT_FREE);
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_bodies = 0;
    b->graph_stream = nullptr;
    if (hipHostMalloc((void **)&b->host_table, sizeof(Slot) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->host_run, sizeof(Slot) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->host_ctls, sizeof(Ctl) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->host_run_ctls, sizeof(Ctl) * max_slots, hipHostMallocDefault) != hipSuccess) {
        gbsub_batch_destroy(b);
        return GBSUB_E_DEVICE;
    }
    std::memset(b->host_table, 0, sizeof(Slot) * max_slots);    // every slot inactive
    if (hipMemcpy(b->table, b->host_table, sizeof(Slot) * max_slots, hipMemcpyHostToDevice) != hipSuccess) {
        gbsub_batch_destroy(b);
        return GBSUB_E_DEVICE;
    }
    *out = b;
    return GBSUB_OK;
}

void gbsub_batch_destroy(gbsub_batch *b)
{
    if (!b) return;
    drop_graph(b);
    for (gbsub_ctx *c : b->owner)
        if (c) c->batch_slot = -1;
    if (b->host_table) (void)hipHostFree(b->host_table);
    if (b->host_run) (void)hipHostFree(b->host_run);
    if (b->host_ctls) (void)hipHostFree(b->host_ctls);
    if (b->host_run_ctls) (void)hipHostFree(b->host_run_ctls);
    delete b;
}

gbsub_status gbsub_batch_admit(gbsub_batch *b, gbsub_ctx *c, const gbsub_catalog *cat, void *ws,
                               uint64_t ws_bytes, void *stream, uint32_t *slot)
{
    if (!b || !slot) return GBSUB_E_INVALID;
    gbsub_status st0 = check_catalog(c, cat, ws, ws_bytes);
    if (st0 != GBSUB_OK) return st0;
    if (c->batch_slot >= 0 || c->device != b->device) return GBSUB_E_INVALID;
    uint32_t k = 0;
    while (k < b->max_slots && b->state[k] != GBSUB_SLOT_FREE) ++k;
    if (k == b->max_slots) return GBSUB_E_NOMEM;
    if (use_device(b->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    Dev d;
    carve(c->g, cat->n, (char *)ws, &d);
    b->host_table[k] = make_slot(c->g, d, cat);
    const Dims one = dims_of(b->host_table[k]);
    Slot *ds = b->table + k;
    hipError_t e = hipMemcpyAsync(ds, &b->host_table[k], sizeof(Slot), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && c->tables_ws != ws) {
        e = launch_grid_tables(ds, one, st);
        if (e == hipSuccess) c->tables_ws = ws;
    }
    if (e == hipSuccess) e = launch_reset(ds, one, st);
    if (e == hipSuccess) e = launch_prep(ds, one, st);
    if (e == hipSuccess) e = launch_xupdate(ds, one, st);
    if (e != hipSuccess) {
        c->tables_ws = nullptr;
        return GBSUB_E_DEVICE;
    }
    c->have_result = false;
    c->batch_slot = (int)k;
    b->owner[k] = c;
    b->ws[k] = ws;
    b->state[k] = GBSUB_SLOT_RUNNING;
    b->run_dirty = true;
    *slot = k;
    return GBSUB_OK;
}

gbsub_status gbsub_batch_step(gbsub_batch *b, uint32_t n, void *stream)
{
    if (!b || n == 0) return GBSUB_E_INVALID;
    if (use_device(b->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    if (b->run_dirty) {
        // loop launches cover the running slots only: a compact descriptor
        // table, grids sized for them, and the median's split threshold
        // shared among them
        if (hipStreamSynchronize(st) != hipSuccess) return GBSUB_E_DEVICE;   // host_run is free
        uint32_t m = 0;
        for (uint32_t k = 0; k < b->max_slots; ++k)
            if (b->owner[k] && b->state[k] == GBSUB_SLOT_RUNNING) {
                b->run_slot[m] = k;
                b->host_run[m++] = b->host_table[k];
            }
        Dims rd{};
        for (uint32_t i = 0; i < m; ++i) {
            Slot &sl = b->host_run[i];
            sl.g.split_tiles = sl.g.split_blocks / ((uint32_t)sl.g.np * m);
            const Dims one = dims_of(sl);
            if (i == 0) rd = one; else widen(rd, one);
        }
        rd.ns = (int)m;
        if (m && hipMemcpyAsync(b->run_table, b->host_run, sizeof(Slot) * m, hipMemcpyHostToDevice, st) != hipSuccess)
            return GBSUB_E_DEVICE;
        b->n_run = m;
        b->run_dims = rd;
        b->run_dirty = false;
    }
    if (b->n_run == 0) return GBSUB_OK;
    if (!st) return enqueue_bodies(b->run_table, b->run_dims, n, st) == hipSuccess ? GBSUB_OK : GBSUB_E_DEVICE;
    if (!b->exec || b->graph_bodies != n || !same_dims(b->graph_dims, b->run_dims) || b->graph_stream != st) {
        drop_graph(b);
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e1 = enqueue_bodies(b->run_table, b->run_dims, n, st);
            e = hipStreamEndCapture(st, &b->graph);
            if (e1 != hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return GBSUB_E_DEVICE;
        }
        b->graph_bodies = n;
        b->graph_dims = b->run_dims;
        b->graph_stream = st;
    }
    return hipGraphLaunch(b->exec, st) == hipSuccess ? GBSUB_OK : GBSUB_E_DEVICE;
}

gbsub_status gbsub_batch_poll(gbsub_batch *b, void *stream, uint8_t *state, uint32_t cap, uint32_t *n_running)
{
    if (!b || !state || cap < b->max_slots) return GBSUB_E_INVALID;
    if (use_device(b->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const bool gathered = !b->run_dirty && b->n_run > 0;
    if (gathered) {
        // only the slots of the last steps can have changed: their control
        // blocks gathered by one kernel, then one copy
        e = launch_gather_ctl(b->run_table, b->n_run, b->ctl_stage, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->host_run_ctls, b->ctl_stage, sizeof(Ctl) * b->n_run, hipMemcpyDeviceToHost, st);
    } else {
        for (uint32_t k = 0; k < b->max_slots && e == hipSuccess; ++k)
            if (b->owner[k])
                e = hipMemcpyAsync(&b->host_ctls[k], b->host_table[k].d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    if (gathered)
        for (uint32_t i = 0; i < b->n_run; ++i) b->host_ctls[b->run_slot[i]] = b->host_run_ctls[i];
    uint32_t running = 0;
    for (uint32_t k = 0; k < b->max_slots; ++k) {
        if (b->owner[k]) {
            const Ctl &h = b->host_ctls[k];
            const uint8_t was = b->state[k];
            b->state[k] = h.bad ? GBSUB_SLOT_INVALID
                        : !h.done ? GBSUB_SLOT_RUNNING
                        : h.status == 6 ? GBSUB_SLOT_MAXITER : GBSUB_SLOT_SETTLED;
            if (was == GBSUB_SLOT_RUNNING && b->state[k] != GBSUB_SLOT_RUNNING) b->run_dirty = true;
            running += b->state[k] == GBSUB_SLOT_RUNNING;
        }
        state[k] = b->state[k];
    }
    if (n_running) *n_running = running;
    return GBSUB_OK;
}

gbsub_status gbsub_batch_retire(gbsub_batch *b, uint32_t k, void *stream, gbsub_summary *out)
{
    if (!b || k >= b->max_slots) return GBSUB_E_INVALID;
    if (!b->owner[k] || b->state[k] == GBSUB_SLOT_RUNNING || b->state[k] == GBSUB_SLOT_FREE)
        return GBSUB_E_STATE;
    if (use_device(b->device) != GBSUB_OK) return GBSUB_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    gbsub_ctx *c = b->owner[k];
    const Slot sl = b->host_table[k];
    Slot *ds = b->table + k;
    const uint8_t outcome = b->state[k];
    hipError_t e = hipSuccess;
    if (outcome == GBSUB_SLOT_SETTLED) e = launch_outputs(ds, dims_of(sl), st);
    if (e == hipSuccess) e = hipMemcpyAsync(&b->host_ctls[k], sl.d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    b->host_table[k].active = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(ds, &b->host_table[k], sizeof(Slot), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return GBSUB_E_DEVICE;
    const Ctl &h = b->host_ctls[k];
    const gbsub_summary s = summary_of(sl.g, h);
    if (out) *out = s;
    b->owner[k] = nullptr;
    const void *wsk = b->ws[k];
    b->ws[k] = nullptr;
    b->state[k] = GBSUB_SLOT_FREE;
    c->batch_slot = -1;
    if (outcome == GBSUB_SLOT_INVALID) return GBSUB_E_INVALID;
    if (outcome == GBSUB_SLOT_MAXITER) return GBSUB_E_MAXITER;
    c->summ = s;
    c->dev = sl.d;
    c->ws = const_cast<void *>(wsk);
    c->n_cand = h.n_cand;
    c->have_result = true;
    return GBSUB_OK;
}

}  // extern "C"
