// gbsub_output.hip -- output kernels of libgbsub: the resolved list and the
// galactic part of the spectrum, computed on the device from the results a
// run leaves in its workspace.
//
// Resolved list (appendix "Subtraction algorithm": the sources taken out,
// with the loop body that took each): stream compaction of the candidate
// records whose loop body is set (per-block counts, one scan, then a ballot
// and prefix inside each block, so the list keeps candidate-slot order),
// then a stable LSD radix sort of the (id, body) pairs by id, 8 bits per
// pass (per-block digit histograms, one scan over (digit, block), a stable
// scatter ranked by ballots inside each wave).

#include "gbsub_internal.h"

namespace gbs {

namespace {

constexpr int OT = 256;              // threads of every output block
constexpr int OE = 16;               // elements per thread
constexpr int OB = OT * OE;          // elements per block
constexpr int SCAN_T = 1024;         // threads of the one-block scan

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

// Count of the resolved candidates of each block of OB slots.
__global__ __launch_bounds__(OT) void k_res_count(const int32_t *iter, uint32_t nc, uint32_t *cnt)
{
    __shared__ uint32_t sw[OT / 64];
    const uint32_t b0 = blockIdx.x * (uint32_t)OB;
    uint32_t c = 0;
    for (int r = 0; r < OE; ++r) {
        const uint32_t j = b0 + (uint32_t)(r * OT) + threadIdx.x;
        c += (j < nc && iter[j] >= 0) ? 1u : 0u;
    }
    for (int o = 32; o >= 1; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
    if (__lane_id() == 0) sw[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = sw[0] + sw[1] + sw[2] + sw[3];
}

// In-place exclusive scan of a[0 .. n) by one block; a[n] gets the total.
__global__ __launch_bounds__(SCAN_T) void k_scan_u32(uint32_t *a, uint32_t n)
{
    __shared__ uint32_t sw[SCAN_T / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (uint32_t base = 0; base < n; base += SCAN_T) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < n ? a[i] : 0u;
        uint32_t inc = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) sw[w] = inc;
        __syncthreads();
        uint32_t pre = carry, tot = 0;
        for (int v = 0; v < SCAN_T / 64; ++v) {
            pre += v < w ? sw[v] : 0u;
            tot += sw[v];
        }
        if (i < n) a[i] = pre + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a[n] = carry;
}

// Writes (id, body) of the resolved candidates of each block from its offset
// off[b], in slot order: per round of OT slots, a ballot gives each lane its
// rank in the wave and a prefix over the waves the wave's start.
__global__ __launch_bounds__(OT) void k_res_scatter(const int32_t *iter, const uint32_t *id, uint32_t nc,
                                                     const uint32_t *off, uint32_t *kout, int32_t *vout)
{
    __shared__ uint32_t sw[OT / 64];
    const int w = threadIdx.x >> 6;
    const uint32_t b0 = blockIdx.x * (uint32_t)OB;
    uint32_t run = off[blockIdx.x];
    for (int r = 0; r < OE; ++r) {
        const uint32_t j = b0 + (uint32_t)(r * OT) + threadIdx.x;
        const int32_t t = j < nc ? iter[j] : -1;
        const bool keep = t >= 0;
        const uint64_t m = (uint64_t)__ballot(keep);
        if (__lane_id() == 0) sw[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int v = 0; v < OT / 64; ++v) {
            pre += v < w ? sw[v] : 0u;
            tot += sw[v];
        }
        if (keep) {
            const uint32_t p = run + pre + (uint32_t)__popcll(m & lanes_below());
            kout[p] = id[j];
            vout[p] = t;
        }
        run += tot;
        __syncthreads();
    }
}

// Digit histogram of each block: hist[d * nb + b] = elements of block b
// whose bits [sh, sh + 8) are d.
__global__ __launch_bounds__(OT) void k_rs_hist(const uint32_t *k, uint32_t m, int sh, uint32_t *hist, uint32_t nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * (uint32_t)OB;
    for (int r = 0; r < OE; ++r) {
        const uint32_t j = b0 + (uint32_t)(r * OT) + threadIdx.x;
        if (j < m) atomicAdd(&h[(k[j] >> sh) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one pass.  Element order inside the block is kept:
// rounds of OT elements; in a round each lane finds the lanes of its wave
// with the same digit (eight ballots, one per digit bit), its rank among the
// lower ones, and the counts of the digit in the waves before its own.
__global__ __launch_bounds__(OT) void k_rs_scatter(const uint32_t *kin, const int32_t *vin, uint32_t m, int sh,
                                                    const uint32_t *hist, uint32_t nb, uint32_t *kout,
                                                    int32_t *vout)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[OT / 64][256];
    const int w = threadIdx.x >> 6;
    run[threadIdx.x] = hist[(size_t)threadIdx.x * nb + blockIdx.x];
    const uint32_t b0 = blockIdx.x * (uint32_t)OB;
    for (int r = 0; r < OE; ++r) {
        for (int v = 0; v < OT / 64; ++v) wc[v][threadIdx.x] = 0;
        __syncthreads();
        const uint32_t j = b0 + (uint32_t)(r * OT) + threadIdx.x;
        const bool in = j < m;
        const uint32_t key = in ? kin[j] : 0u;
        const uint32_t dg = (key >> sh) & 255u;
        uint64_t peers = (uint64_t)__ballot(in);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t ones = (uint64_t)__ballot(in && ((dg >> bit) & 1u));
            peers &= ((dg >> bit) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
        if (in && rank == 0) wc[w][dg] = (uint32_t)__popcll(peers);   // the lowest lane of the group
        __syncthreads();
        if (in) {
            uint32_t pre = 0;
            for (int v = 0; v < OT / 64; ++v) pre += v < w ? wc[v][dg] : 0u;
            const uint32_t p = run[dg] + pre + rank;
            kout[p] = key;
            vout[p] = vin[j];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int v = 0; v < OT / 64; ++v) add += wc[v][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// The control block of each slot of a descriptor table, into out[i].
__global__ __launch_bounds__(64) void k_gather_ctl(const Slot *S, Ctl *out)
{
    static_assert(sizeof(Ctl) % 8 == 0, "Ctl is copied in 8-byte words");
    const uint64_t *src = reinterpret_cast<const uint64_t *>(S[blockIdx.x].d.ctl);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + blockIdx.x);
    for (int w = threadIdx.x; w < (int)(sizeof(Ctl) / 8); w += 64) dst[w] = src[w];
}

__global__ __launch_bounds__(OT) void k_sgal(const double *S, const double *sx, int B, double *out)
{
    const int k = blockIdx.x * OT + threadIdx.x;
    if (k < B) out[k] = S[k] - sx[k];
}

}  // namespace

uint64_t resolved_scratch_words(uint64_t n_max) { return ((n_max + OB - 1) / OB) * 256 + 1; }

hipError_t launch_resolved(const int32_t *iter, const uint32_t *id, uint32_t nc, uint32_t m, uint32_t *hist,
                           uint32_t *kA, int32_t *vA, uint32_t *kB, int32_t *vB, hipStream_t st)
{
    const uint32_t ncb = (nc + OB - 1) / OB;
    if (ncb == 0 || m == 0) return hipSuccess;
    k_res_count<<<ncb, OT, 0, st>>>(iter, nc, hist);
    k_scan_u32<<<1, SCAN_T, 0, st>>>(hist, ncb);
    k_res_scatter<<<ncb, OT, 0, st>>>(iter, id, nc, hist, kA, vA);
    const uint32_t nb = (m + OB - 1) / OB;
    for (int pass = 0; pass < 4; ++pass) {
        const uint32_t *ki = pass & 1 ? kB : kA;
        const int32_t *vi = pass & 1 ? vB : vA;
        uint32_t *ko = pass & 1 ? kA : kB;
        int32_t *vo = pass & 1 ? vA : vB;
        k_rs_hist<<<nb, OT, 0, st>>>(ki, m, 8 * pass, hist, nb);
        k_scan_u32<<<1, SCAN_T, 0, st>>>(hist, 256 * nb);
        k_rs_scatter<<<nb, OT, 0, st>>>(ki, vi, m, 8 * pass, hist, nb, ko, vo);
    }
    return hipGetLastError();
}

hipError_t launch_gather_ctl(const Slot *table, uint32_t n, Ctl *out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    k_gather_ctl<<<n, 64, 0, st>>>(table, out);
    return hipGetLastError();
}

hipError_t launch_sgal(const double *S, const double *sx, int B, double *out, hipStream_t st)
{
    k_sgal<<<(B + OT - 1) / OT, OT, 0, st>>>(S, sx, B, out);
    return hipGetLastError();
}

}  // namespace gbs
