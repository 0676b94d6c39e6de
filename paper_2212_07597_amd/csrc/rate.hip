// rate.hip - rate-based sampling (section 3.2), the scheme the threshold
// sampler is compared with: every byte allocated or freed counts towards the
// next sample, one sample per T bytes, whatever the bytes do to the footprint.
// Deterministic reading: the countdown starts at T instead of a random draw,
// so event i takes floor(V_i / T) - floor(V_(i-1) / T) samples, V being the
// cumulative bytes allocated plus bytes freed by memory events; the samples
// are attributed to the event's line.
//
// Three kernels over the records (one wave per 512-event segment, as in the
// threshold sampler): the volume of each segment; one workgroup's exclusive
// scan of the segment volumes (with the status and the total count); and the
// per-event counts, whose first multiple of T comes from the previous lane's
// quotient, added per line through an LDS cache.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scalene_sampler.h"
#include "sampler_device.h"

namespace smp {
namespace {

constexpr int RATE_SLOTS = 256;            // LDS line cache of the count kernel
constexpr uint32_t NO_LINE = 0xFFFFFFFFu;
constexpr uint64_t VOL_LIMIT = 1ull << 62;  // volumes at or above it: SMP_EOVERFLOW

// Workspace: a header (word 0: flags, bit 0 = a malformed record; words
// 1-16: the scan's span offsets), then one volume per segment (after the
// scan: the volume before the segment, relative to its span).
constexpr uint64_t RATE_HDR = 256;

struct RateRec {
    int64_t delta;
    uint32_t line;
    uint32_t fw;
};

typedef const __attribute__((address_space(1))) uint8_t ru8_t;
typedef const __attribute__((address_space(1))) uint64_t ru64_t;
typedef const __attribute__((address_space(1))) uint32_t ru32_t;

// Lane l's record of window w of the segment at base with nv >= 1 records
// (lanes past nv re-read the last one; their volume is masked).
__device__ __forceinline__ RateRec rate_load(ru8_t* base, int nv, int w) {
    const int k = w * 64 + lane_id();
    ru8_t* p = base + (uint32_t)((k < nv ? k : nv - 1) * 24);
    RateRec r;
    r.delta = (int64_t)*(ru64_t*)p;
    r.line = *(ru32_t*)(p + 12);
    r.fw = *(ru32_t*)(p + 16);
    return r;
}

// |delta| of a well-formed memory record (else 0); bad: a malformed record
// (the checks of the threshold sampler: kind 3, line >= L, delta out of its
// kind's range).
__device__ __forceinline__ uint64_t rate_volume(const RateRec& r, bool valid, uint32_t L, bool& bad) {
    const uint64_t d = (uint64_t)r.delta;
    const uint32_t kind = (r.fw >> 1) & 3;
    const bool okm = d + (uint64_t)(MAX_ABS_DELTA - 1) < (uint64_t)(2 * MAX_ABS_DELTA - 1);
    const bool okc = d < (uint64_t)MAX_ABS_DELTA;
    const bool okt = (d >> 32) == 0;
    const bool good = (r.line < L) & (((kind == 0) & okm) | ((kind == 1) & okc) | ((kind == 2) & okt));
    bad = valid & !good;
    const bool mem = valid & good & (kind == 0);
    return mem ? (r.delta < 0 ? (uint64_t)(-r.delta) : d) : 0;
}

__device__ __forceinline__ int rate_seg_events(uint64_t n, uint64_t j) {
    const uint64_t a = j * SEG;
    return (int)((n - a) < (uint64_t)SEG ? (n - a) : (uint64_t)SEG);
}

__global__ void k_rate_clear(int64_t* counts, uint32_t L, uint64_t* result, uint64_t* flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) gp(counts)[i] = 0;
    if (i < 2) gp(result)[i] = 0;
    if (i == 0) *gp(flags) = 0;
}

// Volume of each segment (one wave per segment).
__global__ __launch_bounds__(BLOCK) void k_rate_sums(const uint8_t* __restrict__ ev, uint64_t n, uint64_t nseg,
                                                     uint32_t L, uint64_t* vol, uint64_t* flags) {
    const uint64_t j = (uint64_t)blockIdx.x * WAVES + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (j >= nseg) return;
    const int nv = rate_seg_events(n, j);
    ru8_t* base = (ru8_t*)(ev + j * SEG * 24);
    RateRec r[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) r[w] = rate_load(base, nv, w);
    uint64_t acc = 0;
    uint64_t badm = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        bool bad;
        acc += rate_volume(r[w], w * 64 + lane_id() < nv, L, bad);  // < 8 x 2^52 per lane
        badm |= ballot(bad);
    }
    const uint64_t s = (uint64_t)wave_sum((int64_t)acc);  // < 2^61
    if (lane_id() == 0) {
        gp(vol)[j] = s;
        if (badm) __hip_atomic_fetch_or(gp(flags), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Exclusive scan of the segment volumes in place, by one workgroup of 16
// waves: wave w scans span w (P consecutive segments) 64 at a time with
// coalesced loads, eight groups in flight, and writes prefixes relative to
// the span start; the span offsets go to hdr[1..16].  The exact total is kept
// as separate sums of the volumes' high and low 32-bit halves, which cannot
// wrap (a segment's volume is below 2^61); every prefix is exact when the
// total is below 2^62, and a larger total is reported as SMP_EOVERFLOW
// (a malformed record wins over it).
__global__ __launch_bounds__(1024) void k_rate_scan(uint64_t* vol, uint64_t nseg, uint64_t P, int64_t T,
                                                    uint64_t* result, uint64_t* hdr) {
    __shared__ uint64_t w_tot[16], w_hi[16], w_lo[16];
    const int wv = threadIdx.x >> 6, l = lane_id();
    const uint64_t b = (uint64_t)wv * P;
    const uint64_t e = b + P < nseg ? b + P : nseg;
    SMP_GLOBAL uint64_t* v = gp(vol);
    uint64_t carry = 0, shi = 0, slo = 0;
    for (uint64_t g = b; g < e; g += 8 * 64) {
        uint64_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint64_t i = g + (uint64_t)(k * 64 + l);
            x[k] = i < e ? v[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            shi += x[k] >> 32;
            slo += x[k] & 0xFFFFFFFFull;
            const uint64_t inc = (uint64_t)wave_incl_sum((int64_t)x[k]);
            const uint64_t i = g + (uint64_t)(k * 64 + l);
            if (i < e) v[i] = carry + inc - x[k];
            carry += readlaneu64(inc, 63);
        }
    }
    shi = (uint64_t)wave_sum((int64_t)shi);
    slo = (uint64_t)wave_sum((int64_t)slo);
    if (l == 0) {
        w_tot[wv] = carry;
        w_hi[wv] = shi;
        w_lo[wv] = slo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t off = 0, H = 0, Lo = 0;
        for (int w = 0; w < 16; ++w) {
            gp(hdr)[1 + w] = off;
            off += w_tot[w];
            H += w_hi[w];  // < 2^53 in all
            Lo += w_lo[w]; // < 2^56 in all
        }
        const bool ovf = H >= (1ull << 30) || (H << 32) + Lo >= VOL_LIMIT;
        const uint64_t f = *gp(hdr);
        gp(result)[1] = (f & 1) ? (uint64_t)SMP_EINVAL : (ovf ? (uint64_t)SMP_EOVERFLOW : (uint64_t)SMP_OK);
        gp(result)[0] = ovf ? 0 : ((H << 32) + Lo) / (uint64_t)T;
    }
}

struct RateCache {
    uint32_t key[RATE_SLOTS];
    unsigned long long cnt[RATE_SLOTS];
};

__device__ __forceinline__ void rate_add(RateCache& c, int64_t* counts, uint32_t line, uint64_t v) {
    const int slot = (int)((line * 2654435761u) >> 24);  // RATE_SLOTS = 256
    uint32_t k = c.key[slot];
    if (k == NO_LINE) k = atomicCAS(&c.key[slot], NO_LINE, line);
    if (k == NO_LINE || k == line)
        atomicAdd(&c.cnt[slot], (unsigned long long)v);
    else
        g_add((uint64_t*)&counts[line], v);
}

// Per-event counts and their per-line sums (grid-stride over segments, one
// wave per segment).  Lane l's count is floor(b_l / T) - floor(b_(l-1) / T),
// b_l the volume through its record; the second quotient is the previous
// lane's first (the previous window's last lane for lane 0).
__global__ __launch_bounds__(BLOCK) void k_rate_count(const uint8_t* __restrict__ ev, uint64_t n, uint64_t nseg,
                                                      uint64_t P, uint32_t L, int64_t T, const uint64_t* vol,
                                                      const uint64_t* hdr, int64_t* counts, const uint64_t* result) {
    __shared__ RateCache c;
    for (int i = threadIdx.x; i < RATE_SLOTS; i += blockDim.x) {
        c.key[i] = NO_LINE;
        c.cnt[i] = 0;
    }
    __syncthreads();
    // nothing to count for a malformed or overflowing trace
    const bool ok = *gp(result + 1) == (uint64_t)SMP_OK;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    const uint64_t uT = (uint64_t)T;
    for (uint64_t j = (uint64_t)blockIdx.x * WAVES + wv; ok && j < nseg; j += stride) {
        const int nv = rate_seg_events(n, j);
        ru8_t* base = (ru8_t*)(ev + j * SEG * 24);
        RateRec r[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) r[w] = rate_load(base, nv, w);
        // the volume before the segment (wave-uniform)
        uint64_t run = readlaneu64(gp(vol)[j] + gp(hdr)[1 + j / P], 0);
        uint64_t q = run / uT;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            bool bad;
            const uint64_t a = rate_volume(r[w], w * 64 + lane_id() < nv, L, bad);
            const uint64_t bv = (uint64_t)wave_incl_sum((int64_t)a) + run;
            const uint64_t qb = bv / uT;
            const uint64_t qa = (uint64_t)wave_shr1((int64_t)qb, (int64_t)q);
            const uint64_t cnt = qb - qa;
            if (cnt) rate_add(c, counts, r[w].line, cnt);
            run = readlaneu64(bv, 63);
            q = readlaneu64(qb, 63);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RATE_SLOTS; i += blockDim.x) {
        const uint32_t k = c.key[i];
        if (k != NO_LINE && c.cnt[i]) g_add((uint64_t*)&counts[k], c.cnt[i]);
    }
}

int g_count_grid = 0;

bool rate_args_ok(const smp_event_t* ev, uint64_t n, int64_t threshold, uint32_t num_lines, int64_t* line_counts,
                  uint64_t* result) {
    return threshold >= 1 && threshold < ((int64_t)1 << 60) && num_lines != 0 && n < 0xFFFFFFFFull && (!n || ev) &&
           line_counts && result;
}

// The launch sequence of one call, with its scratch at ws (RATE_HDR bytes of
// header, then 8 bytes per segment).
int rate_launch(const smp_event_t* ev, uint64_t n, int64_t threshold, uint32_t num_lines, void* ws,
                int64_t* line_counts, uint64_t* result, hipStream_t s) {
    uint64_t* flags = (uint64_t*)ws;
    uint64_t* vol = (uint64_t*)((uint8_t*)ws + RATE_HDR);
    const uint64_t nseg = (n + SEG - 1) / SEG;
    const uint32_t cl = num_lines > 2 ? num_lines : 2;
    // a kernel, not a memset, clears the counts, the result and the flags
    k_rate_clear<<<dim3((cl + 255) / 256), dim3(256), 0, s>>>(line_counts, num_lines, result, flags);
    if (hipGetLastError() != hipSuccess) return SMP_EDEVICE;
    if (nseg == 0) {
        // no events: K = 0, status OK (the clear wrote both)
        return SMP_OK;
    }
    const uint8_t* e = (const uint8_t*)ev;
    k_rate_sums<<<dim3((unsigned)((nseg + WAVES - 1) / WAVES)), dim3(BLOCK), 0, s>>>(e, n, nseg, num_lines, vol, flags);
    const uint64_t P = (nseg + 15) / 16;  // segments per span of the scan
    k_rate_scan<<<dim3(1), dim3(1024), 0, s>>>(vol, nseg, P, threshold, result, flags);
    if (g_count_grid <= 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_rate_count, BLOCK, 0) != hipSuccess)
            return SMP_EDEVICE;
        g_count_grid = cus * (per > 0 ? per : 1);
    }
    const uint64_t wgs = (nseg + WAVES - 1) / WAVES;
    const unsigned grid = (unsigned)(wgs < (uint64_t)g_count_grid ? wgs : (uint64_t)g_count_grid);
    k_rate_count<<<dim3(grid), dim3(BLOCK), 0, s>>>(e, n, nseg, P, num_lines, threshold, vol, flags, line_counts,
                                                    result);
    return hipGetLastError() == hipSuccess ? SMP_OK : SMP_EDEVICE;
}

}  // namespace
}  // namespace smp

// Scratch of the no-allocation entry point: one copy per GPU, held until the
// process ends, shared by every call on that GPU.  Host code never uses this
// name as an address (on the host it only names the symbol); the device
// address comes from hipGetSymbolAddress, once per device.
constexpr uint64_t RATE_SCRATCH_BYTES = smp::RATE_HDR + 8 * (SMP_RATE_NOALLOC_MAX_EVENTS / smp::SEG);
static __device__ __align__(256) uint8_t scratch[RATE_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch (looked up on the device's first
// call, with that device current).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SMP_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SMP_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SMP_OK;
}
}  // namespace

using namespace smp;

extern "C" {

SMP_API uint64_t rate_workspace_bytes(uint64_t n_events) {
    return RATE_HDR + 8 * ((n_events + SEG - 1) / SEG);
}

SMP_API int rate_run(const smp_event_t* ev, uint64_t n, int64_t threshold, uint32_t num_lines, void* workspace,
                     uint64_t workspace_bytes, int64_t* line_counts, uint64_t* result, void* hip_stream) {
    if (!rate_args_ok(ev, n, threshold, num_lines, line_counts, result) || !workspace ||
        workspace_bytes < rate_workspace_bytes(n))
        return SMP_EINVAL;
    return rate_launch(ev, n, threshold, num_lines, workspace, line_counts, result, (hipStream_t)hip_stream);
}

SMP_API int rate_run_noalloc(const smp_event_t* ev, uint64_t n, int64_t threshold, uint32_t num_lines,
                             int64_t* line_counts, uint64_t* result, void* hip_stream) {
    if (!rate_args_ok(ev, n, threshold, num_lines, line_counts, result)) return SMP_EINVAL;
    if (n > SMP_RATE_NOALLOC_MAX_EVENTS) return SMP_ETOOBIG;
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    return rate_launch(ev, n, threshold, num_lines, ws, line_counts, result, (hipStream_t)hip_stream);
}

}  // extern "C"
