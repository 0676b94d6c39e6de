// Device-side data layout and wave64 helpers for the gfx950 sampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smp {

// ---- tiling --------------------------------------------------------------
// A segment is NW windows of 64 events; one wavefront owns a segment at a time
// (lane l of window w holds event 64*w + l of the segment).  The two passes
// that combine segments work on tiles of TILE consecutive segments of one
// trace, one segment per thread.
constexpr int NW = 8;
constexpr int SEG = 64 * NW;
constexpr int WAVES = 4;                 // wavefronts per workgroup of the per-segment passes
constexpr int BLOCK = 64 * WAVES;
constexpr int TILE = 512;                // segments per tile
constexpr int TWAVES = TILE / 64;
constexpr int EMIT_SLOTS = 128;          // emit pass (samples)
constexpr int TRACK_SLOTS = 64;          // and tracked-list pass (mallocs, frees)
constexpr int NCNT = 12;                 // counters cached per slot
constexpr int CHAIN_CAP_MAX = 64;        // chains the all-entry analysis can follow (one per lane)
constexpr uint64_t TILE_MAP_BYTES = 32768;  // map area per tile (in the tracked-list area)

constexpr int64_t MAX_ABS_DELTA = (int64_t)1 << 52;
constexpr int64_t MAX_ABS_F = (int64_t)1 << 61;

// per-line histogram indices (same order as the public SMP_H_* enum)
enum { H_PY = 0, H_NAT, H_GN, H_SN, H_GB, H_SB, H_LEAK_M, H_LEAK_F, H_CS, H_CE, H_PT, H_NT, H_COUNT };
enum { C_PY = 0, C_NAT, C_GN, C_SN, C_GB, C_SB, C_CS, C_CE, C_PT, C_NT, C_LM, C_LF };

// Chain map of a segment over entry offsets: entries in [lo, hi] take no
// sample; every other entry ends at one exit offset (CONST; TOTAL when the
// interval is empty) or depends on the entry (SIM: follow the records).
enum { MAP_SIM = 0, MAP_CONST = 1, MAP_TOTAL = 2 };

// Per-segment values, one int64 plane each (plane p of segment j at
// seg[p * nseg + j]), written once per run by the pass named.
enum {
    // summary pass: sums, extremes of the relative prefixes, chain map (SP_FLG: kind in bits 0-1,
    // bit 2 = copy or timer events present), and the chain after the first forced sample, which is
    // the same for every entry: its node (-1 if none), samples after it, best growth sample after
    // it (value, node or -1), largest sampled footprint after it, last sample node after it (or -1)
    // and the Python footprint there (relative values), the forced window's sample mask after it,
    // the entry offsets [PLO, PHI] that take no sample before it, and the footprint and Python
    // footprint at it
    SP_AF = 0, SP_AP, SP_AC, SP_MXF, SP_MNF, SP_MXP, SP_MNP, SP_LO, SP_HI, SP_KF, SP_FLG,
    SP_FN, SP_ACNT, SP_AGV, SP_AGN, SP_ASMX, SP_ALS, SP_ALP, SP_AMF, SP_PLO, SP_PHI, SP_FFN, SP_PFN,
    // resolve pass: exclusive prefixes, entry and exit offsets of the chain
    SP_F0, SP_P0, SP_C0, SP_EF, SP_XF,
    // chain pass: samples, best growth sample (value, event, ptr), Python footprint at the last sample, flags
    // (BFL_CHAIN until the chain pass has run: the resolve pass writes these planes itself where it can)
    SP_BCNT, SP_BGV, SP_BGI, SP_BGP, SP_LSV, SP_BFL,
    // scan pass: state before the segment (rank base, high-water mark record, flags, last-sample Python footprint)
    SP_XCNT, SP_XHV, SP_XHI, SP_XHP, SP_XFL, SP_XLS,
    NSPLANE
};
constexpr int64_t BFL_CHAIN = 8;

// Look-back status words of one tile (each: 2-bit state | 62-bit payload,
// written once per run; stored plane by plane like the segment values).
enum {
    W_AF = 0, W_AP, W_AC,          // aggregate sums: footprint, Python footprint, copy bytes
    W_IF, W_IP, W_IC,              // inclusive prefixes of the same
    W_XF,                          // exit offset of the chain at the tile end
    W_BCNT, W_BGM, W_BGR, W_BGP,   // aggregate: samples, best growth footprint (2 = present), its event, its ptr
    W_ICNT, W_IGM, W_IGR, W_IGP,   // inclusive of the same
    W_LSA,                         // Python footprint at the tile's last sample (2) or no sample (1)
    W_LSI,                         // Python footprint at the last sample up to the tile's end
    NWORD
};

struct Sample {
    uint32_t event_idx;
    uint32_t line;
    int64_t F;
    int64_t py;
    int64_t nat;
};

struct Tracked {
    uint32_t event_idx;
    uint32_t line;
    uint32_t ptr;
    uint32_t freed;
};

struct Scalars {
    int64_t final_F;
    int64_t peak_F;
    int64_t peak_S;
    uint64_t K;
    uint64_t H;
    uint32_t err;      // bit 0: malformed event, bit 1: overflow, bits 2-3: internal fault
    uint32_t pad;
    uint64_t tmap_done;  // tiles whose tile-map wave has finished (the last one chains them)
    uint64_t reserved;
};

// Per-trace descriptor, built by the host for every launch.
struct Desc {
    const uint8_t* ev;       // n 24-byte records
    uint64_t n;
    int64_t T;
    int64_t Tc;
    int64_t q;
    uint32_t L;
    uint32_t options;
    int32_t tc_shift;        // log2(Tc) if Tc is a power of two, else -1
    uint32_t chain_cap;      // chains the all-entry analysis follows before it gives a segment a SIM map (<= 64)
    uint64_t seg_begin;      // first global segment index of this trace
    uint64_t nseg;
    uint64_t tile_begin;     // first global tile index of this trace
    uint64_t ntile;
    int64_t* seg;            // NSPLANE planes of nseg values
    uint64_t* mask;          // NW sample masks per segment
    uint64_t* tstat;         // NWORD planes of ntile status words
    Sample* samples;         // capacity n + 1
    uint32_t* sample_ptr;    // capacity n + 1, written for tracked samples
    Tracked* tracked;        // capacity n + 1
    uint64_t* tracked_bits;  // by sample rank
    uint64_t* freed_bits;    // by event index
    int64_t* hist;           // H_COUNT * L
    int64_t* leak;           // 4 * L
    uint8_t* gates;          // 2 * L
    Scalars* scal;
    uint64_t* blk;           // compaction block sums
    uint64_t blk_begin;      // first global compaction block of this trace
    uint64_t nblk;
    uint8_t* zero_ptr;       // contiguous range cleared before each launch
    uint64_t zero_bytes;
    uint64_t zero_begin;     // offset of that range in the launch's flattened clear space
    uint64_t line_begin;     // offset of this trace's lines in the flattened line space
    uint32_t tmap;           // 1: tiles that qualify get a tile map before the resolve pass
    uint32_t pad_;
};

// ---- wave64 helpers -------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int readlane32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t readlaneu64(uint64_t v, int l) { return (uint64_t)readlane64((int64_t)v, l); }

__device__ __forceinline__ int shfl32(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
    uint32_t lo = (uint32_t)shfl32((int)(uint32_t)(uint64_t)v, src);
    uint32_t hi = (uint32_t)shfl32((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// DPP move of a 64-bit value (two 32-bit halves).  Lanes whose source is
// outside the row or whose row is masked off receive `old`.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint64_t dpp64(uint64_t v, uint64_t old) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)old, (int)(uint32_t)v, CTRL, ROWS, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(old >> 32), (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

// DPP controls (gfx9 family): row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.
struct OpAdd {
    static constexpr uint64_t id = 0;
    __device__ static int64_t f(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
};
struct OpMax {
    static constexpr uint64_t id = 0x8000000000000000ull;
    __device__ static int64_t f(int64_t a, int64_t b) { return a > b ? a : b; }
};
struct OpMin {
    static constexpr uint64_t id = 0x7FFFFFFFFFFFFFFFull;
    __device__ static int64_t f(int64_t a, int64_t b) { return a < b ? a : b; }
};

// Inclusive wave64 scan: Hillis-Steele inside each row of 16 lanes, then
// row 0's total into row 1 (and row 2's into row 3), then lanes 0-31's total
// into rows 2 and 3.  Must be called with all 64 lanes active.
template <class Op>
__device__ __forceinline__ int64_t wave_scan(int64_t x) {
    x = Op::f(x, (int64_t)dpp64<0x111>((uint64_t)x, Op::id));
    x = Op::f(x, (int64_t)dpp64<0x112>((uint64_t)x, Op::id));
    x = Op::f(x, (int64_t)dpp64<0x114>((uint64_t)x, Op::id));
    x = Op::f(x, (int64_t)dpp64<0x118>((uint64_t)x, Op::id));
    x = Op::f(x, (int64_t)dpp64<0x142, 0xa>((uint64_t)x, Op::id));
    x = Op::f(x, (int64_t)dpp64<0x143, 0xc>((uint64_t)x, Op::id));
    return x;
}

// 64-bit inclusive sum scan as carry-chained DPP adds, in place: each step
// adds the shifted/broadcast value to the lane's own (lanes whose source is
// outside the row, or whose row is masked off, keep their value).  The
// s_nop 1 gives the two wait states a DPP read of a just-written VGPR needs.
__device__ __forceinline__ int64_t wave_incl_sum(int64_t x) {
    uint32_t lo = (uint32_t)(uint64_t)x, hi = (uint32_t)((uint64_t)x >> 32);
    asm volatile(
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:0\n\t"
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_co_u32_dpp %0, vcc, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        : "+v"(lo), "+v"(hi)
        :
        : "vcc");
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// Two (three) inclusive 64-bit sums at once, their DPP steps interleaved: the
// other scans' instructions between two steps of one scan give the DPP read
// its wait states, so only the first step needs an s_nop.
__device__ __forceinline__ void wave_incl_sum2(int64_t& a, int64_t& b) {
    uint32_t alo = (uint32_t)(uint64_t)a, ahi = (uint32_t)((uint64_t)a >> 32);
    uint32_t blo = (uint32_t)(uint64_t)b, bhi = (uint32_t)((uint64_t)b >> 32);
#define SMP_SUM2_STEP(CTRL)                                                    \
    "v_add_co_u32_dpp %0, vcc, %0, %0 " CTRL "\n\t"                              \
    "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " CTRL "\n\t"                        \
    "v_add_co_u32_dpp %2, vcc, %2, %2 " CTRL "\n\t"                              \
    "v_addc_co_u32_dpp %3, vcc, %3, %3, vcc " CTRL "\n\t"
    asm volatile(
        "s_nop 1\n\t"
        SMP_SUM2_STEP("row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM2_STEP("row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM2_STEP("row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM2_STEP("row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM2_STEP("row_bcast:15 row_mask:0xa bank_mask:0xf")
        SMP_SUM2_STEP("row_bcast:31 row_mask:0xc bank_mask:0xf")
        "s_nop 1\n\t"
        : "+v"(alo), "+v"(ahi), "+v"(blo), "+v"(bhi)
        :
        : "vcc");
#undef SMP_SUM2_STEP
    a = (int64_t)(((uint64_t)ahi << 32) | alo);
    b = (int64_t)(((uint64_t)bhi << 32) | blo);
}
__device__ __forceinline__ void wave_incl_sum3(int64_t& a, int64_t& b, int64_t& c) {
    uint32_t alo = (uint32_t)(uint64_t)a, ahi = (uint32_t)((uint64_t)a >> 32);
    uint32_t blo = (uint32_t)(uint64_t)b, bhi = (uint32_t)((uint64_t)b >> 32);
    uint32_t clo = (uint32_t)(uint64_t)c, chi = (uint32_t)((uint64_t)c >> 32);
#define SMP_SUM3_STEP(CTRL)                                                    \
    "v_add_co_u32_dpp %0, vcc, %0, %0 " CTRL "\n\t"                              \
    "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " CTRL "\n\t"                        \
    "v_add_co_u32_dpp %2, vcc, %2, %2 " CTRL "\n\t"                              \
    "v_addc_co_u32_dpp %3, vcc, %3, %3, vcc " CTRL "\n\t"                        \
    "v_add_co_u32_dpp %4, vcc, %4, %4 " CTRL "\n\t"                              \
    "v_addc_co_u32_dpp %5, vcc, %5, %5, vcc " CTRL "\n\t"
    asm volatile(
        "s_nop 1\n\t"
        SMP_SUM3_STEP("row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM3_STEP("row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM3_STEP("row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM3_STEP("row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:0")
        SMP_SUM3_STEP("row_bcast:15 row_mask:0xa bank_mask:0xf")
        SMP_SUM3_STEP("row_bcast:31 row_mask:0xc bank_mask:0xf")
        "s_nop 1\n\t"
        : "+v"(alo), "+v"(ahi), "+v"(blo), "+v"(bhi), "+v"(clo), "+v"(chi)
        :
        : "vcc");
#undef SMP_SUM3_STEP
    a = (int64_t)(((uint64_t)ahi << 32) | alo);
    b = (int64_t)(((uint64_t)bhi << 32) | blo);
    c = (int64_t)(((uint64_t)chi << 32) | clo);
}
__device__ __forceinline__ int64_t wave_incl_max(int64_t x) { return wave_scan<OpMax>(x); }
__device__ __forceinline__ int64_t wave_incl_min(int64_t x) { return wave_scan<OpMin>(x); }

// 32-bit max / min over the wave (DPP steps as in wave_scan, result broadcast).
template <bool MAX>
__device__ __forceinline__ int32_t wave_ext32(int32_t x) {
    const int32_t id = MAX ? INT32_MIN : INT32_MAX;
#define EXT32_STEP(CTRL, ROWS)                                                            \
    {                                                                                     \
        const int32_t y = __builtin_amdgcn_update_dpp(id, x, CTRL, ROWS, 0xf, false);     \
        x = MAX ? (x > y ? x : y) : (x < y ? x : y);                                      \
    }
    EXT32_STEP(0x111, 0xf)
    EXT32_STEP(0x112, 0xf)
    EXT32_STEP(0x114, 0xf)
    EXT32_STEP(0x118, 0xf)
    EXT32_STEP(0x142, 0xa)
    EXT32_STEP(0x143, 0xc)
#undef EXT32_STEP
    return __builtin_amdgcn_readlane(x, 63);
}

// value of the previous lane (lane 0 gets `old`)
__device__ __forceinline__ int64_t wave_shr1(int64_t x, int64_t old) {
    return (int64_t)dpp64<0x138>((uint64_t)x, (uint64_t)old);
}

// unsigned 32-bit max / min over the wave (as wave_ext32)
template <bool MAX>
__device__ __forceinline__ uint32_t wave_extu32(uint32_t x) {
    const uint32_t id = MAX ? 0u : 0xFFFFFFFFu;
#define EXTU32_STEP(CTRL, ROWS)                                                                       \
    {                                                                                                 \
        const uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, CTRL, ROWS, 0xf, false); \
        x = MAX ? (x > y ? x : y) : (x < y ? x : y);                                                  \
    }
    EXTU32_STEP(0x111, 0xf)
    EXTU32_STEP(0x112, 0xf)
    EXTU32_STEP(0x114, 0xf)
    EXTU32_STEP(0x118, 0xf)
    EXTU32_STEP(0x142, 0xa)
    EXTU32_STEP(0x143, 0xc)
#undef EXTU32_STEP
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Signed 64-bit max / min over the wave, exact: the extreme high word (signed),
// then the extreme low word (unsigned) among the lanes that hold it.  Two
// 32-bit reductions cost far fewer instructions than one 64-bit one.
template <bool MAX>
__device__ __forceinline__ int64_t wave_ext64(int64_t x) {
    const int32_t hi = (int32_t)((uint64_t)x >> 32);
    const int32_t mh = wave_ext32<MAX>(hi);
    const uint32_t lo = (uint32_t)(uint64_t)x;
    const uint32_t ml = wave_extu32<MAX>(hi == mh ? lo : (MAX ? 0u : 0xFFFFFFFFu));
    return (int64_t)(((uint64_t)(uint32_t)mh << 32) | ml);
}

// reductions, broadcast
__device__ __forceinline__ int64_t wave_sum(int64_t x) { return readlane64(wave_incl_sum(x), 63); }
__device__ __forceinline__ int64_t wave_max(int64_t x) { return wave_ext64<true>(x); }
__device__ __forceinline__ int64_t wave_min(int64_t x) { return wave_ext64<false>(x); }

// x with lane L's value replaced by the wave-uniform v (v_writelane; this
// compiler exposes no builtin for it).  The lane index is an immediate.
template <int L>
__device__ __forceinline__ int64_t writelane64(int64_t x, int64_t v) {
    uint32_t lo = (uint32_t)(uint64_t)x, hi = (uint32_t)((uint64_t)x >> 32);
    const uint32_t vlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const uint32_t vhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    asm("v_writelane_b32 %0, %2, %4\n\tv_writelane_b32 %1, %3, %4" : "+v"(lo), "+v"(hi) : "s"(vlo), "s"(vhi), "n"(L));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int ctz64(uint64_t m) { return __builtin_ctzll(m); }
__device__ __forceinline__ int top64(uint64_t m) { return 63 - __builtin_clzll(m); }

// ---- status words: 2-bit state in bits 62-63, 62-bit biased payload --------
__device__ __forceinline__ uint64_t pack(int64_t v, uint32_t state) {
    return (((uint64_t)v + ((uint64_t)1 << 61)) & (((uint64_t)1 << 62) - 1)) | ((uint64_t)state << 62);
}
__device__ __forceinline__ int64_t unpack(uint64_t w) {
    return (int64_t)(w & (((uint64_t)1 << 62) - 1)) - ((int64_t)1 << 61);
}
__device__ __forceinline__ uint32_t wstate(uint64_t w) { return (uint32_t)(w >> 62); }

// The tile status words of one trace, stored plane by plane so that a wave
// reading one word of 64 consecutive tiles touches four cache lines.
struct StatusView {
    uint64_t* p;
    int64_t ns;  // tiles in the trace
    __device__ __forceinline__ uint64_t* at(int word, int64_t seg) const { return p + (int64_t)word * ns + seg; }
};

// ---- global memory through global-address-space pointers ------------------
// Descriptor fields are generic pointers; accessed as such they compile to
// flat instructions, which also count against the LDS wait counter, so every
// wait for an LDS result would also wait for outstanding flat stores.
#define SMP_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ SMP_GLOBAL T* gp(T* p) {
    return (SMP_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const SMP_GLOBAL T* gp(const T* p) {
    return (const SMP_GLOBAL T*)p;
}

// relaxed agent-scope atomics on global memory
__device__ __forceinline__ void g_add(uint64_t* p, uint64_t v) {
    __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t g_add_rtn(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_or(uint64_t* p, uint64_t v) {
    __hip_atomic_fetch_or(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_or32(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_or(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_max(int64_t* p, int64_t v) {
    __hip_atomic_fetch_max(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_status(const uint64_t* p) {
    return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
    __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A sample record as four 64-bit words (struct assignment has no overload
// for global-address-space objects).
__device__ __forceinline__ void store_sample(Sample* dst, const Sample& s) {
    SMP_GLOBAL uint64_t* q = (SMP_GLOBAL uint64_t*)dst;
    q[0] = (uint64_t)s.event_idx | ((uint64_t)s.line << 32);
    q[1] = (uint64_t)s.F;
    q[2] = (uint64_t)s.py;
    q[3] = (uint64_t)s.nat;
}
__device__ __forceinline__ Sample load_sample(const Sample* src) {
    const SMP_GLOBAL uint64_t* q = (const SMP_GLOBAL uint64_t*)src;
    const uint64_t w0 = q[0];
    Sample s;
    s.event_idx = (uint32_t)w0;
    s.line = (uint32_t)(w0 >> 32);
    s.F = (int64_t)q[1];
    s.py = (int64_t)q[2];
    s.nat = (int64_t)q[3];
    return s;
}

}  // namespace smp
