// gfx950 kernels of the threshold sampler.
//
// Method (paper sections cited per step):
//  * The footprint F is the running sum of memory-event deltas (section 3.1:
//    every allocation and free is intercepted once, tagged Python or native).
//  * Threshold sampling (section 3.2): after a sample at node r the next one is
//    the first later node j with |F_j - F_r| >= T.  Restated per segment of
//    events: the chain state entering a segment is the reference footprint
//    relative to the segment start, rho in (-T, T); the segment maps it to the
//    state entering the next segment.
//  * Each segment computes that map for all entries at once ("all-entry
//    analysis"): entries that never reach the threshold inside the segment
//    form one interval and are shifted by the segment's footprint change; every
//    other entry starts a chain at a running-maximum or running-minimum node,
//    and chains that sample at the same node coincide from there on.  When all
//    of them coincide the segment's exit is known before its entry is.
//  * Attribution (section 3.3): each sample goes to the triggering event's
//    line with the net Python and native bytes since the previous sample.
//  * Leak rule (section 3.4): a growth sample above the high-water mark of the
//    earlier tracked samples is tracked; frees of its ptr_id before the next
//    tracked sample mark it reclaimed.  The high-water mark and the active
//    tracked object flow between segments as a running "argmax" (the largest
//    growth footprint, earliest on ties).
//  * Copy volume (section 3.5) and the timer split (section 2.1) are
//    per-event histogram updates.
//
// Passes of one launch (no pass over the records waits on another segment):
//   summarize  per segment: sums, prefix extremes, chain map        (records)
//   resolve    per tile:    exclusive sums, entry offset of each segment
//   chain      per segment: samples, best growth sample, last sample (records)
//   scan       per tile:    rank base, high-water mark, last sample before
//   emit       per segment: samples, per-line histograms, leak bits (records)
#include "sampler_device.h"

namespace smp {

__device__ __forceinline__ int cache_to_hist(int c) {
    switch (c) {
        case C_PY: return H_PY;
        case C_NAT: return H_NAT;
        case C_GN: return H_GN;
        case C_SN: return H_SN;
        case C_GB: return H_GB;
        case C_SB: return H_SB;
        case C_CS: return H_CS;
        case C_CE: return H_CE;
        case C_PT: return H_PT;
        case C_NT: return H_NT;
        case C_LM: return H_LEAK_M;
        default: return H_LEAK_F;
    }
}

// Per-workgroup LDS cache of per-line counters, NS slots (a power of two <= 256).
template <int NS>
struct HistCache {
    unsigned long long key[NS];  // (trace << 32) | line, or ~0 when empty
    unsigned long long cnt[NS][NCNT];
};

constexpr unsigned long long EMPTY_KEY = ~0ull;

template <int NS>
__device__ __forceinline__ void hist_init(HistCache<NS>& hc) {
    for (int i = threadIdx.x; i < NS; i += blockDim.x) {
        hc.key[i] = EMPTY_KEY;
        for (int c = 0; c < NCNT; ++c) hc.cnt[i][c] = 0;
    }
}

// Add up to four counters of (trace t, line) through the workgroup's LDS
// cache; a slot held by another line sends the update to global atomics.
template <int NS>
__device__ __forceinline__ void hist_add(HistCache<NS>& hc, const Desc& D, uint32_t t, uint32_t line, int c0,
                                         int64_t v0, int c1, int64_t v1, int c2, int64_t v2, int c3, int64_t v3) {
    const unsigned long long key = ((unsigned long long)t << 32) | line;
    const uint32_t h = (line * 2654435761u) ^ (t * 0x9E3779B9u);
    const int slot = (int)(h >> 24) & (NS - 1);
    unsigned long long k = hc.key[slot];
    if (k == EMPTY_KEY) k = atomicCAS(&hc.key[slot], EMPTY_KEY, key);
    const int cs[4] = {c0, c1, c2, c3};
    const int64_t vs[4] = {v0, v1, v2, v3};
    if (k == EMPTY_KEY || k == key) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (cs[i] >= 0 && vs[i] != 0) atomicAdd(&hc.cnt[slot][cs[i]], (unsigned long long)vs[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (cs[i] >= 0 && vs[i] != 0)
                g_add((uint64_t*)&D.hist[(size_t)cache_to_hist(cs[i]) * D.L + line], (uint64_t)vs[i]);
    }
}

// Move the cache to the per-line histograms (whole workgroup, after a barrier).
template <int NS>
__device__ __forceinline__ void hist_flush(HistCache<NS>& hc, const Desc* desc) {
    for (int i = threadIdx.x; i < NS; i += blockDim.x) {
        const unsigned long long key = hc.key[i];
        if (key == EMPTY_KEY) continue;
        const Desc& D = desc[(uint32_t)(key >> 32)];
        const uint32_t line = (uint32_t)key;
        for (int c = 0; c < NCNT; ++c) {
            const unsigned long long v = hc.cnt[i][c];
            if (v) g_add((uint64_t*)&D.hist[(size_t)cache_to_hist(c) * D.L + line], v);
        }
    }
}

// last trace whose first segment index is <= x
__device__ __forceinline__ int find_trace_seg(const Desc* desc, int lo, int ntraces, uint64_t x) {
    int hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].seg_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// last trace whose first tile index is <= x
__device__ __forceinline__ int find_trace_tile(const Desc* desc, int ntraces, uint64_t x) {
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].tile_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------ event records

// One decoded record (24 bytes: delta i64, ptr u32, line u32, flags u8).
// Flags: bit 0 native (else Python), bits 1-2 kind (0 memory, 1 copy,
// 2 timer).  Memory deltas satisfy |delta| < 2^52, copies 0 <= delta < 2^52,
// timer delays 0 <= delta < 2^32, and line < L; anything else is malformed
// and contributes nothing.
struct Ev {
    int64_t delta;
    int64_t dm;    // footprint delta
    int64_t dp;    // Python footprint delta
    bool mem_ok;   // well-formed memory event
    bool cp;       // well-formed copy event (its bytes: delta)
    bool bad;
    bool aux;      // well-formed copy or timer event
};

// Each kind's range test is made for every lane and the results combined as
// lane masks: cheaper than choosing per-lane bounds by kind.
__device__ __forceinline__ Ev decode(uint64_t r0, uint32_t line, uint32_t fw, bool valid, uint32_t L) {
    Ev e;
    e.delta = (int64_t)r0;
    const uint32_t kind = (fw >> 1) & 3;
    const bool okm = r0 + (uint64_t)(MAX_ABS_DELTA - 1) < (uint64_t)(2 * MAX_ABS_DELTA - 1);
    const bool okc = r0 < (uint64_t)MAX_ABS_DELTA;
    const bool okt = (r0 >> 32) == 0;
    const bool mem = kind == 0, cpy = kind == 1;
    // bitwise, not short-circuit: no branches
    const bool good = valid & (line < L) & ((mem & okm) | (cpy & okc) | ((kind == 2) & okt));
    e.bad = valid & !good;
    e.mem_ok = good & mem;
    e.dm = e.mem_ok ? e.delta : 0;
    e.dp = (fw & 1u) ? 0 : e.dm;
    e.cp = good & cpy;
    e.aux = good & !mem;
    return e;
}

// Global-memory view of the records (the descriptor's generic pointer would
// otherwise compile to flat loads).
typedef const __attribute__((address_space(1))) uint64_t gu64_t;
typedef const __attribute__((address_space(1))) uint8_t gu8_t;

typedef const __attribute__((address_space(1))) int64_t gi64_t;

__device__ __forceinline__ gu64_t* record(const Desc& D, int64_t i) { return (gu64_t*)(D.ev + (size_t)i * 24); }

// Value p of segment j (any lane-varying p; global loads, never flat).
__device__ __forceinline__ int64_t seg_val(const Desc& D, int p, int64_t j) {
    return ((gi64_t*)D.seg)[(int64_t)p * (int64_t)D.nseg + j];
}

// What the summary pass takes from a segment's records.
struct SegScan {
    int64_t sumF, sumP, sumC;
    int64_t mxF, mnF, mxP, mnP;  // extremes of the relative prefixes
    bool any_aux;
    uint32_t err;
};

// A segment's records in registers: lane l holds records 64w + l.  Only the
// words a pass uses are loaded (PTR: the pointer word, LINE: the line word;
// the delta and the flags word always): a loaded word that is never read
// lets the compiler reuse its register while the load is still in flight,
// which makes it wait for every load of the segment before the first window.
struct SegRecs {
    uint64_t d[NW];      // delta
    uint32_t ptr[NW];    // pointer tag
    uint32_t line[NW];
    uint32_t fw[NW];     // flags word (flags in the low byte)
};

typedef const __attribute__((address_space(1))) uint32_t gu32_t;

// Load the words of one record at p into slot w of r.
template <bool PTR, bool LINE>
__device__ __forceinline__ void load_record(gu8_t* p, int w, SegRecs& r) {
    r.d[w] = *(gu64_t*)p;
    if (PTR) r.ptr[w] = *(gu32_t*)(p + 8);
    if (LINE) r.line[w] = *(gu32_t*)(p + 12);
    r.fw[w] = *(gu32_t*)(p + 16);
}

// Address of lane l's record in window w of a segment at base with nv >= 1
// records (lanes past nv re-read record nv-1, a line already fetched).
__device__ __forceinline__ gu8_t* record_addr(gu8_t* base, int nv, int w) {
    const int k = w * 64 + lane_id();
    return base + (uint32_t)((k < nv ? k : nv - 1) * 24);
}

// Issue the loads of one segment's first nv (>= 1) records.  All addresses
// are formed before the first load so that the loads leave back to back.
// Plain loads: the nontemporal hint measured 5-7 % slower on this pattern.
template <bool PTR, bool LINE>
__device__ __forceinline__ void fetch_segment(const Desc& D, int64_t a, int nv, SegRecs& r) {
    gu8_t* base = (gu8_t*)(D.ev + (size_t)a * 24);  // wave-uniform
    gu8_t* ptrs[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) ptrs[w] = record_addr(base, nv, w);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int w = 0; w < NW; ++w) load_record<PTR, LINE>(ptrs[w], w, r);
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ int seg_events(const Desc& D, int64_t j) {
    const uint64_t a = (uint64_t)j * SEG;
    return (int)((D.n - a) < (uint64_t)SEG ? (D.n - a) : (uint64_t)SEG);
}

// ------------------------------------------------------------------- chains

// a > b for wave-uniform values below 2^62 in magnitude, as the sign of
// b - a in scalar arithmetic (the scalar unit has no 64-bit ordered compare,
// so a plain comparison would run on the vector unit).
__device__ __forceinline__ bool sgt64(int64_t a, int64_t b) {
    // the high word's sign (readfirstlane, free on a scalar value, keeps the
    // compiler from turning this back into a 64-bit compare)
    return __builtin_amdgcn_readfirstlane((int)(uint32_t)(((uint64_t)b - (uint64_t)a) >> 32)) < 0;
}

// Lanes whose prefix f is at least T away from ref, from fT = f + (T - 1)
// (formed once per window): |f - ref| >= T as one unsigned compare,
// fT - ref >= 2T - 1 modulo 2^64.  Exact here: prefixes and references stay
// below 2^61 in magnitude and T below 2^61, so the true value of fT - ref lies
// in (-2^63, 2^63) and a negative one wraps above 2^63.
__device__ __forceinline__ uint64_t crossing(int64_t fT, int64_t ref, uint64_t span) {
    return ballot((uint64_t)fT - (uint64_t)ref >= span);
}

// One chain followed through a segment: its reference, sample masks (lane w
// holds window w's mask), the largest growth-sample footprint (earliest on
// ties), the largest sampled footprint and the last sample's index.
struct ChainRun {
    int64_t ref;
    uint64_t mvec;
    int64_t gbest;
    int gnode;
    int64_t smax;
    int lastS;
    int cnt;  // samples recorded
};

// Advance cr through one window whose footprint prefixes f (and Python
// footprint prefixes p) are in registers, after lane st.  FULL also records
// the window's sample mask (lane w), the best growth sample, the largest
// sampled footprint, the last sample node and, in lsp, the Python footprint
// at the last sample.
template <bool FULL>
__device__ __forceinline__ void chain_window(int64_t f, int64_t p, int64_t T, ChainRun& cr, int64_t& lsp, int w,
                                             int st) {
    const int l = lane_id();
    uint64_t m = 0;
    const int64_t fT = (int64_t)((uint64_t)f + (uint64_t)(T - 1));
    const uint64_t span = (uint64_t)(2 * T - 1);
    while (st < 63) {  // (lanes above st: ~0 << (st + 1))
        const uint64_t ex = crossing(fT, cr.ref, span) & (~0ull << (st + 1));
        if (!ex) break;
        const int jj = ctz64(ex);
        const int64_t fj = readlane64(f, jj);
        if (FULL) {
            // (prefixes and references stay below 2^61 in magnitude; smax
            // starts at INT64_MIN)
            if (sgt64(fj, cr.ref) && (cr.gnode < 0 || sgt64(fj, cr.gbest))) {
                cr.gbest = fj;
                cr.gnode = w * 64 + jj;
            }
            if (cr.smax == INT64_MIN || sgt64(fj, cr.smax)) cr.smax = fj;
            m |= 1ull << jj;
            cr.lastS = w * 64 + jj;
        }
        cr.ref = fj;
        st = jj;
    }
    if (FULL && m) {
        lsp = readlane64(p, top64(m));
        if (l == w) cr.mvec |= m;
        cr.cnt += __popcll(m);
    }
}

// Follow one chain through the window held in f (one node per lane), starting
// after lane st.  U holds the lanes where an earlier chain of this window
// sampled; reaching one of them means the chains coincide (returns false).
__device__ __forceinline__ bool follow(int64_t f, int64_t T, int64_t& ref, int st, uint64_t& U) {
    const int64_t fT = (int64_t)((uint64_t)f + (uint64_t)(T - 1));
    const uint64_t span = (uint64_t)(2 * T - 1);
    for (;;) {
        if (st >= 63) return true;
        const uint64_t m = crossing(fT, ref, span) & (~0ull << (st + 1));
        if (!m) return true;
        const int j = ctz64(m);
        if ((U >> j) & 1) return false;
        U |= 1ull << j;
        ref = readlane64(f, j);
        st = j;
    }
}

struct SegMap {
    int64_t lo, hi, kf;
    int kind;
    int fnode;  // first forced event (-1 if none)
};

// All-entry analysis of a segment without forced events (F: relative
// prefixes in LDS), following at most cap distinct chains at once (cap <= 64,
// one per lane; more make the map SIM).
__device__ SegMap analyse_segment(const int64_t* F, int64_t T, int64_t sumF, int cap) {
    const int l = lane_id();
    SegMap m;
    // Entries in [Lo, Hi] have not sampled yet; chain c (lane c < nch) holds
    // the reference of one distinct chain of the entries that have.
    int64_t Lo = -T + 1, Hi = T - 1;
    int nch = 0;
    bool ovf = false;
    int64_t chref = 0;
    for (int w = 0; w < NW; ++w) {
        const int64_t f = F[w * 64 + l];
        if (ovf) {
            if (Lo <= Hi) {
                const int64_t wmx = wave_max(f), wmn = wave_min(f);
                Lo = (wmx - T + 1) > Lo ? (wmx - T + 1) : Lo;
                Hi = (wmn + T - 1) < Hi ? (wmn + T - 1) : Hi;
            }
            continue;
        }
        uint64_t U = 0;
        int nal = 0;
        for (int c = 0; c < nch; ++c) {
            int64_t ref = readlane64(chref, c);
            if (follow(f, T, ref, -1, U)) {
                if (l == nal) chref = ref;
                ++nal;
            }
        }
        if (Lo <= Hi) {
            const int64_t im = wave_incl_max(f), in = wave_incl_min(f);
            const int64_t em = wave_shr1(im, INT64_MIN), en = wave_shr1(in, INT64_MAX);
            // entries still unsampled just before node l
            int64_t lob = Lo, hib = Hi;
            if (l > 0) {
                lob = (em - T + 1) > Lo ? (em - T + 1) : Lo;
                hib = (en + T - 1) < Hi ? (en + T - 1) : Hi;
            }
            const bool ne = lob <= hib;
            const bool up = ne && (f - T >= lob);
            const bool dn = ne && (f + T <= hib);
            // node c is the first sample of some entries: a chain starts there
            uint64_t cm = ballot(up || dn);
            while (cm) {
                const int c = ctz64(cm);
                cm &= cm - 1;
                if ((U >> c) & 1) continue;
                U |= 1ull << c;
                int64_t ref = readlane64(f, c);
                if (follow(f, T, ref, c, U)) {
                    if (nal >= cap) {
                        ovf = true;
                        break;
                    }
                    if (l == nal) chref = ref;
                    ++nal;
                }
            }
            const int64_t wmx = readlane64(im, 63), wmn = readlane64(in, 63);
            Lo = (wmx - T + 1) > Lo ? (wmx - T + 1) : Lo;
            Hi = (wmn + T - 1) < Hi ? (wmn + T - 1) : Hi;
        }
        nch = ovf ? 0 : nal;
    }
    if (Lo > T) Lo = T;
    if (Hi < -T) Hi = -T;
    const bool has_const = !ovf && nch == 1;
    m.fnode = -1;
    m.lo = Lo;
    m.hi = Hi;
    m.kf = has_const ? readlane64(chref, 0) - sumF : 0;
    m.kind = has_const ? (Lo > Hi ? MAP_TOTAL : MAP_CONST) : MAP_SIM;
    return m;
}

// ---------------------------------------------------------------- look-backs

// Every wait on another tile's status polls with a budget and an exponential
// back-off.  Running out of budget (only possible through an internal fault)
// raises the launch-wide abort word, after which every wait returns at once,
// so all waves always exit.
constexpr uint32_t SPIN_BUDGET = 1u << 24;

struct Spin {
    uint32_t budget = SPIN_BUDGET;
    uint32_t reps = 1;
};

__device__ __forceinline__ bool spin_abort(unsigned long long* ctl, Spin& sp) {
    if (ld_status((const uint64_t*)&ctl[1])) return true;
    for (uint32_t i = 0; i < sp.reps; ++i) __builtin_amdgcn_s_sleep(4);
    if (sp.reps < 8) sp.reps <<= 1;
    if (--sp.budget == 0) {
        st_status((uint64_t*)&ctl[1], 1);
        return true;
    }
    return false;
}

// A wait on a flag in LDS (set by another wave of the same workgroup) polls
// with a short sleep and checks the abort word and the budget only every 64
// polls: the exponential back-off above would add up to a microsecond to
// every hand-off.
struct LocalSpin {
    Spin sp;
    uint32_t n = 0;
};

__device__ __forceinline__ bool local_spin_abort(unsigned long long* ctl, LocalSpin& s) {
    __builtin_amdgcn_s_sleep(1);
    if ((++s.n & 63) != 0) return false;
    return spin_abort(ctl, s.sp);
}

// Wait until a status word is published (wave-uniform address).
__device__ bool wait_word(const uint64_t* p, int64_t& v, unsigned long long* ctl) {
    Spin sp;
    for (;;) {
        const uint64_t w = ld_status(p);
        if (wstate(w)) {
            v = unpack(w);
            return true;
        }
        if (spin_abort(ctl, sp)) return false;
    }
}

// Decoupled look-backs over tiles.  Tile g looks at its predecessors g-1-l
// (lane l, nearest first): it needs the nearest one that has published an
// inclusive value and the aggregates of all tiles after it.  Having them, it
// also publishes the inclusive values of those intermediate tiles
// ("helping").  Identical values may be written by several waves.

// Exclusive (F, P, C) prefix of tile g.
__device__ bool scan_sums(const StatusView& sv, int64_t g, int64_t& oF, int64_t& oP, int64_t& oC,
                          unsigned long long* ctl) {
    const int l = lane_id();
    {
        uint64_t v = 0;
        if (l < 3) v = ld_status(sv.at(W_IF + l, g - 1));
        if ((ballot(l < 3 && wstate(v)) & 7ull) == 7ull) {
            oF = unpack(readlaneu64(v, 0));
            oP = unpack(readlaneu64(v, 1));
            oC = unpack(readlaneu64(v, 2));
            return true;
        }
    }
    int64_t accF = 0, accP = 0, accC = 0;
    int64_t base = g - 1;
    bool first = true;
    Spin sp;
    while (base >= 0) {
        const int64_t jj = base - l;
        const bool in = jj >= 0;
        const int64_t js = in ? jj : 0;
        const uint64_t iF = in ? ld_status(sv.at(W_IF, js)) : 0;
        const uint64_t im = ballot(in && wstate(iF));
        const int lim = im ? ctz64(im) : __popcll(ballot(in));
        const bool need = in && l < lim;
        const bool at = im && l == lim;
        uint64_t x0 = 0, x1 = 0, x2 = 0;  // aggregate (need) or inclusive (at) words
        bool have = !(need || at);
        for (;;) {
            if (!have) {
                if (need) {
                    x0 = ld_status(sv.at(W_AF, js));
                    x1 = ld_status(sv.at(W_AP, js));
                    x2 = ld_status(sv.at(W_AC, js));
                } else {
                    x0 = iF;
                    x1 = ld_status(sv.at(W_IP, js));
                    x2 = ld_status(sv.at(W_IC, js));
                }
                have = wstate(x0) && wstate(x1) && wstate(x2);
            }
            if (!ballot(!have)) break;
            if (spin_abort(ctl, sp)) return false;
        }
        const int64_t vF = (need || at) ? unpack(x0) : 0;
        const int64_t vP = (need || at) ? unpack(x1) : 0;
        const int64_t vC = (need || at) ? unpack(x2) : 0;
        // suffix sums toward older tiles: S_l = sum over lanes >= l
        int64_t xF = vF, xP = vP, xC = vC;
        wave_incl_sum3(xF, xP, xC);
        const int64_t tF = readlane64(xF, 63), tP = readlane64(xP, 63), tC = readlane64(xC, 63);
        if (first && im && need) {
            st_status(sv.at(W_IF, js), pack(tF - xF + vF, 1));
            st_status(sv.at(W_IP, js), pack(tP - xP + vP, 1));
            st_status(sv.at(W_IC, js), pack(tC - xC + vC, 1));
        }
        accF += tF;
        accP += tP;
        accC += tC;
        if (im) break;
        base -= 64;
        first = false;
    }
    oF = accF;
    oP = accP;
    oC = accC;
    return true;
}

// (count, best growth record) items, combined in segment order: counts add;
// the record with the larger footprint wins, the earlier one on ties.  The
// state before a trace is a high-water mark of 0 with nothing tracked.
struct Best {
    int64_t cnt;
    bool has;
    int64_t val;
    uint32_t idx, ptr;
};

__device__ __forceinline__ Best with_baseline(Best b) {
    if (b.has && b.val <= 0) b.has = false;  // a high-water mark of 0 beats it
    if (!b.has) b.val = 0;
    return b;
}

// a, then b
__device__ __forceinline__ Best combine(const Best& a, const Best& b) {
    Best r = a;
    r.cnt = a.cnt + b.cnt;
    if (b.has && (!a.has || b.val > a.val)) {
        r.has = true;
        r.val = b.val;
        r.idx = b.idx;
        r.ptr = b.ptr;
    }
    return r;
}

// value of lane l + d (lanes past 63 get `fill`)
__device__ __forceinline__ int64_t lane_down(int64_t x, int d, int64_t fill) {
    const int l = lane_id();
    const int64_t y = shfl64(x, l + d < 64 ? l + d : l);
    return l + d < 64 ? y : fill;
}

// Exclusive Best prefix of tile g (baseline applied), loading as scan_sums.
__device__ bool scan_best(const StatusView& sv, int64_t g, Best& out, unsigned long long* ctl) {
    const int l = lane_id();
    {
        uint64_t v = 0;
        if (l < 4) v = ld_status(sv.at(W_ICNT + l, g - 1));
        if ((ballot(l < 4 && wstate(v)) & 15ull) == 15ull) {
            const uint64_t wg = readlaneu64(v, 1);
            out.cnt = unpack(readlaneu64(v, 0));
            out.has = wstate(wg) == 2;
            out.val = unpack(wg);
            out.idx = (uint32_t)unpack(readlaneu64(v, 2));
            out.ptr = (uint32_t)unpack(readlaneu64(v, 3));
            out = with_baseline(out);
            return true;
        }
    }
    Best acc{0, false, 0, 0, 0};  // later tiles combined so far
    int64_t base = g - 1;
    bool first = true;
    Spin sp;
    while (base >= 0) {
        const int64_t jj = base - l;
        const bool in = jj >= 0;
        const int64_t js = in ? jj : 0;
        const uint64_t ic = in ? ld_status(sv.at(W_ICNT, js)) : 0;
        const uint64_t im = ballot(in && wstate(ic));
        const int lim = im ? ctz64(im) : __popcll(ballot(in));
        const bool need = in && l < lim;
        const bool at = im && l == lim;
        uint64_t c = 0, gm = 0, gr = 0, gp = 0;
        bool have = !(need || at);
        for (;;) {
            if (!have) {
                if (need) {
                    c = ld_status(sv.at(W_BCNT, js));
                    gm = ld_status(sv.at(W_BGM, js));
                    gr = ld_status(sv.at(W_BGR, js));
                    gp = ld_status(sv.at(W_BGP, js));
                } else {
                    c = ic;
                    gm = ld_status(sv.at(W_IGM, js));
                    gr = ld_status(sv.at(W_IGR, js));
                    gp = ld_status(sv.at(W_IGP, js));
                }
                have = wstate(c) && wstate(gm) && wstate(gr) && wstate(gp);
            }
            if (!ballot(!have)) break;
            if (spin_abort(ctl, sp)) return false;
        }
        const bool use = need || at;
        const int64_t cnt = use ? unpack(c) : 0;
        const bool has = use && wstate(gm) == 2;
        const int64_t val = has ? unpack(gm) : INT64_MIN;
        const uint32_t idx = (uint32_t)unpack(gr), ptr = (uint32_t)unpack(gp);
        // suffix (toward older) counts and maxima
        const int64_t xc = wave_incl_sum(cnt);
        const int64_t tc = readlane64(xc, 63);
        const int64_t rev = shfl64(val, 63 - l);
        const int64_t M = shfl64(wave_incl_max(rev), 63 - l);  // max over lanes >= l
        // the earliest holder of M for lane l is the first lane >= l where the
        // suffix maximum drops (or the last lane)
        const int64_t Mn = lane_down(M, 1, INT64_MIN);
        const uint64_t bnd = ballot(M != INT64_MIN && M > Mn);
        const uint64_t ge = bnd & ~lanemask_lt();
        const int src = ge ? ctz64(ge) : l;
        const uint32_t sidx = (uint32_t)shfl32((int)idx, src), sptr = (uint32_t)shfl32((int)ptr, src);
        if (first && im && need) {
            Best inc{tc - xc + cnt, M != INT64_MIN, M, sidx, sptr};
            inc = with_baseline(inc);
            st_status(sv.at(W_ICNT, js), pack(inc.cnt, 1));
            st_status(sv.at(W_IGM, js), pack(inc.val, inc.has ? 2 : 1));
            st_status(sv.at(W_IGR, js), pack((int64_t)inc.idx, 1));
            st_status(sv.at(W_IGP, js), pack((int64_t)inc.ptr, 1));
        }
        // the whole window (lane 0's suffix) comes before everything in acc
        Best win;
        win.cnt = tc;
        const int64_t M0 = readlane64(M, 0);
        win.has = M0 != INT64_MIN;
        win.val = M0;
        win.idx = (uint32_t)readlane32((int)sidx, 0);
        win.ptr = (uint32_t)readlane32((int)sptr, 0);
        acc = combine(win, acc);
        if (im) break;
        base -= 64;
        first = false;
    }
    out = with_baseline(acc);
    return true;
}

// Python footprint at the last sample before tile g (0 if none).
__device__ bool scan_last_sample(const StatusView& sv, int64_t g, int64_t& oP, unsigned long long* ctl) {
    const int l = lane_id();
    int64_t base = g - 1;
    bool first = true;
    Spin sp;
    while (base >= 0) {
        const int64_t jj = base - l;
        const bool in = jj >= 0;
        const int64_t js = in ? jj : 0;
        uint64_t li = 0, la = 0;
        if (in) {
            li = ld_status(sv.at(W_LSI, js));
            la = ld_status(sv.at(W_LSA, js));
        }
        // a lane resolves the search if its tile has a sample or a known exit value
        const bool hit = in && (wstate(la) == 2 || wstate(li) != 0);
        const uint64_t hm = ballot(hit);
        const int lim = hm ? ctz64(hm) : __popcll(ballot(in));
        if (ballot(in && l < lim && wstate(la) == 0)) {
            if (spin_abort(ctl, sp)) return false;
            continue;
        }
        if (hm) {
            const uint64_t src_w = wstate(readlaneu64(la, lim)) == 2 ? readlaneu64(la, lim) : readlaneu64(li, lim);
            const int64_t v = unpack(src_w);
            if (first && in && l < lim && wstate(li) == 0) st_status(sv.at(W_LSI, js), pack(v, 1));
            oP = v;
            return true;
        }
        base -= 64;
        first = false;
    }
    oP = 0;
    return true;
}

// ------------------------------------------------------------ summary pass

// Sums, extremes of the relative prefixes and the chain map of segment g.
// An event with |delta| >= 2T-1 samples for every entry state, so from the
// first such event on the chain is the same for all entries: it is followed
// here, window by window while scanning, with its samples recorded for the
// chain and emit passes.  Segments without one get the all-entry analysis
// over the prefixes kept in LDS.
// The footprint prefixes of SIM segments, kept for the resolve pass in the
// sample area (written only later, by the emit pass): segment j at
// samples + 4 KB * j.  A trace of fewer than 127 events has too small an
// area; the resolve pass then scans such segments from their records.
__device__ __forceinline__ bool prefixes_kept(const Desc& D) {
    return (D.n + 1) * sizeof(Sample) >= (uint64_t)D.nseg * SEG * sizeof(int64_t);
}
__device__ __forceinline__ SMP_GLOBAL int64_t* kept_prefixes(const Desc& D, int64_t j) {
    return gp((int64_t*)D.samples) + j * SEG;
}

__device__ __forceinline__ void summarize_segment(const Desc& D, uint64_t g, int64_t* lF_) {
    const int l = lane_id();
    const int64_t j = (int64_t)(g - D.seg_begin);
    const int64_t a = j * SEG;
    const int nv = seg_events(D, j);
    SegRecs rr;
    fetch_segment<false, true>(D, a, nv, rr);
    const int64_t T = D.T;
    const int64_t two_t = 2 * T - 1;
    int64_t cF = 0, cP = 0, accC = 0;
    int64_t mxF = INT64_MIN, mnF = INT64_MAX, mxP = INT64_MIN, mnP = INT64_MAX;
    uint64_t bad_m = 0, aux_m = 0, cp_m = 0;  // lanes that saw such a record
    int fnode = -1;
    int64_t plo = -T + 1, phi = T - 1, ffn = 0, pfn = 0;
    ChainRun r{0, 0, 0, -1, INT64_MIN, -1, 0};
    int64_t alp = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int k = w * 64 + l;
        const bool valid = k < nv;
        const Ev e = decode(rr.d[w], rr.line[w], rr.fw[w], valid, D.L);
        // malformed, copy and timer records are rare: one test per window
        if (ballot(valid & !e.mem_ok)) {
            bad_m |= ballot(e.bad);
            aux_m |= ballot(e.aux);
            const uint64_t cpw = ballot(e.cp);
            cp_m |= cpw;
            if (cpw) accC += e.cp ? e.delta : 0;
        }
        // forced: |dm| >= 2T - 1, as one unsigned compare (as in crossing)
        const uint64_t fm = ballot((uint64_t)e.dm + (uint64_t)(two_t - 1) >= (uint64_t)(2 * two_t - 1));
        int64_t f = e.dm, p = e.dp;
        wave_incl_sum2(f, p);
        f += cF;
        p += cP;
        cF = readlane64(f, 63);
        cP = readlane64(p, 63);
        lF_[k] = f;
        if (fnode < 0 && fm) {
            // The first forced event: entries in [plo, phi] take no sample
            // before it (the prefix's extremes: earlier windows, then the
            // lanes before it in this one).
            const int fl = ctz64(fm);
            fnode = w * 64 + fl;
            if (fnode > 0) {
                int64_t pmx, pmn;
                if (w == 0 && !ballot(l < fl && (f > INT32_MAX || f < INT32_MIN))) {
                    // the usual case: a first-window prefix of 32-bit values
                    pmx = wave_ext32<true>(l < fl ? (int32_t)f : INT32_MIN);
                    pmn = wave_ext32<false>(l < fl ? (int32_t)f : INT32_MAX);
                } else {
                    pmx = wave_max(l < fl && f > mxF ? f : mxF);
                    pmn = wave_min(l < fl && f < mnF ? f : mnF);
                }
                plo = pmx > 0 ? pmx - T + 1 : -T + 1;
                phi = pmn < 0 ? pmn + T - 1 : T - 1;
            }
            ffn = readlane64(f, fl);
            pfn = readlane64(p, fl);
            r.ref = ffn;
        }
        // lanes past the segment end hold its last prefixes, which are
        // prefixes too: no lane mask needed
        mxF = f > mxF ? f : mxF;
        mnF = f < mnF ? f : mnF;
        mxP = p > mxP ? p : mxP;
        mnP = p < mnP ? p : mnP;
        if (fnode >= w * 64) {
            // the chain from the forced event (the same for every entry)
            chain_window<true>(f, p, T, r, alp, w, fnode - w * 64);
        } else if (fnode >= 0) {
            chain_window<true>(f, p, T, r, alp, w, -1);
        }
    }
    SegScan sc;
    sc.sumF = cF;
    sc.sumP = cP;
    sc.sumC = cp_m ? wave_sum(accC) : 0;
    sc.mxF = wave_max(mxF);
    sc.mnF = wave_min(mnF);
    sc.mxP = wave_max(mxP);
    sc.mnP = wave_min(mnP);
    sc.any_aux = aux_m != 0;
    sc.err = bad_m ? 1u : 0u;
    SegMap m;
    if (fnode >= 0) {
        m.lo = 1;
        m.hi = 0;
        m.kf = r.ref - cF;
        m.kind = MAP_TOTAL;
        m.fnode = fnode;
    } else {
        m = analyse_segment(lF_, T, cF, (int)D.chain_cap);
        if (m.kind == MAP_SIM && prefixes_kept(D)) {
            SMP_GLOBAL int64_t* o = kept_prefixes(D, j);
#pragma unroll
            for (int w = 0; w < NW; ++w) o[w * 64 + l] = lF_[w * 64 + l];
        }
    }
    const int64_t acnt = r.cnt;
    const int64_t amf = fnode >= 0 ? (int64_t)readlaneu64(r.mvec, fnode >> 6) : 0;
    // the plane values (all wave-uniform) into lanes 0..SP_PFN, one store
    int64_t v = 0;
    v = writelane64<SP_AF>(v, sc.sumF);
    v = writelane64<SP_AP>(v, sc.sumP);
    v = writelane64<SP_AC>(v, sc.sumC);
    v = writelane64<SP_MXF>(v, sc.mxF);
    v = writelane64<SP_MNF>(v, sc.mnF);
    v = writelane64<SP_MXP>(v, sc.mxP);
    v = writelane64<SP_MNP>(v, sc.mnP);
    v = writelane64<SP_LO>(v, m.lo);
    v = writelane64<SP_HI>(v, m.hi);
    v = writelane64<SP_KF>(v, m.kf);
    v = writelane64<SP_FLG>(v, m.kind | (sc.any_aux ? 4 : 0));
    v = writelane64<SP_FN>(v, m.fnode);
    v = writelane64<SP_ACNT>(v, acnt);
    v = writelane64<SP_AGV>(v, r.gbest);
    v = writelane64<SP_AGN>(v, r.gnode);
    v = writelane64<SP_ASMX>(v, r.smax);
    v = writelane64<SP_ALS>(v, r.lastS);
    v = writelane64<SP_ALP>(v, r.lastS >= 0 ? alp : 0);
    v = writelane64<SP_AMF>(v, amf);
    v = writelane64<SP_PLO>(v, plo);
    v = writelane64<SP_PHI>(v, phi);
    v = writelane64<SP_FFN>(v, ffn);
    v = writelane64<SP_PFN>(v, pfn);
    if (l <= SP_PFN) gp(D.seg)[(int64_t)l * (int64_t)D.nseg + j] = v;
    if (fnode >= 0 && l < NW) gp(D.mask)[j * NW + l] = r.mvec;
    if (sc.err && l == 0) g_or32(&D.scal->err, sc.err);
}

// One wave per segment, one launch wave per segment (measured faster here
// than a grid-stride loop: the hardware starts a new wave's loads while
// others compute).
__global__ __launch_bounds__(BLOCK) void k_summarize(const Desc* __restrict__ desc, int ntraces,
                                                     uint64_t nseg_total) {
    __shared__ int64_t lF[WAVES][SEG];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const uint64_t g = (uint64_t)blockIdx.x * WAVES + wv;
    if (g >= nseg_total) return;
    summarize_segment(desc[__builtin_amdgcn_readfirstlane(find_trace_seg(desc, 0, ntraces, g))], g, lF[wv]);
}

// ------------------------------------------------------------ resolve pass

constexpr int RING = 12;  // SIM segments pre-scanned ahead of the walker

// Relative footprint prefixes of segment j into F (one wave; lanes past the
// segment end hold its last prefix).
// Two halves of four windows each, to keep the register footprint small.
__device__ __forceinline__ void prescan_segment(const Desc& D, int64_t j, int64_t* F) {
    const int l = lane_id();
    const int nv = seg_events(D, j);
    gu8_t* base = (gu8_t*)(D.ev + (size_t)j * SEG * 24);
    int64_t cF = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint64_t q0[NW / 2];
        uint32_t q2[NW / 2];
#pragma unroll
        for (int w = 0; w < NW / 2; ++w) {
            gu8_t* p = record_addr(base, nv, h * NW / 2 + w);
            q0[w] = *(gu64_t*)p;
            q2[w] = *(gu32_t*)(p + 16);
        }
#pragma unroll
        for (int w = 0; w < NW / 2; ++w) {
            const int k = (h * NW / 2 + w) * 64 + l;
            const uint32_t fl = q2[w];
            const int64_t dm = (k < nv && (fl & 6u) == 0) ? (int64_t)q0[w] : 0;
            const int64_t f = wave_incl_sum(dm) + cF;
            cF = readlane64(f, 63);
            F[k] = f;
        }
    }
}

// The kept prefixes of segment j into F (one wave, one round trip).
__device__ __forceinline__ void copy_prefixes(const Desc& D, int64_t j, int64_t* F) {
    const int l = lane_id();
    const SMP_GLOBAL int64_t* src = kept_prefixes(D, j);
    int64_t v[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) v[w] = src[w * 64 + l];
#pragma unroll
    for (int w = 0; w < NW; ++w) F[w * 64 + l] = v[w];
}

// Exit offset of a segment from entry offset x, following its prefixes F
// window by window (read four windows at a time, so that the LDS reads
// overlap).  A round-based search over all windows at once measured slower:
// walked segments often hold many samples.
__device__ __forceinline__ int64_t walk_prefixes(const int64_t* F, int64_t T, int64_t x) {
    const int l = lane_id();
    const int64_t fend = F[SEG - 1];
    int64_t lsp = 0;
    ChainRun cr{x, 0, 0, -1, INT64_MIN, -1, 0};
#pragma unroll
    for (int h = 0; h < NW; h += 4) {
        int64_t f[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) f[w] = F[(h + w) * 64 + l];
#pragma unroll
        for (int w = 0; w < 4; ++w) chain_window<false>(f[w], 0, T, cr, lsp, h + w, -1);
    }
    return cr.ref - fend;
}

// The kept prefixes of segment j into registers (the loads are issued here;
// the first use of f waits for them).
__device__ __forceinline__ void load_kept(const Desc& D, int64_t j, int64_t (&f)[NW]) {
    const int l = lane_id();
    const SMP_GLOBAL int64_t* F = kept_prefixes(D, j);
#pragma unroll
    for (int w = 0; w < NW; ++w) f[w] = F[w * 64 + l];
}

// Exit offset from entry offset x, following prefixes held in registers.
__device__ __forceinline__ int64_t walk_regs(const int64_t (&f)[NW], int64_t T, int64_t x) {
    int64_t lsp = 0;
    ChainRun cr{x, 0, 0, -1, INT64_MIN, -1, 0};
#pragma unroll
    for (int w = 0; w < NW; ++w) chain_window<false>(f[w], 0, T, cr, lsp, w, -1);
    return cr.ref - readlane64(f[NW - 1], 63);
}

// Exit offset from entry offset x of a segment that moves less than T (its
// prefixes f in registers) when x lies outside its no-sample interval: the
// chain samples once, at the first node at least T above x (x below the
// interval) or at least T below it (above), and never again in the segment.
// The eight windows are tested at once, not one after another.
__device__ __forceinline__ int64_t exit_one_sample(const int64_t (&f)[NW], int64_t T, int64_t x, bool up) {
    uint64_t m[NW];
    if (up) {  // (wave-uniform: one set of compares, not both and a select)
        const int64_t thr = x + T;
#pragma unroll
        for (int w = 0; w < NW; ++w) m[w] = ballot(f[w] >= thr);
    } else {
        const int64_t thr = x - T;
#pragma unroll
        for (int w = 0; w < NW; ++w) m[w] = ballot(f[w] <= thr);
    }
    int64_t fu = x;  // (unreachable for a stop: some node crosses)
#pragma unroll
    for (int w = NW - 1; w >= 0; --w)
        if (m[w]) fu = readlane64(f[w], ctz64(m[w]));
    return fu - readlane64(f[NW - 1], 63);
}

// The same from the kept prefixes in HBM (all windows loaded at once).
__device__ __forceinline__ int64_t walk_kept(const Desc& D, int64_t j, int64_t T, int64_t x) {
    int64_t f[NW];
    load_kept(D, j, f);
    return walk_regs(f, T, x);
}

// Index of the r-th set bit (r < popcount(m)).
__device__ __forceinline__ int nth_bit(uint64_t m, int r) {
    for (; r > 0; --r) m &= m - 1;
    return ctz64(m);
}

// Lanes [lo, hi) of wave w as a mask (tile-wide lane indices).
__device__ __forceinline__ uint64_t range_mask(int w, int lo, int hi) {
    const int a = lo - w * 64, b = hi - w * 64;
    const uint64_t ma = a <= 0 ? ~0ull : (a >= 64 ? 0ull : (~0ull << a));
    const uint64_t mb = b >= 64 ? ~0ull : (b <= 0 ? 0ull : ((1ull << b) - 1));
    return ma & mb;
}

// ------------------------------------------------------------ tile maps
//
// A tile whose segments each move less than T (every SIM map holds at least
// T entries in its no-sample interval) lets an entry sample at most once per
// segment.  For such a tile the chain map over all entry offsets of
// the whole tile is computed by one wave, segment by segment, before the
// resolve pass (section 3.2's rule, restated over entries as in the segment
// analysis):
//  * entries that have not sampled yet form one interval U, which shrinks as
//    the tile's running maximum and minimum footprint grow apart;
//  * at each new running maximum (minimum) node while U is not empty, the
//    entries of U at least T below (above) that node sample there: they form
//    one source interval and start a chain whose reference is that node's
//    footprint;
//  * a chain outside a segment's no-sample interval samples once in it, at
//    the first node at least T above (below) its reference;
//  * chains that sample at the same node coincide from there on and are
//    merged (their sources are joined in a union-find forest).
// Source intervals started at maxima lie below U and grow upward in start
// order; those started at minima lie above it and grow downward.  Runs of
// consecutive sources that end at the same reference are written as (bound,
// exit) pairs, so that the tile's exit for any entry is one search.  The
// last of a trace's tile waves to finish then chains the trace's tile entries
// through the maps in tile order and publishes every tile's exit, so that the
// resolve pass no longer waits for the previous tile's walk.  A tile that
// does not qualify, or whose chains or runs exceed the capacities below, gets
// no map; the resolve pass chains the tiles from it on, by a map lookup where
// a tile has one and by its walk where not.

constexpr int TM_CAP = 1024;   // chains followed at once
constexpr int TM_SRC = 2048;   // source intervals per tile
constexpr int TM_SIDE = 128;   // runs per side (below and above U)
constexpr int64_t TM_WORDS = (int64_t)(TILE_MAP_BYTES / 8);
// Run r of side s (0: below U, 1: above) has its bound at run_word(s, 0, r)
// and its exit at run_word(s, 1, r).  Runs l < 64 of both sides lie in words
// 4l..4l+3 (bound and exit below U, bound and exit above: one lane's words,
// two 16-byte loads), followed by the header (state, runs below, runs above,
// tile change) at word 256; runs 64-127 follow at word 512 the same way.
constexpr int TM_HDR = 256;
constexpr int TM_RUN_HI = 512;
__device__ __forceinline__ int run_word(int side, int which, int r) {
    return (r < 64 ? 0 : TM_RUN_HI) + 4 * (r & 63) + 2 * side + which;
}
constexpr int TM_SB = 1024;    // source bounds (scratch while the map is built)
constexpr int TM_SD = 3072;    // source sides, one byte each: 1 = below U (scratch)
enum { TM_MAPPED = 1, TM_NONE = 2 };
// causes of a tile without a map (control words 7-10 count them)
enum { TMF_QUALIFY = 1, TMF_SOURCES, TMF_CHAINS, TMF_RUNS };

// The map area of tile k: the tracked-list area, unused until the tracked
// list is built at the end of the launch (16 bytes per event against 4 bytes
// per event needed here).
__device__ __forceinline__ SMP_GLOBAL int64_t* tile_map(const Desc& D, int64_t k) {
    return gp((int64_t*)D.tracked) + k * TM_WORDS;
}
// A word of a map that another wave reads in the same launch: stored through
// to memory, as the look-back words are.
__device__ __forceinline__ void st_map(SMP_GLOBAL int64_t* p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First node of a segment (relative prefixes f) whose prefix is >= thr (GE)
// or <= thr (LE); SEG if none.  Branch-free: one compare per window, then a
// select per window from the last one down.
template <bool GE>
__device__ __forceinline__ int first_node(const int64_t (&f)[NW], int64_t thr) {
    uint64_t m[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) m[w] = ballot(GE ? f[w] >= thr : f[w] <= thr);
    int k = SEG;
#pragma unroll
    for (int w = NW - 1; w >= 0; --w) k = m[w] ? w * 64 + ctz64(m[w]) : k;
    return k;
}
// The same for two thresholds at once (independent, so their instructions interleave).
template <bool GE>
__device__ __forceinline__ void first_node2(const int64_t (&f)[NW], int64_t t1, int64_t t2, int& k1, int& k2) {
    uint64_t m1[NW], m2[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        m1[w] = ballot(GE ? f[w] >= t1 : f[w] <= t1);
        m2[w] = ballot(GE ? f[w] >= t2 : f[w] <= t2);
    }
    k1 = SEG;
    k2 = SEG;
#pragma unroll
    for (int w = NW - 1; w >= 0; --w) {
        k1 = m1[w] ? w * 64 + ctz64(m1[w]) : k1;
        k2 = m2[w] ? w * 64 + ctz64(m2[w]) : k2;
    }
}

// The exit of a tile from entry e, from its map's runs (two per lane and
// side: runs l and 64 + l, bound and exit) and header values.
static_assert(TM_SIDE == 128, "map_exit takes two runs per lane and side");
__device__ __forceinline__ int64_t map_exit(int64_t e, int nup, int ndn, int64_t tF, int64_t ub0, int64_t ub1,
                                            int64_t ue0, int64_t ue1, int64_t db0, int64_t db1, int64_t de0,
                                            int64_t de1) {
    const int l = lane_id();
    // below U: the first run whose (upper) bound is >= e
    const uint64_t u0 = ballot(l < nup && ub0 >= e), u1 = ballot(64 + l < nup && ub1 >= e);
    if (u0) return readlane64(ue0, ctz64(u0));
    if (u1) return readlane64(ue1, ctz64(u1));
    // above U: the first run whose (lower) bound is <= e
    const uint64_t d0 = ballot(l < ndn && db0 <= e), d1 = ballot(64 + l < ndn && db1 <= e);
    if (d0) return readlane64(de0, ctz64(d0));
    if (d1) return readlane64(de1, ctz64(d1));
    return e - tF;  // in U: no sample in the tile
}

// The same for a map of at most 64 runs per side (one per lane; vu, vd:
// the lanes that hold one), without branches: both searches, then selects.
__device__ __forceinline__ int64_t map_exit64(int64_t e, uint64_t vu, uint64_t vd, int64_t tF, int64_t ub, int64_t ue,
                                              int64_t db, int64_t de) {
    const uint64_t u = vu & ballot(ub >= e), d = vd & ballot(db <= e);
    const int64_t xu = readlane64(ue, u ? ctz64(u) : 0), xd = readlane64(de, d ? ctz64(d) : 0);
    return u ? xu : (d ? xd : e - tF);
}

// The tile entries of a trace, chained through the maps in tile order by one
// wave (tile 0's entry is 0): each tile's exit is published as the word the
// resolve pass waits for.  It stops at the first tile without a map.  Tiles
// are taken TC_CB at a time, the next ones' words loading while these are
// looked up.
constexpr int TC_CB = 8;
__device__ void chain_maps(const Desc& D, unsigned long long* ctl) {
    const int l = lane_id();
    const int nt = __builtin_amdgcn_readfirstlane((int)D.ntile);
    const StatusView ts{D.tstat, (int64_t)nt};
    // lane l: runs l of both sides (bound, exit below U; bound, exit above);
    // lanes 0-3: the header
    auto load = [&](int t0, int64_t (&w)[TC_CB][4], int64_t (&h)[TC_CB]) {
#pragma unroll
        for (int b = 0; b < TC_CB; ++b) {
            const SMP_GLOBAL int64_t* m = tile_map(D, t0 + b < nt ? t0 + b : nt - 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) w[b][q] = m[4 * l + q];
            h[b] = m[TM_HDR + (l & 3)];
        }
    };
    int64_t nw[TC_CB][4], nh[TC_CB];
    load(0, nw, nh);
    int64_t e = 0;
    int t = 0;
    for (; t < nt;) {
        int64_t cw[TC_CB][4], ch[TC_CB];
#pragma unroll
        for (int b = 0; b < TC_CB; ++b) {
            ch[b] = nh[b];
#pragma unroll
            for (int q = 0; q < 4; ++q) cw[b][q] = nw[b][q];
        }
        if (t + TC_CB < nt) load(t + TC_CB, nw, nh);
        const int nb = (nt - t) < TC_CB ? (nt - t) : TC_CB;
        // everything that does not depend on the entry first: the tiles that
        // can be chained, their runs and tile changes
        int nm = 0;
        int64_t nup[TC_CB], ndn[TC_CB], tFs[TC_CB];
        uint64_t vu[TC_CB], vd[TC_CB];
#pragma unroll
        for (int b = 0; b < TC_CB; ++b) {
            nm += (b == nm && b < nb && readlane64(ch[b], 0) == TM_MAPPED) ? 1 : 0;
            nup[b] = readlane64(ch[b], 1);
            ndn[b] = readlane64(ch[b], 2);
            tFs[b] = readlane64(ch[b], 3);
            vu[b] = ballot(l < nup[b]);
            vd[b] = ballot(l < ndn[b]);
        }
        int done = 0;
        int64_t xs = 0;  // lane b: the exit of tile t + b
#pragma unroll
        for (int b = 0; b < TC_CB; ++b) {
            if (b >= nm) break;
            int64_t x;
            if (nup[b] <= 64 && ndn[b] <= 64) {
                x = map_exit64(e, vu[b], vd[b], tFs[b], cw[b][0], cw[b][1], cw[b][2], cw[b][3]);
            } else {  // more than 64 runs on a side: the rest from the map itself
                const SMP_GLOBAL int64_t* m = tile_map(D, t + b) + TM_RUN_HI + 4 * l;
                x = map_exit(e, (int)nup[b], (int)ndn[b], tFs[b], cw[b][0], m[0], cw[b][1], m[1], cw[b][2], m[2],
                             cw[b][3], m[3]);
            }
            xs = l == b ? x : xs;
            e = x;
            ++done;
        }
        if (l < done) st_status(ts.at(W_XF, t + l), pack(xs, 1));
        t += done;
        if (done < nb) break;  // a tile without a map
    }
    if (l == 0 && t > 0) g_add((uint64_t*)&ctl[6], (uint64_t)t);
}

// One wave per tile (grid: every tile of the launch; tiles of traces without
// maps return at once).
__global__ __launch_bounds__(64) void k_tmap(const Desc* __restrict__ desc, int ntraces, unsigned long long* ctl) {
    __shared__ int64_t cx[TM_CAP];       // live chains: reference (tile coordinates)
    __shared__ uint16_t cr[TM_CAP];      // and the root source of their set
    __shared__ uint16_t par[TM_SRC];     // union-find parent of each source
    // per segment: its prefixes, and per node the chain that sampled there
    // first (see claim below); at the end: the live chain of each root
    __shared__ int64_t lds_u[(SEG * 8 + SEG * 4 > TM_SRC * 2 ? SEG * 8 + SEG * 4 : TM_SRC * 2) / 8];
    int64_t* fl = lds_u;
    uint32_t* claim = (uint32_t*)(lds_u + SEG);
    uint16_t* cidx = (uint16_t*)lds_u;
    const int l = lane_id();
    const uint64_t tk = blockIdx.x;
    const Desc& D = desc[find_trace_tile(desc, ntraces, tk)];
    if (!D.tmap) return;
    const int64_t k = (int64_t)(tk - D.tile_begin);
    const int64_t ns = (int64_t)D.nseg;
    const int nval = (int)((ns - k * TILE) < TILE ? (ns - k * TILE) : TILE);
    const int64_t T = D.T;
    SMP_GLOBAL int64_t* map = tile_map(D, k);
    SMP_GLOBAL uint8_t* sside = (SMP_GLOBAL uint8_t*)(map + TM_SD);
    const SMP_GLOBAL int64_t* sp = gp(D.seg) + k * TILE;
    // every segment SIM, with a no-sample interval of at least T entries
    // (then max - min < T over its prefixes and the entry)
    bool ok = prefixes_kept(D);
    for (int g = 0; g < nval && ok; g += 64) {
        const int s = g + l;
        const bool v = s < nval;
        const int64_t lo = v ? sp[SP_LO * ns + s] : 0, hi = v ? sp[SP_HI * ns + s] : 0;
        const int64_t fl_ = v ? sp[SP_FLG * ns + s] : 0;
        if (ballot(v && ((fl_ & 3) != MAP_SIM || hi < lo || hi - lo < T - 1))) ok = false;
    }
    for (int i = l; i < SEG; i += 64) claim[i] = 0;
    int nch = 0, nsrc = 0;
    int fail = ok ? 0 : TMF_QUALIFY;  // cause, 0 while the map holds
    int64_t Umax = 0, Umin = 0, carry = 0;  // running extremes (from the tile start), footprint change so far
    // segments g..g+63, one per lane: offset, no-sample bounds and extremes in tile coordinates
    int64_t gR = 0, gL = 0, gH = 0, gX = 0, gN = 0;
    auto step = [&](int s, const int64_t (&f)[NW]) {
        if ((s & 63) == 0) {
            const int j = s + l;
            const bool v = j < nval;
            const int64_t af = v ? sp[SP_AF * ns + j] : 0;
            const int64_t lo = v ? sp[SP_LO * ns + j] : 0, hi = v ? sp[SP_HI * ns + j] : 0;
            const int64_t mx = v ? sp[SP_MXF * ns + j] : 0, mn = v ? sp[SP_MNF * ns + j] : 0;
            const int64_t inc = wave_incl_sum(af);
            gR = carry + inc - af;
            carry += readlane64(inc, 63);
            gL = gR + lo;
            gH = gR + hi;
            gX = gR + mx;
            gN = gR + mn;
        }
        const int i = s & 63;
        const int64_t R = readlane64(gR, i), Ls = readlane64(gL, i), Hs = readlane64(gH, i);
        const int64_t Sx = readlane64(gX, i), Sn = readlane64(gN, i);
        // the prefixes in LDS: the value at a sampled node is read from there
#pragma unroll
        for (int w = 0; w < NW; ++w) fl[w * 64 + l] = f[w];
        // Chains that sample at one node merge into the first of them.
        // claim[node] (step numbers from 1): step << 16 | 0x7FFF - chain
        // while chains compete for it (the largest wins: the earliest
        // chain), then step << 16 | 0x8000 | root of the winner's set.
        const uint32_t stag = (uint32_t)(s + 1) << 16;
        // live chains: those outside the no-sample interval sample once here
        // (each group's words load while the one before it is processed:
        // the compaction below never writes past the group it processes)
        int out = 0;
        int64_t Xn = l < nch ? cx[l] : 0;
        int rtn = l < nch ? (int)cr[l] : 0;
        for (int c0 = 0; c0 < nch; c0 += 64) {
            const int c = c0 + l;
            const bool v = c < nch;
            int64_t X = Xn;
            const int rt = rtn;
            if (c0 + 64 < nch) {
                const int cn = c + 64;
                Xn = cn < nch ? cx[cn] : 0;
                rtn = cn < nch ? (int)cr[cn] : 0;
            }
            const uint64_t vm = ballot(v);
            uint64_t alive = vm;
            bool moved = false;  // sampled here and keeps its chain
            const bool up = v && X < Ls;
            const uint64_t sm0 = ballot(up || (v && X > Hs));
            if (sm0) {
                // each sampling chain's node: two chains of one direction at a time
                const uint64_t um = ballot(up), dm = sm0 & ~um;
                const int64_t thr = up ? X - R + T : X - R - T;
                int xnode = SEG;
#define SMP_TM_SEARCH(MASK, GE)                                                 \
    for (uint64_t m_ = (MASK); m_;) {                                           \
        const int q1 = ctz64(m_);                                               \
        m_ &= m_ - 1;                                                           \
        const int64_t th1 = readlane64(thr, q1);                                \
        if (m_) {                                                               \
            const int q2 = ctz64(m_);                                           \
            m_ &= m_ - 1;                                                       \
            int n1, n2;                                                         \
            first_node2<GE>(f, th1, readlane64(thr, q2), n1, n2);               \
            xnode = l == q1 ? n1 : (l == q2 ? n2 : xnode);                      \
        } else {                                                                \
            const int n1 = first_node<GE>(f, th1);                              \
            xnode = l == q1 ? n1 : xnode;                                       \
        }                                                                       \
    }
                SMP_TM_SEARCH(um, true)
                SMP_TM_SEARCH(dm, false)
#undef SMP_TM_SEARCH
                const bool mine = (sm0 >> l) & 1;
                if (ballot(mine && xnode >= SEG)) {  // (unreachable: a chain outside the interval crosses)
                    fail = TMF_QUALIFY;
                    break;
                }
                // merges, for the whole group at once
                const uint32_t key = stag | (uint32_t)(0x7FFF - c);
                if (mine) __hip_atomic_fetch_max(&claim[xnode], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint32_t got =
                    mine ? __hip_atomic_load(&claim[xnode], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0;
                const bool win = mine && got == key;
                if (win)
                    __hip_atomic_store(&claim[xnode], stag | 0x8000u | (uint32_t)rt, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                const bool lose = mine && !win;
                // the winner's root: in the claim once resolved (an earlier
                // group), else held by the winner's lane in this group
                const int wl = (int)(0x7FFFu - (got & 0x7FFFu)) - c0;
                const int wr = shfl32(rt, (got & 0x8000u) ? l : (wl & 63));
                if (lose) par[rt] = (uint16_t)((got & 0x8000u) ? (got & 0x7FFFu) : (uint32_t)wr);
                alive &= ~ballot(lose);
                if (win) X = R + fl[xnode];
                moved = win;
            }
            // compact in place (survivors never move up); while no chain of
            // this step has merged, only the sampled references change
            if (out == c0 && alive == vm) {
                if (moved) cx[c] = X;
            } else if ((alive >> l) & 1) {
                const int o = out + __popcll(alive & lanemask_lt());
                cx[o] = X;
                cr[o] = (uint16_t)rt;
            }
            out += __popcll(alive);
        }
        nch = out;
        // New running extremes while U is not empty start chains.  A window
        // with no node beyond the extremes so far leaves them unchanged; in
        // the others, the extremes before each node come from a scan.
        if (!fail && Umax - Umin <= 2 * T - 2 && (Sx > Umax || Sn < Umin)) {
            int64_t cm = Umax, cn = Umin;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (cm - cn > 2 * T - 2 || fail) break;
                const int64_t gv = R + f[w];
                if (!ballot(gv > cm || gv < cn)) continue;
                int64_t im = wave_incl_max(gv), in = wave_incl_min(gv);
                im = im > cm ? im : cm;
                in = in < cn ? in : cn;
                const int64_t pm = wave_shr1(im, cm), pn = wave_shr1(in, cn);  // before the node
                const bool open = pm - pn <= 2 * T - 2;
                const bool up = open && gv > pm, dn = open && gv < pn;
                const uint64_t spm = ballot(up || dn);
                cm = readlane64(im, 63);
                cn = readlane64(in, 63);
                if (!spm) continue;
                const int cnt = __popcll(spm);
                if (nsrc + cnt > TM_SRC) {
                    fail = TMF_SOURCES;
                    break;
                }
                // sources in node order; the entries of U = [pm - T + 1,
                // pn + T - 1] that sample at this node
                const bool sp_ = (spm >> l) & 1;
                const int src = nsrc + __popcll(spm & lanemask_lt());
                const int64_t bound = up ? ((pn + T - 1) < (gv - T) ? (pn + T - 1) : (gv - T))
                                         : ((pm - T + 1) > (gv + T) ? (pm - T + 1) : (gv + T));
                // a chain that sampled at the same node takes the source into its set
                const uint32_t cl =
                    sp_ ? __hip_atomic_load(&claim[w * 64 + l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0;
                const bool hit = sp_ && (cl >> 16) == (stag >> 16);
                const uint64_t nm = spm & ~ballot(hit);  // new chains
                if (nch + __popcll(nm) > TM_CAP) {
                    fail = TMF_CHAINS;
                    break;
                }
                if (sp_) {
                    map[TM_SB + src] = bound;
                    sside[src] = up ? 1 : 0;
                    par[src] = (uint16_t)(hit ? (cl & 0x7FFFu) : (uint32_t)src);
                }
                if ((nm >> l) & 1) {
                    const int o = nch + __popcll(nm & lanemask_lt());
                    cx[o] = gv;
                    cr[o] = (uint16_t)src;
                }
                nsrc += cnt;
                nch += __popcll(nm);
            }
        }
        Umax = Sx > Umax ? Sx : Umax;
        Umin = Sn < Umin ? Sn : Umin;
    };
    // the next segment's prefixes load while one is processed (into fn,
    // copied out at the start of each step: the only loads then in flight
    // are the ones the copy needs, issued a whole step earlier)
    const int64_t j0 = k * TILE;
    int64_t fn[NW];
    if (!fail) load_kept(D, j0, fn);
    for (int s = 0; s < nval && !fail; ++s) {
        int64_t f[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) f[w] = fn[w];
        load_kept(D, j0 + (s + 1 < nval ? s + 1 : s), fn);
        step(s, f);
    }
    // runs: consecutive sources of one side that end at the same reference
    int nup = 0, ndn = 0;
    if (!fail) {
        const int64_t tF = carry;
        for (int i = l; i < nsrc; i += 64) cidx[i] = 0;
        for (int c0 = 0; c0 < nch; c0 += 64)
            if (c0 + l < nch) cidx[cr[c0 + l]] = (uint16_t)(c0 + l);
        // the source bounds and sides stored above (by this wave), before they are read back
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        int64_t lastU = 0, lastD = 0;  // exit of the previous source of each side
        for (int s0 = 0; s0 < nsrc; s0 += 64) {
            const int s = s0 + l;
            const bool v = s < nsrc;
            int r = s;
            for (int d = 0; v && d < TM_SRC && par[r] != r; ++d) r = par[r];
            const int64_t ex = v ? cx[cidx[r]] - tF : 0;
            const int64_t bnd = v ? map[TM_SB + s] : 0;
            const bool isup = v && sside[s] != 0;
            const bool isdn = v && !isup;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool mine = side == 0 ? isup : isdn;
                const uint64_t sm = ballot(mine);
                if (!sm) continue;
                int& cnt = side == 0 ? nup : ndn;
                int64_t& last = side == 0 ? lastU : lastD;
                // the previous source of this side: an earlier lane, else the carried one
                const uint64_t before = sm & lanemask_lt();
                const int64_t pe = shfl64(ex, before ? top64(before) : 0);
                const bool has_prev = before != 0 || cnt > 0;
                const int64_t prev = before ? pe : last;
                const bool start = mine && (!has_prev || ex != prev);
                const uint64_t stm = ballot(start);
                const int run = cnt + __popcll(stm & (lanemask_lt() | (1ull << l))) - 1;
                // a source whose next source of this side (in this group)
                // starts a new run, or that is the group's last, writes its
                // bound; a later group may still extend its run
                const uint64_t after = sm & ~(lanemask_lt() | (1ull << l));
                const bool ends = mine && (!after || ((stm >> ctz64(after)) & 1));
                const int nr = cnt + __popcll(stm);
                if (nr > TM_SIDE) {
                    fail = TMF_RUNS;
                    break;
                }
                if (start) st_map(map + run_word(side, 1, run), ex);
                if (ends) st_map(map + run_word(side, 0, run), bnd);
                cnt = nr;
                last = readlane64(ex, top64(sm));
            }
            if (fail) break;
        }
        if (!fail && l == 0) {
            st_map(map + TM_HDR + 1, nup);
            st_map(map + TM_HDR + 2, ndn);
            st_map(map + TM_HDR + 3, tF);
        }
    }
    if (l == 0) {
        st_map(map + TM_HDR, fail ? TM_NONE : TM_MAPPED);
        g_add((uint64_t*)&ctl[fail ? 6 + fail : 5], 1ull);
    }
    // The last of the trace's tile waves chains its tiles.  The map's words
    // were stored through to memory (agent-scope stores): it is counted once
    // they are complete, and the last wave drops any stale copies of other
    // tiles' words from its caches before it reads them.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint64_t done = 0;
    if (l == 0) done = g_add_rtn(&D.scal->tmap_done, 1ull);
    if (readlaneu64(done, 0) == D.ntile - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        chain_maps(D, ctl);
    }
}

// One workgroup per tile of TILE segments (tiles taken in ticket order, so a
// tile's predecessors are always running or done): exclusive prefix sums and
// the chain's entry and exit offset of every segment.
//
// Exits of segments with a total map are known at once.  The other segments
// are resolved in order by one wave (the walker), from the segment after the
// tile's first total map to the tile end first (their exits do not depend on
// the tile's entry, so the tile's exit is published before its entry is
// awaited), then from the tile start; the walker takes 64 segments per step
// and stops only at segments whose entry lies outside their no-sample
// interval.  A SIM segment where it stops is followed through its records;
// the other waves scan the SIM segments' footprint prefixes into an LDS ring
// ahead of the walker (skipping those it has already passed), so each one
// costs the walker only a pass over LDS.
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(4))) void k_resolve(const Desc* __restrict__ desc, int ntraces, uint64_t ntile_total,
                                                  unsigned long long* ctl) {
    __shared__ unsigned long long s_tk;
    __shared__ int64_t w_sum[3][TWAVES];
    __shared__ int64_t s_pre[3];
    __shared__ int64_t w_peak[TWAVES], w_peakS[TWAVES];
    __shared__ int w_left[TWAVES];
    __shared__ int64_t m_lo[TILE], m_hi[TILE], m_af[TILE], m_kf[TILE], m_ex[TILE];
    __shared__ int64_t m_R[TILE];  // sparse tiles: the footprint change before each segment
    __shared__ uint64_t w_tot[TWAVES], w_sim[TWAVES];  // valid lanes with TOTAL / SIM maps
    __shared__ int64_t ring[RING][SEG];
    __shared__ int r_ready[RING];  // walk-order SIM index held by each slot
    __shared__ int s_prod, s_cons, s_abort;
    __shared__ int w_wide[TWAVES];
    __shared__ int64_t s_entry;
    const int tid = threadIdx.x, wv = tid >> 6, l = lane_id();
    if (tid == 0) {
        s_tk = g_add_rtn((uint64_t*)&ctl[2], 1ull);
        s_prod = 0;
        s_cons = 0;
        s_abort = 0;
    }
    if (tid < RING) r_ready[tid] = -1;
    __syncthreads();
    const uint64_t tk = s_tk;
    if (tk >= ntile_total) return;
    const Desc& D = desc[find_trace_tile(desc, ntraces, tk)];
    const int64_t k = (int64_t)(tk - D.tile_begin);
    const int64_t ns = (int64_t)D.nseg;
    const int64_t j = k * TILE + tid;
    const bool valid = j < ns;
    const int nval = (int)((ns - k * TILE) < TILE ? (ns - k * TILE) : TILE);  // valid lanes
    const StatusView ts{D.tstat, (int64_t)D.ntile};
    const SMP_GLOBAL int64_t* sp = gp(D.seg) + (valid ? j : 0);
    int64_t af = 0, ap = 0, ac = 0, kf = 0, lo = 0, hi = 0;
    int kind = MAP_CONST;
    if (valid) {
        af = sp[SP_AF * ns];
        ap = sp[SP_AP * ns];
        ac = sp[SP_AC * ns];
        lo = sp[SP_LO * ns];
        hi = sp[SP_HI * ns];
        kf = sp[SP_KF * ns];
        kind = (int)(sp[SP_FLG * ns] & 3);
    }
    m_lo[tid] = lo;
    m_hi[tid] = hi;
    m_af[tid] = af;
    m_kf[tid] = kf;
    m_ex[tid] = kf;  // final for total maps; the walker overwrites the others
    const uint64_t tot = ballot(valid && kind == MAP_TOTAL), sim = ballot(valid && kind == MAP_SIM);
    // sums inside the wave
    int64_t iF = af, iP = ap, iC = ac;
    wave_incl_sum3(iF, iP, iC);
    if (l == 63) {
        w_sum[0][wv] = iF;
        w_sum[1][wv] = iP;
        w_sum[2][wv] = iC;
    }
    // SIM maps whose no-sample interval holds at least half of the entries
    const int nwide_w = __popcll(ballot(valid && kind == MAP_SIM && hi - lo >= D.T));
    if (l == 0) {
        w_tot[wv] = tot;
        w_sim[wv] = sim;
        w_wide[wv] = nwide_w;
    }
    __syncthreads();
    int64_t oF = 0, oP = 0, oC = 0, tF = 0, tP = 0, tC = 0;
    int ft = nval;  // first lane with a total map
    for (int w = TWAVES - 1; w >= 0; --w)
        if (w_tot[w]) ft = w * 64 + ctz64(w_tot[w]);
    for (int w = 0; w < TWAVES; ++w) {
        if (w == wv) {
            oF = tF;
            oP = tP;
            oC = tC;
        }
        tF += w_sum[0][w];
        tP += w_sum[1][w];
        tC += w_sum[2][w];
    }
    // prefixes relative to the tile start (the tile's own prefix is added at the end)
    const int64_t rF = oF + iF - af, rP = oP + iP - ap, rC = oC + iC - ac;
    // SIM segments in walk order: (ft, nval) first, then [0, ft)
    int nA = 0, nsim = 0, nwide = 0;
    for (int w = 0; w < TWAVES; ++w) {
        nA += __popcll(w_sim[w] & range_mask(w, ft + 1, nval));
        nsim += __popcll(w_sim[w]);
        nwide += w_wide[w];
    }
    // publish the tile's sums (inclusive right away for the first tile)
    if (tid < 3) st_status(ts.at(W_AF + tid, k), pack(tid == 0 ? tF : (tid == 1 ? tP : tC), 1));
    if (k == 0 && tid < 3) st_status(ts.at(W_IF + tid, k), pack(tid == 0 ? tF : (tid == 1 ? tP : tC), 1));
    const int64_t T = D.T;

    const bool kept = prefixes_kept(D);
    // Sparse tile: most SIM maps leave at least half of the entries without a
    // sample, so the walker stops at few of them (T far above what a segment
    // moves).  Producers pre-scanning every SIM segment would fall behind the
    // walker, and their loads would queue in the CU's memory pipeline ahead
    // of the walker's own (each stop of the walker waits for one): here the
    // other waves stay idle and the walker reads the kept prefixes itself.
    const bool sparse = kept && nsim > 0 && 4 * nwide >= 3 * nsim;
    if (sparse) {
        // the walker reads footprint offsets inside the tile from LDS instead
        // of scanning each group of 64 segments it enters
        m_R[tid] = rF;
        __syncthreads();
    }
    if (wv == 0) {
        // ---- the walker ----
        int q = 0;  // SIM segments passed, in walk order
        bool ok = true;
        // Sparse tiles: the kept prefixes of the predicted next stop, loaded
        // into pf while the current stop is resolved (pf_lane: its tile lane,
        // -1 if none).  At a stop they are written to ring slot 0 (unused in
        // sparse tiles; the write waits only for loads the stop needs) and
        // the registers take the next prediction's loads at once.
        int64_t pf[NW];
        int pf_lane = -1;
        auto walk = [&](int b, int e, int64_t x) -> int64_t {
            for (int g0 = b & ~63; g0 < e && ok; g0 += 64) {
                const int i = g0 + l;
                const int64_t lo = m_lo[i], hi = m_hi[i], af = m_af[i], kf = m_kf[i];
                const uint64_t sim = w_sim[g0 >> 6], tot = w_tot[g0 >> 6];
                const bool is_tot = (tot >> l) & 1;
                const int64_t S = sparse ? (int64_t)((uint64_t)m_R[i] - (uint64_t)m_R[g0])
                                         : (int64_t)((uint64_t)wave_incl_sum(af) - (uint64_t)af);
                // the last total-map lane before this one, and the entry it gives
                const uint64_t tb = tot & lanemask_lt();
                const int jl = tb ? top64(tb) : -1;
                const int64_t rj = (int64_t)((uint64_t)kf + (uint64_t)S + (uint64_t)af);  // kf_j + S_(j+1) on lane j
                const int64_t xt = (int64_t)((uint64_t)shfl64(rj, jl < 0 ? l : jl) - (uint64_t)S);
                const int ge = e - g0 < 64 ? e - g0 : 64;
                int i0 = b > g0 ? b - g0 : 0;
                while (i0 < ge) {
                    const int64_t xi = jl >= i0 ? xt : (int64_t)((uint64_t)x - ((uint64_t)S - (uint64_t)readlane64(S, i0)));
                    const uint64_t fire = ballot(l >= i0 && l < ge && !is_tot && !(xi >= lo && xi <= hi));
                    const int stop = fire ? ctz64(fire) : ge;
                    const int64_t xo = is_tot ? kf : (int64_t)((uint64_t)xi - (uint64_t)af);
                    if (l >= i0 && l < stop && !is_tot) m_ex[i] = xo;
                    if (!sparse) q += __popcll(sim & range_mask(0, i0, stop));
                    // release the slots passed over before any wait below (a
                    // producer may be waiting for them); every lane stores the
                    // same value (no lane-0-only region inside the loop).  A
                    // sparse tile has no producers, and the release would wait
                    // for every load in flight (the prefetch of the next stop).
                    if (!sparse) __hip_atomic_store(&s_cons, q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (stop > i0) x = readlane64(xo, stop - 1);
                    if (stop < ge) {
                        const int64_t xs = readlane64(xi, stop);
                        int64_t r = readlane64(kf, stop);
                        if ((sim >> stop) & 1 && sparse) {
                            // The exit lies in [xs + T, max] - af for an
                            // entry below lo (one sample at the first node
                            // reaching xs + T; more only where the segment
                            // moves T or more), in [min, xs - T] - af above hi
                            // (max = lo + T - 1, min = hi - T + 1).  The next
                            // stop is predicted as the first later segment
                            // whose no-sample interval does not hold that
                            // whole range, shifted by the footprint changes in
                            // between (this group, else the next one).  A
                            // prediction only decides what is loaded early.
                            const int64_t lo_c = readlane64(lo, stop), hi_c = readlane64(hi, stop);
                            const int64_t af_c = readlane64(af, stop);
                            uint64_t A, B;
                            if (xs < lo_c) {
                                A = (uint64_t)xs + (uint64_t)T - (uint64_t)af_c;
                                B = (uint64_t)lo_c + (uint64_t)(T - 1) - (uint64_t)af_c;
                            } else {
                                A = (uint64_t)hi_c - (uint64_t)(T - 1) - (uint64_t)af_c;
                                B = (uint64_t)xs - (uint64_t)T - (uint64_t)af_c;
                            }
                            const uint64_t base = (uint64_t)readlane64(S, stop) + (uint64_t)af_c;
                            int p = -1;
                            {
                                const uint64_t d = (uint64_t)S - base;
                                const bool cand = l > stop && l < ge &&
                                                  (is_tot || !((int64_t)(A - d) >= lo && (int64_t)(B - d) <= hi));
                                const uint64_t cm = ballot(cand);
                                if (cm) {
                                    const int pl = ctz64(cm);
                                    if ((sim >> pl) & 1) p = g0 + pl;
                                } else if (g0 + 64 < e) {
                                    const int i2 = g0 + 64 + l;
                                    const bool v2 = i2 < e;
                                    const int64_t lo2 = m_lo[v2 ? i2 : 0], hi2 = m_hi[v2 ? i2 : 0];
                                    const uint64_t tot2 = w_tot[(g0 >> 6) + 1], sim2 = w_sim[(g0 >> 6) + 1];
                                    const uint64_t d2 = (uint64_t)m_R[v2 ? i2 : 0] - (uint64_t)m_R[g0] - base;
                                    const bool cand2 = v2 && (((tot2 >> l) & 1) ||
                                                              !((int64_t)(A - d2) >= lo2 && (int64_t)(B - d2) <= hi2));
                                    const uint64_t cm2 = ballot(cand2);
                                    if (cm2 && ((sim2 >> ctz64(cm2)) & 1)) p = g0 + 64 + ctz64(cm2);
                                }
                            }
                            // pf is defined once per stop (the compiler would
                            // otherwise copy it between registers, and a copy
                            // waits for the loads in flight): a miss loads
                            // into a temporary, and the next prefetch is
                            // always issued (of this segment again when there
                            // is no prediction)
                            // A segment that moves less than T samples once
                            // (hi - lo >= T - 1 implies max - min < T): its
                            // exit comes straight from the registers.  Others
                            // are walked from ring slot 0.
                            const int c = g0 + stop;
                            const bool one = (uint64_t)hi_c - (uint64_t)lo_c >= (uint64_t)(T - 1) && hi_c >= lo_c;
                            const bool up = xs < lo_c;
                            if (pf_lane == c) {
                                if (one) {
                                    r = exit_one_sample(pf, T, xs, up);
                                } else {
#pragma unroll
                                    for (int w = 0; w < NW; ++w) ring[0][w * 64 + l] = pf[w];
                                }
                            } else {
                                int64_t tmp[NW];
                                load_kept(D, k * TILE + c, tmp);
                                if (one) {
                                    r = exit_one_sample(tmp, T, xs, up);
                                } else {
#pragma unroll
                                    for (int w = 0; w < NW; ++w) ring[0][w * 64 + l] = tmp[w];
                                }
                            }
                            pf_lane = p;
                            load_kept(D, k * TILE + (p >= 0 ? p : c), pf);
                            if (!one) r = walk_prefixes(ring[0], T, xs);
                        } else if ((sim >> stop) & 1) {
                            const int slot = q % RING;
                            if (kept && __hip_atomic_load(&r_ready[slot], __ATOMIC_ACQUIRE,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP) != q) {
                                // its producer is behind: read the kept prefixes instead of waiting
                                r = walk_kept(D, k * TILE + g0 + stop, T, xs);
                            } else {
                                LocalSpin sp_;
                                while (__hip_atomic_load(&r_ready[slot], __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP) != q) {
                                    if (local_spin_abort(ctl, sp_)) {
                                        ok = false;
                                        break;
                                    }
                                }
                                r = ok ? walk_prefixes(ring[slot], T, xs) : 0;
                            }
                            ++q;
                            __hip_atomic_store(&s_cons, q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        if (l == stop) m_ex[i] = r;
                        x = r;
                    }
                    i0 = stop + 1;
                    if (!ok) break;
                }
            }
            return x;
        };
        // (ft, nval): entry-independent
        if (ft < nval) {
            const int64_t xa = walk(ft + 1, nval, m_kf[ft]);
            st_status(ts.at(W_XF, k), pack(xa, 1));
        }
        // the tile's entry, then [0, ft)
        int64_t e = 0;
        // A tile with a map whose exit the map chain has not published (a
        // tile before it has no map): the exit follows from the entry by one
        // lookup and is published before the walk, so that the next tile
        // need not wait for the walk.  The map loads while the entry is
        // awaited.
        const bool use_map = D.tmap && ft >= nval && k > 0;
        int64_t mh = 0, mr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (use_map) {
            const SMP_GLOBAL int64_t* mp = tile_map(D, k);
            if (l < 4) mh = mp[TM_HDR + l];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                mr[w] = mp[4 * l + w];
                mr[4 + w] = mp[TM_RUN_HI + 4 * l + w];
            }
        }
        if (k > 0 && ok) ok = wait_word(ts.at(W_XF, k - 1), e, ctl);
        if (use_map && ok && readlane64(mh, 0) == TM_MAPPED && !wstate(ld_status(ts.at(W_XF, k)))) {
            const int64_t x = map_exit(e, (int)readlane64(mh, 1), (int)readlane64(mh, 2), readlane64(mh, 3), mr[0],
                                       mr[4], mr[1], mr[5], mr[2], mr[6], mr[3], mr[7]);
            st_status(ts.at(W_XF, k), pack(x, 1));
        }
        const int64_t xb = ok ? walk(0, ft, e) : 0;
        if (ft >= nval) {
            // a tile map may have published the exit already: it must agree
            const uint64_t pw = ld_status(ts.at(W_XF, k));
            if (wstate(pw) && unpack(pw) != xb && l == 0) g_or32(&D.scal->err, 4u);
            st_status(ts.at(W_XF, k), pack(xb, 1));
        }
        if (l == 0) {
            s_entry = e;
            if (!ok) {
                g_or32(&D.scal->err, 8u);
                __hip_atomic_store(&s_abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    } else {
        if (wv == 1) {
            // ---- the tile's prefix sums ----
            int64_t pF = 0, pP = 0, pC = 0;
            bool ok = true;
            if (k > 0) {
                ok = scan_sums(ts, k, pF, pP, pC, ctl);
                if (l < 3) st_status(ts.at(W_IF + l, k), pack(l == 0 ? pF + tF : (l == 1 ? pP + tP : pC + tC), 1));
            }
            if (l == 0) {
                s_pre[0] = pF;
                s_pre[1] = pP;
                s_pre[2] = pC;
                if (!ok) g_or32(&D.scal->err, 8u);
            }
        }
        // ---- producers: pre-scan SIM segments in walk order (dense tiles only) ----
        if (!sparse) for (;;) {
            // every lane takes part (lane 0 adds 1, the others 0): a lane-0-only
            // region here lets the compiler split the wave across loop trips
            const int pidx = __builtin_amdgcn_readfirstlane(
                __hip_atomic_fetch_add(&s_prod, l == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            if (pidx >= nsim) break;
            // its lane: the pidx-th SIM lane of (ft, nval), else of [0, ft)
            int r = pidx < nA ? pidx : pidx - nA;
            const int rlo = pidx < nA ? ft + 1 : 0, rhi = pidx < nA ? nval : ft;
            int lane = -1;
            for (int w = 0; w < TWAVES && lane < 0; ++w) {
                const uint64_t m = w_sim[w] & range_mask(w, rlo, rhi);
                const int c = __popcll(m);
                if (r < c) lane = w * 64 + nth_bit(m, r);
                else r -= c;
            }
            // Wait until the slot is free: the walker has passed its previous
            // occupant (it may pass one without reading it) and that
            // occupant's producer has finished writing.
            const int slot = pidx % RING;
            LocalSpin sp_;
            bool ok = true;
            while (__hip_atomic_load(&s_cons, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <= pidx - RING ||
                   (pidx >= RING &&
                    __hip_atomic_load(&r_ready[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != pidx - RING)) {
                if (__hip_atomic_load(&s_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ||
                    local_spin_abort(ctl, sp_)) {
                    ok = false;
                    break;
                }
            }
            if (!ok) break;
            // a segment the walker has already passed is not scanned
            if (lane >= 0 && __hip_atomic_load(&s_cons, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <= pidx) {
                if (kept) copy_prefixes(D, k * TILE + lane, ring[slot]);
                else prescan_segment(D, k * TILE + lane, ring[slot]);
            }
            __hip_atomic_store(&r_ready[slot], pidx, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    const int64_t ef = tid == 0 ? s_entry : m_ex[tid - 1];
    const int64_t ex = m_ex[tid];
    const int64_t F0 = s_pre[0] + rF;
    const int64_t P0 = s_pre[1] + rP;
    const int64_t C0 = s_pre[2] + rC;
    uint32_t err = 0;
    int64_t pk = 0, pks = 0;
    bool left = false;  // left to the chain pass
    if (valid) {
        const int64_t af = sp[SP_AF * ns], ac = sp[SP_AC * ns];
        const int64_t mxf = sp[SP_MXF * ns], mnf = sp[SP_MNF * ns], mxp = sp[SP_MXP * ns], mnp = sp[SP_MNP * ns];
        SMP_GLOBAL int64_t* o = gp(D.seg) + j;
        o[SP_F0 * ns] = F0;
        o[SP_P0 * ns] = P0;
        o[SP_C0 * ns] = C0;
        o[SP_EF * ns] = ef;
        o[SP_XF * ns] = ex;
        if (F0 + mxf >= MAX_ABS_F || F0 + mnf <= -MAX_ABS_F || P0 + mxp >= MAX_ABS_F || P0 + mnp <= -MAX_ABS_F ||
            C0 + ac >= MAX_ABS_F || F0 >= MAX_ABS_F || F0 <= -MAX_ABS_F)
            err = 2u;
        pk = F0 + mxf;
        if (j == ns - 1) *gp(&D.scal->final_F) = F0 + af;
        // The chain pass's results, here, for a segment whose entry takes no
        // sample before its first forced event (the prefix's only sample is
        // that event's, and from it on the chain is the summary pass's) or,
        // without a forced event, no sample at all.  Every other segment is
        // left to the chain pass.  (Copy and timer events are counted by the
        // emit pass.)
        const int fn = (int)sp[SP_FN * ns];
        if (fn < 0 && ef >= lo && ef <= hi) {
            // no forced event and an entry inside the no-sample interval:
            // the segment takes no sample
            o[SP_BCNT * ns] = 0;
            o[SP_BGV * ns] = 0;
            o[SP_BGI * ns] = 0;
            o[SP_BGP * ns] = 0;
            o[SP_LSV * ns] = 0;
            o[SP_BFL * ns] = 0;
            SMP_GLOBAL uint64_t* mk = gp(D.mask) + j * NW;
#pragma unroll
            for (int w = 0; w < NW; ++w) mk[w] = 0;
        } else if (fn >= 0 && ef >= sp[SP_PLO * ns] && ef <= sp[SP_PHI * ns]) {
            const int64_t ffn = sp[SP_FFN * ns];
            int64_t gbest = 0, smax = ffn, lsrel;
            int gnode = -1;
            if (ffn > ef) {
                gbest = ffn;
                gnode = fn;
            }
            const int64_t agv = sp[SP_AGV * ns], asmx = sp[SP_ASMX * ns];
            const int agn = (int)sp[SP_AGN * ns], als = (int)sp[SP_ALS * ns];
            if (agn >= 0 && (gnode < 0 || agv > gbest)) {
                gbest = agv;
                gnode = agn;
            }
            if (asmx > smax) smax = asmx;
            lsrel = als >= 0 ? sp[SP_ALP * ns] : sp[SP_PFN * ns];
            pks = F0 + smax;
            const int64_t a = j * SEG;
            const bool hg = gnode >= 0 && gnode < seg_events(D, j);
            o[SP_BCNT * ns] = 1 + sp[SP_ACNT * ns];
            o[SP_BGV * ns] = hg ? F0 + gbest : 0;
            o[SP_BGI * ns] = hg ? a + gnode : 0;
            o[SP_BGP * ns] = hg ? (int64_t)(uint32_t)record(D, a + gnode)[1] : 0;
            o[SP_LSV * ns] = P0 + lsrel;
            o[SP_BFL * ns] = (hg ? 1 : 0) | 2;
            // windows before the forced one hold no sample (as the summary
            // pass wrote); the forced window gains the forced sample
            gp(D.mask)[j * NW + (fn >> 6)] = (1ull << (fn & 63)) | (uint64_t)sp[SP_AMF * ns];
        } else {
            o[SP_BFL * ns] = BFL_CHAIN;
            left = true;
        }
    }
    if (ballot(err != 0) && l == 0) g_or32(&D.scal->err, 2u);
    const int nleft = __popcll(ballot(left));
    pk = wave_max(pk);
    pks = wave_max(pks);
    if (l == 0) {
        w_peak[wv] = pk;
        w_peakS[wv] = pks;
        w_left[wv] = nleft;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t p = 0, q = 0;
        uint64_t c = 0;
        for (int w = 0; w < TWAVES; ++w) {
            p = w_peak[w] > p ? w_peak[w] : p;
            q = w_peakS[w] > q ? w_peakS[w] : q;
            c += (uint64_t)w_left[w];
        }
        if (p > 0) g_max(&D.scal->peak_F, (int64_t)p);
        if (q > 0) g_max(&D.scal->peak_S, (int64_t)q);
        if (c) g_add((uint64_t*)&ctl[4], c);
    }
}

// -------------------------------------------------------------- chain pass

// The first two windows of a segment's records (delta, pointer, flags), which
// the chain pass loads one marked segment ahead: in most segments the first
// forced event lies in them, so the walk needs no other record.
constexpr int HEAD_W = 2;  // (the pointer lookup below assumes two)
struct ChainHead {
    uint64_t d[HEAD_W];
    uint32_t ptr[HEAD_W];
    uint32_t fw[HEAD_W];
};

__device__ __forceinline__ void load_head(const Desc& D, int64_t j, ChainHead& h) {
    gu8_t* base = (gu8_t*)(D.ev + (size_t)(j * SEG) * 24);  // wave-uniform
    const int nv = seg_events(D, j);
#pragma unroll
    for (int w = 0; w < HEAD_W; ++w) {
        gu8_t* p = record_addr(base, nv, w);
        h.d[w] = *(gu64_t*)p;
        h.ptr[w] = *(gu32_t*)(p + 8);
        h.fw[w] = *(gu32_t*)(p + 16);
    }
}

// One wave per segment (grid-stride): follow the chain from the segment's
// entry offset; record its samples, count, best growth sample and the Python
// footprint at its last sample.  Copy and timer events are counted here.
__global__ __launch_bounds__(BLOCK) void k_chain(const Desc* __restrict__ desc, int ntraces, uint64_t nseg_total) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int l = lane_id();
    int cur_t = 0;
    int64_t peakS = 0;
    bool have_t = false;
    // lanes 0-4: prefixes, entry and exit from the resolve pass; lanes 5-17:
    // flags, the chain after the first forced sample and the entries that
    // take no sample before it, from the summary pass.  Each wave reads them
    // one segment ahead.
    const int pl_ = l < 5 ? SP_F0 + l : (l == 5 ? SP_FLG : (l < 18 ? SP_FN + (l - 6) : SP_F0));
    // Only the segments the resolve pass left to this pass, grid-stride:
    // each wave reads the flags of its next 64 segments in one load (lane i:
    // the i-th) and visits the marked ones.
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    uint64_t gb = (uint64_t)blockIdx.x * WAVES + wv, cur_gb = 0;
    uint64_t pend = 0;  // marked segments among the last 64 read, not yet taken
    int hint = 0;       // a trace at or before the wave's next segment
    auto next_marked = [&]() -> uint64_t {
        while (!pend) {
            if (gb >= nseg_total) return nseg_total;
            hint = __builtin_amdgcn_readfirstlane(find_trace_seg(desc, hint, ntraces, gb));
            const uint64_t x = gb + (uint64_t)l * stride;
            bool mk = false;
            if (x < nseg_total) {
                const Desc& Dx = desc[find_trace_seg(desc, hint, ntraces, x)];
                mk = seg_val(Dx, SP_BFL, (int64_t)(x - Dx.seg_begin)) == BFL_CHAIN;
            }
            pend = ballot(mk);
            cur_gb = gb;
            gb += 64 * stride;
        }
        const int i = ctz64(pend);
        pend &= pend - 1;
        return cur_gb + (uint64_t)i * stride;
    };
    uint64_t g = next_marked();
    int64_t pv_next = 0;
    ChainHead hd;  // the head of the wave's next segment
    if (g < nseg_total) {
        const Desc& D0 = desc[__builtin_amdgcn_readfirstlane(find_trace_seg(desc, 0, ntraces, g))];
        pv_next = seg_val(D0, pl_, (int64_t)(g - D0.seg_begin));
        load_head(D0, (int64_t)(g - D0.seg_begin), hd);
    }
    for (uint64_t gn; g < nseg_total; g = gn) {
        gn = next_marked();
        const int t = __builtin_amdgcn_readfirstlane(find_trace_seg(desc, cur_t, ntraces, g));
        if (t != cur_t && have_t && l == 0 && peakS > 0)
            g_max(&desc[cur_t].scal->peak_S, (int64_t)peakS);
        if (t != cur_t) peakS = 0;
        cur_t = t;
        have_t = true;
        const Desc& D = desc[t];
        const int64_t j = (int64_t)(g - D.seg_begin);
        const int64_t ns = (int64_t)D.nseg;
        const int64_t a = j * SEG;
        const int nv = seg_events(D, j);
        const int64_t T = D.T;
        const int64_t pv = pv_next;
        const ChainHead cur = hd;
        {
            // past the last segment, this one's again (no branch)
            const uint64_t gq = gn < nseg_total ? gn : g;
            const Desc& Dn = desc[__builtin_amdgcn_readfirstlane(find_trace_seg(desc, t, ntraces, gq))];
            pv_next = seg_val(Dn, pl_, (int64_t)(gq - Dn.seg_begin));
            load_head(Dn, (int64_t)(gq - Dn.seg_begin), hd);
        }
        const int64_t F0 = readlane64(pv, 0), P0 = readlane64(pv, 1);
        const int64_t eF = readlane64(pv, 3), xF = readlane64(pv, 4);
        const int fn = (int)readlane64(pv, 6);
        // The pointer of the summary pass's best growth sample after the forced
        // event, loaded now (it is the segment's best unless the walk below
        // finds a larger one before the forced event).
        const int agn0 = (int)readlane64(pv, 9);
        uint32_t aptr = 0;
        if (fn >= 0 && agn0 >= 0 && agn0 < nv) aptr = (uint32_t)record(D, a + agn0)[1];
        // From a forced sample on the chain is the one the summary pass followed,
        // so only the events up to it are read again.
        const int fwin = fn >= 0 ? fn >> 6 : NW - 1;
        const int nlim = fn >= 0 ? fn + 1 : nv;
        uint32_t err = 0;
        ChainRun cr{eF, 0, 0, -1, INT64_MIN, -1, 0};
        int64_t lsp = 0, cF = 0, cP = 0;
        const int64_t plo = readlane64(pv, 14), phi = readlane64(pv, 15);
        if (fn >= 0 && eF >= plo && eF <= phi) {
            // No sample before the forced event: the prefix's chain is that
            // event's sample alone, known from the summary pass.
            const int64_t ffn = readlane64(pv, 16);
            if (ffn > eF) {
                cr.gbest = ffn;
                cr.gnode = fn;
            }
            cr.smax = ffn;
            cr.lastS = fn;
            cr.ref = ffn;
            if (l == fwin) cr.mvec = 1ull << (fn & 63);
            cr.cnt = 1;
            lsp = readlane64(pv, 17);
        } else {
            // the chain from the entry, window by window while scanning
            // (prefixes in registers): the head from the prefetch, later
            // windows loaded here
            uint64_t rd[NW - HEAD_W];
            uint32_t rfw[NW - HEAD_W];
            if (fwin >= HEAD_W) {
                gu8_t* base = (gu8_t*)(D.ev + (size_t)a * 24);  // wave-uniform
#pragma unroll
                for (int w = HEAD_W; w < NW; ++w) {
                    gu8_t* p = record_addr(base, nlim, w);
                    rd[w - HEAD_W] = *(gu64_t*)p;
                    rfw[w - HEAD_W] = *(gu32_t*)(p + 16);
                }
            }
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (w > fwin) break;
                const int k = w * 64 + l;
                const uint32_t fl = w < HEAD_W ? cur.fw[w] : rfw[w - HEAD_W];
                const uint64_t rdw = w < HEAD_W ? cur.d[w] : rd[w - HEAD_W];
                const int64_t dm = (k < nlim && (fl & 6u) == 0) ? (int64_t)rdw : 0;
                const int64_t dp = (fl & 1u) ? 0 : dm;
                int64_t f = dm, p = dp;
                wave_incl_sum2(f, p);
                f += cF;
                p += cP;
                cF = readlane64(f, 63);
                cP = readlane64(p, 63);
                chain_window<true>(f, p, T, cr, lsp, w, -1);
            }
        }

        int64_t count = cr.cnt;
        int64_t gbest = cr.gbest, smax = cr.smax, lsrel = 0;
        int gnode = cr.gnode, lastS = cr.lastS;
        if (fn >= 0) {
            if (lastS != fn) err |= 4u;  // internal: every entry samples at a forced event
            count += readlane64(pv, 7);
            const int64_t agv = readlane64(pv, 8), asmx = readlane64(pv, 10);
            const int agn = (int)readlane64(pv, 9), als = (int)readlane64(pv, 11);
            if (agn >= 0 && (gnode < 0 || agv > gbest)) {
                gbest = agv;
                gnode = agn;
            }
            if (asmx > smax) smax = asmx;
            if (als >= 0) {
                lastS = als;
                lsrel = readlane64(pv, 12);
            } else {
                lsrel = lsp;  // the forced sample is the prefix's last
            }
        } else {
            if (cr.ref - cF != xF) err |= 4u;  // internal: the resolved exit disagrees with the chain
            if (lastS >= 0) lsrel = lsp;
        }
        if (smax != INT64_MIN && F0 + smax > peakS) peakS = F0 + smax;
        const bool hg = gnode >= 0 && gnode < nv;  // nodes past the trace end never sample
        uint32_t gptr = 0;
        if (hg) {
            if (fn >= 0 && gnode > fn)
                gptr = aptr;  // the summary pass's sample (gnode == agn0)
            else if (gnode < HEAD_W * 64)
                gptr = (uint32_t)readlane32((int)((gnode >> 6) == 0 ? cur.ptr[0] : cur.ptr[1]), gnode & 63);
            else
                gptr = (uint32_t)record(D, a + gnode)[1];
        }
        const int64_t lsv = lastS >= 0 ? P0 + lsrel : 0;
        if (l < 6) {
            int64_t v;
            switch (l) {
                case 0: v = count; break;
                case 1: v = hg ? F0 + gbest : 0; break;
                case 2: v = hg ? a + gnode : 0; break;
                case 3: v = gptr; break;
                case 4: v = lsv; break;
                default: v = (hg ? 1 : 0) | (lastS >= 0 ? 2 : 0); break;
            }
            gp(D.seg)[(SP_BCNT + l) * ns + j] = v;
        }
        // windows after the forced sample's keep the summary pass's masks
        const uint64_t amf = fn >= 0 ? (uint64_t)readlane64(pv, 13) : 0ull;
        if (l < NW && l <= fwin) gp(D.mask)[j * NW + l] = cr.mvec | (l == fwin ? amf : 0ull);
        if (err && l == 0) g_or32(&D.scal->err, err);
    }
    if (have_t && l == 0 && peakS > 0) g_max(&desc[cur_t].scal->peak_S, (int64_t)peakS);
}

// --------------------------------------------------------------- scan pass

// (count, best growth record, last-sample Python footprint) of a run of segments.
struct BItem {
    Best b;
    bool lsh;
    int64_t ls;
};

__device__ __forceinline__ BItem bcombine(const BItem& a, const BItem& b) {
    BItem r;
    r.b = combine(a.b, b.b);
    r.lsh = a.lsh || b.lsh;
    r.ls = b.lsh ? b.ls : a.ls;
    return r;
}

// One workgroup per tile (ticket order): the state before every segment.
__global__ __launch_bounds__(TILE) void k_bscan(const Desc* __restrict__ desc, int ntraces, uint64_t ntile_total,
                                                unsigned long long* ctl) {
    __shared__ unsigned long long s_tk;
    __shared__ int64_t w_cnt[TWAVES], w_val[TWAVES], w_ls[TWAVES];
    __shared__ uint32_t w_idx[TWAVES], w_ptr[TWAVES];
    __shared__ int w_flags[TWAVES];
    __shared__ int64_t s_pre_cnt, s_pre_val, s_pre_ls;
    __shared__ uint32_t s_pre_idx, s_pre_ptr;
    __shared__ int s_pre_has;
    const int tid = threadIdx.x, wv = tid >> 6, l = lane_id();
    if (tid == 0) s_tk = g_add_rtn((uint64_t*)&ctl[3], 1ull);
    __syncthreads();
    const uint64_t tk = s_tk;
    if (tk >= ntile_total) return;
    const Desc& D = desc[find_trace_tile(desc, ntraces, tk)];
    const int64_t k = (int64_t)(tk - D.tile_begin);
    const int64_t ns = (int64_t)D.nseg;
    const int64_t j = k * TILE + tid;
    const bool valid = j < ns;
    const StatusView ts{D.tstat, (int64_t)D.ntile};
    int64_t cnt = 0, gv = 0, gi = 0, gpt = 0, lsv = 0, fl = 0;
    if (valid) {
        const SMP_GLOBAL int64_t* sp = gp(D.seg) + j;
        cnt = sp[SP_BCNT * ns];
        gv = sp[SP_BGV * ns];
        gi = sp[SP_BGI * ns];
        gpt = sp[SP_BGP * ns];
        lsv = sp[SP_LSV * ns];
        fl = sp[SP_BFL * ns];
    }
    const bool hg = (fl & 1) != 0, hs = (fl & 2) != 0;
    // inclusive within the wave
    const int64_t icnt = wave_incl_sum(cnt);
    const int64_t M = wave_incl_max(hg ? gv : INT64_MIN);
    const int64_t Mp = wave_shr1(M, INT64_MIN);
    const uint64_t le = lanemask_lt() | (1ull << l);
    const uint64_t bnd = ballot(M != INT64_MIN && M > Mp) & le;  // where the running maximum rises
    const int src = bnd ? top64(bnd) : l;
    const uint32_t iidx = (uint32_t)shfl32((int)(uint32_t)gi, src), iptr = (uint32_t)shfl32((int)(uint32_t)gpt, src);
    const uint64_t lsm = ballot(hs) & le;
    const int lsrc = lsm ? top64(lsm) : l;
    const int64_t ils = shfl64(lsv, lsrc);
    if (l == 63) {
        w_cnt[wv] = icnt;
        w_val[wv] = M;
        w_idx[wv] = iidx;
        w_ptr[wv] = iptr;
        w_ls[wv] = ils;
        w_flags[wv] = (M != INT64_MIN ? 1 : 0) | (lsm ? 2 : 0);
    }
    __syncthreads();
    BItem wpre{{0, false, 0, 0, 0}, false, 0}, agg{{0, false, 0, 0, 0}, false, 0};
    for (int w = 0; w < TWAVES; ++w) {
        if (w == wv) wpre = agg;
        const BItem it{{w_cnt[w], (w_flags[w] & 1) != 0, w_val[w], w_idx[w], w_ptr[w]}, (w_flags[w] & 2) != 0, w_ls[w]};
        agg = bcombine(agg, it);
    }
    if (tid == 0) {
        st_status(ts.at(W_BCNT, k), pack(agg.b.cnt, 1));
        st_status(ts.at(W_BGM, k), pack(agg.b.has ? agg.b.val : 0, agg.b.has ? 2 : 1));
        st_status(ts.at(W_BGR, k), pack((int64_t)agg.b.idx, 1));
        st_status(ts.at(W_BGP, k), pack((int64_t)agg.b.ptr, 1));
        st_status(ts.at(W_LSA, k), pack(agg.ls, agg.lsh ? 2 : 1));
    }
    if (wv == 0) {
        Best pre{0, false, 0, 0, 0};
        int64_t eP = 0;
        bool ok = true;
        if (k > 0) {
            ok = scan_best(ts, k, pre, ctl);
            if (ok) ok = scan_last_sample(ts, k, eP, ctl);
        }
        const Best inc = with_baseline(combine(pre, agg.b));
        if (l == 0) {
            st_status(ts.at(W_ICNT, k), pack(inc.cnt, 1));
            st_status(ts.at(W_IGM, k), pack(inc.val, inc.has ? 2 : 1));
            st_status(ts.at(W_IGR, k), pack((int64_t)inc.idx, 1));
            st_status(ts.at(W_IGP, k), pack((int64_t)inc.ptr, 1));
            st_status(ts.at(W_LSI, k), pack(agg.lsh ? agg.ls : eP, 1));
            s_pre_cnt = pre.cnt;
            s_pre_has = pre.has ? 1 : 0;
            s_pre_val = pre.val;
            s_pre_idx = pre.idx;
            s_pre_ptr = pre.ptr;
            s_pre_ls = eP;
            if (!ok) g_or32(&D.scal->err, 8u);
        }
    }
    __syncthreads();
    // state before this segment: tile prefix, waves before, lanes before
    const BItem tpre{{s_pre_cnt, s_pre_has != 0, s_pre_val, s_pre_idx, s_pre_ptr}, true, s_pre_ls};
    const int pl = l > 0 ? l - 1 : 0;
    const int64_t pcnt = shfl64(icnt, pl);
    const uint32_t pidx = (uint32_t)shfl32((int)iidx, pl), pptr = (uint32_t)shfl32((int)iptr, pl);
    const int64_t pls = shfl64(ils, pl);
    const bool plsh = l > 0 && (lsm & ~(1ull << l)) != 0;
    BItem lpre{{l > 0 ? pcnt : 0, l > 0 && Mp != INT64_MIN, Mp, pidx, pptr}, plsh, pls};
    const BItem st = bcombine(bcombine(tpre, wpre), lpre);
    const Best b = with_baseline(st.b);
    if (valid) {
        SMP_GLOBAL int64_t* o = gp(D.seg) + j;
        o[SP_XCNT * ns] = b.cnt;
        o[SP_XHV * ns] = b.val;
        o[SP_XHI * ns] = b.idx;
        o[SP_XHP * ns] = b.ptr;
        o[SP_XFL * ns] = b.has ? 1 : 0;
        o[SP_XLS * ns] = st.ls;
        if (j == ns - 1) *gp(&D.scal->K) = (uint64_t)(b.cnt + cnt);
    }
}

// --------------------------------------------------------------- emit pass

// One wave per segment (grid-stride): write the segment's samples with their
// attribution, per-line counters, tracked samples and the frees that reclaim
// them.
constexpr int STAGE = 128;  // staged sample records per wave
// The emit pass: four waves per workgroup around one line cache (30 KB of
// LDS) and at most 96 VGPRs, so five waves share each SIMD.
constexpr int EMIT_WAVES = 4;
constexpr int EMIT_BLOCK = EMIT_WAVES * 64;

// Write staged samples [0, cnt) (cnt <= 64) to ranks r0.. and add them to
// their lines' counters, one sample per lane.
__device__ __forceinline__ void flush_stage(const Desc& D, uint32_t t, const Sample* stg, int cnt, int64_t r0,
                                            HistCache<EMIT_SLOTS>& hc) {
    const int l = lane_id();
    if (l < cnt && r0 + l < (int64_t)D.n) {
        const Sample smp = stg[l];
        store_sample(D.samples + r0 + l, smp);
        if (smp.line < D.L) {
            const int64_t dl = smp.py + smp.nat;
            const bool gr = dl > 0;
            hist_add(hc, D, t, smp.line, C_PY, smp.py, C_NAT, smp.nat, gr ? C_GN : C_SN, 1, gr ? C_GB : C_SB,
                     gr ? dl : -dl);
        }
    }
}

// What the emit pass loads for a segment: its records, its plane values
// (lanes 0-3: F0, P0, C0, entry offset; lanes 4-9: the scan state before
// the segment; lane 18: its copy bytes; lane 19: its summary flags) and its
// sample masks (lane w: window w).
// The emit pass carries each window's records from one segment to the next
// as one 16-byte vector (delta, pointer, line) and the flags word: the
// registers a refill load writes are then the ones the next segment reads,
// with no copy (a copy would wait for the load).  pv holds, on lanes 0-3,
// F0, P0, C0 and the entry offset, on lanes 4-9 the scan state before the
// segment, on lanes 10-17 the sample masks of windows 0-7, on lane 18 the
// segment's copy bytes and on lane 19 its summary flags.
typedef uint32_t v4u32 __attribute__((ext_vector_type(4), aligned(8)));
typedef const __attribute__((address_space(1))) v4u32 gv4u32_t;

struct EmitIn {
    v4u32 q[NW];
    uint32_t fw[NW];
    int64_t pv;
};

__device__ __forceinline__ void emit_load_record(gu8_t* p, int w, EmitIn& in) {
    in.q[w] = *(gv4u32_t*)p;
    in.fw[w] = *(gu32_t*)(p + 16);
}

// A segment of the emit pass: trace t, index j in the trace, nv records.
struct EmitSeg {
    int t;
    int64_t j;
    int nv;
};

__device__ __forceinline__ void emit_fetch_meta(const Desc& D, int64_t j, EmitIn& in) {
    const int l = lane_id();
    const int pl = l < 4 ? SP_F0 + (l == 3 ? SP_EF - SP_F0 : l) : (l == 18 ? SP_AC : (l == 19 ? SP_FLG : SP_XCNT + (l - 4)));
    gi64_t* src = (l < 10 || l == 18 || l == 19) ? (gi64_t*)D.seg + (int64_t)pl * (int64_t)D.nseg + j
                                                 : (gi64_t*)D.mask + j * NW + ((l - 10) & (NW - 1));
    in.pv = *src;
}

// Emit segment s from in: its samples (staged in stg), the tracked and freed
// bits of its growth samples and its lines' counters.  When hn, the wave's
// next segment sn is loaded into in as this one is consumed: its planes at
// the start, its records window by window as each window's registers free up
// (so the next segment's loads are in flight while this one computes).
__device__ __forceinline__ void emit_segment(const Desc* __restrict__ desc, const EmitSeg& s, HistCache<EMIT_SLOTS>& hc,
                                             Sample* stg, EmitIn& in, bool hn, const EmitSeg& sn) {
    const int l = lane_id();
    const int t = s.t;
    const Desc& D = desc[t];
    const int64_t a = s.j * SEG;
    const int nv = s.nv;
    const int64_t pv = in.pv;
    const Desc& Dn = desc[sn.t];
    gu8_t* nbase = (gu8_t*)(Dn.ev + (size_t)(sn.j * SEG) * 24);  // wave-uniform
    const int64_t F0 = readlane64(pv, 0), P0 = readlane64(pv, 1), eF = readlane64(pv, 3);
    // Copy volume (section 3.5: one Tc sample per multiple of Tc crossed by
    // the cumulative copy bytes) and the timer split (section 2.1: Python
    // time += quantum, native time += delay) go to the lines' counters here.
    // Only a segment that holds such events (summary flag bit 2) looks for
    // them, and only one whose copy bytes cross a multiple of Tc holds a copy
    // sample and scans its copy bytes.
    const bool has_aux = (readlane64(pv, 19) & 4) != 0;
    int64_t cc = 0;
    bool csmp = false;
    if (has_aux) {
        cc = readlane64(pv, 2);
        const uint64_t c0u = (uint64_t)cc, c1u = c0u + (uint64_t)readlane64(pv, 18);
        csmp = D.tc_shift >= 0 ? (c1u >> D.tc_shift) != (c0u >> D.tc_shift)
                               : c1u / (uint64_t)D.Tc != c0u / (uint64_t)D.Tc;
    }
    int64_t base = readlane64(pv, 4);
    const int64_t hv = readlane64(pv, 5);
    const uint32_t hidx = (uint32_t)readlane64(pv, 6), hptr = (uint32_t)readlane64(pv, 7);
    const bool hh = (readlane64(pv, 8) & 1) != 0;
    const int64_t eP = readlane64(pv, 9);
    uint64_t wm[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) wm[w] = readlaneu64((uint64_t)pv, 10 + w);
    if (hn) emit_fetch_meta(Dn, sn.j, in);
    uint32_t err = 0;
    if (base < 0 || base > (int64_t)D.n) {  // only reachable after an internal fault
        err |= 8u;
        base = 0;
    }
    int64_t refF = eF, refP = eP - P0;
    int64_t cnt = 0;
    bool cur_has = hh;
    uint32_t cur_ptr = hptr, cur_idx = hidx;
    int64_t hwm = hh ? hv : 0;
    int64_t cF = 0, cP = 0;
    // Sample records are staged in LDS in rank order and written (with their
    // per-line counters) 64 at a time, all lanes busy.
    int staged = 0;
    int64_t stage_rank = base;
    // Window by window: decode and scan (prefixes stay in registers), then
    // the window's samples and frees.
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int k = w * 64 + l;
        const uint32_t fl = in.fw[w];
        const int64_t dm = (k < nv && (fl & 6u) == 0) ? (int64_t)(((uint64_t)in.q[w].y << 32) | in.q[w].x) : 0;
        const int64_t dp = (fl & 1u) ? 0 : dm;
        int64_t f = dm, p = dp;
        wave_incl_sum2(f, p);
        f += cF;
        p += cP;
        cF = readlane64(f, 63);
        cP = readlane64(p, 63);
        const uint64_t fm = ballot(dm < 0);
        const uint64_t m = wm[w];
        if (m != 0 || (fm != 0 && cur_has)) {
            const uint32_t pt = in.q[w].z, wline = in.q[w].w;
            const uint64_t below = m & lanemask_lt();
            uint64_t tmask = 0;
            if (m) {
                const int pl = below ? top64(below) : l;
                int64_t fprev = shfl64(f, pl), pprev = shfl64(p, pl);
                if (!below) {
                    fprev = refF;
                    pprev = refP;
                }
                const bool is_s = ((m >> l) & 1) && k < nv;
                const int64_t dl = f - fprev;
                const int64_t pyb = p - pprev;
                const int64_t nat = dl - pyb;
                const int64_t Fabs = F0 + f;
                const int64_t rank = base + cnt + __popcll(below);
                if (is_s) {
                    Sample smp;
                    smp.event_idx = (uint32_t)(a + k);
                    smp.line = wline;
                    smp.F = Fabs;
                    smp.py = pyb;
                    smp.nat = nat;
                    stg[staged + __popcll(below)] = smp;
                }
                uint64_t cand = ballot(is_s && dl > 0 && Fabs > hwm);
                while (cand) {
                    const int c = ctz64(cand);
                    cand &= cand - 1;
                    const int64_t Fc = readlane64(Fabs, c);
                    if (Fc > hwm) {
                        hwm = Fc;
                        tmask |= 1ull << c;
                    }
                }
                if (((tmask >> l) & 1) && rank < (int64_t)D.n) {
                    g_or(&D.tracked_bits[rank >> 6], 1ull << (rank & 63));
                    gp(D.sample_ptr)[rank] = pt;
                }
                const int ls = top64(m);
                refF = readlane64(f, ls);
                refP = readlane64(p, ls);
            }
            if (fm && tmask) {
                // a new tracked object in this window: each free compares
                // with the last one tracked before it
                const uint64_t tb = tmask & lanemask_lt();
                const int al = tb ? top64(tb) : l;
                const uint32_t spt = (uint32_t)shfl32((int)pt, al);
                const uint32_t aptr = tb ? spt : cur_ptr;
                const uint32_t aidx = tb ? (uint32_t)(a + w * 64 + al) : cur_idx;
                const bool ahas = tb != 0 || cur_has;
                if (((fm >> l) & 1) && ahas && pt == aptr && aidx < D.n)
                    g_or(&D.freed_bits[aidx >> 6], 1ull << (aidx & 63));
            } else if (fm && cur_has) {
                // (the usual case) every free compares with the active object
                if (((fm >> l) & 1) && pt == cur_ptr && cur_idx < D.n)
                    g_or(&D.freed_bits[cur_idx >> 6], 1ull << (cur_idx & 63));
            }
            if (tmask) {
                const int tl = top64(tmask);
                cur_ptr = (uint32_t)readlane32((int)pt, tl);
                cur_idx = (uint32_t)(a + w * 64 + tl);
                cur_has = true;
            }
            cnt += __popcll(m);
            staged += __popcll(m);
        }
        // the window's copy and timer events (validated as in the summary pass)
        if (has_aux) {
            const uint32_t kind = (fl >> 1) & 3u;
            const uint64_t r0 = ((uint64_t)in.q[w].y << 32) | in.q[w].x;
            const uint32_t line = in.q[w].w;
            const bool lok = k < nv && line < D.L;
            const bool cp = lok && kind == 1u && r0 < (uint64_t)MAX_ABS_DELTA;
            const bool tm = lok && kind == 2u && (r0 >> 32) == 0;
            if (ballot(cp || tm)) {
                int64_t vcs = 0;  // bytes of the copy samples this event triggers
                if (csmp) {
                    const int64_t dc = cp ? (int64_t)r0 : 0;
                    const int64_t sc_ = wave_incl_sum(dc) + cc;
                    cc = readlane64(sc_, 63);
                    const uint64_t cout = (uint64_t)sc_, cin = cout - (uint64_t)dc;
                    const uint64_t nsmp = D.tc_shift >= 0 ? (cout >> D.tc_shift) - (cin >> D.tc_shift)
                                                          : cout / (uint64_t)D.Tc - cin / (uint64_t)D.Tc;
                    vcs = (int64_t)(nsmp * (uint64_t)D.Tc);
                }
                if (cp || tm)
                    hist_add(hc, D, (uint32_t)t, line, cp ? C_CS : C_PT, cp ? vcs : D.q, cp ? C_CE : C_NT, (int64_t)r0,
                             -1, 0, -1, 0);
            }
        }
        // this window's registers take the next segment's window w (after
        // their last use here, so no copies and no early wait)
        if (hn) emit_load_record(record_addr(nbase, sn.nv, w), w, in);
        if (staged >= 64) {
            flush_stage(D, (uint32_t)t, stg, 64, stage_rank, hc);
            stage_rank += 64;
            staged -= 64;
            Sample rest;
            if (l < staged) rest = stg[64 + l];
            if (l < staged) stg[l] = rest;
        }
    }
    if (staged) flush_stage(D, (uint32_t)t, stg, staged, stage_rank, hc);
    if (err && l == 0) g_or32(&D.scal->err, err);
}

__global__ __launch_bounds__(EMIT_BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_emit(
    const Desc* __restrict__ desc, int ntraces, uint64_t nseg_total) {
    __shared__ HistCache<EMIT_SLOTS> hc;
    __shared__ Sample stage[EMIT_WAVES][STAGE];
    hist_init(hc);
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    // A batch of several traces: each workgroup takes one contiguous run of
    // segments (its waves interleaved in it), so that it sees the lines of
    // one or two traces and its line cache holds their hot lines; spread over
    // the grid, it would fill the cache with the first keys seen and send
    // nearly every later update to global atomics.  A single trace: segments
    // grid-stride (consecutive waves, consecutive segments), which streams
    // HBM faster than one run per workgroup.  Each wave loads its next
    // segment while it emits the current.
    uint64_t g, g_end, stride;
    if (ntraces > 1) {
        const uint64_t per = (nseg_total + (uint64_t)gridDim.x * EMIT_WAVES - 1) / ((uint64_t)gridDim.x * EMIT_WAVES);
        const uint64_t e0 = ((uint64_t)blockIdx.x + 1) * per * EMIT_WAVES;
        g = (uint64_t)blockIdx.x * per * EMIT_WAVES + wv;
        g_end = e0 < nseg_total ? e0 : nseg_total;
        stride = EMIT_WAVES;
    } else {
        g = (uint64_t)blockIdx.x * EMIT_WAVES + wv;
        g_end = nseg_total;
        stride = (uint64_t)gridDim.x * EMIT_WAVES;
    }
    if (g < g_end) {
        auto locate = [&](uint64_t x, int from) {
            EmitSeg r;
            r.t = __builtin_amdgcn_readfirstlane(find_trace_seg(desc, from, ntraces, x));
            r.j = (int64_t)(x - desc[r.t].seg_begin);
            r.nv = seg_events(desc[r.t], r.j);
            return r;
        };
        EmitSeg s = locate(g, 0);
        EmitIn in;
        emit_fetch_meta(desc[s.t], s.j, in);
        {
            gu8_t* base = (gu8_t*)(desc[s.t].ev + (size_t)(s.j * SEG) * 24);
#pragma unroll
            for (int w = 0; w < NW; ++w) emit_load_record(record_addr(base, s.nv, w), w, in);
        }
        for (;;) {
            const uint64_t gn = g + stride;
            const bool hn = gn < g_end;
            const EmitSeg sn = hn ? locate(gn, s.t) : s;
            emit_segment(desc, s, hc, stage[wv], in, hn, sn);
            if (!hn) break;
            g = gn;
            s = sn;
        }
    }
    __syncthreads();
    hist_flush(hc, desc);
}

// ----------------------------------------------------------------- clearing

__global__ void k_clear(const Desc* __restrict__ desc, int ntraces, uint64_t total_bytes, unsigned long long* ctl) {
    const uint64_t chunk = 1ull << 16;
    const uint64_t begin = (uint64_t)blockIdx.x * chunk;
    if (blockIdx.x == 0 && threadIdx.x < 32) gp(ctl)[threadIdx.x] = 0;
    if (begin >= total_bytes) return;
    const uint64_t end = begin + chunk < total_bytes ? begin + chunk : total_bytes;
    // traces overlapping [begin, end)
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].zero_begin <= begin) lo = mid; else hi = mid - 1;
    }
    for (int t = lo; t < ntraces; ++t) {
        const Desc& D = desc[t];
        if (D.zero_begin >= end) break;
        const uint64_t s = D.zero_begin > begin ? D.zero_begin : begin;
        const uint64_t e = (D.zero_begin + D.zero_bytes) < end ? (D.zero_begin + D.zero_bytes) : end;
        if (s >= e) continue;
        SMP_GLOBAL uint64_t* p = gp((uint64_t*)(D.zero_ptr + (s - D.zero_begin)));
        const uint64_t nw = (e - s) >> 3;
        for (uint64_t i = threadIdx.x; i < nw; i += blockDim.x) p[i] = 0;
    }
}

// ------------------------------------------------ tracked-list compaction

constexpr int CBLK_WORDS = 256;    // bitmap words per compaction block (one per thread)
constexpr int TRACK_UNROLL = 4;    // tracked entries per thread and trip of the fill

__device__ __forceinline__ int find_trace_blk(const Desc* desc, int ntraces, uint64_t x) {
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].blk_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Count before compaction block b of a trace's tracked bitmap, by a
// decoupled look-back over its earlier blocks (one wave; status words st:
// state 1 = a block's own count, 2 = the count through it).
__device__ bool count_lookback(const uint64_t* st, int64_t b, uint64_t& excl, unsigned long long* ctl) {
    const int l = lane_id();
    uint64_t acc = 0;
    int64_t base = b - 1;
    Spin sp;
    while (base >= 0) {
        const int64_t jj = base - l;
        const bool in = jj >= 0;
        const uint64_t w = in ? ld_status(st + (in ? jj : 0)) : 0;
        const uint32_t stt = wstate(w);
        const uint64_t incl = ballot(in && stt == 2);
        // lanes before the nearest inclusive word need their blocks' own counts
        const int lim = incl ? ctz64(incl) : 64;
        const uint64_t need = ballot(in && l < lim);
        if ((ballot(in && stt != 0) & need) != need) {
            if (spin_abort(ctl, sp)) return false;
            continue;
        }
        acc += (uint64_t)wave_sum(in && l <= lim && (l < lim || incl) ? unpack(w) : 0);
        if (incl) break;
        base -= 64;
    }
    excl = acc;
    return true;
}

// Ordered tracked list (the samples that set a new high-water mark, section
// 3.4) in one pass: the entries in rank order, each with the event, line and
// ptr_id of its sample and whether a free reclaimed it, and the per-line
// (mallocs, frees) counts.  Grid-stride over the compaction blocks of every
// trace's tracked bitmap (only the blocks that hold words below the trace's
// sample count do work), each workgroup taking its blocks in increasing
// order.  A block counts its set bits, publishes that count (status words in
// D.blk, cleared per launch), takes the count before it from a look-back
// over the trace's earlier blocks and writes its entries; the block holding
// the bitmap's last word writes H.  The grid never exceeds what the device
// holds at once, so every block a look-back waits on belongs to a running
// workgroup that reaches it in order.  Every reclaimed object is counted
// here; the last one of a trace (unresolved unless RESOLVE_AT_END) is taken
// back out by k_finish.
__global__ __launch_bounds__(256) void k_track(const Desc* __restrict__ desc, int ntraces, uint64_t nblk_total,
                                               unsigned long long* ctl) {
    __shared__ HistCache<TRACK_SLOTS> hc;
    __shared__ uint64_t s_excl;
    __shared__ uint64_t w_cnt[4];
    hist_init(hc);
    __syncthreads();
    const int tid = threadIdx.x, l = lane_id(), wv = tid >> 6;
    constexpr int PER = CBLK_WORDS / 256;  // each thread owns PER consecutive words
    for (uint64_t b = blockIdx.x; b < nblk_total; b += gridDim.x) {
        const uint32_t t = (uint32_t)find_trace_blk(desc, ntraces, b);
        const Desc& D = desc[t];
        const uint64_t lb = b - D.blk_begin;
        const uint64_t Kr = *gp(&D.scal->K);
        const uint64_t K = Kr < D.n ? Kr : D.n;
        const uint64_t nwords = (K + 63) >> 6;
        const uint64_t w0 = lb * CBLK_WORDS;
        if (w0 >= nwords) continue;  // (workgroup-uniform) no sample of this trace in the block
        uint64_t words[PER];
        uint64_t c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint64_t wi = w0 + (uint64_t)tid * PER + i;
            words[i] = wi < nwords ? gp(D.tracked_bits)[wi] : 0;
            c += __popcll(words[i]);
        }
        const uint64_t ci = (uint64_t)wave_incl_sum((int64_t)c);
        if (l == 63) w_cnt[wv] = ci;
        __syncthreads();
        uint64_t woff = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wv) woff += w_cnt[w];
            total += w_cnt[w];
        }
        uint64_t* st = D.blk;
        if (wv == 0) {
            uint64_t excl = 0;
            bool ok = true;
            if (lb == 0) {
                if (l == 0) st_status(st, pack((int64_t)total, 2));
            } else {
                if (l == 0) st_status(st + lb, pack((int64_t)total, 1));
                ok = count_lookback(st, (int64_t)lb, excl, ctl);
                if (l == 0) st_status(st + lb, pack((int64_t)(excl + total), 2));
            }
            if (l == 0) {
                s_excl = excl;
                if (!ok) g_or32(&D.scal->err, 8u);
            }
        }
        __syncthreads();
        const uint64_t h0 = s_excl, h1 = s_excl + total;
        if (tid == 0 && w0 + CBLK_WORDS >= nwords) *gp(&D.scal->H) = h1;
        // First the sample rank of each entry (tracked samples cluster, so a
        // thread may own many), then the entries, spread over all threads.
        uint64_t h = h0 + woff + ci - c;
        SMP_GLOBAL uint32_t* tq = (SMP_GLOBAL uint32_t*)D.tracked;
        for (int i = 0; i < PER; ++i) {
            uint64_t m = words[i];
            const uint64_t wi = w0 + (uint64_t)tid * PER + i;
            while (m) {
                const int bit = __builtin_ctzll(m);
                m &= m - 1;
                const uint64_t r = wi * 64 + bit;
                tq[4 * h] = r < K ? (uint32_t)r : 0xFFFFFFFFu;  // (r >= K only after an internal fault)
                ++h;
            }
        }
        __syncthreads();
        // TRACK_UNROLL entries per thread and trip, each step's loads issued
        // for all of them before the first is used: a block may hold many
        // thousands of entries, and one at a time its three dependent loads
        // (rank, sample, freed bit) would each cost a full round trip.
        for (uint64_t hb = h0 + tid; hb < h1; hb += 256 * TRACK_UNROLL) {
            uint32_t r[TRACK_UNROLL], ptr[TRACK_UNROLL];
            uint64_t sw[TRACK_UNROLL], fw[TRACK_UNROLL];
#pragma unroll
            for (int u = 0; u < TRACK_UNROLL; ++u) {
                const uint64_t hh = hb + 256 * (uint64_t)u;
                r[u] = hh < h1 ? tq[4 * hh] : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int u = 0; u < TRACK_UNROLL; ++u) {
                const uint32_t rr = r[u] < K ? r[u] : 0u;
                sw[u] = *(const SMP_GLOBAL uint64_t*)(D.samples + rr);  // event index, line
                ptr[u] = gp(D.sample_ptr)[rr];
            }
#pragma unroll
            for (int u = 0; u < TRACK_UNROLL; ++u) {
                const uint32_t ev = (uint32_t)sw[u];
                fw[u] = r[u] < K && ev < D.n ? gp(D.freed_bits)[ev >> 6] : 0;
            }
#pragma unroll
            for (int u = 0; u < TRACK_UNROLL; ++u) {
                if (r[u] >= K) continue;  // (past the block's entries, or after an internal fault)
                const uint64_t hh = hb + 256 * (uint64_t)u;
                const uint32_t ev = (uint32_t)sw[u], line = (uint32_t)(sw[u] >> 32);
                const uint32_t freed = (uint32_t)((fw[u] >> (ev & 63)) & 1);
                tq[4 * hh] = ev;
                tq[4 * hh + 1] = line;
                tq[4 * hh + 2] = ptr[u];
                tq[4 * hh + 3] = freed;
                if (line < D.L) hist_add(hc, D, t, line, C_LM, 1, C_LF, (int64_t)freed, -1, 0, -1, 0);
            }
        }
        __syncthreads();  // w_cnt and s_excl are reused by the next block
    }
    __syncthreads();
    hist_flush(hc, desc);
}

// ------------------------------------------------ leak likelihood per line

__device__ int64_t gcd64(int64_t x, int64_t y) {
    if (x < 0) x = -x;
    while (y) {
        const int64_t r = x % y;
        x = y;
        y = r;
    }
    return x;
}

// After the tracked list: per line, exact reduced rationals of the leak
// likelihood (section 3.4) - Laplace's rule of succession (m-f+1)/(m+2) and
// the formula as printed (m-2f+1)/(m-f+2) - and their gates, likelihood >
// 0.95.  The last tracked object of a trace stays unresolved (its free does
// not count) unless RESOLVE_AT_END, so the thread of its line takes it back
// out of that line's frees.  Threads below 8 x ntraces also gather every
// trace's scalars (final from here on) into one array, which may live in
// pinned host memory (the host reads it once the launch has completed).
__global__ void k_finish(const Desc* __restrict__ desc, int ntraces, uint64_t total_lines, Scalars* gather) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint64_t)ntraces * 8) {
        const uint64_t t = i >> 3, w = i & 7;  // 8 words per Scalars
        gp((uint64_t*)(gather + t))[w] = gp((const uint64_t*)desc[t].scal)[w];
    }
    if (i >= total_lines) return;
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].line_begin <= i) lo = mid; else hi = mid - 1;
    }
    const Desc& D = desc[lo];
    const uint64_t line = i - D.line_begin;
    if (line >= D.L) return;
    SMP_GLOBAL int64_t* hist = gp(D.hist);
    const int64_t m = hist[(size_t)H_LEAK_M * D.L + line];
    int64_t f = hist[(size_t)H_LEAK_F * D.L + line];
    if (m > 0 && (D.options & 2u) == 0) {
        const uint64_t H = *gp(&D.scal->H);
        if (H > 0) {
            const SMP_GLOBAL uint32_t* last = (const SMP_GLOBAL uint32_t*)(D.tracked + (H - 1));
            if (last[1] == (uint32_t)line && last[3] != 0) {
                f -= 1;
                hist[(size_t)H_LEAK_F * D.L + line] = f;
            }
        }
    }
    SMP_GLOBAL int64_t* out = gp(D.leak);
    SMP_GLOBAL uint8_t* gates = gp(D.gates);
    if (m <= 0) {
        out[line] = 0;
        out[D.L + line] = 0;
        out[2 * (size_t)D.L + line] = 0;
        out[3 * (size_t)D.L + line] = 0;
        gates[line] = 0;
        gates[D.L + line] = 0;
        return;
    }
    int64_t n1 = m - f + 1, d1 = m + 2;
    int64_t n2 = m - 2 * f + 1, d2 = m - f + 2;
    const uint8_t g1 = 20 * n1 > 19 * d1;
    const uint8_t g2 = 20 * n2 > 19 * d2;
    if (n1 == 0) { d1 = 1; } else { const int64_t g = gcd64(n1, d1); n1 /= g; d1 /= g; }
    if (n2 == 0) { d2 = 1; } else { const int64_t g = gcd64(n2, d2); n2 /= g; d2 /= g; }
    out[line] = n1;
    out[D.L + line] = d1;
    out[2 * (size_t)D.L + line] = n2;
    out[3 * (size_t)D.L + line] = d2;
    gates[line] = g1;
    gates[D.L + line] = g2;
}

// ------------------------------------------------------------ launchers

static int occupancy_grid(const void* fn, int block) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, block, 0) != hipSuccess) return 0;
    return cus * (per > 0 ? per : 1);
}

int chain_grid_limit() { return occupancy_grid((const void*)k_chain, BLOCK); }
int emit_grid_limit() { return occupancy_grid((const void*)k_emit, EMIT_BLOCK); }
// workgroups of k_track the device holds at once (its look-back needs all of them resident)
int track_grid_limit() { return occupancy_grid((const void*)k_track, 256); }

hipError_t launch_clear(const Desc* desc, int ntraces, uint64_t total_bytes, unsigned long long* ctl, hipStream_t s) {
    const uint64_t blocks = (total_bytes + (1ull << 16) - 1) >> 16;
    k_clear<<<dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s>>>(desc, ntraces, total_bytes, ctl);
    return hipGetLastError();
}

hipError_t launch_tmap(const Desc* desc, int ntraces, uint64_t ntile_total, unsigned long long* ctl, hipStream_t s) {
    if (ntile_total == 0) return hipSuccess;
    k_tmap<<<dim3((unsigned)ntile_total), dim3(64), 0, s>>>(desc, ntraces, ctl);
    return hipGetLastError();
}

hipError_t launch_pass(int pass, const Desc* desc, int ntraces, uint64_t nseg_total, uint64_t ntile_total,
                       unsigned long long* ctl, int grid_limit, hipStream_t s) {
    if (nseg_total == 0) return hipSuccess;
    const uint64_t wgs = (nseg_total + WAVES - 1) / WAVES;
    const unsigned pgrid = (unsigned)(wgs < (uint64_t)grid_limit ? wgs : (uint64_t)grid_limit);
    switch (pass) {
        case 0: k_summarize<<<dim3((unsigned)wgs), dim3(BLOCK), 0, s>>>(desc, ntraces, nseg_total); break;
        case 1: k_resolve<<<dim3((unsigned)ntile_total), dim3(TILE), 0, s>>>(desc, ntraces, ntile_total, ctl); break;
        case 2: k_chain<<<dim3(pgrid), dim3(BLOCK), 0, s>>>(desc, ntraces, nseg_total); break;
        case 3: k_bscan<<<dim3((unsigned)ntile_total), dim3(TILE), 0, s>>>(desc, ntraces, ntile_total, ctl); break;
        default: {
            const uint64_t ewgs = (nseg_total + EMIT_WAVES - 1) / EMIT_WAVES;
            const unsigned egrid = (unsigned)(ewgs < (uint64_t)grid_limit ? ewgs : (uint64_t)grid_limit);
            k_emit<<<dim3(egrid), dim3(EMIT_BLOCK), 0, s>>>(desc, ntraces, nseg_total);
            break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_finish(const Desc* desc, int ntraces, uint64_t nblk_total, uint64_t total_lines,
                         unsigned long long* ctl, int track_grid, Scalars* gather, hipStream_t s) {
    if (nblk_total) {
        const unsigned g = (unsigned)(nblk_total < (uint64_t)track_grid ? nblk_total : (uint64_t)track_grid);
        k_track<<<dim3(g), dim3(256), 0, s>>>(desc, ntraces, nblk_total, ctl);
    }
    const uint64_t items = total_lines > (uint64_t)ntraces * 8 ? total_lines : (uint64_t)ntraces * 8;
    k_finish<<<dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s>>>(desc, ntraces, total_lines, gather);
    return hipGetLastError();
}

}  // namespace smp
