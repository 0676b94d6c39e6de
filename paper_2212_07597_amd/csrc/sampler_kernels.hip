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
//    of them coincide the segment's exit is known before its entry is, so
//    segments hand their state on without waiting (a decoupled look-back over
//    maps instead of sums).
//  * Attribution (section 3.3): each sample goes to the triggering event's
//    line with the net Python and native bytes since the previous sample.
//  * Leak rule (section 3.4): a growth sample above the high-water mark of the
//    earlier tracked samples is tracked; frees of its ptr_id before the next
//    tracked sample mark it reclaimed.  The high-water mark and the active
//    tracked object flow between segments as a running "argmax" (the largest
//    growth footprint, earliest on ties).
//  * Copy volume (section 3.5) and the timer split (section 2.1) are
//    per-event histogram updates.
#include "sampler_device.h"

// Optional per-phase cycle counters (diagnostic builds only, -DSMP_PHASE_STATS):
// each wave accumulates shader-clock cycles per phase and a few event counts,
// then adds them once to ctl[8 + i] at exit.
#ifdef SMP_PHASE_STATS
#define PH_DECL uint64_t ph[16] = {0}; uint64_t ph_t = clock64();
#define PH_MARK(i) do { const uint64_t _n = clock64(); ph[i] += _n - ph_t; ph_t = _n; } while (0)
#define PH_COUNT(i, v) ph[i] += (uint64_t)(v)
#define PH_FLUSH(ctl) do { if (lane_id() == 0) for (int _i = 0; _i < 16; ++_i) atomicAdd(&(ctl)[8 + _i], ph[_i]); } while (0)
#else
#define PH_DECL
#define PH_MARK(i) do {} while (0)
#define PH_COUNT(i, v) do {} while (0)
#define PH_FLUSH(ctl) do {} while (0)
#endif

namespace smp {

#ifdef SMP_PHASE_STATS
// look-back diagnostics: [0] sums iterations, [1] sums spins, [2] sums lim total,
// [3] best iterations, [4] best spins, [5] best lim total, [6] ls spins, [7] chain slow path
__device__ unsigned long long g_lbstat[8];
#define LB_COUNT(i, v) do { if (lane_id() == 0) atomicAdd(&g_lbstat[i], (unsigned long long)(v)); } while (0)
#else
#define LB_COUNT(i, v) do {} while (0)
#endif

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
        default: return H_NT;
    }
}

struct SegLds {
    int64_t F[SEG];     // footprint after each event, relative to the segment start
    int64_t P[SEG];     // Python footprint after each event, relative
    uint32_t ptr[SEG];  // line ids are re-read from the records at samples
};

struct HistCache {
    unsigned long long key[NSLOT];  // (trace << 32) | line, or ~0 when empty
    unsigned long long cnt[NSLOT][NCNT];
};

constexpr unsigned long long EMPTY_KEY = ~0ull;

// Add up to four counters of (trace t, line) through the workgroup's LDS
// cache; a slot held by another line sends the update to global atomics.
__device__ __forceinline__ void hist_add(HistCache& hc, const Desc& D, uint32_t t, uint32_t line, int c0, int64_t v0,
                                         int c1, int64_t v1, int c2, int64_t v2, int c3, int64_t v3) {
    const unsigned long long key = ((unsigned long long)t << 32) | line;
    const uint32_t h = (line * 2654435761u) ^ (t * 0x9E3779B9u);
    const int slot = (int)(h >> (32 - 7)) & (NSLOT - 1);
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
                atomicAdd((unsigned long long*)&D.hist[(size_t)cache_to_hist(cs[i]) * D.L + line],
                          (unsigned long long)vs[i]);
    }
}

// ---------------------------------------------------------------- look-backs

// Every wait on another segment's status polls with a budget and an
// exponential back-off.  Running out of budget (only possible through an
// internal fault) raises the launch-wide abort word, after which every wait
// returns at once, so all waves always exit.
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

// ------------------------------------------------- decoupled look-backs
//
// Segment g looks at its predecessors g-1-l (lane l, nearest first).  It
// needs the nearest one that has published an inclusive value and the
// aggregates of all segments after it.  Having them, it can also compute the
// inclusive values of those intermediate segments, and it publishes them
// ("helping"): the resolved frontier then advances as fast as aggregates
// appear instead of one look-back at a time.  Identical values may be
// written by several waves; a reader sees either copy.

// Exclusive (F, P, C) prefix of segment g.  Loads are kept small: the
// predecessor's inclusive first (three lanes), then one state word per lane to
// find the nearest published inclusive, then the aggregates of the segments
// after it; a wait re-reads only the lanes still missing.
__device__ bool scan_sums(const StatusView& sv, int64_t g, int64_t& oF, int64_t& oP, int64_t& oC, unsigned long long* ctl) {
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
        uint64_t x0 = 0, x1 = 0, x2 = 0;   // aggregate (need) or inclusive (at) words
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
            LB_COUNT(1, 1);
            if (spin_abort(ctl, sp)) return false;
        }
        LB_COUNT(0, 1);
        LB_COUNT(2, lim);
        const int64_t vF = (need || at) ? unpack(x0) : 0;
        const int64_t vP = (need || at) ? unpack(x1) : 0;
        const int64_t vC = (need || at) ? unpack(x2) : 0;
        // suffix sums toward older segments: S_l = sum over lanes >= l
        const int64_t xF = wave_incl_sum(vF), xP = wave_incl_sum(vP), xC = wave_incl_sum(vC);
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

// value of lane l + d (lanes past 63 get `fill`)
__device__ __forceinline__ int64_t lane_down(int64_t x, int d, int64_t fill) {
    const int l = lane_id();
    const int64_t y = shfl64(x, l + d < 64 ? l + d : l);
    return l + d < 64 ? y : fill;
}

// Exclusive Best prefix of segment g (baseline applied), loading as scan_sums.
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
    Best acc{0, false, 0, 0, 0};  // later segments combined so far
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
            LB_COUNT(4, 1);
            if (spin_abort(ctl, sp)) return false;
        }
        LB_COUNT(3, 1);
        LB_COUNT(5, lim);
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
        Best r = win;
        r.cnt = win.cnt + acc.cnt;
        if (acc.has && (!win.has || acc.val > win.val)) {
            r.has = true;
            r.val = acc.val;
            r.idx = acc.idx;
            r.ptr = acc.ptr;
        }
        acc = r;
        if (im) break;
        base -= 64;
        first = false;
    }
    out = with_baseline(acc);
    return true;
}

// Absolute Python footprint at the last sample before segment g (0 if none).
__device__ bool scan_last_sample(const StatusView& sv, int64_t g, int64_t& oP, unsigned long long* ctl) {
    const int l = lane_id();
    int64_t base = g - 1;
    bool first = true;
    Spin sp;
    while (base >= 0) {
        const int64_t jj = base - l;
        const bool in = jj >= 0;
        uint64_t li = 0, la = 0;
        const int64_t js = in ? jj : 0;
        if (in) {
            li = ld_status(sv.at(W_LSI, js));
            la = ld_status(sv.at(W_LSA, js));
        }
        // a lane resolves the search if its segment has a sample or a known exit value
        const bool hit = in && (wstate(la) == 2 || wstate(li) != 0);
        const uint64_t hm = ballot(hit);
        const int lim = hm ? ctz64(hm) : __popcll(ballot(in));
        if (ballot(in && l < lim && wstate(la) == 0)) {
            LB_COUNT(6, 1);
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

// Entry reference offset of segment g (relative to its first event).
__device__ bool lookback_chain(const const StatusView& sv, int64_t g, int64_t& eF, unsigned long long* ctl) {
    const int l = lane_id();
    Spin sp;
    int i0;
    uint64_t xF;
    // fast path: the predecessor's exit (published early when its map is total)
    for (int tries = 0; tries < 3; ++tries) {
        const uint64_t a = ld_status(sv.at(W_XF, g - 1));
        if (wstate(a)) {
            eF = unpack(a);
            return true;
        }
        if (spin_abort(ctl, sp)) return false;
    }
    LB_COUNT(7, 1);
    // nearest predecessor (within 64) that has published its exit
    for (;;) {
        const int64_t jj = g - 1 - l;
        const bool in = jj >= 0;
        xF = in ? ld_status(sv.at(W_XF, jj)) : 0;
        const uint64_t xm = ballot(in && wstate(xF));
        if (xm) {
            i0 = ctz64(xm);
            break;
        }
        if (spin_abort(ctl, sp)) return false;
    }
    int64_t F = unpack(readlaneu64(xF, i0));
    // apply the maps of the segments after it, oldest first
    for (int i = i0 - 1; i >= 0; --i) {
        const int64_t js = g - 1 - i;
        Spin sp2;
        for (;;) {
            const uint64_t x0 = ld_status(sv.at(W_XF, js));
            if (wstate(x0)) {
                F = unpack(x0);
                break;
            }
            const uint64_t lo = ld_status(sv.at(W_MLO, js)), hi = ld_status(sv.at(W_MHI, js)), cf = ld_status(sv.at(W_MCF, js));
            const uint64_t sf = ld_status(sv.at(W_AF, js));
            if (wstate(lo) && wstate(hi) && wstate(cf) && wstate(sf)) {
                if (F >= unpack(lo) && F <= unpack(hi)) {
                    F -= unpack(sf);
                    break;
                }
                if (wstate(cf) == 2) {
                    F = unpack(cf);
                    break;
                }
            }
            if (spin_abort(ctl, sp2)) return false;
        }
    }
    eF = F;
    return true;
}

// -------------------------------------------------------- all-entry analysis

// Follow one chain through the window held in f (one node per lane), starting
// after lane st.  U holds the lanes where an earlier chain of this window
// sampled; reaching one of them means the chains coincide (returns false).
__device__ __forceinline__ bool follow(int64_t f, int64_t T, int64_t& ref, int& last, int st, uint64_t& U, int w) {
    const int l = lane_id();
    for (;;) {
        const int64_t d = f - ref;
        const uint64_t m = ballot(l > st && (d >= T || d <= -T));
        if (!m) return true;
        const int j = ctz64(m);
        if ((U >> j) & 1) return false;
        U |= 1ull << j;
        ref = readlane64(f, j);
        last = w * 64 + j;
        st = j;
    }
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
};

// Follow cr from window w0 (after lane st0) through window wend (below lane
// stend), sampling wherever the footprint is at least T away from the
// reference (section 3.2).
__device__ void run_chain(const int64_t* F, int64_t T, ChainRun& cr, int w0, int st0, int wend, int stend) {
    const int l = lane_id();
    for (int w = w0; w <= wend; ++w) {
        const int64_t f = F[w * 64 + l];
        int stl = w == w0 ? st0 : -1;
        const int lim = w == wend ? stend : 64;
        uint64_t m = 0;
        for (;;) {
            const int64_t d = f - cr.ref;
            const uint64_t ex = ballot(l > stl && l < lim && (d >= T || d <= -T));
            if (!ex) break;
            const int jj = ctz64(ex);
            const int64_t fj = readlane64(f, jj);
            if (fj > cr.ref && (cr.gnode < 0 || fj > cr.gbest)) {
                cr.gbest = fj;
                cr.gnode = w * 64 + jj;
            }
            if (fj > cr.smax) cr.smax = fj;
            cr.ref = fj;
            m |= 1ull << jj;
            stl = jj;
            cr.lastS = w * 64 + jj;
        }
        if (l == w) cr.mvec |= m;
    }
}

// ------------------------------------------------------------------ main kernel

// last trace whose first segment (or block, line) index is <= x
__device__ __forceinline__ int find_trace_seg(const Desc* desc, int ntraces, uint64_t x) {
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].seg_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(BLOCK) void k_sample(const Desc* __restrict__ desc, int ntraces, uint64_t nseg_total,
                                                 unsigned long long* ctl) {
    __shared__ SegLds lds_seg[WAVES];
    __shared__ HistCache hc;

    for (int i = threadIdx.x; i < NSLOT; i += BLOCK) {
        hc.key[i] = EMPTY_KEY;
        for (int c = 0; c < NCNT; ++c) hc.cnt[i][c] = 0;
    }
    __syncthreads();

    const int wv = threadIdx.x >> 6;
    const int l = lane_id();
    SegLds& S = lds_seg[wv];

    int cur_t = -1;
    int64_t peakF = 0, peakS = 0;
    PH_DECL

    for (;;) {
        unsigned long long tk = 0;
        if (l == 0) tk = atomicAdd(&ctl[0], 1ull);
        tk = readlaneu64(tk, 0);
        if (tk >= nseg_total) break;
        // tickets only grow, so the owning trace only moves forward
        int tt = cur_t < 0 ? find_trace_seg(desc, ntraces, tk) : cur_t;
        while (tt + 1 < ntraces && desc[tt + 1].seg_begin <= tk) ++tt;
        const uint32_t t = (uint32_t)tt;
        const Desc& D = desc[t];
        if ((int)t != cur_t) {
            if (cur_t >= 0 && l == 0) {
                atomicMax((long long*)&desc[cur_t].scal->peak_F, (long long)peakF);
                atomicMax((long long*)&desc[cur_t].scal->peak_S, (long long)peakS);
            }
            cur_t = (int)t;
            peakF = 0;
            peakS = 0;
        }
        const int64_t g0 = (int64_t)D.seg_begin;
        const int64_t g = (int64_t)tk;
        const int64_t j = g - g0;
        const int64_t a = j * SEG;
        const int nv = (int)((D.n - (uint64_t)a) < (uint64_t)SEG ? (D.n - (uint64_t)a) : (uint64_t)SEG);
        const int64_t T = D.T;
        const uint32_t L = D.L;
        const StatusView sv{D.status, (int64_t)D.nseg};
        uint32_t err = 0;
        PH_MARK(0);
        PH_COUNT(12, 1);

        // ---- P1: load, decode, validate, scan ----------------------------
        uint64_t q0[NW], q1[NW], q2[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int k = w * 64 + l;
            if (k < nv) {
                const uint64_t* p = (const uint64_t*)(D.ev + (size_t)(a + k) * 24);
                q0[w] = __builtin_nontemporal_load(p);
                q1[w] = __builtin_nontemporal_load(p + 1);
                q2[w] = __builtin_nontemporal_load(p + 2);
            } else {
                q0[w] = 0;
                q1[w] = 0;
                q2[w] = 0;
            }
        }
        int64_t cF = 0, cP = 0, cC = 0;
        int64_t mxF = INT64_MIN, mnF = INT64_MAX, mxP = INT64_MIN, mnP = INT64_MAX;
        uint64_t forced_v = 0, free_v = 0;   // lane w: mask of window w
        int64_t accC = 0;                     // per-lane copy bytes
        bool any_aux = false;                 // segment holds copy or timer events
        const int64_t two_t = 2 * T - 1;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int k = w * 64 + l;
            const bool valid = k < nv;
            const int64_t delta = (int64_t)q0[w];
            const uint32_t ptr = (uint32_t)q1[w];
            const uint32_t line = (uint32_t)(q1[w] >> 32);
            const uint32_t flags = (uint32_t)(q2[w] & 0xFF);
            const uint32_t kind = (flags >> 1) & 3;
            const bool py = (flags & 1) == 0;
            // memory: |delta| < 2^52; copy: 0 <= delta < 2^52; timer: 0 <= delta < 2^32
            const uint64_t shifted = (uint64_t)delta + (kind == 0 ? (uint64_t)(MAX_ABS_DELTA - 1) : 0ull);
            const uint64_t span = kind == 0 ? (uint64_t)(2 * MAX_ABS_DELTA - 1)
                                            : (kind == 1 ? (uint64_t)MAX_ABS_DELTA : (1ull << 32));
            const bool bad = valid && (kind == 3 || line >= L || shifted >= span);
            const bool ok = valid && !bad;
            const int64_t dm = (ok && kind == 0) ? delta : 0;
            const int64_t dp = py ? dm : 0;
            const int64_t dc = (ok && kind == 1) ? delta : 0;
            if (ballot(bad)) err |= 1u;
            const uint64_t fm = ballot(dm >= two_t || dm <= -two_t);
            const uint64_t frm = ballot(dm < 0);
            if (l == w) {
                forced_v = fm;
                free_v = frm;
            }
            const int64_t sF = wave_incl_sum(dm) + cF;
            const int64_t sP = wave_incl_sum(dp) + cP;
            cF = readlane64(sF, 63);
            cP = readlane64(sP, 63);
            accC += dc;
            if (ballot(ok && kind != 0)) any_aux = true;
            S.F[k] = sF;
            S.P[k] = sP;
            S.ptr[k] = ptr;
            if (valid) {
                mxF = sF > mxF ? sF : mxF;
                mnF = sF < mnF ? sF : mnF;
                mxP = sP > mxP ? sP : mxP;
                mnP = sP < mnP ? sP : mnP;
            }
        }
        cC = wave_sum(accC);
        const int64_t sumF = cF, sumP = cP, sumC = cC;
        if (l < 3) st_status(sv.at(W_AF + l, j), pack(l == 0 ? sumF : (l == 1 ? sumP : sumC), 1));
        PH_MARK(1);

        // ---- prefix sums from the preceding segments ------------------------
        int64_t F0 = 0, P0 = 0, C0 = 0;
        if (j > 0 && !scan_sums(sv, j, F0, P0, C0, ctl)) err |= 8u;
        if (l < 3) st_status(sv.at(W_IF + l, j), pack(l == 0 ? F0 + sumF : (l == 1 ? P0 + sumP : C0 + sumC), 1));
        PH_MARK(2);

        // ---- P2: all-entry analysis: the segment's map on entry states --------
        bool map_total = false;
        int64_t map_kF = 0;
        // An event with |delta| >= 2T-1 samples for every entry state, so the
        // chain from the first such event onwards is the same for all entries.
        int fwin = -1, flane = -1;
        ChainRun p2run{0, 0, 0, -1, INT64_MIN, -1};
        if (j > 0) {
            const uint64_t wf = ballot(l < NW && forced_v != 0);
            if (wf) {
                fwin = ctz64(wf);
                flane = ctz64(readlaneu64(forced_v, fwin));
                p2run.ref = readlane64(S.F[fwin * 64 + l], flane);
                run_chain(S.F, T, p2run, fwin, flane, NW - 1, 64);
                map_total = true;
                map_kF = p2run.ref - sumF;
                if (l == 0) st_status(sv.at(W_MLO, j), pack(1, 1));
                if (l == 1) st_status(sv.at(W_MHI, j), pack(0, 1));
                if (l == 2) st_status(sv.at(W_MCF, j), pack(map_kF, 2));
                if (l == 3) st_status(sv.at(W_XF, j), pack(map_kF, 1));
                PH_COUNT(13, 1);
                PH_COUNT(15, 1);
            }
        }
        if (j > 0 && fwin < 0) {
            int64_t Lo = -T + 1, Hi = T - 1;
            int nch = 0;
            bool ovf = false;
            int64_t chref = 0;
            int chlast = -1;
            for (int w = 0; w < NW; ++w) {
                const int64_t f = S.F[w * 64 + l];
                uint64_t U = 0;
                int first_st = -1;
                if (ovf) {
                    const uint64_t fm = readlaneu64(forced_v, w);
                    if (!fm) {
                        if (Lo <= Hi) {
                            const int64_t wmx = wave_max(f), wmn = wave_min(f);
                            Lo = (wmx - T + 1) > Lo ? (wmx - T + 1) : Lo;
                            Hi = (wmn + T - 1) < Hi ? (wmn + T - 1) : Hi;
                        }
                        continue;
                    }
                    // every chain samples at a forced event: one chain remains
                    const int fj = ctz64(fm);
                    const int64_t r = readlane64(f, fj);
                    if (l == 0) {
                        chref = r;
                        chlast = w * 64 + fj;
                    }
                    nch = 1;
                    ovf = false;
                    Lo = 1;
                    Hi = 0;
                    U = 1ull << fj;
                    first_st = fj;
                }
                int nal = 0;
                for (int c = 0; c < nch; ++c) {
                    int64_t ref = readlane64(chref, c);
                    int last = readlane32(chlast, c);
                    if (follow(f, T, ref, last, c == 0 ? first_st : -1, U, w)) {
                        if (l == nal) {
                            chref = ref;
                            chlast = last;
                        }
                        ++nal;
                    }
                }
                if (Lo <= Hi) {
                    const int64_t im = wave_incl_max(f), in = wave_incl_min(f);
                    const int64_t em = wave_shr1(im, INT64_MIN), en = wave_shr1(in, INT64_MAX);
                    int64_t lob = Lo, hib = Hi;
                    if (l > 0) {
                        lob = (em - T + 1) > Lo ? (em - T + 1) : Lo;
                        hib = (en + T - 1) < Hi ? (en + T - 1) : Hi;
                    }
                    const bool ne = lob <= hib;
                    const bool up = ne && (f - T >= lob);
                    const bool dn = ne && (f + T <= hib);
                    uint64_t cm = ballot(up || dn);
                    while (cm) {
                        const int c = ctz64(cm);
                        cm &= cm - 1;
                        if ((U >> c) & 1) continue;
                        U |= 1ull << c;
                        int64_t ref = readlane64(f, c);
                        int last = w * 64 + c;
                        if (follow(f, T, ref, last, c, U, w)) {
                            if (nal >= CHAIN_CAP) {
                                ovf = true;
                                break;
                            }
                            if (l == nal) {
                                chref = ref;
                                chlast = last;
                            }
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
            bool has_const = !ovf && nch == 1;
            int64_t kF = 0;
            if (has_const) kF = readlane64(chref, 0) - sumF;
            // publish the map
            if (l == 0) st_status(sv.at(W_MLO, j), pack(Lo, 1));
            if (l == 1) st_status(sv.at(W_MHI, j), pack(Hi, 1));
            if (l == 2) st_status(sv.at(W_MCF, j), pack(kF, has_const ? 2 : 1));
            PH_COUNT(13, has_const ? 1 : 0);
            PH_COUNT(14, ovf ? 1 : 0);
            if (has_const && Lo > Hi) {
                PH_COUNT(15, 1);
                map_total = true;
                map_kF = kF;
                if (l == 0) st_status(sv.at(W_XF, j), pack(kF, 1));
            }
        }

        PH_MARK(4);


        {
            const int64_t hiF = wave_max(mxF), loF = wave_min(mnF);
            const int64_t hiP = wave_max(mxP), loP = wave_min(mnP);
            if (F0 + hiF >= MAX_ABS_F || F0 + loF <= -MAX_ABS_F || P0 + hiP >= MAX_ABS_F || P0 + loP <= -MAX_ABS_F ||
                C0 + sumC >= MAX_ABS_F || F0 >= MAX_ABS_F || F0 <= -MAX_ABS_F)
                err |= 2u;
            if (nv > 0 && F0 + hiF > peakF) peakF = F0 + hiF;
        }

        // Copy volume (section 3.5: one Tc sample per multiple of Tc crossed by
        // the cumulative copy bytes) and the timer split (section 2.1: Python
        // time += quantum, native time += delay).  Only segments that hold such
        // events re-read their records here.
        if (any_aux) {
            int64_t cc = C0;
            for (int w = 0; w < NW; ++w) {
                const int k = w * 64 + l;
                uint64_t r0 = 0, r1 = 0, r2 = 0;
                if (k < nv) {
                    const uint64_t* rp = (const uint64_t*)(D.ev + (size_t)(a + k) * 24);
                    r0 = rp[0];
                    r1 = rp[1];
                    r2 = rp[2];
                }
                const int64_t delta = (int64_t)r0;
                const uint32_t line = (uint32_t)(r1 >> 32);
                const uint32_t kind = ((uint32_t)r2 >> 1) & 3;
                const bool lok = k < nv && line < L;
                const bool cp = lok && kind == 1 && delta >= 0 && delta < MAX_ABS_DELTA;
                const bool tm = lok && kind == 2 && delta >= 0 && delta <= (int64_t)0xFFFFFFFFll;
                const int64_t dc = cp ? delta : 0;
                const int64_t sc = wave_incl_sum(dc) + cc;
                cc = readlane64(sc, 63);
                if (cp || tm) {
                    int c0 = C_PT, c1 = C_NT;
                    int64_t v0 = D.q, v1 = delta;
                    if (cp) {
                        const uint64_t cout = (uint64_t)sc, cin = cout - (uint64_t)dc;
                        uint64_t ns;
                        if (D.tc_shift >= 0)
                            ns = (cout >> D.tc_shift) - (cin >> D.tc_shift);
                        else
                            ns = cout / (uint64_t)D.Tc - cin / (uint64_t)D.Tc;
                        c0 = C_CS;
                        c1 = C_CE;
                        v0 = (int64_t)(ns * (uint64_t)D.Tc);
                        v1 = dc;
                    }
                    hist_add(hc, D, t, line, c0, v0, c1, v1, -1, 0, -1, 0);
                }
            }
        }

        PH_MARK(3);

        // ---- P4: entry state, then the segment's own samples -----------------
        int64_t eF = 0;
        if (j > 0 && !lookback_chain(sv, j, eF, ctl)) err |= 8u;
        PH_MARK(5);
        ChainRun cr{eF, 0, 0, -1, INT64_MIN, -1};
        if (fwin >= 0) {
            // entry-dependent samples come only before the forced event
            run_chain(S.F, T, cr, 0, -1, fwin, flane);
            const int64_t fc = readlane64(S.F[fwin * 64 + l], flane);
            if (fc > cr.ref && (cr.gnode < 0 || fc > cr.gbest)) {
                cr.gbest = fc;
                cr.gnode = fwin * 64 + flane;
            }
            if (fc > cr.smax) cr.smax = fc;
            if (l == fwin) cr.mvec |= 1ull << flane;
            cr.mvec |= p2run.mvec;
            if (p2run.gnode >= 0 && (cr.gnode < 0 || p2run.gbest > cr.gbest)) {
                cr.gbest = p2run.gbest;
                cr.gnode = p2run.gnode;
            }
            if (p2run.smax > cr.smax) cr.smax = p2run.smax;
            cr.lastS = p2run.lastS >= 0 ? p2run.lastS : fwin * 64 + flane;
            cr.ref = p2run.ref;
        } else {
            run_chain(S.F, T, cr, 0, -1, NW - 1, 64);
        }
        const uint64_t smask_v = cr.mvec;
        const int64_t ref = cr.ref;
        const int lastS = cr.lastS;
        const int64_t gbest = cr.gbest;
        const int gnode = cr.gnode;
        const int64_t smax = cr.smax;
        const int64_t xF = ref - sumF;
        if (!map_total) {
            if (l == 0) st_status(sv.at(W_XF, j), pack(xF, 1));
        } else if (xF != map_kF) {
            err |= 4u;  // internal: the all-entry map disagrees with the simulated chain
        }
        const int count = (int)wave_sum(l < NW ? (int64_t)__popcll(smask_v) : 0);
        if (smax != INT64_MIN && F0 + smax > peakS) peakS = F0 + smax;

        PH_MARK(6);
        // ---- P5: publish (count, best growth record, last-sample Python footprint) ----
        {
            const bool hg = gnode >= 0;
            const int64_t gval = F0 + gbest;
            const uint32_t gidx = hg ? (uint32_t)(a + gnode) : 0u;
            const uint32_t gptr = hg ? S.ptr[gnode] : 0u;
            if (l == 0) st_status(sv.at(W_BCNT, j), pack(count, 1));
            if (l == 1) st_status(sv.at(W_BGM, j), pack(hg ? gval : 0, hg ? 2 : 1));
            if (l == 2) st_status(sv.at(W_BGR, j), pack((int64_t)gidx, 1));
            if (l == 3) st_status(sv.at(W_BGP, j), pack((int64_t)gptr, 1));
            const int64_t lsP = lastS >= 0 ? P0 + S.P[lastS] : 0;
            if (l == 4) st_status(sv.at(W_LSA, j), pack(lsP, lastS >= 0 ? 2 : 1));
            Best pre{0, false, 0, 0, 0};
            if (j > 0 && !scan_best(sv, j, pre, ctl)) err |= 8u;
            {
                Best inc = pre;
                inc.cnt += count;
                if (hg && gval > (pre.has ? pre.val : 0)) {
                    inc.has = true;
                    inc.val = gval;
                    inc.idx = gidx;
                    inc.ptr = gptr;
                }
                if (l == 0) st_status(sv.at(W_ICNT, j), pack(inc.cnt, 1));
                if (l == 1) st_status(sv.at(W_IGM, j), pack(inc.has ? inc.val : 0, inc.has ? 2 : 1));
                if (l == 2) st_status(sv.at(W_IGR, j), pack((int64_t)inc.idx, 1));
                if (l == 3) st_status(sv.at(W_IGP, j), pack((int64_t)inc.ptr, 1));
            }
            int64_t eP = 0;
            if (j > 0 && !scan_last_sample(sv, j, eP, ctl)) err |= 8u;
            if (l == 0) st_status(sv.at(W_LSI, j), pack(lastS >= 0 ? lsP : eP, 1));
            int64_t base = pre.cnt, hv = pre.val;
            bool hh = pre.has;
            uint32_t hidx = pre.idx, hptr = pre.ptr;
            PH_MARK(7);
            if (base < 0 || base > (int64_t)D.n) {  // only reachable after an internal fault
                err |= 8u;
                base = 0;
            }
            if ((uint64_t)j == D.nseg - 1 && l == 0) {
                D.scal->K = (uint64_t)(base + count);
                D.scal->final_F = F0 + sumF;
            }

            // ---- P7: emit samples, per-line attribution, leak tracking ----
            int64_t refF = eF, refP = eP - P0;
            int64_t cnt = 0;
            bool cur_has = hh;
            uint32_t cur_ptr = hptr, cur_idx = hidx;
            int64_t hwm = hh ? hv : 0;
            for (int w = 0; w < NW; ++w) {
                const uint64_t m = readlaneu64(smask_v, w);
                const uint64_t fm = readlaneu64(free_v, w);
                if (m == 0 && (fm == 0 || !cur_has)) continue;
                const int k = w * 64 + l;
                const int64_t f = S.F[k];
                const int64_t p = S.P[k];
                const uint32_t pt = S.ptr[k];
                const uint64_t below = m & lanemask_lt();
                uint64_t tmask = 0;
                if (m) {
                    const int pl = below ? top64(below) : l;
                    int64_t fprev = shfl64(f, pl), pprev = shfl64(p, pl);
                    if (!below) {
                        fprev = refF;
                        pprev = refP;
                    }
                    const bool is_s = (m >> l) & 1;
                    const int64_t dl = f - fprev;
                    const int64_t pyb = p - pprev;
                    const int64_t nat = dl - pyb;
                    const int64_t Fabs = F0 + f;
                    const int64_t rank = base + cnt + __popcll(below);
                    if (is_s && rank < (int64_t)D.n) {
                        const uint32_t ln = ((const uint32_t*)(D.ev + (size_t)(a + k) * 24))[3];
                        Sample smp;
                        smp.event_idx = (uint32_t)(a + k);
                        smp.line = ln;
                        smp.F = Fabs;
                        smp.py = pyb;
                        smp.nat = nat;
                        D.samples[rank] = smp;
                        if (ln < L) {
                            const bool gr = dl > 0;
                            hist_add(hc, D, t, ln, C_PY, pyb, C_NAT, nat, gr ? C_GN : C_SN, 1, gr ? C_GB : C_SB,
                                     gr ? dl : -dl);
                        }
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
                        atomicOr((unsigned long long*)&D.tracked_bits[rank >> 6], 1ull << (rank & 63));
                        D.sample_ptr[rank] = pt;
                    }
                    const int ls = top64(m);
                    refF = readlane64(f, ls);
                    refP = readlane64(p, ls);
                }
                if (fm && (cur_has || tmask)) {
                    const uint64_t tb = tmask & lanemask_lt();
                    const int al = tb ? top64(tb) : l;
                    const uint32_t sp = (uint32_t)shfl32((int)pt, al);
                    const uint32_t aptr = tb ? sp : cur_ptr;
                    const uint32_t aidx = tb ? (uint32_t)(a + w * 64 + al) : cur_idx;
                    const bool ahas = tb != 0 || cur_has;
                    if (((fm >> l) & 1) && ahas && pt == aptr && aidx < D.n)
                        atomicOr((unsigned long long*)&D.freed_bits[aidx >> 6], 1ull << (aidx & 63));
                }
                if (tmask) {
                    const int tl = top64(tmask);
                    cur_ptr = (uint32_t)readlane32((int)pt, tl);
                    cur_idx = (uint32_t)(a + w * 64 + tl);
                    cur_has = true;
                }
                cnt += __popcll(m);
            }
        }
        PH_MARK(8);
        if (err && l == 0) atomicOr(&D.scal->err, err);
    }
    PH_FLUSH(ctl);
    if (cur_t >= 0 && l == 0) {
        atomicMax((long long*)&desc[cur_t].scal->peak_F, (long long)peakF);
        atomicMax((long long*)&desc[cur_t].scal->peak_S, (long long)peakS);
    }
    __syncthreads();
    // flush the LDS histogram cache
    for (int i = threadIdx.x; i < NSLOT; i += BLOCK) {
        const unsigned long long key = hc.key[i];
        if (key == EMPTY_KEY) continue;
        const Desc& D = desc[(uint32_t)(key >> 32)];
        const uint32_t line = (uint32_t)key;
        for (int c = 0; c < NCNT; ++c) {
            const unsigned long long v = hc.cnt[i][c];
            if (v) atomicAdd((unsigned long long*)&D.hist[(size_t)cache_to_hist(c) * D.L + line], v);
        }
    }
}

// ----------------------------------------------------------------- clearing

__global__ void k_clear(const Desc* __restrict__ desc, int ntraces, uint64_t total_bytes, unsigned long long* ctl) {
    const uint64_t chunk = 1ull << 16;
    const uint64_t begin = (uint64_t)blockIdx.x * chunk;
    if (blockIdx.x == 0 && threadIdx.x < 32) ctl[threadIdx.x] = 0;
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
        uint64_t* p = (uint64_t*)(D.zero_ptr + (s - D.zero_begin));
        const uint64_t nw = (e - s) >> 3;
        for (uint64_t i = threadIdx.x; i < nw; i += blockDim.x) p[i] = 0;
    }
}

// ------------------------------------------------ tracked-list compaction

constexpr int CBLK_WORDS = 1024;   // bitmap words per compaction block

__device__ __forceinline__ int find_trace_blk(const Desc* desc, int ntraces, uint64_t x) {
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].blk_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_track_count(const Desc* __restrict__ desc, int ntraces, uint64_t nblk_total) {
    const uint64_t b = blockIdx.x;
    if (b >= nblk_total) return;
    const Desc& D = desc[find_trace_blk(desc, ntraces, b)];
    const uint64_t lb = b - D.blk_begin;
    const uint64_t K = D.scal->K < D.n ? D.scal->K : D.n;
    const uint64_t nwords = (K + 63) >> 6;
    const uint64_t w0 = lb * CBLK_WORDS;
    uint64_t c = 0;
    for (uint64_t i = threadIdx.x; i < CBLK_WORDS; i += blockDim.x)
        if (w0 + i < nwords) c += __popcll(D.tracked_bits[w0 + i]);
    __shared__ uint64_t red[256];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) D.blk[lb] = red[0];
}

__global__ void k_track_scan(const Desc* __restrict__ desc) {
    const Desc& D = desc[blockIdx.x];
    __shared__ uint64_t part[256];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < D.nblk; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t v = i < D.nblk ? D.blk[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < (int)blockDim.x; s <<= 1) {
            uint64_t x = (int)threadIdx.x >= s ? part[threadIdx.x - s] : 0;
            __syncthreads();
            part[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < D.nblk) D.blk[i] = carry + part[threadIdx.x] - v;  // exclusive
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += part[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) D.scal->H = carry;
}

__global__ void k_track_emit(const Desc* __restrict__ desc, int ntraces, uint64_t nblk_total) {
    const uint64_t b = blockIdx.x;
    if (b >= nblk_total) return;
    const Desc& D = desc[find_trace_blk(desc, ntraces, b)];
    const uint64_t lb = b - D.blk_begin;
    const uint64_t K = D.scal->K < D.n ? D.scal->K : D.n;
    const uint64_t nwords = (K + 63) >> 6;
    const uint64_t w0 = lb * CBLK_WORDS;
    if (w0 >= nwords) return;
    const uint64_t H = D.scal->H;
    // each thread owns 4 consecutive words
    constexpr int PER = CBLK_WORDS / 256;
    uint64_t words[PER];
    uint64_t c = 0;
    for (int i = 0; i < PER; ++i) {
        const uint64_t wi = w0 + threadIdx.x * PER + i;
        words[i] = wi < nwords ? D.tracked_bits[wi] : 0;
        c += __popcll(words[i]);
    }
    __shared__ uint64_t part[256];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
        uint64_t x = (int)threadIdx.x >= s ? part[threadIdx.x - s] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    uint64_t h = D.blk[lb] + part[threadIdx.x] - c;
    const bool resolve_last = (D.options & 2u) != 0;
    for (int i = 0; i < PER; ++i) {
        uint64_t m = words[i];
        const uint64_t wi = w0 + threadIdx.x * PER + i;
        while (m) {
            const int bit = __builtin_ctzll(m);
            m &= m - 1;
            const uint64_t r = wi * 64 + bit;
            if (r >= K || h >= H) break;  // only reachable after an internal fault
            const Sample s = D.samples[r];
            const uint32_t freed =
                s.event_idx < D.n ? (uint32_t)((D.freed_bits[s.event_idx >> 6] >> (s.event_idx & 63)) & 1) : 0u;
            Tracked tr;
            tr.event_idx = s.event_idx;
            tr.line = s.line;
            tr.ptr = D.sample_ptr[r];
            tr.freed = freed;
            D.tracked[h] = tr;
            if (s.line < D.L) {
                atomicAdd((unsigned long long*)&D.hist[(size_t)H_LEAK_M * D.L + s.line], 1ull);
                if (freed && (h + 1 < H || resolve_last))
                    atomicAdd((unsigned long long*)&D.hist[(size_t)H_LEAK_F * D.L + s.line], 1ull);
            }
            ++h;
        }
    }
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

// Exact reduced rationals: Laplace's rule of succession (m-f+1)/(m+2) and the
// formula as printed (m-2f+1)/(m-f+2); gate: likelihood > 0.95 (section 3.4).
__global__ void k_leak_finalize(const Desc* __restrict__ desc, int ntraces, uint64_t total_lines) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total_lines) return;
    int lo = 0, hi = ntraces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].line_begin <= i) lo = mid; else hi = mid - 1;
    }
    const Desc& D = desc[lo];
    const uint64_t line = i - D.line_begin;
    if (line >= D.L) return;
    const int64_t m = D.hist[(size_t)H_LEAK_M * D.L + line];
    const int64_t f = D.hist[(size_t)H_LEAK_F * D.L + line];
    int64_t* out = D.leak;
    if (m <= 0) {
        out[line] = 0;
        out[D.L + line] = 0;
        out[2 * (size_t)D.L + line] = 0;
        out[3 * (size_t)D.L + line] = 0;
        D.gates[line] = 0;
        D.gates[D.L + line] = 0;
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
    D.gates[line] = g1;
    D.gates[D.L + line] = g2;
}

// ------------------------------------------------------------ launchers

#ifdef SMP_PHASE_STATS
int read_lbstat(unsigned long long* out8, bool reset) {
    if (hipMemcpyFromSymbol(out8, HIP_SYMBOL(g_lbstat), 8 * sizeof(unsigned long long)) != hipSuccess) return -1;
    if (reset) {
        unsigned long long z[8] = {0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_lbstat), z, sizeof(z)) != hipSuccess) return -1;
    }
    return 0;
}
#endif

int sample_grid_limit() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sample, BLOCK, 0) != hipSuccess) return 0;
    return cus * (per > 0 ? per : 1);
}

hipError_t launch_clear(const Desc* desc, int ntraces, uint64_t total_bytes, unsigned long long* ticket,
                        hipStream_t s) {
    const uint64_t blocks = (total_bytes + (1ull << 16) - 1) >> 16;
    k_clear<<<dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s>>>(desc, ntraces, total_bytes, ticket);
    return hipGetLastError();
}

hipError_t launch_sample(const Desc* desc, int ntraces, uint64_t nseg_total, unsigned long long* ticket, int grid,
                         hipStream_t s) {
    if (nseg_total == 0) return hipSuccess;
    k_sample<<<dim3((unsigned)grid), dim3(BLOCK), 0, s>>>(desc, ntraces, nseg_total, ticket);
    return hipGetLastError();
}

hipError_t launch_finish(const Desc* desc, int ntraces, uint64_t nblk_total, uint64_t total_lines, hipStream_t s) {
    if (nblk_total) {
        k_track_count<<<dim3((unsigned)nblk_total), dim3(256), 0, s>>>(desc, ntraces, nblk_total);
        k_track_scan<<<dim3((unsigned)ntraces), dim3(256), 0, s>>>(desc);
        k_track_emit<<<dim3((unsigned)nblk_total), dim3(256), 0, s>>>(desc, ntraces, nblk_total);
    }
    if (total_lines) {
        const uint64_t blocks = (total_lines + 255) / 256;
        k_leak_finalize<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(desc, ntraces, total_lines);
    }
    return hipGetLastError();
}

}  // namespace smp
