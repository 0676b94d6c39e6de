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
        default: return H_NT;
    }
}

struct SegLds {
    int64_t F[SEG];     // footprint after each event, relative to the segment start
    int64_t P[SEG];     // Python footprint after each event, relative
    uint32_t line[SEG];
    uint32_t ptr[SEG];
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

// Every wait on another segment's status polls with a budget.  Running out
// (only possible through an internal fault) raises the launch-wide abort word,
// after which every wait returns at once, so all waves always exit.
constexpr uint32_t SPIN_BUDGET = 1u << 27;

__device__ __forceinline__ bool spin_abort(unsigned long long* ctl, uint32_t& budget) {
    if (ld_status((const uint64_t*)&ctl[1])) return true;
    __builtin_amdgcn_s_sleep(2);
    if (--budget == 0) {
        st_status((uint64_t*)&ctl[1], 1);
        return true;
    }
    return false;
}

// Exclusive prefix of (footprint, Python footprint, copy bytes) for segment g.
__device__ bool lookback_sums(uint64_t* status, int64_t g, int64_t g0, int64_t& oF, int64_t& oP, int64_t& oC,
                              unsigned long long* ctl) {
    const int l = lane_id();
    uint32_t budget = SPIN_BUDGET;
    int64_t accF = 0, accP = 0, accC = 0;
    int64_t base = g - 1;
    for (;;) {
        const int64_t jj = base - l;
        const bool in = jj >= g0;
        uint64_t iF = 0, iP = 0, iC = 0;
        if (in) {
            const uint64_t* w = status + jj * NWORD;
            iF = ld_status(w + W_IF);
            iP = ld_status(w + W_IP);
            iC = ld_status(w + W_IC);
        }
        const bool has_incl = in && wstate(iF) && wstate(iP) && wstate(iC);
        const uint64_t im = ballot(has_incl);
        const uint64_t inm = ballot(in);
        const int lim = im ? ctz64(im) : __popcll(inm);
        const bool need = in && l < lim;
        uint64_t aF = 0, aP = 0, aC = 0;
        if (need) {
            const uint64_t* w = status + jj * NWORD;
            aF = ld_status(w + W_AF);
            aP = ld_status(w + W_AP);
            aC = ld_status(w + W_AC);
        }
        if (ballot(need && !(wstate(aF) && wstate(aP) && wstate(aC)))) {
            if (spin_abort(ctl, budget)) return false;
            continue;
        }
        int64_t vF = 0, vP = 0, vC = 0;
        if (need) {
            vF = unpack(aF);
            vP = unpack(aP);
            vC = unpack(aC);
        } else if (im && l == lim) {
            vF = unpack(iF);
            vP = unpack(iP);
            vC = unpack(iC);
        }
        accF += wave_sum(vF);
        accP += wave_sum(vP);
        accC += wave_sum(vC);
        if (im || base - 64 < g0) break;
        base -= 64;
    }
    oF = accF;
    oP = accP;
    oC = accC;
    return true;
}

// Combine (count, best growth record) over the segments before g.
// Record order: value > wins; ties keep the earlier segment.
__device__ bool lookback_best(uint64_t* status, int64_t g, int64_t g0, int64_t& oCnt, bool& oHas, int64_t& oVal,
                              uint32_t& oIdx, uint32_t& oPtr, unsigned long long* ctl) {
    const int l = lane_id();
    uint32_t budget = SPIN_BUDGET;
    int64_t cnt = 0;
    bool has = false;   // running best from later segments (processed first)
    int64_t val = 0;
    uint32_t idx = 0, ptr = 0;
    int64_t base = g - 1;
    bool reached_start = false;
    for (;;) {
        const int64_t jj = base - l;
        const bool in = jj >= g0;
        uint64_t ic = 0, ig = 0, ir = 0, ip = 0;
        if (in) {
            const uint64_t* w = status + jj * NWORD;
            ic = ld_status(w + W_ICNT);
            ig = ld_status(w + W_IGM);
            ir = ld_status(w + W_IGR);
            ip = ld_status(w + W_IGP);
        }
        const bool has_incl = in && wstate(ic) && wstate(ig) && wstate(ir) && wstate(ip);
        const uint64_t im = ballot(has_incl);
        const uint64_t inm = ballot(in);
        const int lim = im ? ctz64(im) : __popcll(inm);
        const bool need = in && l < lim;
        uint64_t ac = 0, ag = 0, ar = 0, ap = 0;
        if (need) {
            const uint64_t* w = status + jj * NWORD;
            ac = ld_status(w + W_BCNT);
            ag = ld_status(w + W_BGM);
            ar = ld_status(w + W_BGR);
            ap = ld_status(w + W_BGP);
        }
        if (ballot(need && !(wstate(ac) && wstate(ag) && wstate(ar) && wstate(ap)))) {
            if (spin_abort(ctl, budget)) return false;
            continue;
        }
        uint64_t c = 0, gm = 0, gr = 0, gp = 0;
        bool use = false;
        if (need) {
            c = ac; gm = ag; gr = ar; gp = ap;
            use = true;
        } else if (im && l == lim) {
            c = ic; gm = ig; gr = ir; gp = ip;
            use = true;
        }
        cnt += wave_sum(use ? unpack(c) : 0);
        const bool lh = use && wstate(gm) == 2;
        const int64_t lv = lh ? unpack(gm) : INT64_MIN;
        const int64_t mx = wave_max(lv);
        const uint64_t at = ballot(lh && lv == mx);
        if (at) {
            const int src = top64(at);  // highest lane = earliest segment
            if (!has || mx >= val) {
                has = true;
                val = mx;
                idx = (uint32_t)unpack(readlaneu64(gr, src));
                ptr = (uint32_t)unpack(readlaneu64(gp, src));
            }
        }
        if (im) break;
        if (base - 64 < g0) {
            reached_start = true;
            break;
        }
        base -= 64;
    }
    (void)reached_start;
    // the state before the trace is a high-water mark of 0 with nothing tracked
    if (has && val <= 0) has = false;
    oCnt = cnt;
    oHas = has;
    oVal = has ? val : 0;
    oIdx = idx;
    oPtr = ptr;
    return true;
}

// Entry state (reference offset, absolute Python reference) of segment g.
__device__ bool lookback_chain(uint64_t* status, int64_t g, int64_t g0, int64_t& eF, int64_t& eP,
                               unsigned long long* ctl) {
    const int l = lane_id();
    uint32_t budget = SPIN_BUDGET;
    int i0;
    uint64_t xF, xP;
    // nearest predecessor (within 64) that has published its exit
    for (;;) {
        const int64_t jj = g - 1 - l;
        const bool in = jj >= g0;
        xF = 0;
        xP = 0;
        if (in) {
            const uint64_t* w = status + jj * NWORD;
            xF = ld_status(w + W_XF);
            xP = ld_status(w + W_XP);
        }
        const uint64_t xm = ballot(in && wstate(xF) && wstate(xP));
        if (xm) {
            i0 = ctz64(xm);
            break;
        }
        if (spin_abort(ctl, budget)) return false;
    }
    int64_t F = unpack(readlaneu64(xF, i0));
    int64_t P = unpack(readlaneu64(xP, i0));
    // apply the maps of the segments after it, oldest first
    for (int i = i0 - 1; i >= 0; --i) {
        const uint64_t* w = status + (g - 1 - i) * NWORD;
        for (;;) {
            const uint64_t x0 = ld_status(w + W_XF), x1 = ld_status(w + W_XP);
            if (wstate(x0) && wstate(x1)) {
                F = unpack(x0);
                P = unpack(x1);
                break;
            }
            const uint64_t lo = ld_status(w + W_MLO), hi = ld_status(w + W_MHI);
            const uint64_t cf = ld_status(w + W_MCF), cp = ld_status(w + W_MCP);
            const uint64_t sf = ld_status(w + W_AF);
            if (wstate(lo) && wstate(hi) && wstate(cf) && wstate(cp) && wstate(sf)) {
                if (F >= unpack(lo) && F <= unpack(hi)) {
                    F -= unpack(sf);
                    break;
                }
                if (wstate(cf) == 2) {
                    F = unpack(cf);
                    P = unpack(cp);
                    break;
                }
            }
            if (spin_abort(ctl, budget)) return false;
        }
    }
    eF = F;
    eP = P;
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
        uint64_t* st = D.status + j * NWORD;
        uint32_t err = 0;

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
        int64_t sC[NW], dC[NW];
        uint32_t lnC[NW];
        uint64_t copym[NW];
        bool any_copy = false;
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
            bool bad = valid && (kind == 3 || line >= L);
            if (valid && kind == 0) bad |= delta >= MAX_ABS_DELTA || delta <= -MAX_ABS_DELTA;
            if (valid && kind == 1) bad |= delta < 0 || delta >= MAX_ABS_DELTA;
            if (valid && kind == 2) bad |= delta < 0 || delta > (int64_t)0xFFFFFFFFll;
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
            const uint64_t cm = ballot(dc != 0);
            copym[w] = cm;
            if (cm) {
                any_copy = true;
                sC[w] = wave_incl_sum(dc) + cC;
                cC = readlane64(sC[w], 63);
            } else {
                sC[w] = cC;
            }
            dC[w] = dc;
            lnC[w] = line;
            S.F[k] = sF;
            S.P[k] = sP;
            S.line[k] = line;
            S.ptr[k] = ptr;
            if (valid) {
                mxF = sF > mxF ? sF : mxF;
                mnF = sF < mnF ? sF : mnF;
                mxP = sP > mxP ? sP : mxP;
                mnP = sP < mnP ? sP : mnP;
            }
            // timer events: Python time += quantum, native time += delay (section 2.1)
            const bool tim = ok && kind == 2;
            if (ballot(tim) && tim) hist_add(hc, D, t, line, C_PT, D.q, C_NT, delta, -1, 0, -1, 0);
        }
        const int64_t sumF = cF, sumP = cP, sumC = cC;
        if (l < 3) st_status(st + W_AF + l, pack(l == 0 ? sumF : (l == 1 ? sumP : sumC), 1));

        // ---- prefix sums from the preceding segments ------------------------
        int64_t F0 = 0, P0 = 0, C0 = 0;
        if (j > 0 && !lookback_sums(D.status, j, 0, F0, P0, C0, ctl)) err |= 8u;
        if (l < 3) st_status(st + W_IF + l, pack(l == 0 ? F0 + sumF : (l == 1 ? P0 + sumP : C0 + sumC), 1));

        {
            const int64_t hiF = wave_max(mxF), loF = wave_min(mnF);
            const int64_t hiP = wave_max(mxP), loP = wave_min(mnP);
            if (F0 + hiF >= MAX_ABS_F || F0 + loF <= -MAX_ABS_F || P0 + hiP >= MAX_ABS_F || P0 + loP <= -MAX_ABS_F ||
                C0 + sumC >= MAX_ABS_F || F0 >= MAX_ABS_F || F0 <= -MAX_ABS_F)
                err |= 2u;
            if (nv > 0 && F0 + hiF > peakF) peakF = F0 + hiF;
        }

        // copy volume: one Tc sample per multiple of Tc crossed (section 3.5)
        if (any_copy) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (copym[w] && dC[w] != 0) {
                    const uint64_t cout = (uint64_t)(C0 + sC[w]);
                    const uint64_t cin = cout - (uint64_t)dC[w];
                    uint64_t ns;
                    if (D.tc_shift >= 0)
                        ns = (cout >> D.tc_shift) - (cin >> D.tc_shift);
                    else
                        ns = cout / (uint64_t)D.Tc - cin / (uint64_t)D.Tc;
                    hist_add(hc, D, t, lnC[w], C_CS, (int64_t)(ns * (uint64_t)D.Tc), C_CE, dC[w], -1, 0, -1, 0);
                }
            }
        }

        // ---- P2: all-entry analysis: the segment's map on entry states --------
        bool map_total = false;
        int64_t map_kF = 0, map_kP = 0;
        if (j > 0) {
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
                    int64_t em = shfl64(im, l > 0 ? l - 1 : 0), en = shfl64(in, l > 0 ? l - 1 : 0);
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
            int64_t kF = 0, kP = 0;
            if (has_const) {
                const int64_t r = readlane64(chref, 0);
                const int lst = readlane32(chlast, 0);
                kF = r - sumF;
                kP = P0 + S.P[lst];
            }
            // publish the map
            if (l == 0) st_status(st + W_MLO, pack(Lo, 1));
            if (l == 1) st_status(st + W_MHI, pack(Hi, 1));
            if (l == 2) st_status(st + W_MCF, pack(kF, has_const ? 2 : 1));
            if (l == 3) st_status(st + W_MCP, pack(kP, 1));
            if (has_const && Lo > Hi) {
                map_total = true;
                map_kF = kF;
                map_kP = kP;
                if (l == 0) st_status(st + W_XF, pack(kF, 1));
                if (l == 1) st_status(st + W_XP, pack(kP, 1));
            }
        }

        // ---- P4: entry state, then the segment's own samples -----------------
        int64_t eF = 0, eP = 0;
        if (j > 0 && !lookback_chain(D.status, j, 0, eF, eP, ctl)) err |= 8u;
        uint64_t smask_v = 0;  // lane w: sample mask of window w
        int64_t ref = eF;
        int lastS = -1;
        int64_t gbest = 0;
        int gnode = -1;
        int64_t smax = INT64_MIN;
        for (int w = 0; w < NW; ++w) {
            const int64_t f = S.F[w * 64 + l];
            int stl = -1;
            uint64_t m = 0;
            for (;;) {
                const int64_t d = f - ref;
                const uint64_t ex = ballot(l > stl && (d >= T || d <= -T));
                if (!ex) break;
                const int jj = ctz64(ex);
                const int64_t fj = readlane64(f, jj);
                if (fj > ref && (gnode < 0 || fj > gbest)) {
                    gbest = fj;
                    gnode = w * 64 + jj;
                }
                if (fj > smax) smax = fj;
                ref = fj;
                m |= 1ull << jj;
                stl = jj;
                lastS = w * 64 + jj;
            }
            if (l == w) smask_v = m;
        }
        const int64_t xF = ref - sumF;
        const int64_t xP = lastS >= 0 ? P0 + S.P[lastS] : eP;
        if (!map_total) {
            if (l == 0) st_status(st + W_XF, pack(xF, 1));
            if (l == 1) st_status(st + W_XP, pack(xP, 1));
        } else if (xF != map_kF || xP != map_kP) {
            err |= 4u;  // internal: the all-entry map disagrees with the simulated chain
        }
        const int count = (int)wave_sum(l < NW ? (int64_t)__popcll(smask_v) : 0);
        if (smax != INT64_MIN && F0 + smax > peakS) peakS = F0 + smax;

        // ---- P5: publish (count, best growth record), then combine ------------
        {
            const bool hg = gnode >= 0;
            const int64_t gval = F0 + gbest;
            const uint32_t gidx = hg ? (uint32_t)(a + gnode) : 0u;
            const uint32_t gptr = hg ? S.ptr[gnode] : 0u;
            if (l == 0) st_status(st + W_BCNT, pack(count, 1));
            if (l == 1) st_status(st + W_BGM, pack(hg ? gval : 0, hg ? 2 : 1));
            if (l == 2) st_status(st + W_BGR, pack((int64_t)gidx, 1));
            if (l == 3) st_status(st + W_BGP, pack((int64_t)gptr, 1));
            int64_t base = 0, hv = 0;
            bool hh = false;
            uint32_t hidx = 0, hptr = 0;
            if (j > 0 && !lookback_best(D.status, j, 0, base, hh, hv, hidx, hptr, ctl)) err |= 8u;
            if (base < 0 || base > (int64_t)D.n) {  // only reachable after an internal fault
                err |= 8u;
                base = 0;
            }
            // inclusive record
            bool nh = hh;
            int64_t nvv = hv;
            uint32_t nidx = hidx, nptr = hptr;
            if (hg && gval > (hh ? hv : 0)) {
                nh = true;
                nvv = gval;
                nidx = gidx;
                nptr = gptr;
            }
            if (l == 0) st_status(st + W_ICNT, pack(base + count, 1));
            if (l == 1) st_status(st + W_IGM, pack(nh ? nvv : 0, nh ? 2 : 1));
            if (l == 2) st_status(st + W_IGR, pack((int64_t)nidx, 1));
            if (l == 3) st_status(st + W_IGP, pack((int64_t)nptr, 1));
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
                const uint32_t ln = S.line[k];
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
                        Sample smp;
                        smp.event_idx = (uint32_t)(a + k);
                        smp.line = ln;
                        smp.F = Fabs;
                        smp.py = pyb;
                        smp.nat = nat;
                        D.samples[rank] = smp;
                        if (ln < L) {
                            if (dl > 0)
                                hist_add(hc, D, t, ln, C_PY, pyb, C_NAT, nat, C_GN, 1, C_GB, dl);
                            else
                                hist_add(hc, D, t, ln, C_PY, pyb, C_NAT, nat, C_SN, 1, C_SB, -dl);
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
        if (err && l == 0) atomicOr(&D.scal->err, err);
    }
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
    if (blockIdx.x == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0;
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
