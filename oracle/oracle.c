/*
 * oracle.c - plain, sequential CPU reference for the threshold sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * What it computes, step by step in the paper's own terms (Berger, Stern,
 * Altmayer Pizzorno, "Triangulating Python Performance Issues with Scalene",
 * OSDI 2023, arXiv:2212.07597):
 *
 *  - Threshold-based sampling (section 3.2): the sampler keeps A, the bytes
 *    allocated, and F, the bytes freed, since the last sample.  When
 *    |A - F| >= T it takes a sample and resets both counters.  The loop below
 *    keeps exactly those two counters (named A and Fr here so that F stays the
 *    footprint) in 128-bit integers so they cannot overflow.
 *  - Sample contents (section 3.3): each sample records whether it was growth
 *    or shrink, the Python/native split of the bytes in the sample and the
 *    line it is attributed to; the footprint at each crossing is recorded for
 *    the timeline and the maximum footprint is tracked.
 *  - Leak detection (section 3.4): at a growth sample that sets a new
 *    high-water mark the sampled allocation is tracked; every later free is
 *    compared with it; at the next new maximum the site's leak score
 *    (frees, mallocs) is updated - mallocs when tracking starts, frees only if
 *    the object was reclaimed - and a new object is tracked.
 *  - Leak likelihood (section 3.4, Rule of Succession): reported as exact
 *    rationals in two readings, Laplace's rule 1 - (f+1)/(m+2) and the
 *    formula as printed, 1 - (f+1)/(m-f+2), plus the 95 % report gate.
 *  - Copy volume (section 3.5): rate-based sampling of memcpy bytes, one
 *    sample of Tc bytes per multiple of Tc crossed by the cumulative count.
 *  - Python/native time (section 2.1): each timer sample adds the quantum q
 *    to the line's Python time and the signal delay to its native time.
 *  - Rate-based sampling (section 3.2, the scheme threshold sampling is
 *    compared with; oracle_rate below): one sample per T bytes allocated or
 *    freed, counted over the cumulative volume of memory events.
 *
 * Readings where the paper is silent (all stated in the design notes):
 *  start state 0 before event 0; ">=" triggers; reset discards overshoot; the
 *  sample is attributed to the triggering event's line; only memory events
 *  move the footprint; the Python/native split is the signed net bytes of
 *  each kind over the sample's window; the high-water mark is the maximum
 *  footprint over earlier tracked samples, starting at 0, compared with ">";
 *  a tracked object counts as reclaimed if a free of its pointer id occurs
 *  before the next tracked sample; the last tracked object stays unresolved
 *  unless OPT_RESOLVE_AT_END; per-line sums wrap modulo 2^64.
 *
 * Input contract: |delta| < 2^52 for memory and copy events, timer delays in
 * [0, 2^32), kind < 3, line < num_lines (else OR_EINVAL, which wins over
 * overflow); every prefix of the footprint, of its Python part and of the
 * copy bytes must stay inside (-2^61, 2^61) (else OR_EOVERFLOW).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* status codes (same numbering as the library's, defined independently) */
enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 7, OR_EOVERFLOW = 6 };

enum { OR_OPT_PRIME_T = 1u, OR_OPT_RESOLVE_AT_END = 2u };

#define OR_MAX_ABS_DELTA ((int64_t)1 << 52)
#define OR_MAX_ABS_F ((int64_t)1 << 61)
#define OR_MAX_T ((int64_t)1 << 60)

typedef struct {
    int64_t delta;
    uint32_t ptr_id;
    uint32_t line_id;
    uint8_t flags;
    uint8_t pad[7];
} or_event;

typedef struct {
    int64_t threshold;
    int64_t copy_threshold;
    uint32_t num_lines;
    uint32_t quantum_us;
    uint32_t options;
    uint32_t reserved;
} or_params;

typedef struct {
    uint32_t event_idx;
    uint32_t line;
    int64_t F;
    int64_t py;
    int64_t nat;
} or_sample;

typedef struct {
    uint32_t event_idx;
    uint32_t line;
    uint32_t ptr;
    uint32_t freed;
} or_tracked;

enum {
    H_PY_BYTES, H_NAT_BYTES, H_GROWTH_N, H_SHRINK_N, H_GROWTH_BYTES, H_SHRINK_BYTES,
    H_LEAK_MALLOCS, H_LEAK_FREES, H_COPY_SAMPLED, H_COPY_EXACT, H_PY_TIME, H_NAT_TIME,
    H_COUNT
};

typedef struct {
    int status;
    uint32_t num_lines;
    int64_t threshold_used;
    uint64_t n_samples;
    uint64_t n_tracked;
    int64_t final_F;
    int64_t peak_F;
    int64_t peak_sampled_F;
    or_sample *samples;
    or_tracked *tracked;
    int64_t *hist; /* H_COUNT arrays of num_lines, back to back */
    uint64_t samples_cap, tracked_cap;
} or_result;

static int is_prime(uint64_t v) {
    if (v < 2) return 0;
    if (v % 2 == 0) return v == 2;
    for (uint64_t d = 3; d * d <= v; d += 2)
        if (v % d == 0) return 0;
    return 1;
}

/* smallest prime >= t (the paper sets T to a prime to avoid stride effects) */
OR_EXPORT int64_t oracle_prime_at_least(int64_t t) {
    uint64_t v = t < 2 ? 2 : (uint64_t)t;
    while (!is_prime(v)) ++v;
    return (int64_t)v;
}

static int push_sample(or_result *r, or_sample s) {
    if (r->n_samples == r->samples_cap) {
        uint64_t cap = r->samples_cap ? 2 * r->samples_cap : 1024;
        or_sample *p = (or_sample *)realloc(r->samples, cap * sizeof(or_sample));
        if (!p) return -1;
        r->samples = p;
        r->samples_cap = cap;
    }
    r->samples[r->n_samples++] = s;
    return 0;
}

static int push_tracked(or_result *r, or_tracked t) {
    if (r->n_tracked == r->tracked_cap) {
        uint64_t cap = r->tracked_cap ? 2 * r->tracked_cap : 256;
        or_tracked *p = (or_tracked *)realloc(r->tracked, cap * sizeof(or_tracked));
        if (!p) return -1;
        r->tracked = p;
        r->tracked_cap = cap;
    }
    r->tracked[r->n_tracked++] = t;
    return 0;
}

/* wrapping add for per-line sums (two's complement, modulo 2^64) */
static inline void wadd(int64_t *dst, int64_t v) { *dst = (int64_t)((uint64_t)*dst + (uint64_t)v); }

OR_EXPORT void oracle_free(or_result *r) {
    if (!r) return;
    free(r->samples);
    free(r->tracked);
    free(r->hist);
    free(r);
}

OR_EXPORT int oracle_run(const void *events, uint64_t n, const or_params *p, or_result **out) {
    *out = NULL;
    or_result *r = (or_result *)calloc(1, sizeof(or_result));
    if (!r) return OR_ENOMEM;
    *out = r;
    if (!p || p->threshold < 1 || p->threshold >= OR_MAX_T || p->copy_threshold < 1 ||
        p->num_lines == 0 || n >= 0xFFFFFFFFull || (n && !events)) {
        r->status = OR_EINVAL;
        return r->status;
    }
    const uint32_t L = p->num_lines;
    r->num_lines = L;
    r->hist = (int64_t *)calloc((size_t)H_COUNT * L, sizeof(int64_t));
    if (!r->hist) { r->status = OR_ENOMEM; return r->status; }
    int64_t *h[H_COUNT];
    for (int k = 0; k < H_COUNT; ++k) h[k] = r->hist + (size_t)k * L;

    const int64_t T = (p->options & OR_OPT_PRIME_T) ? oracle_prime_at_least(p->threshold) : p->threshold;
    r->threshold_used = T;
    const int64_t Tc = p->copy_threshold;
    const int64_t q = (int64_t)p->quantum_us;

    const or_event *ev = (const or_event *)events;
    __int128 A = 0, Fr = 0;      /* bytes allocated / freed since the last sample */
    int64_t cur = 0;             /* footprint */
    int64_t wpy = 0, wnat = 0;   /* net Python / native bytes since the last sample */
    int64_t hwm = 0;             /* high-water mark over tracked samples */
    int have_tracked = 0;
    uint64_t tracked_slot = 0;   /* index of the tracked object in r->tracked */
    int64_t C = 0;               /* cumulative copy bytes */
    int64_t peak = 0, peak_s = 0;
    int64_t pycur = 0;           /* footprint of Python memory (range check only) */
    int status = OR_OK;
    int overflow = 0;            /* once set, events are only validated */

    for (uint64_t i = 0; i < n; ++i) {
        const or_event e = ev[i];
        const int kind = (e.flags >> 1) & 3;
        const int pn = e.flags & 1;
        const uint32_t line = e.line_id;
        const int64_t d = e.delta;
        if (kind == 3 || line >= L) { status = OR_EINVAL; break; }
        if (kind == 0) {
            if (d >= OR_MAX_ABS_DELTA || d <= -OR_MAX_ABS_DELTA) { status = OR_EINVAL; break; }
            if (overflow) continue;
            cur += d;
            if (pn == 0) pycur += d;
            if (cur >= OR_MAX_ABS_F || cur <= -OR_MAX_ABS_F || pycur >= OR_MAX_ABS_F || pycur <= -OR_MAX_ABS_F) {
                overflow = 1;
                continue;
            }
            if (d > 0) A += d; else Fr += -(__int128)d;
            if (pn == 0) wpy += d; else wnat += d;
            if (d < 0 && have_tracked && e.ptr_id == r->tracked[tracked_slot].ptr)
                r->tracked[tracked_slot].freed = 1;
            if (cur > peak) peak = cur;
            __int128 diff = A - Fr;
            __int128 mag = diff < 0 ? -diff : diff;
            if (mag >= T) {
                or_sample s = { (uint32_t)i, line, cur, wpy, wnat };
                if (push_sample(r, s)) { status = OR_ENOMEM; break; }
                wadd(&h[H_PY_BYTES][line], wpy);
                wadd(&h[H_NAT_BYTES][line], wnat);
                if (diff > 0) {
                    wadd(&h[H_GROWTH_N][line], 1);
                    wadd(&h[H_GROWTH_BYTES][line], (int64_t)diff);
                } else {
                    wadd(&h[H_SHRINK_N][line], 1);
                    wadd(&h[H_SHRINK_BYTES][line], (int64_t)(-diff));
                }
                if (cur > peak_s) peak_s = cur;
                if (diff > 0 && cur > hwm) {
                    /* new high-water mark: settle the previous object's score
                     * and start tracking the sampled allocation */
                    if (have_tracked) {
                        const or_tracked *t = &r->tracked[tracked_slot];
                        wadd(&h[H_LEAK_FREES][t->line], (int64_t)t->freed);
                    }
                    or_tracked t = { (uint32_t)i, line, e.ptr_id, 0 };
                    if (push_tracked(r, t)) { status = OR_ENOMEM; break; }
                    tracked_slot = r->n_tracked - 1;
                    have_tracked = 1;
                    wadd(&h[H_LEAK_MALLOCS][line], 1);
                    hwm = cur;
                }
                A = 0;
                Fr = 0;
                wpy = 0;
                wnat = 0;
            }
        } else if (kind == 1) {
            if (d < 0 || d >= OR_MAX_ABS_DELTA) { status = OR_EINVAL; break; }
            if (overflow) continue;
            if (C + d >= OR_MAX_ABS_F) { overflow = 1; continue; }
            wadd(&h[H_COPY_EXACT][line], d);
            int64_t nsamp = (C + d) / Tc - C / Tc;
            wadd(&h[H_COPY_SAMPLED][line], (int64_t)((uint64_t)nsamp * (uint64_t)Tc));
            C += d;
        } else { /* timer */
            if (d < 0 || d > 0xFFFFFFFFll) { status = OR_EINVAL; break; }
            if (overflow) continue;
            wadd(&h[H_PY_TIME][line], q);
            wadd(&h[H_NAT_TIME][line], d);
        }
    }
    if (status == OR_OK && overflow) status = OR_EOVERFLOW;
    if (status == OR_OK && have_tracked && (p->options & OR_OPT_RESOLVE_AT_END)) {
        const or_tracked *t = &r->tracked[tracked_slot];
        wadd(&h[H_LEAK_FREES][t->line], (int64_t)t->freed);
    }
    r->final_F = cur;
    r->peak_F = peak;
    r->peak_sampled_F = peak_s;
    r->status = status;
    return status;
}

static int64_t gcd64(int64_t a, int64_t b) {
    if (a < 0) a = -a;
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a;
}

static void reduce(int64_t num, int64_t den, int64_t *on, int64_t *od) {
    if (num == 0) { *on = 0; *od = 1; return; }
    int64_t g = gcd64(num, den);
    *on = num / g;
    *od = den / g;
}

/* Leak likelihood per line from the (frees, mallocs) pair, as exact reduced
 * rationals with a positive denominator.  Laplace's rule of succession with
 * frees as successes: 1 - (f+1)/(m+2) = (m-f+1)/(m+2).  The formula as
 * printed in the paper: 1 - (f+1)/(m-f+2) = (m-2f+1)/(m-f+2).  The report
 * gate is "likelihood > 0.95", i.e. 20*num > 19*den.  Lines with m = 0 get
 * 0/0 and gate 0. */
OR_EXPORT void oracle_leak_scores(const int64_t *mallocs, const int64_t *frees, uint32_t n,
                                  int64_t *lap_num, int64_t *lap_den, int64_t *lit_num,
                                  int64_t *lit_den, uint8_t *lap_gate, uint8_t *lit_gate) {
    for (uint32_t i = 0; i < n; ++i) {
        const int64_t m = mallocs[i], f = frees[i];
        if (m <= 0) {
            lap_num[i] = lap_den[i] = lit_num[i] = lit_den[i] = 0;
            lap_gate[i] = lit_gate[i] = 0;
            continue;
        }
        reduce(m - f + 1, m + 2, &lap_num[i], &lap_den[i]);
        reduce(m - 2 * f + 1, m - f + 2, &lit_num[i], &lit_den[i]);
        lap_gate[i] = (uint8_t)(20 * (m - f + 1) > 19 * (m + 2));
        lit_gate[i] = (uint8_t)(20 * (m - 2 * f + 1) > 19 * (m - f + 2));
    }
}

/*
 * Rate-based sampling (section 3.2): every byte allocated or freed counts
 * towards the next sample, one sample per T bytes, whatever it does to the
 * footprint.  Deterministic reading: the countdown starts at T instead of a
 * random draw, so the event that brings V, the cumulative bytes allocated
 * plus bytes freed (memory events only), to or past a multiple of T takes one
 * sample per multiple reached: n_i = floor(V_i / T) - floor(V_{i-1} / T),
 * attributed to the event's line.  line_counts (num_lines entries) receives
 * the samples per line and *K their total.  Input contract as for oracle_run
 * (OR_EINVAL wins); V must stay below 2^62 (else OR_EOVERFLOW).
 */
OR_EXPORT int oracle_rate(const void *events, uint64_t n, int64_t T, uint32_t L, int64_t *line_counts, uint64_t *K) {
    *K = 0;
    if (T < 1 || T >= OR_MAX_T || L == 0 || n >= 0xFFFFFFFFull || (n && !events) || !line_counts) return OR_EINVAL;
    memset(line_counts, 0, sizeof(int64_t) * L);
    const or_event *ev = (const or_event *)events;
    __int128 V = 0;
    int overflow = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const or_event e = ev[i];
        const int kind = (e.flags >> 1) & 3;
        const int64_t d = e.delta;
        if (kind == 3 || e.line_id >= L) return OR_EINVAL;
        if (kind == 1 && (d < 0 || d >= OR_MAX_ABS_DELTA)) return OR_EINVAL;
        if (kind == 2 && (d < 0 || d > 0xFFFFFFFFll)) return OR_EINVAL;
        if (kind != 0) continue;
        if (d >= OR_MAX_ABS_DELTA || d <= -OR_MAX_ABS_DELTA) return OR_EINVAL;
        if (overflow) continue;
        const __int128 Vn = V + (d < 0 ? -(__int128)d : (__int128)d);
        if (Vn >= ((__int128)1 << 62)) { overflow = 1; continue; }
        const int64_t ni = (int64_t)(Vn / T - V / T);
        line_counts[e.line_id] += ni;
        *K += (uint64_t)ni;
        V = Vn;
    }
    return overflow ? OR_EOVERFLOW : OR_OK;
}
