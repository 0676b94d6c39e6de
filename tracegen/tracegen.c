/*
 * tracegen.c - seeded synthetic allocation/free/copy/timer event traces.
 *
 * This module only synthesises inputs.  It holds none of the sampler's
 * arithmetic: it never computes a footprint, a threshold crossing, an
 * attribution or a leak score.  Both the CPU oracle and the GPU path consume
 * the byte buffers it writes.
 *
 * Record layout (24 bytes, little endian, array of structs):
 *   int64  delta     signed bytes for memory events (alloc > 0, free < 0),
 *                    bytes copied for copy events, delay in microseconds for
 *                    timer events
 *   uint32 ptr_id    allocation identity; unique per allocation, 0 for
 *                    copy/timer events
 *   uint32 line_id   source line the event is attributed to
 *   uint8  flags     bit 0: 0 = Python, 1 = native; bits 1-2: kind
 *                    (0 memory, 1 copy, 2 timer)
 *   uint8  pad[7]    zero
 *
 * Determinism: every random draw comes from xoshiro256** seeded through
 * splitmix64 (both published generators by Vigna).  The few transcendental
 * functions (log, exp) are computed here from basic IEEE-754 double
 * operations only (no libm), so the same seed gives the same bytes on every
 * x86-64 host regardless of which libm variant the loader picks.  Build with
 * -ffp-contract=off so no fused multiply-add changes a rounding.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h> /* sqrt only: correctly rounded by IEEE-754 */

#define TG_EXPORT __attribute__((visibility("default")))

typedef struct {
    int64_t delta;
    uint32_t ptr_id;
    uint32_t line_id;
    uint8_t flags;
    uint8_t pad[7];
} tg_event;

_Static_assert(sizeof(tg_event) == 24, "event record must be 24 bytes");

/* ---------------------------------------------------------------- PRNG -- */

static uint64_t splitmix64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

TG_EXPORT uint64_t tg_splitmix64(uint64_t x) {
    uint64_t s = x;
    return splitmix64_next(&s);
}

typedef struct { uint64_t s[4]; } rng_t;

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t rng_u64(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_u64(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n), Lemire's multiply-shift (bias < n / 2^64) */
static inline uint64_t rng_below(rng_t *r, uint64_t n) {
    return (uint64_t)(((unsigned __int128)rng_u64(r) * n) >> 64);
}

/* ------------------------------------------- deterministic log and exp -- */

static const double LN2 = 0.6931471805599453094;

static double make_pow2(int k) {
    /* 2^k for k in the normal exponent range */
    uint64_t bits = (uint64_t)(k + 1023) << 52;
    double d;
    memcpy(&d, &bits, 8);
    return d;
}

/* Series coefficients, filled once by coef_init(): 1/(2k+1) for the atanh
 * series of log and 1/i! for the Taylor series of exp.  Evaluating with
 * Horner's rule on these tables uses only IEEE-754 add and multiply. */
static double LOG_COEF[13];
static double EXP_COEF[15];
static int coef_ready = 0;

static void coef_init(void) {
    if (coef_ready) return;
    for (int k = 0; k < 13; ++k) LOG_COEF[k] = 1.0 / (double)(2 * k + 1);
    double f = 1.0;
    EXP_COEF[0] = 1.0;
    for (int i = 1; i < 15; ++i) { f *= (double)i; EXP_COEF[i] = 1.0 / f; }
    coef_ready = 1;
}

/* natural log of x > 0 (normal range): x = m * 2^e with m in
 * [sqrt(1/2), sqrt(2)), log m = 2 atanh(s), s = (m-1)/(m+1). */
static double det_log(double x) {
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    bits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull; /* m in [1,2) */
    double m;
    memcpy(&m, &bits, 8);
    if (m > 1.4142135623730951) { m *= 0.5; e += 1; }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double acc = LOG_COEF[12];
    for (int k = 11; k >= 0; --k) acc = acc * s2 + LOG_COEF[k];
    return 2.0 * s * acc + (double)e * LN2;
}

/* e^x for |x| < 700: x = k ln2 + r, |r| <= ln2/2, Taylor series for e^r. */
static double det_exp(double x) {
    double kd = x / LN2;
    int k = (int)(kd < 0 ? kd - 0.5 : kd + 0.5);
    double r = x - (double)k * LN2;
    double acc = EXP_COEF[14];
    for (int i = 13; i >= 0; --i) acc = acc * r + EXP_COEF[i];
    if (k > 1020) { acc *= make_pow2(k - 1020); k = 1020; }
    if (k < -1020) { acc *= make_pow2(k + 1020); k = -1020; }
    return acc * make_pow2(k);
}

/* ----------------------------------------------------------- samplers -- */

/* floor of a log-uniform draw on [lo, hi] */
static int64_t draw_log_uniform(rng_t *r, double loglo, double loghi, int64_t lo, int64_t hi) {
    double v = det_exp(loglo + rng_unif(r) * (loghi - loglo));
    int64_t s = (int64_t)v;
    if (s < lo) s = lo;
    if (s > hi) s = hi;
    return s;
}

/* exponential with the given mean, as a double >= 0 */
static double draw_exp(rng_t *r, double mean) {
    return -mean * det_log(1.0 - rng_unif(r)); /* 1-u in (0, 1] */
}

/* standard normal, Marsaglia's polar method (log and sqrt only) */
static double draw_normal(rng_t *r) {
    for (;;) {
        double x = 2.0 * rng_unif(r) - 1.0;
        double y = 2.0 * rng_unif(r) - 1.0;
        double s = x * x + y * y;
        if (s > 0.0 && s < 1.0) return x * sqrt(-2.0 * det_log(s) / s);
    }
}

/* Zipf over ranks 0..n-1 with weight (rank+1)^-s, Vose's alias method.  The
 * rank is mapped to a line id by a fixed bijection so hot lines are spread
 * over the id space rather than packed at 0. */
typedef struct { double prob; uint32_t id_self; uint32_t id_alias; } zslot_t;

typedef struct {
    uint32_t n;
    zslot_t *tab;
    uint64_t mult, add;
    /* the next draw is started one call ahead so its table slot can be
     * prefetched: rank candidate and its acceptance uniform */
    uint32_t next_k;
    double next_u;
} zipf_t;

static int zipf_init(zipf_t *z, uint32_t n, double s) {
    z->n = n;
    z->tab = (zslot_t *)malloc(sizeof(zslot_t) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!z->tab || !w || !small || !large) return -1;
    double total = 0.0;
    for (uint32_t k = 0; k < n; ++k) {
        w[k] = det_exp(-s * det_log((double)k + 1.0));
        total += w[k];
    }
    uint32_t ns = 0, nl = 0;
    for (uint32_t k = 0; k < n; ++k) {
        w[k] = w[k] * (double)n / total;
        if (w[k] < 1.0) small[ns++] = k; else large[nl++] = k;
    }
    while (ns > 0 && nl > 0) {
        uint32_t l = small[--ns], g = large[--nl];
        z->tab[l].prob = w[l];
        z->tab[l].id_alias = g;
        w[g] = (w[g] + w[l]) - 1.0;
        if (w[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { uint32_t g = large[--nl]; z->tab[g].prob = 1.0; z->tab[g].id_alias = g; }
    while (ns > 0) { uint32_t l = small[--ns]; z->tab[l].prob = 1.0; z->tab[l].id_alias = l; }
    free(w); free(small); free(large);
    /* multiplier coprime with n for the rank -> id bijection */
    uint64_t m = 7919;
    for (;;) {
        uint64_t a = m % n, b = n;
        while (b) { uint64_t t = a % b; a = b; b = t; }
        if (a == 1 || n == 1) break;
        m += 2;
    }
    z->mult = m % (n ? n : 1);
    z->add = 17 % (n ? n : 1);
    /* store mapped line ids in the table so a draw needs no division */
    for (uint32_t k = 0; k < n; ++k) {
        z->tab[k].id_self = (uint32_t)(((uint64_t)k * z->mult + z->add) % n);
        z->tab[k].id_alias = (uint32_t)(((uint64_t)z->tab[k].id_alias * z->mult + z->add) % n);
    }
    return 0;
}

static void zipf_free(zipf_t *z) { free(z->tab); }

static inline void zipf_start(zipf_t *z, rng_t *r) {
    z->next_k = (uint32_t)rng_below(r, z->n);
    z->next_u = rng_unif(r);
    __builtin_prefetch(&z->tab[z->next_k]);
}

static inline uint32_t zipf_draw(zipf_t *z, rng_t *r) {
    const zslot_t *s = &z->tab[z->next_k];
    uint32_t id = z->next_u >= s->prob ? s->id_alias : s->id_self;
    zipf_start(z, r);
    return id;
}

/* --------------------------------------------------------- event mixes -- */

enum { KIND_MEM = 0, KIND_COPY = 1, KIND_TIMER = 2 };

static inline void put(tg_event *e, int64_t delta, uint32_t ptr, uint32_t line, int pn, int kind) {
    e->delta = delta;
    e->ptr_id = ptr;
    e->line_id = line;
    e->flags = (uint8_t)((pn & 1) | (kind << 1));
    memset(e->pad, 0, sizeof e->pad);
}

/* "Uniform-live" mix: each memory event allocates with probability
 * alloc_frac (log-uniform size, Python with probability py_frac) or frees a
 * uniformly chosen live pointer (the negated size); a fraction leak_frac of
 * allocations is never freed.  copy_frac / timer_frac of all events are copy
 * events (log-uniform bytes) and timer events (exponential delay). */
typedef struct {
    uint32_t num_lines;
    double zipf_s;
    double alloc_frac;
    double py_frac;
    double leak_frac;
    int64_t size_lo, size_hi;
    double copy_frac;
    double timer_frac;
    double timer_mean_us;
} tg_mix_params;

typedef struct { uint32_t ptr; uint32_t pn; int64_t size; } live_t;

TG_EXPORT int tg_mix(uint64_t seed, uint64_t n, const tg_mix_params *p, void *out) {
    coef_init();
    if (!p || (!out && n) || p->num_lines == 0 || p->size_lo < 1 || p->size_hi < p->size_lo) return -1;
    if (n >= 0xFFFFFFFFull) return -1;
    rng_t r;
    rng_seed(&r, seed);
    zipf_t z;
    if (zipf_init(&z, p->num_lines, p->zipf_s)) return -2;
    zipf_start(&z, &r);
    size_t cap = 1024, nlive = 0;
    live_t *live = (live_t *)malloc(cap * sizeof(live_t));
    if (!live) return -2;
    tg_event *ev = (tg_event *)out;
    double loglo = det_log((double)p->size_lo), loghi = det_log((double)p->size_hi + 1.0);
    uint32_t next_ptr = 1;
    /* The uniform word that picks the next freed pointer is drawn one free
     * ahead so its live-set slot can be prefetched (the live set of a long
     * trace is far larger than the caches). */
    uint64_t upick = rng_u64(&r);
    for (uint64_t i = 0; i < n; ++i) {
        double u = rng_unif(&r);
        if (u < p->copy_frac) {
            int64_t b = draw_log_uniform(&r, loglo, loghi, p->size_lo, p->size_hi);
            uint32_t line = zipf_draw(&z, &r);
            int pn = rng_unif(&r) < p->py_frac ? 0 : 1;
            put(&ev[i], b, 0, line, pn, KIND_COPY);
            continue;
        }
        if (u < p->copy_frac + p->timer_frac) {
            double d = draw_exp(&r, p->timer_mean_us) + 0.5;
            int64_t delay = (int64_t)d;
            if (delay > 0xFFFFFFFFll) delay = 0xFFFFFFFFll;
            uint32_t line = zipf_draw(&z, &r);
            put(&ev[i], delay, 0, line, 0, KIND_TIMER);
            continue;
        }
        if (nlive == 0 || rng_unif(&r) < p->alloc_frac) {
            int64_t size = draw_log_uniform(&r, loglo, loghi, p->size_lo, p->size_hi);
            int pn = rng_unif(&r) < p->py_frac ? 0 : 1;
            uint32_t line = zipf_draw(&z, &r);
            uint32_t ptr = next_ptr++;
            put(&ev[i], size, ptr, line, pn, KIND_MEM);
            if (rng_unif(&r) >= p->leak_frac) {
                if (nlive == cap) {
                    cap *= 2;
                    live_t *nl = (live_t *)realloc(live, cap * sizeof(live_t));
                    if (!nl) { free(live); zipf_free(&z); return -2; }
                    live = nl;
                }
                live[nlive].ptr = ptr;
                live[nlive].pn = (uint32_t)pn;
                live[nlive].size = size;
                ++nlive;
            }
        } else {
            size_t k = (size_t)(((unsigned __int128)upick * nlive) >> 64);
            live_t o = live[k];
            live[k] = live[--nlive];
            upick = rng_u64(&r);
            if (nlive) __builtin_prefetch(&live[(size_t)(((unsigned __int128)upick * nlive) >> 64)]);
            uint32_t line = zipf_draw(&z, &r);
            put(&ev[i], -o.size, o.ptr, line, (int)o.pn, KIND_MEM);
        }
    }
    free(live);
    zipf_free(&z);
    return 0;
}

/* "Lifetime" mix: allocations are small Python objects (16*k bytes, k-1
 * geometric with success probability geo_p, truncated at k_max) with
 * probability small_frac, else native arrays with log-uniform size on
 * [big_lo, big_hi].  Each non-leaked allocation dies after an exponential
 * lifetime (in events); a due death is emitted as a free before any new
 * allocation. */
typedef struct {
    uint32_t num_lines;
    double zipf_s;
    double small_frac;
    double geo_p;
    uint32_t k_max;
    int64_t big_lo, big_hi;
    double life_mean;
    double leak_frac;
} tg_life_params;

typedef struct { uint64_t death; uint32_t ptr; uint32_t pn; int64_t size; } death_t;

static void heap_push(death_t *h, size_t *n, death_t v) {
    size_t i = (*n)++;
    while (i > 0) {
        size_t par = (i - 1) / 2;
        if (h[par].death < v.death || (h[par].death == v.death && h[par].ptr < v.ptr)) break;
        h[i] = h[par];
        i = par;
    }
    h[i] = v;
}

static death_t heap_pop(death_t *h, size_t *n) {
    death_t top = h[0];
    death_t v = h[--(*n)];
    size_t i = 0;
    for (;;) {
        size_t c = 2 * i + 1;
        if (c >= *n) break;
        if (c + 1 < *n && (h[c + 1].death < h[c].death || (h[c + 1].death == h[c].death && h[c + 1].ptr < h[c].ptr))) ++c;
        if (v.death < h[c].death || (v.death == h[c].death && v.ptr < h[c].ptr)) break;
        h[i] = h[c];
        i = c;
    }
    h[i] = v;
    return top;
}

TG_EXPORT int tg_lifetime(uint64_t seed, uint64_t n, const tg_life_params *p, void *out) {
    coef_init();
    if (!p || (!out && n) || p->num_lines == 0 || p->k_max < 1 || p->big_lo < 1 || p->big_hi < p->big_lo) return -1;
    if (n >= 0xFFFFFFFFull) return -1;
    rng_t r;
    rng_seed(&r, seed);
    zipf_t z;
    if (zipf_init(&z, p->num_lines, p->zipf_s)) return -2;
    zipf_start(&z, &r);
    size_t cap = 1024, nh = 0;
    death_t *h = (death_t *)malloc(cap * sizeof(death_t));
    if (!h) return -2;
    tg_event *ev = (tg_event *)out;
    double loglo = det_log((double)p->big_lo), loghi = det_log((double)p->big_hi + 1.0);
    double log_q = det_log(1.0 - p->geo_p);
    uint32_t next_ptr = 1;
    for (uint64_t i = 0; i < n; ++i) {
        if (nh > 0 && h[0].death <= i) {
            death_t d = heap_pop(h, &nh);
            uint32_t line = zipf_draw(&z, &r);
            put(&ev[i], -d.size, d.ptr, line, (int)d.pn, KIND_MEM);
            continue;
        }
        int64_t size;
        int pn;
        if (rng_unif(&r) < p->small_frac) {
            /* k - 1 = number of failures before the first success */
            double g = det_log(1.0 - rng_unif(&r)) / log_q;
            uint64_t k = (uint64_t)g + 1;
            if (k > p->k_max) k = p->k_max;
            size = 16 * (int64_t)k;
            pn = 0;
        } else {
            size = draw_log_uniform(&r, loglo, loghi, p->big_lo, p->big_hi);
            pn = 1;
        }
        uint32_t line = zipf_draw(&z, &r);
        uint32_t ptr = next_ptr++;
        put(&ev[i], size, ptr, line, pn, KIND_MEM);
        if (rng_unif(&r) >= p->leak_frac) {
            double life = draw_exp(&r, p->life_mean);
            death_t d;
            d.death = i + 1 + (uint64_t)life;
            d.ptr = ptr;
            d.pn = (uint32_t)pn;
            d.size = size;
            if (nh == cap) {
                cap *= 2;
                death_t *nh2 = (death_t *)realloc(h, cap * sizeof(death_t));
                if (!nh2) { free(h); zipf_free(&z); return -2; }
                h = nh2;
            }
            heap_push(h, &nh, d);
        }
    }
    free(h);
    zipf_free(&z);
    return 0;
}

/* ------------------------------------------------------ workload plans -- */

/* Batch of n traces: length floor(10^(lo_exp + (hi_exp-lo_exp) u)), a
 * threshold index uniform in [0, n_thresholds) and a per-trace seed
 * splitmix64(base ^ t). */
TG_EXPORT int tg_plan_batch(uint64_t base_seed, uint32_t n, double lo_exp, double hi_exp,
                            uint32_t n_thresholds, uint64_t *out_len, uint32_t *out_tidx,
                            uint64_t *out_seed) {
    coef_init();
    if (n_thresholds == 0) return -1;
    rng_t r;
    rng_seed(&r, base_seed);
    const double LN10 = 2.302585092994045684;
    for (uint32_t t = 0; t < n; ++t) {
        double e = lo_exp + (hi_exp - lo_exp) * rng_unif(&r);
        out_len[t] = (uint64_t)det_exp(e * LN10);
        if (out_len[t] < 1) out_len[t] = 1;
        out_tidx[t] = (uint32_t)rng_below(&r, n_thresholds);
        out_seed[t] = tg_splitmix64(base_seed ^ (uint64_t)t);
    }
    return 0;
}

/* Served requests: Poisson arrivals at rate_per_s (arrival time in ns from
 * the first request), lengths LogNormal(log(median), sigma) clamped to
 * [1, cap], per-request seed splitmix64(base ^ i). */
TG_EXPORT int tg_plan_serve(uint64_t base_seed, uint32_t n, double rate_per_s, double median,
                            double sigma, uint64_t cap, uint64_t *out_len, uint64_t *out_arrival_ns,
                            uint64_t *out_seed) {
    coef_init();
    if (rate_per_s <= 0 || median <= 0) return -1;
    rng_t r;
    rng_seed(&r, base_seed);
    double t_ns = 0.0, logm = det_log(median);
    for (uint32_t i = 0; i < n; ++i) {
        if (i > 0) t_ns += draw_exp(&r, 1e9 / rate_per_s);
        out_arrival_ns[i] = (uint64_t)t_ns;
        double len = det_exp(logm + sigma * draw_normal(&r));
        uint64_t l = (uint64_t)len;
        if (l < 1) l = 1;
        if (l > cap) l = cap;
        out_len[i] = l;
        out_seed[i] = tg_splitmix64(base_seed ^ (uint64_t)i);
    }
    return 0;
}

/* 64-bit digest of a byte buffer, for pinning generated traces: each 8-byte
 * little-endian word is folded through a splitmix64 round. */
TG_EXPORT uint64_t tg_digest(const void *buf, uint64_t bytes) {
    const uint8_t *b = (const uint8_t *)buf;
    uint64_t h = 0x243F6A8885A308D3ull ^ bytes;
    uint64_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        memcpy(&w, b + i, 8);
        h = tg_splitmix64(h ^ w);
    }
    uint64_t tail = 0;
    for (uint64_t k = 0; i + k < bytes; ++k) tail |= (uint64_t)b[i + k] << (8 * k);
    return tg_splitmix64(h ^ tail ^ 0x13198A2E03707344ull);
}

/* exposed for tests of the deterministic math */
TG_EXPORT double tg_det_log(double x) { coef_init(); return det_log(x); }
TG_EXPORT double tg_det_exp(double x) { coef_init(); return det_exp(x); }
