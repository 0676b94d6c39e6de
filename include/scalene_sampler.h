/*
 * scalene_sampler.h - C ABI of the MI355X threshold sampler.
 *
 * The library runs the memory-profiling core of Scalene (Berger, Stern,
 * Altmayer Pizzorno, arXiv:2212.07597) offline over recorded event traces on
 * one gfx950 GPU:
 *   - threshold-based sampling of the footprint (section 3.2): a sample is
 *     taken when the bytes allocated minus the bytes freed since the last
 *     sample reach T in absolute value, and the counters restart;
 *   - per-sample attribution to the triggering line with the Python/native
 *     split of the sample's bytes, footprint timeline and maximum (section 3.3);
 *   - the leak rule (track the sampled allocation at each new high-water mark,
 *     check every free against it) and the (frees, mallocs) leak score with
 *     its rule-of-succession likelihood (section 3.4);
 *   - copy volume by rate-based sampling of copied bytes (section 3.5);
 *   - the Python/native time split from timer-signal delays (section 2.1).
 *
 * All functions are callable from C; none throws.  Pointers marked "device"
 * must be device memory of the sampler's GPU; "host" pointers are ordinary
 * host memory.  Every function returns an SMP_* status unless noted.
 *
 * Readings where the paper is silent (identical in the CPU oracle):
 *   the footprint and the sample reference start at 0 before event 0; ">="
 *   triggers; a sample resets the reference to the footprint at the sample
 *   (overshoot discarded); the sample belongs to the triggering event's line;
 *   only memory events move the footprint; the Python/native split is the
 *   signed net bytes of each kind in the sample's window; the high-water mark
 *   is the largest footprint of an earlier tracked sample (initially 0) and a
 *   growth sample is tracked when its footprint is strictly greater; a tracked
 *   object is reclaimed if a free of its ptr_id occurs before the next tracked
 *   sample; the last tracked object is unresolved unless
 *   SMP_OPT_RESOLVE_AT_END; per-line sums wrap modulo 2^64.
 */
#ifndef SCALENE_SAMPLER_H
#define SCALENE_SAMPLER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMP_API __attribute__((visibility("default")))

/* ---- status codes ---------------------------------------------------- */
#define SMP_OK 0
#define SMP_EINVAL 1    /* bad argument, or a malformed event (reported by fetch) */
#define SMP_EBUDGET 2   /* not enough free budget now; fetch a finished trace and retry */
#define SMP_ETOOBIG 3   /* the trace alone exceeds the whole budget */
#define SMP_EAGAIN 4    /* trace not finished yet */
#define SMP_EDEVICE 5   /* a HIP call failed; the sampler is unusable and must be destroyed */
#define SMP_EOVERFLOW 6 /* a footprint, Python-footprint or copy prefix left (-2^61, 2^61) */
#define SMP_ENOMEM 7    /* host allocation failed */
#define SMP_ESTATE 8    /* call not valid in the trace's current state (unknown id, not run, ...) */

/* ---- options ----------------------------------------------------------- */
#define SMP_OPT_PRIME_T 1u        /* use the smallest prime >= threshold (section 3.2) */
#define SMP_OPT_RESOLVE_AT_END 2u /* also score the last tracked object at the end of the trace */

/* ---- event record: 24 bytes, array of structs --------------------------
 * delta   : memory event: signed bytes (allocation > 0, free < 0), |delta| < 2^52
 *           copy event  : bytes copied, 0 <= delta < 2^52
 *           timer event : signal delay in microseconds, 0 <= delta < 2^32
 * ptr_id  : identity of the allocation (compared on frees by the leak rule)
 * line_id : source line, < num_lines
 * flags   : bit 0 = 0 Python / 1 native; bits 1-2 = kind (0 memory, 1 copy, 2 timer)
 */
typedef struct {
    int64_t delta;
    uint32_t ptr_id;
    uint32_t line_id;
    uint8_t flags;
    uint8_t pad[7];
} smp_event_t;

/* ---- per-trace parameters ----------------------------------------------
 * threshold      : T >= 1 and < 2^60 (section 3.2)
 * copy_threshold : Tc >= 1, bytes per copy-volume sample (section 3.5)
 * num_lines      : line ids are < num_lines, 1 <= num_lines <= 2^31
 * quantum_us     : timer quantum q added to Python time per timer event (section 2.1)
 * options        : SMP_OPT_* bits
 */
typedef struct {
    int64_t threshold;
    int64_t copy_threshold;
    uint32_t num_lines;
    uint32_t quantum_us;
    uint32_t options;
    uint32_t reserved; /* must be 0 */
} smp_params_t;

/* one sample (section 3.3): event index of the triggering event, its line,
 * footprint after it, and the net Python / native bytes since the previous
 * sample (py + nat = F - F_previous_sample) */
typedef struct {
    uint32_t event_idx;
    uint32_t line;
    int64_t F;
    int64_t py;
    int64_t nat;
} smp_sample_t;

/* one tracked object (section 3.4): the sample that tracked it, its line and
 * ptr_id, and whether a free of it was seen before the next tracked sample
 * (for the last one: before the end of the trace) */
typedef struct {
    uint32_t event_idx;
    uint32_t line;
    uint32_t ptr;
    uint32_t freed;
} smp_tracked_t;

/* per-line histogram order inside smp_profile_t.hist (num_lines entries each) */
enum {
    SMP_H_PY_BYTES = 0,   /* sum of py over samples attributed to the line */
    SMP_H_NAT_BYTES,      /* sum of nat */
    SMP_H_GROWTH_N,       /* number of growth samples */
    SMP_H_SHRINK_N,       /* number of shrink samples */
    SMP_H_GROWTH_BYTES,   /* sum of |F - F_prev| over growth samples */
    SMP_H_SHRINK_BYTES,   /* sum of |F - F_prev| over shrink samples */
    SMP_H_LEAK_MALLOCS,   /* leak score: objects tracked at this line */
    SMP_H_LEAK_FREES,     /* leak score: tracked objects found reclaimed */
    SMP_H_COPY_SAMPLED,   /* copy volume: Tc per copy sample */
    SMP_H_COPY_EXACT,     /* copy volume: exact bytes copied */
    SMP_H_PY_TIME,        /* q per timer event (microseconds) */
    SMP_H_NAT_TIME,       /* delay per timer event (microseconds) */
    SMP_H_COUNT
};

/* leak likelihood order inside smp_profile_t.leak (num_lines entries each):
 * reduced rationals num/den with den > 0 (0/0 for lines with no tracked object)
 *   Laplace's rule of succession, frees as successes: 1-(f+1)/(m+2)
 *   the formula as printed in the paper:             1-(f+1)/(m-f+2)   */
enum { SMP_L_LAP_NUM = 0, SMP_L_LAP_DEN, SMP_L_LIT_NUM, SMP_L_LIT_DEN, SMP_L_COUNT };
/* report gates inside smp_profile_t.gates: likelihood > 95 % (section 3.4) */
enum { SMP_G_LAP = 0, SMP_G_LIT, SMP_G_COUNT };

typedef struct {
    uint64_t n_samples;
    uint64_t n_tracked;
    uint32_t num_lines;
    int32_t status;    /* SMP_OK, SMP_EINVAL (malformed event) or SMP_EOVERFLOW */
} smp_profile_sizes_t;

/* caller-owned host buffers, sized from smp_profile_sizes_t; any array
 * pointer may be NULL to skip it */
typedef struct {
    smp_sample_t *samples;   /* n_samples */
    smp_tracked_t *tracked;  /* n_tracked */
    int64_t *hist;           /* SMP_H_COUNT * num_lines */
    int64_t *leak;           /* SMP_L_COUNT * num_lines */
    uint8_t *gates;          /* SMP_G_COUNT * num_lines */
    /* filled scalars */
    int64_t final_F;         /* footprint after the last event */
    int64_t peak_F;          /* max(0, max footprint over all events) */
    int64_t peak_sampled_F;  /* max(0, max footprint over samples) */
    int64_t threshold_used;  /* T, or the prime chosen by SMP_OPT_PRIME_T */
    uint64_t n_samples;
    uint64_t n_tracked;
    int32_t status;
    int32_t reserved;
} smp_profile_t;

typedef struct smp_sampler smp_sampler_t; /* opaque, owned by the library */

/* Device bytes one trace of n_events needs inside the workspace (exact; the
 * admission rule of submit_trace).  ev_on_device != 1 adds room for a device
 * copy of the events.  Returns 0 for invalid params. */
SMP_API uint64_t workspace_bytes(uint64_t n_events, const smp_params_t *params, int ev_on_device);

/* Create a sampler on HIP device `device` that launches on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream) and carves all its device
 * state out of `workspace` (device, caller-owned, at least 256-byte aligned,
 * `workspace_size` bytes; it must outlive the sampler).  mem_budget caps the
 * bytes admitted traces may hold at once (0 = the whole workspace minus the
 * sampler's fixed part).  On success *out receives the sampler. */
SMP_API int sampler_create(int device, void *hip_stream, uint64_t mem_budget, void *workspace,
                           uint64_t workspace_size, smp_sampler_t **out);

/* Admit one trace.  ev: n events.  ev_on_device = 0: host memory, copied
 * into the workspace before this returns (the buffer may be reused at once);
 * 1: device memory, borrowed (must stay valid and unchanged until the trace's
 * fetch_profile); 2: pinned host memory (hipHostMalloc), copied asynchronously
 * on the caller's stream (must stay unchanged until the trace's
 * fetch_profile).  n < 2^32 - 1.  Returns
 * SMP_ETOOBIG if workspace_bytes(n) exceeds the budget, SMP_EBUDGET if it does
 * not fit now.  *trace_id receives a handle.  The trace waits for run(). */
SMP_API int submit_trace(smp_sampler_t *s, const smp_event_t *ev, uint64_t n, const smp_params_t *params,
                         int ev_on_device, uint64_t *trace_id);

/* Admit count traces with one call (a batch of many small traces): as
 * submit_trace(s, ev[i], n[i], &params[i], ev_on_device, &trace_ids[i]) for
 * i in order, stopping at the first one refused.  *submitted receives how
 * many were admitted (their ids are trace_ids[0 .. *submitted-1]); the
 * return value is SMP_OK when all were, else the refused trace's code. */
SMP_API int submit_traces(smp_sampler_t *s, uint32_t count, const smp_event_t *const *ev, const uint64_t *n,
                          const smp_params_t *params, int ev_on_device, uint64_t *trace_ids, uint32_t *submitted);

/* Launch every submitted, not yet launched trace as one batch (each pass of
 * the launch sequence covers the segments of all of them).  Launches
 * alternate between the sampler's two internal streams, each ordered after
 * all work queued so far on the caller's stream, so two consecutive batches
 * may overlap on the device (a third queues behind the first).
 * blocking = 1 waits for completion. */
SMP_API int run(smp_sampler_t *s, int blocking);

/* SMP_OK if the trace's batch finished, SMP_EAGAIN if still running,
 * SMP_ESTATE for unknown or not launched ids. */
SMP_API int poll(smp_sampler_t *s, uint64_t trace_id);

/* Two-call fetch.  With out == NULL: waits for the trace, fills *sizes.
 * With out != NULL: copies the profile into the caller's host buffers (sized
 * from *sizes), fills the scalars, releases the trace's workspace and
 * invalidates trace_id.  The returned status is the call's; the trace's own
 * status (SMP_OK / SMP_EINVAL / SMP_EOVERFLOW) is in sizes->status and
 * out->status. */
SMP_API int fetch_profile(smp_sampler_t *s, uint64_t trace_id, smp_profile_sizes_t *sizes, smp_profile_t *out);

/* Release count launched traces without copying their profiles out, with
 * one call: as fetch_profile with no output buffers for each, in order.
 * n_samples[i] and status[i] (either may be NULL) receive each trace's
 * sample count and own status.  Stops at the first call that fails (an id
 * that is not a launched trace: SMP_ESTATE; a device error: SMP_EDEVICE) and
 * returns its code; *released receives how many were released. */
SMP_API int release_traces(smp_sampler_t *s, uint32_t count, const uint64_t *trace_ids, uint64_t *n_samples,
                           int32_t *status, uint32_t *released);

/* Device pointers of a finished trace's results, for callers that keep them
 * on the GPU (valid until fetch_profile releases the trace).  Any out pointer
 * may be NULL. */
SMP_API int trace_device_results(smp_sampler_t *s, uint64_t trace_id, void **samples, void **hist,
                                 uint64_t *n_samples);

/* Timing of the last run() (milliseconds, HIP events on the launch's
 * stream): the five sampling passes together (summarize, resolve, chain,
 * scan, emit; -1 unless the events before the first and after the last pass
 * are recorded, see sampler_set_pass_events), and the whole launch sequence
 * including clearing, the tracked-list compaction and the leak rationals
 * (-1 unless the start event is recorded). */
SMP_API int sampler_last_timing(smp_sampler_t *s, float *main_kernel_ms, float *total_ms);

/* Which timing events later runs record: bit p (0-4) = the event before
 * sampling pass p, bit 5 = the event after the last pass, bit 6 = the
 * launch's start event (total_ms of sampler_last_timing).  Default 0x7F
 * (all).  Each event between two kernels idles the GPU for a few
 * microseconds, so a timed loop may keep only the two around the pass it
 * measures (0x30: the emit pass).  Returns SMP_EINVAL for bits above 6. */
SMP_API int sampler_set_pass_events(smp_sampler_t *s, uint32_t mask);

/* Per-pass timing of the last run(): pass_ms[0..4] = summarize, resolve,
 * chain, scan, emit (milliseconds, HIP events around each kernel on the
 * launch's stream; -1 for a pass whose two events were not recorded).
 * pass_ms must hold 5 floats. */
SMP_API int sampler_last_pass_timing(smp_sampler_t *s, float *pass_ms);

/* Diagnostics: the 32 control words of the last launch (word 1: abort flag,
 * words 2 and 3: tiles taken by the resolve and scan passes, word 4:
 * segments the chain pass followed through their records (the resolve pass
 * finishes the others), word 5: tiles given a tile map, word 6: tiles whose
 * exit was chained through tile maps before the resolve pass, words 7-10:
 * tiles of traces with tile maps that got none because a segment moves T or
 * more (or is not followed by chains), or because the tile needs more source
 * intervals, live chains or runs than a map holds; the other words are 0). */
SMP_API int sampler_last_counters(smp_sampler_t *s, uint64_t *out32);

/* Launch parameters of later runs.  None changes any result (every
 * choice computes the same profile); they trade work between passes:
 *   chain_cap  : distinct chains the summary pass follows through a segment
 *                before it gives up and leaves the segment to be followed
 *                from its actual entry (1..64, default 16)
 *   chain_grid : workgroups of the chain pass (0 = as many as the device
 *                holds at once, the default)
 *   emit_grid  : workgroups of the emit pass (0 = the same default)
 *   graphs     : 1 (default) = a run slot replays a launch sequence whose
 *                shape (trace count, segment, tile, block and line totals,
 *                grids, timing events) it launched before as a HIP graph,
 *                captured on the second launch of that shape; launches that
 *                record timing events between passes (sampler_set_pass_events
 *                bits 0-5) are always plain; 0 = plain launches only
 *   tile_map_tiles : traces of at least this many tiles (of 512 segments of
 *                512 events) get tile maps: for every tile whose segments
 *                each move the footprint by less than T, its chain map over
 *                all entries (section 3.2), built for all tiles at once
 *                before the resolve pass, so that tile entries follow by one
 *                lookup per tile instead of a walk per tile (0 = the default,
 *                64; 0xFFFFFFFF = never)
 * sampler_set_tuning returns SMP_EINVAL for values out of range;
 * sampler_get_tuning reports the current ones with the defaults resolved. */
typedef struct {
    uint32_t chain_cap;
    uint32_t chain_grid;
    uint32_t emit_grid;
    uint32_t graphs;
    uint32_t tile_map_tiles;
} smp_tuning_t;
SMP_API int sampler_set_tuning(smp_sampler_t *s, const smp_tuning_t *t);
SMP_API int sampler_get_tuning(smp_sampler_t *s, smp_tuning_t *t);

/* Launch counts since the sampler was created: out3[0] launch sequences
 * issued plainly, out3[1] graphs captured, out3[2] graph replays (a capture
 * is followed by its first replay). */
SMP_API int sampler_launch_stats(smp_sampler_t *s, uint64_t *out3);

/* Bytes of the workspace the sampler keeps for itself (descriptor tables,
 * counters); the rest is the trace budget. */
SMP_API uint64_t sampler_fixed_bytes(void);

SMP_API void sampler_destroy(smp_sampler_t *s);

/* Static string for a status code. */
SMP_API const char *error_string(int status);

/* ---- rate-based sampling (section 3.2) --------------------------------
 * The scheme threshold sampling is compared with: every byte allocated or
 * freed counts towards the next sample, one sample per T bytes, whatever the
 * bytes do to the footprint.  Read deterministically (the countdown starts at
 * T, not at a random draw): memory event i takes
 * floor(V_i / T) - floor(V_(i-1) / T) samples, V the cumulative bytes
 * allocated plus bytes freed by memory events, attributed to the event's
 * line.  Copy and timer events add nothing.  Independent of a sampler
 * object: the caller owns every buffer and the stream. */

/* Device workspace bytes rate_run needs for a trace of n_events events
 * (256 bytes plus 8 per 512 events). */
SMP_API uint64_t rate_workspace_bytes(uint64_t n_events);

/* Rate-based sampling of one trace, asynchronous on hip_stream (a
 * hipStream_t; NULL = the null stream).
 *   ev          : device pointer to n records (layout smp_event_t), read only
 *   n           : < 2^32 events (0 allowed)
 *   threshold   : T, 1 <= T < 2^60, used as given
 *   num_lines   : L >= 1; every record's line must be < L
 *   workspace   : device scratch of at least rate_workspace_bytes(n) bytes,
 *                 owned by the caller, contents not preserved
 *   line_counts : device array of L int64, written: samples per line
 *   result      : device array of 2 uint64, written: [0] = K, the total
 *                 number of samples; [1] = SMP_OK, SMP_EINVAL (a malformed
 *                 record, as fetch_profile reports it) or SMP_EOVERFLOW (V
 *                 reaches 2^62); counts are meaningful only with SMP_OK
 * Returns SMP_EINVAL for invalid arguments (nothing launched), SMP_EDEVICE
 * if a launch failed, else SMP_OK; the results are complete when the stream
 * reaches them.  Concurrent calls must use separate workspaces. */
SMP_API int rate_run(const smp_event_t *ev, uint64_t n, int64_t threshold, uint32_t num_lines, void *workspace,
                     uint64_t workspace_bytes, int64_t *line_counts, uint64_t *result, void *hip_stream);

/* ---- rate-based sampling without allocation ----------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rate_run
 * with its scratch in a device array inside the library instead of a
 * workspace argument.  The library holds one such array of
 * 256 + 8 * (SMP_RATE_NOALLOC_MAX_EVENTS / 512) bytes (8 MiB + 256 B) on
 * each GPU it runs on, until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and clears what
 * must start at zero with a kernel.  Every call on one GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be
 * serialised by the caller.  The array's device address is looked up on a
 * device's first call, with that device current.
 * Arguments, results and errors as rate_run, with n <= SMP_RATE_NOALLOC_MAX_EVENTS;
 * a larger n returns SMP_ETOOBIG and launches nothing. */
#define SMP_RATE_NOALLOC_MAX_EVENTS (1ull << 29)
SMP_API int rate_run_noalloc(const smp_event_t *ev, uint64_t n, int64_t threshold, uint32_t num_lines,
                             int64_t *line_counts, uint64_t *result, void *hip_stream);

/* ---- report line filter (section 5) -----------------------------------
 * The lines a profile shows: those with at least 1 % of the execution time
 * or at least 1 % of the memory, each with the line before and the line
 * after it.  Readings: a line's time is py_time_us + nat_time_us (timer
 * samples), its memory growth_bytes (bytes of its growth samples), both as
 * fetch_profile returns them; "at least 1 %" is 100 x >= the total of the
 * lines' positive values (a line with x <= 0 never qualifies; a zero total
 * selects nothing); neighbours are the ids one below and one above, inside
 * [0, num_lines).  The paper bounds a profile at 300 lines: at most 100
 * lines can hold 1 % of one total, but the two criteria together can admit
 * 200, so when more than 100 qualify the 100 with the largest share stay (a
 * line's share: the larger of its time share and its memory share, compared
 * exactly; equal shares keep the lower id) before neighbours are added.
 *   py_time_us, nat_time_us, growth_bytes : host arrays of num_lines values
 *   out_lines : host array with room for num_lines ids, written in
 *               increasing order; *n_out receives their number
 * Host-only; returns SMP_EINVAL for missing pointers, else SMP_OK. */
SMP_API int report_lines(const int64_t *py_time_us, const int64_t *nat_time_us, const int64_t *growth_bytes,
                         uint32_t num_lines, uint32_t *out_lines, uint32_t *n_out);

/* ---- leak report filter (section 3.4) ---------------------------------
 * Leaks are reported only when their likelihood passes its gate and overall
 * memory grows by at least 1 %.  Reading of the growth test: the
 * least-squares line of the sampled footprint F against the event index
 * over the K samples passes when its rise over the sampled span is at least
 * 1 % of the peak sampled footprint, 100 b (x_K - x_1) >= max F with
 * b = (K Sxy - Sx Sy) / (K Sxx - Sx^2), decided exactly (K < 2 or a peak
 * <= 0 never passes).  The leak rate of a line (bytes allocated at it per
 * elapsed time; bytes per microsecond is MB/s) divides its growth_bytes by
 * *elapsed_us, the trace's total Python plus native time.
 *   samples, n_samples : the profile's samples in rank order (host)
 *   gate               : num_lines report gates (SMP_G_LAP or SMP_G_LIT row)
 *   py_time_us, nat_time_us : num_lines values (host)
 *   slope_ok  : out, 1 if the growth test passes
 *   reported  : out, num_lines flags: gate and growth test
 *   elapsed_us: out, the sum of py_time_us + nat_time_us modulo 2^64
 * Host-only; returns SMP_EINVAL for missing pointers or n_samples >= 2^32. */
SMP_API int leak_report(const smp_sample_t *samples, uint64_t n_samples, const uint8_t *gate,
                        const int64_t *py_time_us, const int64_t *nat_time_us, uint32_t num_lines,
                        int32_t *slope_ok, uint8_t *reported, int64_t *elapsed_us);

/* ---- per-line memory timelines (section 5) ----------------------------
 * Each line's footprint log (its samples in rank order, as points (event
 * index, footprint)) reduced by Ramer-Douglas-Peucker to at most max_points
 * points (the paper uses 100).  A point is kept when its distance from the
 * chord of its run exceeds eps, decided exactly (cross^2 > eps^2 len^2); the
 * farthest point of a run, the first on ties, splits it; eps is the smallest
 * of {0, 1, 2, 4, ..., 2^62} that leaves at most max_points points, so the
 * random downsampling the paper applies after an approximate eps is never
 * needed.  Samples whose line is >= num_lines belong to no timeline.
 *   samples, n_samples : the profile's samples in rank order (host)
 *   max_points         : >= 2
 *   keep               : out, n_samples flags: 1 = the sample is a point of
 *                        its line's reduced timeline
 * Host-only; returns SMP_EINVAL for missing pointers, max_points < 2 or
 * n_samples >= 2^32. */
SMP_API int timeline_points(const smp_sample_t *samples, uint64_t n_samples, uint32_t num_lines,
                            uint32_t max_points, uint8_t *keep);

/* The same timelines by the paper's own procedure (section 5): RDP with an
 * approximate eps, the line's footprint range over max_points (integer
 * division), then every log still longer than max_points randomly
 * downsampled to exactly max_points of its RDP points.  The subset is a
 * uniform one drawn by selection sampling (Knuth, TAOCP vol. 2, 3.4.2,
 * Algorithm S): with m of k = max_points chosen, the t-th of the N RDP points
 * is chosen when floor(x (N - t) / 2^64) < k - m, x the next output of
 * splitmix64 (Steele, Lea and Flood, 2014) started at state seed + line
 * (modulo 2^64), so a seed fixes the result.  Arguments and errors as
 * timeline_points. */
SMP_API int timeline_points_sampled(const smp_sample_t *samples, uint64_t n_samples, uint32_t num_lines,
                                    uint32_t max_points, uint64_t seed, uint8_t *keep);

#ifdef __cplusplus
}
#endif

#endif
