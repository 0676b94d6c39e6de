// Host side of the C ABI: workspace arena, trace admission, batch launch,
// completion tracking and result copy-out.  Every computation on trace data
// runs in the kernels of sampler_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "sampler_device.h"
#include "scalene_sampler.h"

namespace smp {
int chain_grid_limit();
int emit_grid_limit();
int track_grid_limit();
hipError_t launch_clear(const Desc* desc, int ntraces, uint64_t total_bytes, unsigned long long* ctl, hipStream_t s);
hipError_t launch_pass(int pass, const Desc* desc, int ntraces, uint64_t nseg_total, uint64_t ntile_total,
                       unsigned long long* ctl, int grid_limit, hipStream_t s);
hipError_t launch_finish(const Desc* desc, int ntraces, uint64_t nblk_total, uint64_t total_lines,
                         unsigned long long* ctl, int track_grid, Scalars* gather, hipStream_t s);
hipError_t launch_tmap(const Desc* desc, int ntraces, uint64_t ntile_total, unsigned long long* ctl, hipStream_t s);
}  // namespace smp

using namespace smp;

static_assert(sizeof(smp_event_t) == 24, "event record layout");
static_assert(sizeof(smp_sample_t) == sizeof(Sample), "sample layout");
static_assert(sizeof(smp_tracked_t) == sizeof(Tracked), "tracked layout");
static_assert(sizeof(Scalars) == 64, "scalars are gathered as 8 words");

namespace {

constexpr uint64_t ALIGN = 256;
constexpr int RUN_SLOTS = 8;
// Launches alternate between two streams created together, so that two
// launches in flight sit on two hardware queues and overlap on the device.
// The runtime spreads streams over a small pool of hardware queues (four by
// default); with a stream per run slot, two slots' streams could share a
// queue, and launches on one queue never overlap.
constexpr int LAUNCH_STREAMS = 2;
constexpr int MAX_TRACES_PER_RUN = 4096;
constexpr uint64_t CBLK_WORDS = 256;
constexpr int NPASS = 5;  // summarize, resolve, chain, scan, emit
constexpr uint32_t TILE_MAP_TILES_DEFAULT = 64;  // traces of at least this many tiles get tile maps

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ---- deterministic Miller-Rabin for 64-bit integers ----
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }
uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}
bool is_prime_mr(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : small) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : small) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

// Byte layout of one trace's region in the workspace.
struct Layout {
    uint64_t nseg, ntile, words, nblk;
    uint64_t ev, samples, sample_ptr, tracked, seg, mask;  // offsets
    uint64_t zero, tstat, tracked_bits, freed_bits, hist, leak, gates, scal, blk, zero_end;
    uint64_t total;
};

Layout make_layout(uint64_t n, uint32_t L, bool ev_copy) {
    Layout y{};
    y.nseg = (n + SEG - 1) / SEG;
    y.ntile = (y.nseg + TILE - 1) / TILE;
    y.words = (n + 1 + 63) / 64;
    y.nblk = (y.words + CBLK_WORDS - 1) / CBLK_WORDS;
    uint64_t o = 0;
    y.ev = o;
    if (ev_copy) o = align_up(o + 24 * n, ALIGN);
    y.samples = o;
    o = align_up(o + sizeof(Sample) * (n + 1), ALIGN);
    y.sample_ptr = o;
    o = align_up(o + 4 * (n + 1), ALIGN);
    y.tracked = o;
    o = align_up(o + sizeof(Tracked) * (n + 1), ALIGN);
    y.seg = o;
    o = align_up(o + 8 * (uint64_t)NSPLANE * y.nseg, ALIGN);
    y.mask = o;
    o = align_up(o + 8 * (uint64_t)NW * y.nseg, ALIGN);
    y.zero = o;
    y.tstat = o;
    o += 8 * (uint64_t)NWORD * y.ntile;
    y.tracked_bits = o;
    o += 8 * y.words;
    y.freed_bits = o;
    o += 8 * y.words;
    y.hist = o;
    o += 8 * (uint64_t)H_COUNT * L;
    y.leak = o;
    o += 8 * 4 * (uint64_t)L;
    y.gates = o;
    o = align_up(o + 2 * (uint64_t)L, 8);
    y.scal = o;
    o += sizeof(Scalars);
    y.blk = o;
    o += 8 * y.nblk;
    o = align_up(o, ALIGN);
    y.zero_end = o;
    y.total = o;
    return y;
}

bool params_ok(const smp_params_t* p) {
    return p && p->threshold >= 1 && p->threshold < ((int64_t)1 << 60) && p->copy_threshold >= 1 && p->num_lines >= 1 &&
           p->num_lines <= (1u << 31) && p->reserved == 0 && (p->options & ~3u) == 0;
}

enum TraceState { PENDING = 0, LAUNCHED = 1 };

struct TraceRec {
    uint64_t id = 0;
    int state = PENDING;
    uint64_t n = 0;
    smp_params_t params{};
    int64_t T_used = 0;
    uint64_t off = 0, bytes = 0;
    Layout lay{};
    const uint8_t* ev = nullptr;
    int slot = -1;
    uint64_t run_seq = 0;
    bool have_scal = false;  // scalars copied to the host when its launch retired
    Scalars scal{};
};

// Timing events: bit p (0-4) the event before pass p, bit 5 the event after
// the last pass, bit 6 the launch's start event.
constexpr uint32_t PASS_EVENTS_ALL = 0x7F;
constexpr int START_EVENT_BIT = NPASS + 1;
constexpr uint32_t PASS_EVENT_BITS = (1u << (NPASS + 1)) - 1;  // the events between passes

// Shape of one launch sequence: everything its kernel arguments and grids
// depend on besides the slot's own buffers.
struct LaunchKey {
    uint64_t cnt, seg, tile, blk, zero, lines, ev_mask, chain_grid, emit_grid, track_grid, tmap;
    bool operator==(const LaunchKey& o) const { return memcmp(this, &o, sizeof(LaunchKey)) == 0; }
};

struct RunSlot {
    Desc* host_desc = nullptr;   // pinned staging
    Desc* dev_desc = nullptr;
    Desc* last_desc = nullptr;   // what dev_desc holds (host copy), to skip an unchanged upload
    size_t last_cnt = 0;
    // every trace's scalars, gathered by the last kernel of the launch straight
    // into pinned, coherent host memory (no copy in the launch sequence)
    Scalars* host_scal = nullptr;
    Scalars* host_scal_dev = nullptr;  // its device address
    std::vector<uint64_t> ids;     // the launch's traces, in descriptor order
    unsigned long long* dev_ticket = nullptr;
    hipStream_t stream = nullptr;  // the slot's current launch (one of the sampler's launch streams)
    hipEvent_t e_ready = nullptr;  // recorded on the caller's stream at run()
    hipEvent_t e_start = nullptr, e_end = nullptr;
    hipEvent_t e_pass[NPASS + 1] = {};  // around each pass of the sampling kernels
    uint32_t ev_mask = 0;               // which e_pass events this launch recorded
    bool busy = false;
    uint64_t seq = 0;
    LaunchKey last_key{};               // shape of the slot's previous launch
    bool last_valid = false;
    hipGraphExec_t gexec = nullptr;     // the captured launch sequence of shape gkey
    LaunchKey gkey{};
    bool gkey_valid = false;
};

}  // namespace

struct smp_sampler {
    int device = 0;
    hipStream_t stream = nullptr;
    uint8_t* ws = nullptr;
    uint64_t ws_size = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    uint64_t arena_base = 0;  // offset of the trace arena inside the workspace
    std::map<uint64_t, uint64_t> free_list;  // offset -> size
    std::map<uint64_t, TraceRec> traces;
    RunSlot slots[RUN_SLOTS];
    hipStream_t streams[LAUNCH_STREAMS] = {};  // launches, ordered after the caller's stream
    int next_stream = 0;
    uint64_t next_id = 1;
    uint64_t run_seq = 0;
    int grid_chain = 0, grid_emit = 0, grid_track = 0;
    bool failed = false;
    float last_main_ms = 0, last_total_ms = 0;
    float last_pass_ms[NPASS] = {};
    uint32_t pass_events = PASS_EVENTS_ALL;  // timing events to record (all by default)
    smp_tuning_t tuning{16, 0, 0, 1, 0};
    bool graphs_ok = true;                   // off after a failed capture
    uint64_t n_plain = 0, n_captured = 0, n_replayed = 0;
    uint64_t last_seq = 0;
};

namespace {

// Per run slot: descriptors, 32 control words, gathered scalars.
uint64_t slot_bytes() { return align_up(sizeof(Desc) * MAX_TRACES_PER_RUN, ALIGN) + ALIGN; }

uint64_t fixed_bytes() { return align_up((uint64_t)RUN_SLOTS * slot_bytes(), ALIGN); }

bool arena_alloc(smp_sampler* s, uint64_t bytes, uint64_t* off) {
    for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t noff = it->first + bytes;
            s->free_list.erase(it);
            if (rest) s->free_list[noff] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(smp_sampler* s, uint64_t off, uint64_t bytes) {
    auto it = s->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_list.erase(nx);
    }
    if (it != s->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_list.erase(it);
        }
    }
}

int fail(smp_sampler* s) {
    s->failed = true;
    return SMP_EDEVICE;
}

// Whether a trace gets tile maps: long enough (the maps are built for all
// tiles at once, in about the time a few tiles take to walk one after
// another) and with room for them in its tracked-list area.
bool wants_tile_maps(const smp_sampler* s, const TraceRec& t) {
    const uint64_t min_tiles = s->tuning.tile_map_tiles ? s->tuning.tile_map_tiles : TILE_MAP_TILES_DEFAULT;
    return t.lay.ntile >= min_tiles && t.lay.ntile > 1 &&
           sizeof(Tracked) * (t.n + 1) >= t.lay.ntile * TILE_MAP_BYTES;
}

#define HIPCHK(expr)                          \
    do {                                      \
        if ((expr) != hipSuccess) return fail(s); \
    } while (0)

// Wait for a slot's launch to finish and record its timing.
int retire_slot(smp_sampler* s, RunSlot& r) {
    if (!r.busy) return SMP_OK;
    HIPCHK(hipEventSynchronize(r.e_end));
    // intervals whose two events were not recorded read -1
    float a = -1, b = -1, p[NPASS];
    const uint32_t m = r.ev_mask;
    if ((m & 1u) && ((m >> NPASS) & 1u)) HIPCHK(hipEventElapsedTime(&a, r.e_pass[0], r.e_pass[NPASS]));
    if ((m >> START_EVENT_BIT) & 1u) HIPCHK(hipEventElapsedTime(&b, r.e_start, r.e_end));
    for (int i = 0; i < NPASS; ++i) {
        p[i] = -1;
        if (((m >> i) & 1u) && ((m >> (i + 1)) & 1u)) HIPCHK(hipEventElapsedTime(&p[i], r.e_pass[i], r.e_pass[i + 1]));
    }
    if (r.seq >= s->last_seq) {
        s->last_seq = r.seq;
        s->last_main_ms = a;
        s->last_total_ms = b;
        for (int i = 0; i < NPASS; ++i) s->last_pass_ms[i] = p[i];
    }
    for (size_t k = 0; k < r.ids.size(); ++k) {
        auto it = s->traces.find(r.ids[k]);
        if (it != s->traces.end() && it->second.run_seq == r.seq) {
            it->second.scal = r.host_scal[k];
            it->second.have_scal = true;
        }
    }
    r.busy = false;
    return SMP_OK;
}

}  // namespace

extern "C" {

uint64_t sampler_fixed_bytes(void) { return fixed_bytes(); }

uint64_t workspace_bytes(uint64_t n_events, const smp_params_t* params, int ev_on_device) {
    if (!params_ok(params) || n_events >= 0xFFFFFFFFull) return 0;
    return make_layout(n_events, params->num_lines, ev_on_device == 0).total;
}

const char* error_string(int status) {
    switch (status) {
        case SMP_OK: return "ok";
        case SMP_EINVAL: return "invalid argument or malformed event";
        case SMP_EBUDGET: return "not enough free workspace budget now";
        case SMP_ETOOBIG: return "trace exceeds the whole workspace budget";
        case SMP_EAGAIN: return "trace not finished";
        case SMP_EDEVICE: return "HIP device error; destroy the sampler";
        case SMP_EOVERFLOW: return "footprint, Python footprint or copy prefix outside (-2^61, 2^61)";
        case SMP_ENOMEM: return "host allocation failed";
        case SMP_ESTATE: return "unknown trace id or wrong trace state";
        default: return "unknown status";
    }
}

int sampler_create(int device, void* hip_stream, uint64_t mem_budget, void* workspace, uint64_t workspace_size,
                   smp_sampler_t** out) {
    if (!out) return SMP_EINVAL;
    *out = nullptr;
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return SMP_EINVAL;
    const uint64_t fixed = fixed_bytes();
    if (workspace_size < fixed + ALIGN) return SMP_EINVAL;
    smp_sampler* s = new (std::nothrow) smp_sampler();
    if (!s) return SMP_ENOMEM;
    s->device = device;
    s->stream = (hipStream_t)hip_stream;
    s->ws = (uint8_t*)workspace;
    s->ws_size = workspace_size;
    s->arena_base = fixed;
    const uint64_t arena = (workspace_size - fixed) / ALIGN * ALIGN;
    s->budget = mem_budget == 0 || mem_budget > arena ? arena : mem_budget;
    s->free_list[fixed] = arena;
    if (hipSetDevice(device) != hipSuccess) {
        delete s;
        return SMP_EDEVICE;
    }
    for (auto& st : s->streams) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            st = nullptr;
            sampler_destroy(s);
            return SMP_EDEVICE;
        }
    }
    for (int i = 0; i < RUN_SLOTS; ++i) {
        RunSlot& r = s->slots[i];
        uint8_t* base = s->ws + i * slot_bytes();
        r.dev_desc = (Desc*)base;
        r.dev_ticket = (unsigned long long*)(base + align_up(sizeof(Desc) * MAX_TRACES_PER_RUN, ALIGN));
        if (hipHostMalloc((void**)&r.host_desc, sizeof(Desc) * MAX_TRACES_PER_RUN, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&r.host_scal, sizeof(Scalars) * MAX_TRACES_PER_RUN, hipHostMallocCoherent) !=
                hipSuccess ||
            hipHostGetDevicePointer((void**)&r.host_scal_dev, r.host_scal, 0) != hipSuccess ||
            hipEventCreateWithFlags(&r.e_ready, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&r.e_start) != hipSuccess || hipEventCreate(&r.e_end) != hipSuccess ||
            !(r.last_desc = new (std::nothrow) Desc[MAX_TRACES_PER_RUN])) {
            sampler_destroy(s);
            return SMP_EDEVICE;
        }
        for (auto& e : r.e_pass) {
            if (hipEventCreate(&e) != hipSuccess) {
                sampler_destroy(s);
                return SMP_EDEVICE;
            }
        }
    }
    s->grid_chain = chain_grid_limit();
    s->grid_emit = emit_grid_limit();
    s->grid_track = track_grid_limit();
    if (s->grid_chain <= 0 || s->grid_emit <= 0 || s->grid_track <= 0) {
        sampler_destroy(s);
        return SMP_EDEVICE;
    }
    *out = s;
    return SMP_OK;
}

void sampler_destroy(smp_sampler_t* s) {
    if (!s) return;
    if (!s->failed) {
        for (auto& r : s->slots)
            if (r.busy && r.e_end) (void)hipEventSynchronize(r.e_end);
    }
    for (auto& r : s->slots) {
        if (r.host_desc) (void)hipHostFree(r.host_desc);
        delete[] r.last_desc;
        r.last_desc = nullptr;
        if (r.host_scal) (void)hipHostFree(r.host_scal);
        if (r.e_ready) (void)hipEventDestroy(r.e_ready);
        if (r.e_start) (void)hipEventDestroy(r.e_start);
        for (auto& e : r.e_pass)
            if (e) (void)hipEventDestroy(e);
        if (r.e_end) (void)hipEventDestroy(r.e_end);
        if (r.gexec) (void)hipGraphExecDestroy(r.gexec);
    }
    for (auto& st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    delete s;
}

int submit_trace(smp_sampler_t* s, const smp_event_t* ev, uint64_t n, const smp_params_t* params, int ev_on_device,
                 uint64_t* trace_id) {
    if (!s || !trace_id || !params_ok(params) || n >= 0xFFFFFFFFull || (n && !ev)) return SMP_EINVAL;
    if (s->failed) return SMP_EDEVICE;
    if (ev_on_device < 0 || ev_on_device > 2) return SMP_EINVAL;
    const bool copy = ev_on_device != 1;
    const Layout lay = make_layout(n, params->num_lines, copy);
    if (lay.total > s->budget) return SMP_ETOOBIG;
    if (s->used + lay.total > s->budget) return SMP_EBUDGET;
    uint64_t off = 0;
    if (!arena_alloc(s, lay.total, &off)) return SMP_EBUDGET;
    TraceRec t;
    t.id = s->next_id++;
    t.n = n;
    t.params = *params;
    t.T_used = params->threshold;
    if (params->options & SMP_OPT_PRIME_T) {
        uint64_t v = (uint64_t)params->threshold;
        while (!is_prime_mr(v)) ++v;
        t.T_used = (int64_t)v;
    }
    t.off = off;
    t.bytes = lay.total;
    t.lay = lay;
    if (copy) {
        t.ev = s->ws + off + lay.ev;
        if (n) {
            // mode 0: pageable source, wait for the copy; mode 2: pinned source, leave it queued
            if (hipSetDevice(s->device) != hipSuccess ||
                hipMemcpyAsync((void*)t.ev, ev, 24 * n, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
                (ev_on_device == 0 && hipStreamSynchronize(s->stream) != hipSuccess)) {
                arena_free(s, off, lay.total);
                return fail(s);
            }
        }
    } else {
        t.ev = (const uint8_t*)ev;
    }
    s->used += lay.total;
    *trace_id = t.id;
    s->traces.emplace(t.id, t);
    return SMP_OK;
}

// The kernels of one launch, in stream order on r.stream, with the timing
// events between passes that k asks for (captured into a graph when called
// between hipStreamBeginCapture and hipStreamEndCapture, which is done only
// for launches without such events).
static hipError_t issue_launch(RunSlot& r, const LaunchKey& k) {
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
        return e == hipSuccess;
    };
    auto record = [&](hipEvent_t ev) { return hipEventRecord(ev, r.stream); };
    const int cnt = (int)k.cnt;
    if (!ok(launch_clear(r.dev_desc, cnt, k.zero, r.dev_ticket, r.stream))) return e;
    for (int p = 0; p < NPASS; ++p) {
        if ((k.ev_mask >> p) & 1u && !ok(record(r.e_pass[p]))) return e;
        const int lim = p == 2 ? (int)k.chain_grid : (int)k.emit_grid;
        if (p == 1 && k.tmap && !ok(launch_tmap(r.dev_desc, cnt, k.tile, r.dev_ticket, r.stream))) return e;
        if (!ok(launch_pass(p, r.dev_desc, cnt, k.seg, k.tile, r.dev_ticket, lim, r.stream))) return e;
    }
    if ((k.ev_mask >> NPASS) & 1u && !ok(record(r.e_pass[NPASS]))) return e;
    ok(launch_finish(r.dev_desc, cnt, k.blk, k.lines, r.dev_ticket, (int)k.track_grid, r.host_scal_dev, r.stream));
    return e;
}

// Capture the launch sequence of key k into the slot's graph (updating the
// instantiated graph in place when it allows).  On any failure graphs are
// switched off for the sampler and the caller launches plainly.
static bool capture_graph(smp_sampler* s, RunSlot& r, const LaunchKey& k) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(r.stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        s->graphs_ok = false;
        return false;
    }
    const hipError_t ei = issue_launch(r, k);
    const hipError_t ee = hipStreamEndCapture(r.stream, &g);
    bool ok = ei == hipSuccess && ee == hipSuccess && g != nullptr;
    if (ok && r.gexec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(r.gexec, g, &err_node, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(r.gexec);
            r.gexec = nullptr;
        }
    }
    if (ok && !r.gexec) ok = hipGraphInstantiate(&r.gexec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        (void)hipGetLastError();
        if (r.gexec) (void)hipGraphExecDestroy(r.gexec);
        r.gexec = nullptr;
        r.gkey_valid = false;
        s->graphs_ok = false;
        return false;
    }
    r.gkey = k;
    r.gkey_valid = true;
    ++s->n_captured;
    return true;
}

int run(smp_sampler_t* s, int blocking) {
    if (!s) return SMP_EINVAL;
    if (s->failed) return SMP_EDEVICE;
    std::vector<TraceRec*> pend;
    for (auto& kv : s->traces)
        if (kv.second.state == PENDING) pend.push_back(&kv.second);
    if (pend.empty()) return SMP_OK;
    HIPCHK(hipSetDevice(s->device));
    size_t done = 0;
    while (done < pend.size()) {
        const size_t cnt = std::min<size_t>(MAX_TRACES_PER_RUN, pend.size() - done);
        // the launch's shape
        LaunchKey key{};
        key.cnt = cnt;
        for (size_t k = 0; k < cnt; ++k) {
            const TraceRec& t = *pend[done + k];
            key.seg += t.lay.nseg;
            key.tile += t.lay.ntile;
            key.blk += t.lay.nblk;
            key.zero += t.lay.zero_end - t.lay.zero;
            key.lines += t.params.num_lines;
            key.tmap += wants_tile_maps(s, t) ? 1 : 0;
        }
        key.ev_mask = s->pass_events;
        key.chain_grid = s->tuning.chain_grid ? s->tuning.chain_grid : (uint64_t)s->grid_chain;
        key.emit_grid = s->tuning.emit_grid ? s->tuning.emit_grid : (uint64_t)s->grid_emit;
        key.track_grid = (uint64_t)s->grid_track;
        // A free slot that launched this shape before (its graph or its
        // descriptors may be reused), else the free slot used longest ago,
        // else the busy slot launched longest ago (waited for below).
        int si = -1;
        for (int i = 0; i < RUN_SLOTS; ++i) {
            const RunSlot& c = s->slots[i];
            if (!c.busy && ((c.gkey_valid && c.gkey == key) || (c.last_valid && c.last_key == key)) &&
                (si < 0 || c.seq > s->slots[si].seq))
                si = i;
        }
        if (si < 0) {
            for (int i = 0; i < RUN_SLOTS; ++i)
                if (!s->slots[i].busy && (si < 0 || s->slots[i].seq < s->slots[si].seq)) si = i;
        }
        if (si < 0) {
            si = 0;
            for (int i = 1; i < RUN_SLOTS; ++i)
                if (s->slots[i].seq < s->slots[si].seq) si = i;
        }
        RunSlot& r = s->slots[si];
        if (int rc = retire_slot(s, r)) return rc;
        r.stream = s->streams[s->next_stream];
        s->next_stream = (s->next_stream + 1) % LAUNCH_STREAMS;
        uint64_t seg = 0, tile = 0, blk = 0, zero = 0, lines = 0;
        r.ids.clear();
        for (size_t k = 0; k < cnt; ++k) {
            TraceRec& t = *pend[done + k];
            Desc& D = r.host_desc[k];
            std::memset(&D, 0, sizeof(Desc));
            uint8_t* base = s->ws + t.off;
            D.ev = t.ev;
            D.n = t.n;
            D.T = t.T_used;
            D.Tc = t.params.copy_threshold;
            D.q = t.params.quantum_us;
            D.L = t.params.num_lines;
            D.options = t.params.options;
            D.tc_shift = -1;
            D.chain_cap = s->tuning.chain_cap;
            if ((D.Tc & (D.Tc - 1)) == 0) D.tc_shift = __builtin_ctzll((uint64_t)D.Tc);
            D.seg_begin = seg;
            D.nseg = t.lay.nseg;
            D.tile_begin = tile;
            D.ntile = t.lay.ntile;
            D.seg = (int64_t*)(base + t.lay.seg);
            D.mask = (uint64_t*)(base + t.lay.mask);
            D.tstat = (uint64_t*)(base + t.lay.tstat);
            D.samples = (Sample*)(base + t.lay.samples);
            D.sample_ptr = (uint32_t*)(base + t.lay.sample_ptr);
            D.tracked = (Tracked*)(base + t.lay.tracked);
            D.tracked_bits = (uint64_t*)(base + t.lay.tracked_bits);
            D.freed_bits = (uint64_t*)(base + t.lay.freed_bits);
            D.hist = (int64_t*)(base + t.lay.hist);
            D.leak = (int64_t*)(base + t.lay.leak);
            D.gates = base + t.lay.gates;
            D.scal = (Scalars*)(base + t.lay.scal);
            D.blk = (uint64_t*)(base + t.lay.blk);
            D.blk_begin = blk;
            D.nblk = t.lay.nblk;
            D.zero_ptr = base + t.lay.zero;
            D.zero_bytes = t.lay.zero_end - t.lay.zero;
            D.zero_begin = zero;
            D.line_begin = lines;
            D.tmap = wants_tile_maps(s, t) ? 1u : 0u;
            seg += D.nseg;
            tile += D.ntile;
            blk += D.nblk;
            zero += D.zero_bytes;
            lines += D.L;
            t.state = LAUNCHED;
            t.slot = si;
            t.have_scal = false;
            r.ids.push_back(t.id);
        }
        r.seq = ++s->run_seq;
        for (size_t k = 0; k < cnt; ++k) pend[done + k]->run_seq = r.seq;
        // everything the caller queued on its stream (event copies) comes first
        HIPCHK(hipEventRecord(r.e_ready, s->stream));
        HIPCHK(hipStreamWaitEvent(r.stream, r.e_ready, 0));
        // the slot's previous launch has retired, and kernels never write the
        // descriptors: an unchanged table need not be uploaded again
        if (r.last_cnt != cnt || memcmp(r.last_desc, r.host_desc, sizeof(Desc) * cnt) != 0) {
            HIPCHK(hipMemcpyAsync(r.dev_desc, r.host_desc, sizeof(Desc) * cnt, hipMemcpyHostToDevice, r.stream));
            memcpy(r.last_desc, r.host_desc, sizeof(Desc) * cnt);
            r.last_cnt = cnt;
        }
        // an event between two kernels costs a few microseconds of idle GPU
        r.ev_mask = s->pass_events;
        // A shape this slot launched before is replayed as a HIP graph (the
        // kernels read the descriptors uploaded above; no memset nodes: the
        // clearing is a kernel); a new shape, or a launch that records timing
        // events between its passes, is launched plainly.  The start and end
        // events are recorded outside the graph.
        if ((r.ev_mask >> START_EVENT_BIT) & 1u) HIPCHK(hipEventRecord(r.e_start, r.stream));
        bool graphed = false;
        if (s->tuning.graphs && s->graphs_ok && (key.ev_mask & PASS_EVENT_BITS) == 0) {
            if (r.gkey_valid && r.gkey == key)
                graphed = true;
            else if (r.last_valid && r.last_key == key)
                graphed = capture_graph(s, r, key);
        }
        if (graphed) {
            HIPCHK(hipGraphLaunch(r.gexec, r.stream));
            ++s->n_replayed;
        } else {
            HIPCHK(issue_launch(r, key));
            ++s->n_plain;
        }
        r.last_key = key;
        r.last_valid = true;
        HIPCHK(hipEventRecord(r.e_end, r.stream));
        r.busy = true;
        done += cnt;
    }
    if (blocking) {
        for (auto& r : s->slots)
            if (int rc = retire_slot(s, r)) return rc;
    }
    return SMP_OK;
}

int poll(smp_sampler_t* s, uint64_t trace_id) {
    if (!s) return SMP_EINVAL;
    auto it = s->traces.find(trace_id);
    if (it == s->traces.end() || it->second.state != LAUNCHED) return SMP_ESTATE;
    if (s->failed) return SMP_EDEVICE;
    RunSlot& r = s->slots[it->second.slot];
    if (!r.busy || r.seq != it->second.run_seq) return SMP_OK;
    const hipError_t q = hipEventQuery(r.e_end);
    if (q == hipSuccess) return SMP_OK;
    if (q == hipErrorNotReady) return SMP_EAGAIN;
    return fail(s);
}

static int wait_trace(smp_sampler_t* s, TraceRec& t) {
    RunSlot& r = s->slots[t.slot];
    if (r.busy && r.seq == t.run_seq) return retire_slot(s, r);
    return SMP_OK;
}

int fetch_profile(smp_sampler_t* s, uint64_t trace_id, smp_profile_sizes_t* sizes, smp_profile_t* out) {
    if (!s || !sizes) return SMP_EINVAL;
    auto it = s->traces.find(trace_id);
    if (it == s->traces.end() || it->second.state != LAUNCHED) return SMP_ESTATE;
    if (s->failed) return SMP_EDEVICE;
    TraceRec& t = it->second;
    HIPCHK(hipSetDevice(s->device));
    if (int rc = wait_trace(s, t)) return rc;
    uint8_t* base = s->ws + t.off;
    Scalars sc = t.scal;
    if (!t.have_scal) HIPCHK(hipMemcpy(&sc, base + t.lay.scal, sizeof(sc), hipMemcpyDeviceToHost));
    int32_t status = SMP_OK;
    if (sc.err & 1u) status = SMP_EINVAL;
    else if (sc.err & 2u) status = SMP_EOVERFLOW;
    else if (sc.err & 12u) status = SMP_EDEVICE;  // internal consistency fault
    sizes->n_samples = sc.K;
    sizes->n_tracked = sc.H;
    sizes->num_lines = t.params.num_lines;
    sizes->status = status;
    if (!out) return SMP_OK;
    const uint64_t L = t.params.num_lines;
    if (out->samples && sc.K)
        HIPCHK(hipMemcpy(out->samples, base + t.lay.samples, sizeof(Sample) * sc.K, hipMemcpyDeviceToHost));
    if (out->tracked && sc.H)
        HIPCHK(hipMemcpy(out->tracked, base + t.lay.tracked, sizeof(Tracked) * sc.H, hipMemcpyDeviceToHost));
    if (out->hist) HIPCHK(hipMemcpy(out->hist, base + t.lay.hist, 8 * H_COUNT * L, hipMemcpyDeviceToHost));
    if (out->leak) HIPCHK(hipMemcpy(out->leak, base + t.lay.leak, 8 * 4 * L, hipMemcpyDeviceToHost));
    if (out->gates) HIPCHK(hipMemcpy(out->gates, base + t.lay.gates, 2 * L, hipMemcpyDeviceToHost));
    out->final_F = sc.final_F;
    out->peak_F = sc.peak_F;
    out->peak_sampled_F = sc.peak_S;
    out->threshold_used = t.T_used;
    out->n_samples = sc.K;
    out->n_tracked = sc.H;
    out->status = status;
    arena_free(s, t.off, t.bytes);
    s->used -= t.bytes;
    s->traces.erase(it);
    return SMP_OK;
}

int submit_traces(smp_sampler_t* s, uint32_t count, const smp_event_t* const* ev, const uint64_t* n,
                  const smp_params_t* params, int ev_on_device, uint64_t* trace_ids, uint32_t* submitted) {
    if (submitted) *submitted = 0;
    if (!s || (count && (!ev || !n || !params || !trace_ids))) return SMP_EINVAL;
    for (uint32_t i = 0; i < count; ++i) {
        if (int rc = submit_trace(s, ev[i], n[i], &params[i], ev_on_device, &trace_ids[i])) return rc;
        if (submitted) *submitted = i + 1;
    }
    return SMP_OK;
}

int release_traces(smp_sampler_t* s, uint32_t count, const uint64_t* trace_ids, uint64_t* n_samples, int32_t* status,
                   uint32_t* released) {
    if (released) *released = 0;
    if (!s || (count && !trace_ids)) return SMP_EINVAL;
    for (uint32_t i = 0; i < count; ++i) {
        smp_profile_sizes_t sz{};
        smp_profile_t none{};
        if (int rc = fetch_profile(s, trace_ids[i], &sz, &none)) return rc;
        if (n_samples) n_samples[i] = sz.n_samples;
        if (status) status[i] = sz.status;
        if (released) *released = i + 1;
    }
    return SMP_OK;
}

int trace_device_results(smp_sampler_t* s, uint64_t trace_id, void** samples, void** hist, uint64_t* n_samples) {
    if (!s) return SMP_EINVAL;
    auto it = s->traces.find(trace_id);
    if (it == s->traces.end() || it->second.state != LAUNCHED) return SMP_ESTATE;
    if (s->failed) return SMP_EDEVICE;
    TraceRec& t = it->second;
    if (int rc = wait_trace(s, t)) return rc;
    uint8_t* base = s->ws + t.off;
    if (samples) *samples = base + t.lay.samples;
    if (hist) *hist = base + t.lay.hist;
    if (n_samples) {
        Scalars sc = t.scal;
        if (!t.have_scal) HIPCHK(hipMemcpy(&sc, base + t.lay.scal, sizeof(sc), hipMemcpyDeviceToHost));
        *n_samples = sc.K;
    }
    return SMP_OK;
}

int sampler_last_counters(smp_sampler_t* s, uint64_t* out32) {
    if (!s || !out32) return SMP_EINVAL;
    if (s->failed) return SMP_EDEVICE;
    int si = -1;
    for (int i = 0; i < RUN_SLOTS; ++i)
        if (s->slots[i].seq && (si < 0 || s->slots[i].seq > s->slots[si].seq)) si = i;
    if (si < 0) return SMP_ESTATE;
    if (int rc = retire_slot(s, s->slots[si])) return rc;
    HIPCHK(hipMemcpy(out32, s->slots[si].dev_ticket, 32 * sizeof(uint64_t), hipMemcpyDeviceToHost));
    return SMP_OK;
}

int sampler_last_timing(smp_sampler_t* s, float* main_kernel_ms, float* total_ms) {
    if (!s) return SMP_EINVAL;
    if (s->failed) return SMP_EDEVICE;
    for (auto& r : s->slots)
        if (int rc = retire_slot(s, r)) return rc;
    if (main_kernel_ms) *main_kernel_ms = s->last_main_ms;
    if (total_ms) *total_ms = s->last_total_ms;
    return SMP_OK;
}

int sampler_set_pass_events(smp_sampler_t* s, uint32_t mask) {
    if (!s || (mask & ~PASS_EVENTS_ALL) != 0) return SMP_EINVAL;
    s->pass_events = mask;
    return SMP_OK;
}

int sampler_set_tuning(smp_sampler_t* s, const smp_tuning_t* t) {
    if (!s || !t || t->chain_cap < 1 || t->chain_cap > (uint32_t)CHAIN_CAP_MAX || t->chain_grid > (1u << 20) ||
        t->emit_grid > (1u << 20) || t->graphs > 1)
        return SMP_EINVAL;
    s->tuning = *t;
    return SMP_OK;
}

int sampler_get_tuning(smp_sampler_t* s, smp_tuning_t* t) {
    if (!s || !t) return SMP_EINVAL;
    *t = s->tuning;
    if (!t->chain_grid) t->chain_grid = (uint32_t)s->grid_chain;
    if (!t->emit_grid) t->emit_grid = (uint32_t)s->grid_emit;
    return SMP_OK;
}

int sampler_launch_stats(smp_sampler_t* s, uint64_t* out3) {
    if (!s || !out3) return SMP_EINVAL;
    out3[0] = s->n_plain;
    out3[1] = s->n_captured;
    out3[2] = s->n_replayed;
    return SMP_OK;
}

int sampler_last_pass_timing(smp_sampler_t* s, float* pass_ms) {
    if (!s || !pass_ms) return SMP_EINVAL;
    if (s->failed) return SMP_EDEVICE;
    for (auto& r : s->slots)
        if (int rc = retire_slot(s, r)) return rc;
    for (int i = 0; i < NPASS; ++i) pass_ms[i] = s->last_pass_ms[i];
    return SMP_OK;
}

}  // extern "C"
