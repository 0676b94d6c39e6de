// report.cpp - host-side report layer over fetched profiles: the report
// line filter (section 5), the leak report filter (section 3.4) and the
// per-line memory timelines (section 5).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "scalene_sampler.h"

// ---------------------------------------------------------------------------
// Leak report filter (section 3.4): leaks are reported only when overall
// memory grows by at least 1 %.  Read as the least-squares line of the
// sampled footprint F against the event index x over the K samples: it
// passes when its rise over the sampled span, b (x_K - x_1) with
// b = (K Sxy - Sx Sy) / (K Sxx - Sx^2), is at least 1 % of the peak sampled
// footprint.  The sums fit in 128 bits (x < 2^32, |F| < 2^61, K < 2^32); the
// comparison 100 num span >= peak den needs up to ~197 bits, done here on
// four 64-bit limbs with signs kept apart.

namespace {

struct U256 {
    uint64_t w[4];
};

U256 u256(unsigned __int128 v) { return U256{{(uint64_t)v, (uint64_t)(v >> 64), 0, 0}}; }

U256 add(const U256& a, const U256& b) {
    U256 r{};
    unsigned __int128 c = 0;
    for (int i = 0; i < 4; ++i) {
        const unsigned __int128 s = (unsigned __int128)a.w[i] + b.w[i] + c;
        r.w[i] = (uint64_t)s;
        c = s >> 64;
    }
    return r;
}

U256 sub(const U256& a, const U256& b) {  // a >= b
    U256 r{};
    uint64_t borrow = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t d = a.w[i] - b.w[i] - borrow;
        borrow = (a.w[i] < b.w[i] || (a.w[i] == b.w[i] && borrow)) ? 1 : 0;
        r.w[i] = d;
    }
    return r;
}

int cmp(const U256& a, const U256& b) {
    for (int i = 3; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

bool is_zero(const U256& a) { return !(a.w[0] | a.w[1] | a.w[2] | a.w[3]); }

U256 mul64(const U256& a, uint64_t b) {  // the product stays below 2^256 here
    U256 r{};
    unsigned __int128 c = 0;
    for (int i = 0; i < 4; ++i) {
        const unsigned __int128 p = (unsigned __int128)a.w[i] * b + c;
        r.w[i] = (uint64_t)p;
        c = p >> 64;
    }
    return r;
}

U256 mul128(unsigned __int128 a, unsigned __int128 b) {
    const U256 lo = mul64(u256(a), (uint64_t)b);
    const U256 hi = mul64(u256(a), (uint64_t)(b >> 64));
    return add(lo, U256{{0, hi.w[0], hi.w[1], hi.w[2]}});
}

unsigned __int128 mag(__int128 v) { return v < 0 ? (unsigned __int128)(-(v + 1)) + 1 : (unsigned __int128)v; }

}  // namespace

// ---------------------------------------------------------------------------
// Report line filter (section 5): a profile shows only the lines that take at
// least 1 % of the execution time or at least 1 % of the memory, each with
// the line before and the line after it, and never more than 300 lines.  A
// line's time is its Python plus native time, its memory the bytes of its
// growth samples; "at least 1 %" is 100 x >= the total of the lines'
// positive values.  Each criterion alone admits at most 100 lines, the two
// together up to 200, so when more than 100 qualify the 100 with the largest
// share stay (a line's share: the larger of its time and memory shares,
// compared exactly; equal shares: the lower id), which keeps the bound.

namespace {

constexpr size_t MAX_QUALIFYING = 100;

// a fraction num/den (den > 0) of one criterion's total
struct Share {
    unsigned __int128 num, den;
};

bool share_less(const Share& a, const Share& b) { return cmp(mul128(a.num, b.den), mul128(b.num, a.den)) < 0; }

}  // namespace

extern "C" SMP_API int report_lines(const int64_t* py_time_us, const int64_t* nat_time_us, const int64_t* growth_bytes,
                                    uint32_t num_lines, uint32_t* out_lines, uint32_t* n_out) {
    if (!n_out) return SMP_EINVAL;
    *n_out = 0;
    if (num_lines == 0) return SMP_OK;
    if (!py_time_us || !nat_time_us || !growth_bytes || !out_lines) return SMP_EINVAL;
    auto line_time = [&](uint32_t l) { return (__int128)py_time_us[l] + (__int128)nat_time_us[l]; };
    unsigned __int128 tot_time = 0, tot_mem = 0;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const __int128 t = line_time(l);
        if (t > 0) tot_time += (unsigned __int128)t;
        if (growth_bytes[l] > 0) tot_mem += (unsigned __int128)growth_bytes[l];
    }
    std::vector<uint32_t> q;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const __int128 t = line_time(l);
        const int64_t m = growth_bytes[l];
        if ((t > 0 && (unsigned __int128)t * 100u >= tot_time) || (m > 0 && (unsigned __int128)m * 100u >= tot_mem))
            q.push_back(l);
    }
    if (q.size() > MAX_QUALIFYING) {
        auto share = [&](uint32_t l) {
            const __int128 t = line_time(l);
            const int64_t m = growth_bytes[l];
            const Share ts{t > 0 ? (unsigned __int128)t : 0, tot_time ? tot_time : 1};
            const Share ms{m > 0 ? (unsigned __int128)m : 0, tot_mem ? tot_mem : 1};
            return share_less(ts, ms) ? ms : ts;
        };
        std::vector<std::pair<Share, uint32_t>> ranked;
        ranked.reserve(q.size());
        for (uint32_t l : q) ranked.emplace_back(share(l), l);
        std::sort(ranked.begin(), ranked.end(), [](const auto& a, const auto& b) {
            if (share_less(b.first, a.first)) return true;   // larger share first
            if (share_less(a.first, b.first)) return false;
            return a.second < b.second;                        // then the lower id
        });
        q.clear();
        for (size_t i = 0; i < MAX_QUALIFYING; ++i) q.push_back(ranked[i].second);
        std::sort(q.begin(), q.end());
    }
    // the kept lines and their neighbours, ascending and once each
    uint32_t k = 0;
    for (uint32_t l : q) {
        const uint32_t lo = l > 0 ? l - 1 : 0, hi = l + 1 < num_lines ? l + 1 : l;
        for (uint32_t c = lo; c <= hi; ++c)
            if (k == 0 || c > out_lines[k - 1]) out_lines[k++] = c;
    }
    *n_out = k;
    return SMP_OK;
}

extern "C" SMP_API int leak_report(const smp_sample_t* samples, uint64_t n_samples, const uint8_t* gate,
                                   const int64_t* py_time_us, const int64_t* nat_time_us, uint32_t num_lines,
                                   int32_t* slope_ok, uint8_t* reported, int64_t* elapsed_us) {
    if (!slope_ok || !elapsed_us || (n_samples && !samples) ||
        (num_lines && (!gate || !py_time_us || !nat_time_us || !reported)))
        return SMP_EINVAL;
    if (n_samples >= (1ull << 32)) return SMP_EINVAL;
    bool ok = false;
    if (n_samples >= 2) {
        unsigned __int128 Sx = 0, Sxx = 0;
        __int128 Sy = 0, Sxy = 0;
        int64_t peak = samples[0].F;
        for (uint64_t k = 0; k < n_samples; ++k) {
            const uint64_t x = samples[k].event_idx;
            const int64_t y = samples[k].F;
            Sx += x;
            Sxx += (unsigned __int128)x * x;
            Sy += y;
            Sxy += (__int128)x * y;
            if (y > peak) peak = y;
        }
        const uint64_t K = n_samples;
        const uint64_t x0 = samples[0].event_idx, x1 = samples[n_samples - 1].event_idx;
        if (peak > 0 && x1 > x0) {
            // num = K Sxy - Sx Sy as (sign, magnitude)
            const bool a_neg = Sxy < 0, b_neg = Sy < 0;
            const U256 A = mul128(K, mag(Sxy)), B = mul128(Sx, mag(Sy));
            bool n_neg;
            U256 N;
            if (a_neg != b_neg) {
                n_neg = a_neg;
                N = add(A, B);
            } else if (cmp(A, B) >= 0) {
                n_neg = a_neg;
                N = sub(A, B);
            } else {
                n_neg = !a_neg;
                N = sub(B, A);
            }
            const U256 KSxx = mul128(K, Sxx), Sx2 = mul128(Sx, Sx);
            if (!n_neg && !is_zero(N) && cmp(KSxx, Sx2) > 0) {
                const U256 den = sub(KSxx, Sx2);
                const U256 lhs = mul64(mul64(N, x1 - x0), 100);
                const U256 rhs = mul64(den, (uint64_t)peak);
                ok = cmp(lhs, rhs) >= 0;
            }
        }
    }
    *slope_ok = ok ? 1 : 0;
    uint64_t el = 0;
    for (uint32_t l = 0; l < num_lines; ++l) {
        el += (uint64_t)py_time_us[l] + (uint64_t)nat_time_us[l];  // modulo 2^64, as the per-line sums
        reported[l] = (ok && gate[l]) ? 1 : 0;
    }
    *elapsed_us = (int64_t)el;
    return SMP_OK;
}

// ---------------------------------------------------------------------------
// Per-line memory timelines (section 5): each line's footprint log (its
// samples in rank order, as points (event index, footprint)) reduced by
// Ramer-Douglas-Peucker to at most max_points points.  A point is kept when
// its distance from the chord of its run exceeds eps, decided exactly as
// cross^2 > eps^2 (dx^2 + dy^2) on 256-bit integers; the farthest point of a
// run (the first on ties) splits it.  eps is the smallest of
// {0, 1, 2, 4, ..., 2^62} that leaves at most max_points points: the kept set
// only shrinks as eps grows, so a binary search over the candidates finds it.

namespace {

struct Run {
    uint32_t i, j;
};

// RDP over pts[0..n) at eps; marks kept points in keep (if given) and
// returns their number.  stack: scratch for the runs.
uint64_t rdp(const uint32_t* xs, const int64_t* ys, uint32_t n, uint64_t eps, uint8_t* keep, std::vector<Run>& stack) {
    if (n <= 2) {
        if (keep)
            for (uint32_t k = 0; k < n; ++k) keep[k] = 1;
        return n;
    }
    const unsigned __int128 e2 = (unsigned __int128)eps * eps;
    uint64_t kept = 2;
    if (keep) keep[0] = keep[n - 1] = 1;
    stack.clear();
    stack.push_back(Run{0, n - 1});
    while (!stack.empty()) {
        const Run r = stack.back();
        stack.pop_back();
        if (r.j - r.i < 2) continue;
        const int64_t dx = (int64_t)xs[r.j] - (int64_t)xs[r.i];
        const __int128 dy = (__int128)ys[r.j] - ys[r.i];
        unsigned __int128 best = 0;
        uint32_t bk = 0;
        bool any = false;
        for (uint32_t k = r.i + 1; k < r.j; ++k) {
            const __int128 c = (__int128)dx * ((__int128)ys[k] - ys[r.i]) - dy * ((int64_t)xs[k] - (int64_t)xs[r.i]);
            const unsigned __int128 a = mag(c);
            if (!any || a > best) {
                best = a;
                bk = k;
                any = true;
            }
        }
        const unsigned __int128 len2 = (unsigned __int128)((__int128)dx * dx) + mag(dy) * mag(dy);
        if (cmp(mul128(best, best), mul128(e2, len2)) > 0) {
            ++kept;
            if (keep) keep[bk] = 1;
            stack.push_back(Run{r.i, bk});
            stack.push_back(Run{bk, r.j});
        }
    }
    return kept;
}

}  // namespace

extern "C" SMP_API int timeline_points(const smp_sample_t* samples, uint64_t n_samples, uint32_t num_lines,
                                       uint32_t max_points, uint8_t* keep) {
    if (max_points < 2 || (n_samples && (!samples || !keep)) || n_samples >= (1ull << 32)) return SMP_EINVAL;
    for (uint64_t r = 0; r < n_samples; ++r) keep[r] = 0;
    if (!n_samples || !num_lines) return SMP_OK;
    // group the samples by line, rank order kept (counting sort)
    std::vector<uint32_t> start((size_t)num_lines + 1, 0), order(n_samples);
    for (uint64_t r = 0; r < n_samples; ++r)
        if (samples[r].line < num_lines) ++start[samples[r].line + 1];
    for (uint32_t l = 0; l < num_lines; ++l) start[l + 1] += start[l];
    std::vector<uint32_t> fill(start.begin(), start.end() - 1);
    for (uint64_t r = 0; r < n_samples; ++r)
        if (samples[r].line < num_lines) order[fill[samples[r].line]++] = (uint32_t)r;
    std::vector<uint32_t> xs;
    std::vector<int64_t> ys;
    std::vector<uint8_t> mark;
    std::vector<Run> stack;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const uint32_t b = start[l], n = start[l + 1] - b;
        if (!n) continue;
        xs.resize(n);
        ys.resize(n);
        for (uint32_t k = 0; k < n; ++k) {
            xs[k] = samples[order[b + k]].event_idx;
            ys[k] = samples[order[b + k]].F;
        }
        // candidates c(0) = 0, c(e + 1) = 2^e: the first with at most max_points
        auto cand = [](int i) -> uint64_t { return i == 0 ? 0 : (1ull << (i - 1)); };
        int lo = 0, hi = 63;  // rdp at c(63) = 2^62 keeps the two endpoints only
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (rdp(xs.data(), ys.data(), n, cand(mid), nullptr, stack) <= max_points) hi = mid;
            else lo = mid + 1;
        }
        mark.assign(n, 0);
        rdp(xs.data(), ys.data(), n, cand(lo), mark.data(), stack);
        for (uint32_t k = 0; k < n; ++k)
            if (mark[k]) keep[order[b + k]] = 1;
    }
    return SMP_OK;
}

// ---------------------------------------------------------------------------
// Per-line memory timelines by the paper's own procedure (section 5): RDP
// with an approximate eps, then a random downsampling of every log that is
// still longer than max_points to exactly max_points points.  The eps of a
// line is its footprint range over max_points (integer division).  The
// downsampling keeps a uniform random subset of the RDP points by selection
// sampling (Knuth, TAOCP vol. 2, section 3.4.2, Algorithm S): with m of k
// points chosen, the t-th of the N candidates is chosen when
// floor(x (N - t) / 2^64) < k - m, x the next output of splitmix64 (Steele,
// Lea and Flood, 2014) whose state starts at seed + line, modulo 2^64.

namespace {

uint64_t splitmix64_next(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" SMP_API int timeline_points_sampled(const smp_sample_t* samples, uint64_t n_samples, uint32_t num_lines,
                                               uint32_t max_points, uint64_t seed, uint8_t* keep) {
    if (max_points < 2 || (n_samples && (!samples || !keep)) || n_samples >= (1ull << 32)) return SMP_EINVAL;
    for (uint64_t r = 0; r < n_samples; ++r) keep[r] = 0;
    if (!n_samples || !num_lines) return SMP_OK;
    std::vector<uint32_t> start((size_t)num_lines + 1, 0), order(n_samples);
    for (uint64_t r = 0; r < n_samples; ++r)
        if (samples[r].line < num_lines) ++start[samples[r].line + 1];
    for (uint32_t l = 0; l < num_lines; ++l) start[l + 1] += start[l];
    std::vector<uint32_t> fill(start.begin(), start.end() - 1);
    for (uint64_t r = 0; r < n_samples; ++r)
        if (samples[r].line < num_lines) order[fill[samples[r].line]++] = (uint32_t)r;
    std::vector<uint32_t> xs;
    std::vector<int64_t> ys;
    std::vector<uint8_t> mark;
    std::vector<Run> stack;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const uint32_t b = start[l], n = start[l + 1] - b;
        if (!n) continue;
        xs.resize(n);
        ys.resize(n);
        int64_t ymin = samples[order[b]].F, ymax = ymin;
        for (uint32_t k = 0; k < n; ++k) {
            xs[k] = samples[order[b + k]].event_idx;
            ys[k] = samples[order[b + k]].F;
            ymin = ys[k] < ymin ? ys[k] : ymin;
            ymax = ys[k] > ymax ? ys[k] : ymax;
        }
        const uint64_t eps = (uint64_t)((unsigned __int128)((__int128)ymax - ymin) / max_points);
        mark.assign(n, 0);
        const uint64_t kept = rdp(xs.data(), ys.data(), n, eps, mark.data(), stack);
        if (kept > max_points) {
            uint64_t state = seed + l, chosen = 0, t = 0;
            for (uint32_t k = 0; k < n; ++k) {
                if (!mark[k]) continue;
                bool take = false;
                if (chosen < max_points) {
                    const uint64_t x = splitmix64_next(state);
                    take = (uint64_t)(((unsigned __int128)x * (kept - t)) >> 64) < max_points - chosen;
                }
                ++t;
                if (take) ++chosen;
                else mark[k] = 0;
            }
        }
        for (uint32_t k = 0; k < n; ++k)
            if (mark[k]) keep[order[b + k]] = 1;
    }
    return SMP_OK;
}
