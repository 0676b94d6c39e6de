// report.cpp - the report line filter (section 5), host side: a profile
// shows only the lines that take at least 1 % of the execution time or at
// least 1 % of the memory, together with the line before and the line after
// each.  A line's time is its Python plus native time, its memory the bytes
// of its growth samples; "at least 1 %" is 100 x >= the total of the lines'
// positive values.  One pass over the lines decides each line from its
// neighbours' tests (a window of three), so the output comes out in order.
#include <cstdint>

#include "scalene_sampler.h"

namespace {

struct Shares {
    unsigned __int128 time = 0, mem = 0;
};

inline __int128 line_time(const int64_t* py, const int64_t* nat, uint32_t l) {
    return (__int128)py[l] + (__int128)nat[l];
}

}  // namespace

extern "C" SMP_API int report_lines(const int64_t* py_time_us, const int64_t* nat_time_us, const int64_t* growth_bytes,
                                    uint32_t num_lines, uint32_t* out_lines, uint32_t* n_out) {
    if (!n_out) return SMP_EINVAL;
    *n_out = 0;
    if (num_lines == 0) return SMP_OK;
    if (!py_time_us || !nat_time_us || !growth_bytes || !out_lines) return SMP_EINVAL;
    Shares tot;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const __int128 t = line_time(py_time_us, nat_time_us, l);
        if (t > 0) tot.time += (unsigned __int128)t;
        if (growth_bytes[l] > 0) tot.mem += (unsigned __int128)growth_bytes[l];
    }
    auto qualifies = [&](uint32_t l) -> bool {
        const __int128 t = line_time(py_time_us, nat_time_us, l);
        if (t > 0 && (unsigned __int128)t * 100u >= tot.time) return true;
        const int64_t m = growth_bytes[l];
        return m > 0 && (unsigned __int128)m * 100u >= tot.mem;
    };
    // q_prev, q_cur, q_next: the tests of lines l-1, l, l+1
    bool q_prev = false, q_cur = qualifies(0);
    uint32_t k = 0;
    for (uint32_t l = 0; l < num_lines; ++l) {
        const bool q_next = l + 1 < num_lines && qualifies(l + 1);
        if (q_prev || q_cur || q_next) out_lines[k++] = l;
        q_prev = q_cur;
        q_cur = q_next;
    }
    *n_out = k;
    return SMP_OK;
}
