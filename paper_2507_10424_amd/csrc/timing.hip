// Optional per-kernel timing with HIP events, for benchmarks.  When enabled,
// every launch of a timed kernel is bracketed by two events recorded on the
// launch stream; ldpc_timing_read sums their elapsed times.  Decoding results
// do not depend on it.
#include <mutex>
#include <tuple>

#include "ldpc_internal.h"

namespace ldpc {

namespace {
struct TimerState {
    std::mutex mu;
    bool on = false;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> recs;
};
TimerState &state() {
    static TimerState s;
    return s;
}
void clear_locked(TimerState &s) {
    for (auto &r : s.recs) {
        (void)hipEventDestroy(std::get<1>(r));
        (void)hipEventDestroy(std::get<2>(r));
    }
    s.recs.clear();
}
} // namespace

bool timing_on() { return state().on; }

void timing_record(int kid, hipEvent_t a, hipEvent_t b) {
    TimerState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    s.recs.emplace_back(kid, a, b);
}

} // namespace ldpc

extern "C" int ldpc_timing_enable(int on) {
    ldpc::TimerState &s = ldpc::state();
    std::lock_guard<std::mutex> lk(s.mu);
    ldpc::clear_locked(s);
    s.on = on != 0;
    return LDPC_OK;
}

extern "C" int ldpc_timing_read(int32_t kernel, double *total_ms, int64_t *launches) {
    if (kernel < 0 || kernel >= ldpc::K_COUNT) return LDPC_EINVAL;
    ldpc::TimerState &s = ldpc::state();
    std::lock_guard<std::mutex> lk(s.mu);
    double ms = 0.0;
    int64_t cnt = 0;
    for (auto &r : s.recs) {
        if (std::get<0>(r) != kernel) continue;
        float e = 0.0f;
        if (hipEventSynchronize(std::get<2>(r)) != hipSuccess ||
            hipEventElapsedTime(&e, std::get<1>(r), std::get<2>(r)) != hipSuccess)
            return LDPC_EHIP;
        ms += e;
        ++cnt;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    return LDPC_OK;
}
