// Event-bracketed kernel timing used by the benchmark: per-launch durations
// of the operator kernels measured on the stream they run on.
#include "internal.hpp"

namespace trbdg {

namespace {
hipEvent_t take(const tbdg_ctx* c) {
    auto& pool = c->timer.pool;
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    TBDG_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

// Every kSampleStride-th launch of each kernel class is timed (stride 3 is
// coprime with the launch pattern of the GMRES cycles, so the sample keeps
// their mix of plain and fused launches); a timed dispatch costs a few
// microseconds of its own, about 4 % of the benchmark step if every launch
// is timed.
constexpr uint64_t kSampleStride = 3;

TimedLaunch::TimedLaunch(const tbdg_ctx* c, int which, double bytes) : c_(c), which_(which) {
    if (!c_->timer.on) return;
    static thread_local uint64_t seen[2] = {0, 0};
    if (seen[which_]++ % kSampleStride != 0) return;
    e1_ = take(c_);
    e2_ = take(c_);
    c_->timer.bytes[which_] += bytes;
}

TimedLaunch::~TimedLaunch() {
    if (!e1_) return;
    c_->timer.pending[which_].emplace_back(e1_, e2_);
    if (c_->timer.pending[which_].size() >= 4096) {
        try {
            timer_collect(c_);
        } catch (...) {
        }
    }
}

void timer_collect(const tbdg_ctx* c) {
    for (int w = 0; w < 2; ++w) {
        for (auto& pr : c->timer.pending[w]) {
            TBDG_HIP(hipEventSynchronize(pr.second));
            float ms = 0.0f;
            TBDG_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
            c->timer.total_ms[w] += ms;
            c->timer.count[w] += 1;
            c->timer.pool.push_back(pr.first);
            c->timer.pool.push_back(pr.second);
        }
        c->timer.pending[w].clear();
    }
}

void timer_release(const tbdg_ctx* c) {
    for (int w = 0; w < 2; ++w) {
        for (auto& pr : c->timer.pending[w]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        c->timer.pending[w].clear();
    }
    for (hipEvent_t e : c->timer.pool) (void)hipEventDestroy(e);
    c->timer.pool.clear();
}

}  // namespace trbdg
