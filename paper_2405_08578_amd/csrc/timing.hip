// Optional per-kernel timing: while enabled, the launchers bracket the
// launches of the path's main kernels with HIP events recorded on the launch
// stream; lpsift_timing_read waits for the recorded events and returns the
// summed device time per kernel. Host-side state, guarded by one mutex.
#include <mutex>
#include <vector>

#include "internal.h"

namespace lpsift {
namespace {

struct Pending {
    int kernel;
    hipEvent_t a, b;
};

struct TimingState {
    std::mutex mu;
    bool on = false;
    bool failed = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    double ms[LPSIFT_KERNEL_COUNT] = {};
    int64_t launches[LPSIFT_KERNEL_COUNT] = {};
};

TimingState& state()
{
    static TimingState* s = new TimingState();   // never destroyed: usable at exit
    return *s;
}

hipEvent_t take_event(TimingState& s)
{
    if (!s.free_events.empty()) {
        hipEvent_t e = s.free_events.back();
        s.free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Waits for every pending pair and folds it into the sums (lock held).
void drain(TimingState& s)
{
    for (const Pending& p : s.pending) {
        float t = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            s.ms[p.kernel] += t;
            s.launches[p.kernel] += 1;
        } else {
            s.failed = true;
        }
        s.free_events.push_back(p.a);
        s.free_events.push_back(p.b);
    }
    s.pending.clear();
}

}  // namespace

TimedScope::TimedScope(int kernel, hipStream_t stream) : kernel_(kernel), stream_(stream)
{
    TimingState& s = state();
    std::lock_guard<std::mutex> g(s.mu);
    if (!s.on) return;
    a_ = take_event(s);
    b_ = take_event(s);
    if (!a_ || !b_ || hipEventRecord(a_, stream_) != hipSuccess) {
        if (a_) s.free_events.push_back(a_);
        if (b_) s.free_events.push_back(b_);
        a_ = b_ = nullptr;
        s.failed = true;
    }
}

TimedScope::~TimedScope()
{
    if (!a_) return;
    TimingState& s = state();
    std::lock_guard<std::mutex> g(s.mu);
    if (hipEventRecord(b_, stream_) != hipSuccess) {
        s.failed = true;
        s.free_events.push_back(a_);
        s.free_events.push_back(b_);
        return;
    }
    s.pending.push_back(Pending{kernel_, a_, b_});
}

}  // namespace lpsift

using namespace lpsift;

extern "C" {

int lpsift_timing_enable(int32_t on)
{
    TimingState& s = state();
    std::lock_guard<std::mutex> g(s.mu);
    drain(s);
    for (int k = 0; k < LPSIFT_KERNEL_COUNT; ++k) {
        s.ms[k] = 0.0;
        s.launches[k] = 0;
    }
    s.failed = false;
    s.on = on != 0;
    return LPSIFT_OK;
}

int lpsift_timing_read(int32_t kernel, double* ms, int64_t* launches)
{
    if (kernel < 0 || kernel >= LPSIFT_KERNEL_COUNT || !ms || !launches) return LPSIFT_EINVAL;
    TimingState& s = state();
    std::lock_guard<std::mutex> g(s.mu);
    drain(s);
    *ms = s.ms[kernel];
    *launches = s.launches[kernel];
    return s.failed ? LPSIFT_EHIP : LPSIFT_OK;
}

}  // extern "C"
