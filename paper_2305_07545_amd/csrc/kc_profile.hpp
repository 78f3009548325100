// Optional per-kernel timing with HIP events recorded on the launch stream.
// The events only time the work between them: they are created without the
// system-scope fence, so waiting for one does not order memory for the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace kc {

class Profiler {
  public:
    bool on = false;
    uint32_t mask = ~0u;  // phases timed while on (bit per phase)

    // Record a start event for `phase` on stream s (no-op when off or when
    // the phase is masked out).
    void begin(int phase, hipStream_t s) {
        if (!on || phase < 0 || phase >= 32 || !((mask >> phase) & 1u))
            return;
        Rec r;
        r.phase = phase;
        r.a = take();
        r.b = take();
        if (!r.a || !r.b)
            return;
        (void)hipEventRecord(r.a, s);
        recs_.push_back(r);
        open_ = true;
    }

    void end(hipStream_t s) {
        if (!on || !open_)
            return;
        (void)hipEventRecord(recs_.back().b, s);
        open_ = false;
    }

    // Wait for every recorded pair, add its time to ms[phase] and count the
    // launch; events go back to the pool.
    void collect(double *ms, uint64_t *launches, uint32_t n_phases) {
        for (auto &r : recs_) {
            float t = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess &&
                hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && (uint32_t)r.phase < n_phases) {
                if (ms)
                    ms[r.phase] += t;
                if (launches)
                    launches[r.phase] += 1;
            }
            pool_.push_back(r.a);
            pool_.push_back(r.b);
        }
        recs_.clear();
        open_ = false;
    }

    void release() {
        for (auto &r : recs_) {
            (void)hipEventSynchronize(r.b);
            pool_.push_back(r.a);
            pool_.push_back(r.b);
        }
        recs_.clear();
        for (auto e : pool_)
            (void)hipEventDestroy(e);
        pool_.clear();
    }

  private:
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs_;
    std::vector<hipEvent_t> pool_;
    bool open_ = false;

    hipEvent_t take() {
        if (!pool_.empty()) {
            hipEvent_t e = pool_.back();
            pool_.pop_back();
            return e;
        }
        // timing only: no system-scope fence (and its L2 writeback and
        // invalidate) when an event is recorded
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            return nullptr;
        return e;
    }
};

}  // namespace kc
