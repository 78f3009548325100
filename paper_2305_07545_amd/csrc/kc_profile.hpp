// Optional per-kernel timing with HIP events recorded on the launch stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace kc {

class Profiler {
  public:
    bool on = false;

    // Record a start event for `phase` on stream s (no-op when off).
    void begin(int phase, hipStream_t s) {
        if (!on)
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
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
};

}  // namespace kc
