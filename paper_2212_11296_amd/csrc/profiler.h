// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

namespace vq {

class Profiler {
   public:
    static Profiler& get();
    bool enabled() const { return on_; }
    void enable(bool on);
    void reset();
    // Brackets one kernel launch on `st` (no-op when disabled).
    void begin(const char* name, hipStream_t st);
    void end(hipStream_t st);
    // Waits for recorded events and folds them into the totals.
    int read(char* names, int name_len, double* total_ms, long long* count,
             int max);

   private:
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    void fold();
    bool on_ = false;
    std::mutex mu_;
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> free_;
    std::vector<std::string> names_;
    std::vector<double> ms_;
    std::vector<long long> cnt_;
    std::string cur_;
    hipEvent_t cur_a_ = nullptr;
};

// Exponentials per second the device's vector units issue (v_exp_f32 on
// independent chains, all SIMDs busy); synchronises `st`.  sink: one float
// of device memory the kernel writes.
hipError_t probe_exp_rate(float* sink, hipStream_t st, double* per_s);

}  // namespace vq
