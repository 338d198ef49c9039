#include "profiler.h"

#include <cstring>

namespace vq {

Profiler& Profiler::get() {
    static Profiler p;
    return p;
}

void Profiler::enable(bool on) {
    std::lock_guard<std::mutex> g(mu_);
    on_ = on;
}

void Profiler::reset() {
    std::lock_guard<std::mutex> g(mu_);
    fold();
    names_.clear();
    ms_.clear();
    cnt_.clear();
}

static hipEvent_t take(std::vector<hipEvent_t>& pool) {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Profiler::begin(const char* name, hipStream_t st) {
    if (!on_) return;
    std::lock_guard<std::mutex> g(mu_);
    cur_ = name;
    cur_a_ = take(free_);
    if (cur_a_) (void)hipEventRecord(cur_a_, st);
}

void Profiler::end(hipStream_t st) {
    if (!on_ || !cur_a_) return;
    std::lock_guard<std::mutex> g(mu_);
    hipEvent_t b = take(free_);
    if (!b) return;
    (void)hipEventRecord(b, st);
    pending_.push_back({cur_, cur_a_, b});
    cur_a_ = nullptr;
    if (pending_.size() > 4096) fold();
}

void Profiler::fold() {
    for (auto& p : pending_) {
        (void)hipEventSynchronize(p.b);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        size_t k = 0;
        while (k < names_.size() && names_[k] != p.name) ++k;
        if (k == names_.size()) {
            names_.push_back(p.name);
            ms_.push_back(0.0);
            cnt_.push_back(0);
        }
        ms_[k] += ms;
        cnt_[k] += 1;
        free_.push_back(p.a);
        free_.push_back(p.b);
    }
    pending_.clear();
}

int Profiler::read(char* names, int name_len, double* total_ms,
                   long long* count, int max) {
    std::lock_guard<std::mutex> g(mu_);
    fold();
    const int n = (int)names_.size() < max ? (int)names_.size() : max;
    for (int k = 0; k < n; ++k) {
        if (names) {
            std::strncpy(names + (size_t)k * name_len, names_[k].c_str(),
                         name_len - 1);
            names[(size_t)k * name_len + name_len - 1] = 0;
        }
        if (total_ms) total_ms[k] = ms_[k];
        if (count) count[k] = cnt_[k];
    }
    return (int)names_.size();
}

// ------------------------------------------------ exponential issue rate
// Every lane runs eight independent chains x <- 2^x on the vector unit's
// exponential instruction (v_exp_f32); the chains saturate to +inf after a
// few steps, which does not change the instruction's issue rate.  Lane 0
// of block 0 writes its sum so the chains stay live.
__global__ void __launch_bounds__(256) k_exp_probe(float* sink, int iters) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = -1.0f - 1e-3f * (float)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(x[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) sink[0] = s;
}

hipError_t probe_exp_rate(float* sink, hipStream_t st, double* per_s) {
    // 8 waves per SIMD on 256 CUs x 4 SIMDs
    const int blocks = 256 * 8, threads = 256, iters = 1 << 16;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // warm-up launch, then the timed one
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_exp_probe, dim3(blocks), dim3(threads), 0, st,
                           sink, 256);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_exp_probe, dim3(blocks), dim3(threads), 0, st,
                           sink, iters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess)
        *per_s = (double)blocks * threads * 8.0 * iters / (ms * 1e-3);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return e;
}

}  // namespace vq
