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

}  // namespace vq
