// Local energy for callers that cannot allocate device memory: the call's
// workspace is a fixed array of device memory owned by the library.
//
// The array lives in this file's code object, so every device the library
// runs on holds one copy of kScratchBytes from the first use of that copy
// until the process ends.  Host code never takes the array's name as a
// device address: the device address of each device's copy is looked up
// once with hipGetSymbolAddress (with that device current) and kept.
#include <mutex>

#include "engine.h"

namespace {

constexpr size_t kScratchBytes = (size_t)VQNQS_STATIC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_addr[kMaxDevices];   // device address of `scratch` per device

// Device address of the current device's copy of `scratch`.
hipError_t scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

// The call's status to the caller: the first int32 of the workspace is a
// flag that the spin validation sets on a value other than +-1.
__global__ void k_status_out(const int32_t* ws_flag, int32_t* out) {
    if (threadIdx.x == 0) *out = *ws_flag ? VQNQS_ERR_BAD_SPIN : VQNQS_OK;
}

}  // namespace

namespace vq {

vqnqs_status local_energy_static(const ModelDims& m, const void* params,
                                 const int8_t* spins, int64_t batch, int mode,
                                 double* eloc, double* stats, double* ratios,
                                 int64_t* counters, int32_t* status,
                                 hipStream_t st) {
    // one sample's workspace must fit: larger problems are refused before
    // anything is enqueued
    if (workspace_bytes(m, mode, 1) > kScratchBytes)
        return VQNQS_ERR_EXCEEDS_STATIC_SCRATCH;
    void* ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return VQNQS_ERR_HIP;
    // every workspace word the call reads is written by the call first
    // (status word, list counters, counters), so the previous call's
    // contents do not matter
    vqnqs_status s = local_energy(m, params, spins, batch, mode, eloc, stats,
                                  ratios, counters, ws, kScratchBytes, st);
    if (s) return s;
    if (status) {
        hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st,
                           static_cast<const int32_t*>(ws), status);
        if (hipGetLastError() != hipSuccess) return VQNQS_ERR_HIP;
    }
    return VQNQS_OK;
}

}  // namespace vq
