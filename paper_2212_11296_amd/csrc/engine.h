// Internal interface between the C ABI and the kernel orchestration.
#pragma once
#include "common.h"

namespace vq {

int64_t param_count(const ModelDims& m);
size_t workspace_bytes(const ModelDims& m, int mode, int64_t chunk);
size_t vmc_workspace_bytes(const ModelDims& m, int64_t batch, int64_t chunk);
int64_t pick_chunk(const ModelDims& m, int mode, int64_t batch, size_t ws);
int64_t max_overlay_rows_per_sample(const ModelDims& m);

vqnqs_status local_energy(const ModelDims& m, const void* params,
                          const int8_t* spins, int64_t batch, int mode,
                          double* eloc, double* stats, double* ratios,
                          int64_t* counters, void* ws, size_t ws_bytes,
                          hipStream_t st);
// local_energy with the library's static device array as its workspace
vqnqs_status local_energy_static(const ModelDims& m, const void* params,
                                 const int8_t* spins, int64_t batch, int mode,
                                 double* eloc, double* stats, double* ratios,
                                 int64_t* counters, int32_t* status,
                                 hipStream_t st);
// attn: nullable [batch][nl][N][d] attention outputs (activation type)
vqnqs_status forward_logpsi(const ModelDims& m, const void* params,
                            const int8_t* spins, int64_t batch, double* logpsi,
                            int32_t* codes, void* attn, void* ws,
                            size_t ws_bytes, hipStream_t st);
vqnqs_status sample(const ModelDims& m, const void* params,
                    const double* uniforms, int64_t batch, int8_t* spins,
                    double* logpsi, void* ws, size_t ws_bytes,
                    hipStream_t st);
vqnqs_status vmc_step(const ModelDims& m, void* params, void* opt_state,
                      int64_t step, double lr, const double* uniforms,
                      int64_t B, int8_t* spins_out, double* eloc_out,
                      double* stats_out, void* ws, size_t ws_bytes,
                      hipStream_t st);
vqnqs_status grad_logpsi(const ModelDims& m, const void* params,
                         const int8_t* spins, int64_t batch,
                         const double* weights, void* grad, double* logpsi,
                         void* ws, size_t ws_bytes, hipStream_t st);
vqnqs_status autotune(const ModelDims& m, const void* params,
                      const int8_t* spins, int64_t batch, int mode, void* ws,
                      size_t ws_bytes, hipStream_t st, int32_t* choices);
size_t workspace_bytes_multi(const ModelDims* ms, const vqnqs_job* jobs,
                             int njobs, int mode);
vqnqs_status local_energy_multi(const ModelDims* ms, const vqnqs_job* jobs,
                                int njobs, int mode, int flags, void* ws,
                                size_t ws_bytes, hipStream_t st);
vqnqs_status neighbours(const ModelDims& m, const int8_t* spins, int64_t batch,
                        int16_t* bonds, int32_t* count, double* diag, void* ws,
                        size_t ws_bytes, hipStream_t st);

}  // namespace vq
