// C ABI entry points: argument validation (host only, before any HIP call)
// and dispatch to the engine.
#include <cmath>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "profiler.h"

namespace {

bool dims_from(const vqnqs_config* c, vq::ModelDims* m, vqnqs_status* err) {
    if (!c) {
        *err = VQNQS_ERR_NULL_POINTER;
        return false;
    }
    *err = VQNQS_ERR_INVALID_CONFIG;
    if (c->hamiltonian != VQNQS_HEISENBERG_2D && c->hamiltonian != VQNQS_TFIM_1D)
        return false;
    const bool chain = c->hamiltonian == VQNQS_TFIM_1D;
    if (c->L < (chain ? 2 : 1) || c->L > (chain ? 1024 : 32)) return false;
    if (c->periodic != 0 && c->periodic != 1) return false;
    if (c->marshall != 0 && c->marshall != 1) return false;
    if (c->periodic && c->L < 3) return false;              // repeated bonds
    if (c->periodic && c->marshall && (c->L & 1)) return false;  // not bipartite
    if (chain && (c->marshall || !std::isfinite(c->gamma))) return false;
    if (c->attn_tail != 0 && c->attn_tail != 1) return false;
    if (c->encoder != 0 && c->encoder != 1) return false;
    if (c->encoder && c->attn_tail) return false;
    if (!std::isfinite(c->J)) return false;
    if (c->d_model < 1 || c->n_layers < 0 || c->n_heads < 1 || c->d_ff < 1 ||
        c->codebook_size < 1 || c->vq_heads < 1)
        return false;
    if (c->d_model % c->n_heads || c->d_model % c->vq_heads) return false;
    if (c->precision < VQNQS_F64 || c->precision > VQNQS_BF16) return false;
    if (c->flags & ~(VQNQS_FLAG_CERTIFIED_VQ | VQNQS_FLAG_INCREMENTAL_ATTN |
                     VQNQS_INC_LAYERS(255)))
        return false;
    *err = VQNQS_ERR_UNSUPPORTED;
    if (c->encoder && (c->flags & VQNQS_FLAG_INCREMENTAL_ATTN)) return false;
    const int dh = c->d_model / c->n_heads;
    if (dh != 4 && dh != 8 && dh != 16 && dh != 32 && dh != 64) return false;
    if (c->d_model > 512 || c->d_ff > 4096 || c->n_layers > VQNQS_NCOUNTERS - 17 ||
        c->codebook_size > 65536)
        return false;
    const int S = chain ? c->L : c->L * c->L;
    const int K = c->group ? c->group : 1;
    if (K < 1 || K > 4) {
        *err = VQNQS_ERR_INVALID_CONFIG;
        return false;
    }
    if (S % K) {
        *err = VQNQS_ERR_INVALID_CONFIG;
        return false;
    }
    const int N = S / K;
    const size_t act = c->precision == VQNQS_F64 ? 8 : 4;
    if (2 * (size_t)N * dh * act > 128 * 1024) return false;  // attention K/V in LDS
    m->L = c->L;
    m->N = N;
    m->S = S;
    m->K = K;
    m->enc = c->encoder;
    m->d = c->d_model;
    m->nl = c->n_layers;
    m->nh = c->n_heads;
    m->dh = dh;
    m->dff = c->d_ff;
    m->Q = c->codebook_size;
    m->H = c->vq_heads;
    m->dseg = c->d_model / c->vq_heads;
    m->periodic = c->periodic;
    m->marshall = c->marshall;
    m->precision = c->precision;
    m->flags = c->flags;
    m->J = c->J;
    m->chain = chain ? 1 : 0;
    m->tail = c->attn_tail;
    m->gamma = chain ? c->gamma : 0.0;
    m->mfma = 0;
    m->mfma = c->precision == VQNQS_BF16 && vq::mfma_shapes_ok(*m);
    *err = VQNQS_OK;
    return true;
}

}  // namespace

extern "C" {

int64_t vqnqs_param_count(const vqnqs_config* cfg) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return -(int64_t)e;
    return vq::param_count(m);
}

vqnqs_status vqnqs_workspace_size(const vqnqs_config* cfg, int64_t batch,
                                  int32_t mode, int64_t chunk, size_t* bytes) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (!bytes) return VQNQS_ERR_NULL_POINTER;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (mode != VQNQS_PLAIN && mode != VQNQS_DEDUP &&
        mode != VQNQS_WS_FORWARD && mode != VQNQS_WS_GRAD &&
        mode != VQNQS_WS_SAMPLE && mode != VQNQS_WS_VMC)
        return VQNQS_ERR_INVALID_CONFIG;
    if (mode == VQNQS_WS_VMC) {
        // the step's own buffers hold the whole batch; the calls inside
        // it process `chunk` samples at a time
        const int64_t c = chunk <= 0 || chunk > batch ? (batch > 0 ? batch : 1)
                                                      : chunk;
        *bytes = vq::vmc_workspace_bytes(m, batch > 0 ? batch : 1, c);
        return VQNQS_OK;
    }
    if (chunk <= 0 || chunk > batch) chunk = batch > 0 ? batch : 1;
    *bytes = vq::workspace_bytes(m, mode, chunk);
    return VQNQS_OK;
}

vqnqs_status vqnqs_neighbours(const vqnqs_config* cfg, const int8_t* spins,
                              int64_t batch, int16_t* bonds, int32_t* count,
                              double* diag, void* ws, size_t ws_bytes,
                              void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (batch < 0 || batch > ((int64_t)1 << 31) - 1) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!spins || !bonds || !count)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::neighbours(m, spins, batch, bonds, count, diag, ws, ws_bytes,
                          (hipStream_t)stream);
}

vqnqs_status vqnqs_forward_logpsi(const vqnqs_config* cfg, const void* params,
                                  const int8_t* spins, int64_t batch,
                                  double* logpsi, int32_t* codes, void* ws,
                                  size_t ws_bytes, void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!params || !spins || !logpsi)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::forward_logpsi(m, params, spins, batch, logpsi, codes, nullptr,
                              ws, ws_bytes, (hipStream_t)stream);
}

vqnqs_status vqnqs_forward_activations(const vqnqs_config* cfg,
                                       const void* params,
                                       const int8_t* spins, int64_t batch,
                                       double* logpsi, int32_t* codes,
                                       void* attn, void* ws, size_t ws_bytes,
                                       void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!params || !spins || !logpsi || !attn)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::forward_logpsi(m, params, spins, batch, logpsi, codes, attn,
                              ws, ws_bytes, (hipStream_t)stream);
}

vqnqs_status vqnqs_local_energy(const vqnqs_config* cfg, const void* params,
                                const int8_t* spins, int64_t batch,
                                int32_t mode, double* eloc, double* stats,
                                double* ratios, int64_t* counters, void* ws,
                                size_t ws_bytes, void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (mode != VQNQS_PLAIN && mode != VQNQS_DEDUP) return VQNQS_ERR_INVALID_CONFIG;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!params || !spins || !eloc)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::local_energy(m, params, spins, batch, mode, eloc, stats, ratios,
                            counters, ws, ws_bytes, (hipStream_t)stream);
}

vqnqs_status vqnqs_local_energy_static(const vqnqs_config* cfg,
                                       const void* params,
                                       const int8_t* spins, int64_t batch,
                                       int32_t mode, double* eloc,
                                       double* stats, double* ratios,
                                       int64_t* counters, int32_t* status,
                                       void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (mode != VQNQS_PLAIN && mode != VQNQS_DEDUP) return VQNQS_ERR_INVALID_CONFIG;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (batch > 0 && (!params || !spins || !eloc)) return VQNQS_ERR_NULL_POINTER;
    return vq::local_energy_static(m, params, spins, batch, mode, eloc, stats,
                                   ratios, counters, status,
                                   (hipStream_t)stream);
}

vqnqs_status vqnqs_sample(const vqnqs_config* cfg, const void* params,
                          const double* uniforms, int64_t batch,
                          int8_t* spins, double* logpsi, void* ws,
                          size_t ws_bytes, void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (m.enc) return VQNQS_ERR_UNSUPPORTED;     // not autoregressive
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!params || !uniforms || !spins)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::sample(m, params, uniforms, batch, spins, logpsi, ws, ws_bytes,
                      (hipStream_t)stream);
}

vqnqs_status vqnqs_vmc_step(const vqnqs_config* cfg, void* params,
                            void* opt_state, int64_t step, double lr,
                            const double* uniforms, int64_t batch,
                            int8_t* spins, double* eloc, double* stats,
                            void* ws, size_t ws_bytes, void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (m.enc) return VQNQS_ERR_UNSUPPORTED;     // needs direct samples
    if (batch < 1) return VQNQS_ERR_INVALID_SHAPE;
    if (!std::isfinite(lr) || (opt_state && step < 1))
        return VQNQS_ERR_INVALID_CONFIG;
    if (!ws || !params || !uniforms) return VQNQS_ERR_NULL_POINTER;
    return vq::vmc_step(m, params, opt_state, step, lr, uniforms, batch, spins,
                        eloc, stats, ws, ws_bytes, (hipStream_t)stream);
}

vqnqs_status vqnqs_grad_logpsi(const vqnqs_config* cfg, const void* params,
                               const int8_t* spins, int64_t batch,
                               const double* weights, void* grad,
                               double* logpsi, void* ws, size_t ws_bytes,
                               void* stream) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || !grad || (batch > 0 && (!params || !spins)))
        return VQNQS_ERR_NULL_POINTER;
    return vq::grad_logpsi(m, params, spins, batch, weights, grad, logpsi, ws,
                           ws_bytes, (hipStream_t)stream);
}

static vqnqs_status multi_dims(const vqnqs_job* jobs, int32_t njobs,
                               int32_t mode, std::vector<vq::ModelDims>& ms) {
    if (!jobs) return VQNQS_ERR_NULL_POINTER;
    if (njobs < 1 || njobs > 64) return VQNQS_ERR_INVALID_SHAPE;
    if (mode != VQNQS_PLAIN && mode != VQNQS_DEDUP) return VQNQS_ERR_INVALID_CONFIG;
    ms.resize(njobs);
    for (int i = 0; i < njobs; ++i) {
        vqnqs_status e;
        if (!dims_from(&jobs[i].cfg, &ms[i], &e)) return e;
        if (jobs[i].batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    }
    return VQNQS_OK;
}

vqnqs_status vqnqs_workspace_size_multi(const vqnqs_job* jobs, int32_t njobs,
                                        int32_t mode, size_t* bytes) {
    std::vector<vq::ModelDims> ms;
    vqnqs_status e = multi_dims(jobs, njobs, mode, ms);
    if (e) return e;
    if (!bytes) return VQNQS_ERR_NULL_POINTER;
    *bytes = vq::workspace_bytes_multi(ms.data(), jobs, njobs, mode);
    return VQNQS_OK;
}

vqnqs_status vqnqs_local_energy_multi(const vqnqs_job* jobs, int32_t njobs,
                                      int32_t mode, int32_t flags, void* ws,
                                      size_t ws_bytes, void* stream) {
    std::vector<vq::ModelDims> ms;
    vqnqs_status e = multi_dims(jobs, njobs, mode, ms);
    if (e) return e;
    if (flags & ~(VQNQS_MULTI_CONCURRENT | VQNQS_MULTI_GRAPH))
        return VQNQS_ERR_INVALID_CONFIG;
    if (!ws) return VQNQS_ERR_NULL_POINTER;
    for (int i = 0; i < njobs; ++i)
        if (jobs[i].batch > 0 &&
            (!jobs[i].params || !jobs[i].spins || !jobs[i].eloc))
            return VQNQS_ERR_NULL_POINTER;
    return vq::local_energy_multi(ms.data(), jobs, njobs, mode, flags, ws,
                                  ws_bytes, (hipStream_t)stream);
}

vqnqs_status vqnqs_autotune(const vqnqs_config* cfg, const void* params,
                            const int8_t* spins, int64_t batch, int32_t mode,
                            void* ws, size_t ws_bytes, void* stream,
                            int32_t* choices) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (mode != VQNQS_PLAIN && mode != VQNQS_DEDUP) return VQNQS_ERR_INVALID_CONFIG;
    if (batch < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (!ws || (batch > 0 && (!params || !spins))) return VQNQS_ERR_NULL_POINTER;
    return vq::autotune(m, params, spins, batch, mode, ws, ws_bytes,
                        (hipStream_t)stream, choices);
}

vqnqs_status vqnqs_set_tuning(const vqnqs_config* cfg, const int32_t* choices) {
    vq::ModelDims m;
    vqnqs_status e;
    if (!dims_from(cfg, &m, &e)) return e;
    if (!choices) return VQNQS_ERR_NULL_POINTER;
    vq::Tuning t;
    t.qkv_mb = choices[0];
    t.mlp_mb = choices[1];
    t.vq_mb = choices[2];
    if (!vq::tuning_valid(m, t)) return VQNQS_ERR_INVALID_CONFIG;
    vq::tuning_set(m, t);
    return VQNQS_OK;
}

vqnqs_status vqnqs_workspace_status(const void* ws, void* stream) {
    if (!ws) return VQNQS_ERR_NULL_POINTER;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return VQNQS_ERR_HIP;
    int32_t v = 0;
    if (hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
        return VQNQS_ERR_HIP;
    return v ? VQNQS_ERR_BAD_SPIN : VQNQS_OK;
}

void vqnqs_profile_enable(int on) { vq::Profiler::get().enable(on != 0); }

void vqnqs_profile_reset(void) { vq::Profiler::get().reset(); }

int vqnqs_profile_read(char* names, int name_len, double* total_ms,
                       long long* count, int max) {
    if (max < 0 || (names && name_len < 2)) return -1;
    return vq::Profiler::get().read(names, name_len, total_ms, count, max);
}

vqnqs_status vqnqs_probe_exp_rate(float* sink, void* stream,
                                  double* exps_per_s) {
    if (!sink || !exps_per_s) return VQNQS_ERR_NULL_POINTER;
    if (vq::probe_exp_rate(sink, (hipStream_t)stream, exps_per_s) != hipSuccess)
        return VQNQS_ERR_HIP;
    return VQNQS_OK;
}

vqnqs_status vqnqs_probe_gelu(const float* x, float* y, int64_t n,
                              void* stream) {
    if (n < 0) return VQNQS_ERR_INVALID_SHAPE;
    if (n == 0) return VQNQS_OK;
    if (!x || !y) return VQNQS_ERR_NULL_POINTER;
    if (vq::launch_probe_gelu(x, y, n, (hipStream_t)stream) != hipSuccess)
        return VQNQS_ERR_HIP;
    return VQNQS_OK;
}

const char* vqnqs_status_string(vqnqs_status s) {
    switch (s) {
        case VQNQS_OK: return "ok";
        case VQNQS_ERR_NULL_POINTER: return "null pointer";
        case VQNQS_ERR_INVALID_CONFIG: return "invalid config";
        case VQNQS_ERR_INVALID_SHAPE: return "invalid shape";
        case VQNQS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case VQNQS_ERR_UNSUPPORTED: return "unsupported configuration";
        case VQNQS_ERR_BAD_SPIN: return "spin value other than +1/-1";
        case VQNQS_ERR_HIP: return "HIP runtime error";
        case VQNQS_ERR_EXCEEDS_STATIC_SCRATCH:
            return "one sample's workspace exceeds the static scratch";
    }
    return "unknown status";
}

}  // extern "C"
