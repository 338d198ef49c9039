// BF16 matrix-core kernels (gfx950 v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the per-location products of the VQ transformer
// (paper Sec. 3.1): LN1 + QKV projection, the fused output-projection /
// residual / MLP block, and the codebook distance search of the quantizer
// (eqs. 4-6).
//
// Weights are bfloat16 (the BF16 mode evaluates the network at the
// bfloat16-rounded parameters, so they are exact).  Activations are kept in
// FP32 and enter the matrix core as a pair hi + lo of bfloat16 values
// (hi = bf16(x), lo = bf16(x - hi)), i.e. two MFMA passes into one FP32
// accumulator; this keeps ~16 significant bits of every activation.
//
// Operand layout of the 16x16x32 MFMA (wave64): lane l holds
//   A[l % 16][8*(l/16) + j], B[8*(l/16) + j][l % 16]  (j = 0..7), and
//   D[4*(l/16) + r][l % 16]                            (r = 0..3).
// Weight matrices W[K][Nout] are packed once per call into fragments
// frag(nb, kb) = 64 lanes x 8 bf16, stored contiguously so one fragment is
// one 16-byte load per lane.
#include <map>
#include <mutex>

#include "kernels.h"

namespace vq {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kMT = 256;          // threads per workgroup (4 waves)
constexpr int kMGridCap = 8192;

static inline unsigned mgrid(int64_t units) {
    if (units <= 0) return 1;
    return (unsigned)(units < kMGridCap ? units : kMGridCap);
}

__device__ inline int64_t rs_n(const RowSet& r) {
    return r.n_dev ? (int64_t)(*r.n_dev) * r.mult : r.n_host;
}
__device__ inline int64_t rs_slot(const RowSet& r, int64_t k) {
    return r.idx ? r.idx[k] : k;
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline void split1(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}
// split1 of two values with paired conversions (the same per-value result).
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
__device__ inline void split2(float a, float b, bf16x2& hi, bf16x2& lo) {
    hi = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const f32x2 back = __builtin_convertvector(hi, f32x2);
    lo = __builtin_convertvector(f32x2{a - back[0], b - back[1]}, bf16x2);
}

// ---------------------------------------------------------------- packing
// out[((nb*KB + kb)*64 + l)*8 + j] = W[kb*32 + kk(8*(l/16) + j)][nb*16 + l%16]
// with W[k][c] read at src[k*sk + c*sc] (K x Nout logical matrix).  kk is
// the identity, or with hperm the order in which a transposed product leaves
// 32 rows in a lane's A fragment: 8g + j holds row 4g + j for j < 4 and row
// 16 + 4g + (j - 4) otherwise (the 4 rows of each of two 16-row blocks).
__global__ void k_pack_b(const float* __restrict__ src, int K, int Nout,
                         int64_t sk, int64_t sc, int hperm,
                         __bf16* __restrict__ out) {
    const int64_t total = (int64_t)K * Nout;
    const int KB = K / 32;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e & 7);
        const int l = (int)((e >> 3) & 63);
        const int64_t f = e >> 9;             // fragment id nb*KB + kb
        const int kb = (int)(f % KB);
        const int nb = (int)(f / KB);
        const int g = l >> 4;
        const int k = kb * 32 + (hperm ? (j < 4 ? 4 * g + j : 12 + 4 * g + j)
                                       : 8 * g + j);
        const int c = nb * 16 + (l & 15);
        out[e] = (__bf16)src[k * sk + (int64_t)c * sc];
    }
}

// BF16 mode: every parameter rounded to bfloat16 (kept as FP32 values).
__global__ void k_round_bf16(const float* __restrict__ src, int64_t n,
                             float* __restrict__ dst) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = (float)(__bf16)src[e];
}

hipError_t launch_round_bf16(const float* src, int64_t n, float* dst,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_round_bf16, dim3(mgrid((n + 255) / 256)), dim3(256),
                       0, st, src, n, dst);
    return hipGetLastError();
}

// out[e] = -cnorm[e]/2 (exact: halving a normal float), the quantizer
// search's accumulator input.
__global__ void k_pack_cnorm(const float* __restrict__ cnorm, int64_t n,
                             float* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = -0.5f * cnorm[e];
}

hipError_t launch_pack_layer(const ModelDims& m, const LayerW<float>& w,
                             bf16* Wqkv_p, bf16* W1_p, bf16* W2_p, bf16* cb_p,
                             float* cnh, hipStream_t st) {
    const int d = m.d, F = m.dff;
    auto go = [&](const float* src, int K, int Nout, int64_t sk, int64_t sc,
                  bf16* out, int hperm = 0) {
        const int64_t total = (int64_t)K * Nout;
        hipLaunchKernelGGL(k_pack_b, dim3(mgrid((total + 255) / 256)),
                           dim3(256), 0, st, src, K, Nout, sk, sc, hperm,
                           reinterpret_cast<__bf16*>(out));
    };
    go(w.W_qkv, d, 3 * d, 3 * d, 1, Wqkv_p);
    go(w.W1, d, F, F, 1, W1_p);
    go(w.W2, F, d, d, 1, W2_p, 1);    // rows in the hidden layer's lane order
    // codebook head h as B[k][c] = cb[h][c][k]
    for (int h = 0; h < m.H; ++h)
        go(w.codebook + (int64_t)h * m.Q * m.dseg, m.dseg, m.Q, 1, m.dseg,
           cb_p + (int64_t)h * m.Q * m.dseg);
    const int64_t nc = (int64_t)m.H * m.Q;
    hipLaunchKernelGGL(k_pack_cnorm, dim3(mgrid((nc + 255) / 256)), dim3(256),
                       0, st, w.cnorm, nc, cnh);
    return hipGetLastError();
}

hipError_t launch_pack_qkv(const ModelDims& m, const float* W_qkv, bf16* out,
                           hipStream_t st) {
    const int d = m.d;
    const int64_t total = (int64_t)d * 3 * d;
    hipLaunchKernelGGL(k_pack_b, dim3(mgrid((total + 255) / 256)), dim3(256),
                       0, st, W_qkv, d, 3 * d, (int64_t)3 * d, (int64_t)1, 0,
                       reinterpret_cast<__bf16*>(out));
    return hipGetLastError();
}

bool mfma_shapes_ok(const ModelDims& m) {
    const int KB = m.d / 32;
    return m.d % 32 == 0 && m.dff % 32 == 0 && m.dseg % 32 == 0 &&
           m.Q % 16 == 0 && (KB == 2 || KB == 4 || KB == 8) &&
           (m.dff == 4 * m.d) && (m.dseg / 32 == 1 || m.dseg / 32 == 2 ||
                                  m.dseg / 32 == 4 || m.dseg / 32 == 8);
}

// ------------------------------------------------------------- LN stats
__device__ inline void row_ln(const float* x, int d, float& mean, float& rstd) {
    const int lane = threadIdx.x & 63;
    float s = 0;
    for (int k = lane; k < d; k += 64) s += x[k];
    mean = wave_sum(s) / (float)d;
    float v = 0;
    for (int k = lane; k < d; k += 64) {
        const float t = x[k] - mean;
        v += t * t;
    }
    v = wave_sum(v) / (float)d;
    rstd = 1.0f / sqrtf(v + 1e-5f);
}

// A fragment (rows mb*16.., k-block kb) from a row-major LDS tile.
__device__ inline bf16x8 lds_frag(const __bf16* base, int ld, int mb, int kb,
                                  int lane) {
    return *reinterpret_cast<const bf16x8*>(
        base + (mb * 16 + (lane & 15)) * ld + kb * 32 + 8 * (lane >> 4));
}

// ------------------------------------------------- per-wave A fragments
// A fragments (hi/lo) of 16*MB rows x D = 32*KB columns held by one wave:
// lane l holds row i*16 + l%16, columns kb*32 + 8*(l/16) + j.  The row's
// LayerNorm statistics combine the four lanes sharing the row.
template <int KB, int MB>
__device__ inline void ln_frags(const float* const (&xr)[MB], const float* g,
                                const float* b, bf16x8 (&ah)[MB][KB],
                                bf16x8 (&al)[MB][KB]) {
    constexpr int D = KB * 32;
    const int lane = threadIdx.x & 63, gq = lane >> 4;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        float v[KB][8];
        float s = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            if (xr[i]) {
                const float4* p = reinterpret_cast<const float4*>(xr[i] + kb * 32 + 8 * gq);
                const float4 v0 = p[0], v1 = p[1];
                v[kb][0] = v0.x; v[kb][1] = v0.y; v[kb][2] = v0.z; v[kb][3] = v0.w;
                v[kb][4] = v1.x; v[kb][5] = v1.y; v[kb][6] = v1.z; v[kb][7] = v1.w;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[kb][j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[kb][j];
        }
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        const float mean = s / (float)D;
        float q = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float t = v[kb][j] - mean;
                q += t * t;
            }
        q += __shfl_xor(q, 16, 64);
        q += __shfl_xor(q, 32, 64);
        const float rstd = 1.0f / sqrtf(q / (float)D + 1e-5f);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb * 32 + 8 * gq + j;
                const float y = (v[kb][j] - mean) * rstd * g[k] + b[k];
                __bf16 h, l;
                split1(y, h, l);
                ah[i][kb][j] = h;
                al[i][kb][j] = l;
            }
    }
}

// Same as ln_frags for row values already in registers (A positions).
template <int KB, int MB>
__device__ inline void ln_frags_v(const float (&v)[MB][KB][8], const float* g,
                                  const float* b, bf16x8 (&ah)[MB][KB],
                                  bf16x8 (&al)[MB][KB]) {
    constexpr int D = KB * 32;
    const int gq = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[i][kb][j];
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        const float mean = s / (float)D;
        float q = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float t = v[i][kb][j] - mean;
                q += t * t;
            }
        q += __shfl_xor(q, 16, 64);
        q += __shfl_xor(q, 32, 64);
        const float rstd = 1.0f / sqrtf(q / (float)D + 1e-5f);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb * 32 + 8 * gq + j;
                const float y = (v[i][kb][j] - mean) * rstd * g[k] + b[k];
                __bf16 h, l;
                split1(y, h, l);
                ah[i][kb][j] = h;
                al[i][kb][j] = l;
            }
    }
}

// Cooperative copy of `cnt` fragment lanes (16 B each) into an LDS stage.
// The loads are unconditional (indices past cnt are clamped to the last
// lane; those entries are never used), so nothing consumes a loaded value
// before the stage is stored: the loads stay in flight over the caller's
// work between fetch and store.
template <int PER>
__device__ inline void stage_fetch(bf16x8 (&pre)[PER], const bf16x8* src,
                                   int64_t cnt) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t e = threadIdx.x + k * kMT;
        pre[k] = src[e < cnt ? e : cnt - 1];
    }
}
template <int PER>
__device__ inline void stage_store(const bf16x8 (&pre)[PER], bf16x8* dst) {
#pragma unroll
    for (int k = 0; k < PER; ++k) dst[threadIdx.x + k * kMT] = pre[k];
}

// Global-to-LDS loads (gfx950): lane l's 16 (4) bytes at gsrc land at
// lds + 16 l (4 l); lds is the wave's base address, the same in every lane.
// They complete in order with the vector memory loads (vmcnt).
__device__ inline void lds_dma16(const void* gsrc, void* lds) {
    __builtin_amdgcn_global_load_lds(
        gsrc, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
__device__ inline void lds_dma4(const void* gsrc, void* lds) {
    __builtin_amdgcn_global_load_lds(
        gsrc, (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}
// s_waitcnt vmcnt(0): this wave's vector memory loads, global-to-LDS loads
// included, have completed (expcnt and lgkmcnt left at their maxima).
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// s_waitcnt lgkmcnt(0) alone (vector memory loads stay in flight).
__device__ inline void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// --------------------------------------------------------------- LN1 + QKV
// Each wave: 16*MB rows (LN1 output as register A fragments).  The 3d/16
// output column blocks stream through two LDS stages, NBC blocks (64
// columns) per chunk with their biases, shared by the four waves and filled
// like the VQ search's: global-to-LDS loads one chunk ahead (the next tile's
// first chunk after the last), a wait for them and a barrier at each chunk
// start.  A chunk's outputs stay in registers and are stored after the next
// chunk's loads have been issued, so that wait never covers fresh stores.
// With one row tile per wave up to d = 128 the kernel fits 168 VGPRs (a few
// spills at tile level), which allows three waves per SIMD.
template <int KB, int MB>
__global__ void __launch_bounds__(kMT)
    __attribute__((amdgpu_waves_per_eu(MB == 1 && KB <= 4 ? 3 : 1)))
    k_qkv_mfma(ModelDims m, LayerW<float> w, RowSet rows,
               BlockIO<PrecBF16> io, const bf16x8* __restrict__ Bp) {
    constexpr int D = KB * 32, WR = MB * 16, NBC = 4;
    constexpr int CHUNK = NBC * KB * 64, PER = CHUNK / kMT;
    constexpr int NBT = 3 * D / 16;
    constexpr int nchunk = NBT / NBC;
    static_assert(NBT % NBC == 0, "whole chunks");
    __shared__ bf16x8 stage0[CHUNK], stage1[CHUNK];
    __shared__ float bias0[NBC * 16], bias1[NBC * 16];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gq = lane >> 4, c16 = lane & 15;
    const int64_t n = rs_n(rows);
    const int64_t ntile = (n + 4 * WR - 1) / (4 * WR);
    auto fetch = [&](int c, bf16x8* st, float* bs) {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            lds_dma16(Bp + (int64_t)c * CHUNK + threadIdx.x + k * kMT,
                      st + wave * 64 + k * kMT);
        if (wave == 0) lds_dma4(w.b_qkv + c * NBC * 16 + lane, bs);
    };
    bool ahead = false;      // the tile's first chunk is in stage0
    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        int64_t slot[MB];
        const float* xr[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int64_t r = t * 4 * WR + wave * WR + i * 16 + c16;
            slot[i] = r < n ? rs_slot(rows, r) : -1;
            xr[i] = slot[i] >= 0 ? io.x + slot[i] * D : nullptr;
        }
        bf16x8 ah[MB][KB], al[MB][KB];
        ln_frags<KB, MB>(xr, w.ln1_g, w.ln1_b, ah, al);
        int64_t oslot[MB][4];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) oslot[i][r] = __shfl(slot[i], 4 * gq + r, 64);
        if (!ahead) {
            __syncthreads();                 // both stages free
            fetch(0, stage0, bias0);
        }
        float ov[MB][NBC][4];                // outputs of the pending chunk
        auto flush = [&](int c) {
#pragma unroll
            for (int nbl = 0; nbl < NBC; ++nbl) {
                const int col = (c * NBC + nbl) * 16 + c16;
                float* dst = col < D ? io.q : (col < 2 * D ? io.k : io.v);
                const int cc = col < D ? col : (col < 2 * D ? col - D : col - 2 * D);
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (oslot[i][r] >= 0) dst[oslot[i][r] * D + cc] = ov[i][nbl][r];
            }
        };
        auto chunk = [&](int c, const bf16x8* sb, const float* bs, bf16x8* nsb,
                         float* nbs, bool into0) {
            wait_vmem();
            __syncthreads();
            if (c + 1 < nchunk) {
                fetch(c + 1, nsb, nbs);
            } else {
                ahead = into0 && t + gridDim.x < ntile;
                if (ahead) fetch(0, nsb, nbs);
            }
            if (c > 0) flush(c - 1);
#pragma unroll
            for (int nbl = 0; nbl < NBC; ++nbl) {
                f32x4 acc[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) acc[i] = f32x4{0, 0, 0, 0};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const bf16x8 b = sb[(nbl * KB + kb) * 64 + lane];
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        acc[i] = mfma(ah[i][kb], b, acc[i]);
                        acc[i] = mfma(al[i][kb], b, acc[i]);
                    }
                }
                const float bias = bs[nbl * 16 + c16];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ov[i][nbl][r] = acc[i][r] + bias;
            }
        };
        // the two stages are distinct arrays named statically in each copy
        // of the chunk body (see k_vq_mfma)
        for (int c = 0; c < nchunk; c += 2) {
            chunk(c, stage0, bias0, stage1, bias1, false);
            if (c + 1 < nchunk) chunk(c + 1, stage1, bias1, stage0, bias0, true);
        }
        flush(nchunk - 1);
    }
}

// ------------------------------------------ out-projection + residual + MLP
// Each wave: 16*MB rows.  x' = x_in + b_o + sum_h table[h][code_h] is formed
// in the A-fragment layout, written to the output rows, and LN2(x') kept as
// register fragments.  The hidden layer is produced 64 columns at a time and
// transposed: with the W1 fragments as the left operand and the LN2 rows as
// the right one the matrix core returns H^T, so a lane holds 4 consecutive
// hidden units of one row of each 16-unit block.  Two such blocks, GELU'd
// and split, are directly a lane's A fragment of the second product (the W2
// rows are packed in that order), with no transposition through memory.
// The W1/W2 fragments of a chunk are staged in LDS for the four waves.
// GELU with erf from Abramowitz & Stegun 7.1.26 (absolute error of erf at
// most 1.5e-7): with y = |x|/sqrt(2), t = 1/(1 + p y) and
// (a1 t + ... + a5 t^5) exp(-y^2) ~ erfc(y).  The constants are folded:
// t = 1/(1 + (p/sqrt 2)|x|), the coefficients are halved so that
// q = (a1/2 t + ... + a5/2 t^5) 2^(-(log2 e)/2 x^2) ~ erfc(y)/2 = Phi(-|x|),
// and GELU(x) = x Phi(x) = max(x, 0) - |x| q: x q for x < 0 (no
// cancellation) and x - x q otherwise, one FMA either way.  Branch-free.
__device__ inline float gelu_as(float x) {
    const float ax = __builtin_fabsf(x);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(ax, 0.231641888f, 1.0f));
    const float poly =
        t * (0.127414796f +
             t * (-0.142248368f +
                  t * (0.710706871f + t * (-0.726576014f + t * 0.530702714f))));
    const float q = poly * __builtin_amdgcn_exp2f(x * x * -0.72134752044448169f);
    return __builtin_fmaf(-ax, q, __builtin_elementwise_maximum(x, 0.0f));
}

__global__ void k_probe_gelu(const float* __restrict__ x, float* __restrict__ y,
                             int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = gelu_as(x[i]);
}

hipError_t launch_probe_gelu(const float* x, float* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_probe_gelu, dim3(mgrid((n + 255) / 256)), dim3(256), 0, st,
                       x, y, n);
    return hipGetLastError();
}

template <int KB1, int MB>
__global__ void __launch_bounds__(kMT) __attribute__((amdgpu_waves_per_eu(2))) k_mlp_mfma(ModelDims m, LayerW<float> w,
                                                 RowSet rows, BlockIO<PrecBF16> io,
                                                 const bf16x8* __restrict__ B1,
                                                 const bf16x8* __restrict__ B2) {
    constexpr int D = KB1 * 32, F = 4 * D, KB2 = F / 32;
    constexpr int WR = MB * 16, HC = 64, NB1C = HC / 16, KB2C = HC / 32;
    constexpr int NBO = D / 16;                    // output column blocks
    constexpr int C1 = NB1C * KB1 * 64;            // W1 fragment lanes per chunk
    constexpr int C2 = KB2C * NBO * 64;            // W2 fragment lanes per chunk
    constexpr int PER1 = C1 / kMT, PER2 = C2 / kMT;
    __shared__ bf16x8 s1[C1];
    __shared__ bf16x8 s2[C2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gq = lane >> 4, c16 = lane & 15;
    const int64_t n = rs_n(rows);
    const int64_t ntile = (n + 4 * WR - 1) / (4 * WR);
    // W1 columns and W2 rows of one hidden chunk, fetched into registers
    bf16x8 p1[PER1], p2[PER2];
    auto fetch_w = [&](int hc) {
        stage_fetch<PER1>(p1, B1 + (int64_t)hc * C1, C1);
        // W2 rows of the chunk: k-blocks hc*KB2C .. +KB2C of every output
        // block nb; packed index (nb*KB2 + kb)*64 + lane
#pragma unroll
        for (int k = 0; k < PER2; ++k) {
            const int e = threadIdx.x + k * kMT;
            const int ln = e & 63, f = e >> 6;
            const int kbl = f % KB2C, nb = f / KB2C;
            p2[k] = B2[((int64_t)nb * KB2 + hc * KB2C + kbl) * 64 + ln];
        }
    };
    fetch_w(0);
    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        int64_t slot[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int64_t r = t * 4 * WR + wave * WR + i * 16 + c16;
            slot[i] = r < n ? rs_slot(rows, r) : -1;
        }
        // x' = x_in + (b_o + sum_h table) in A-fragment positions, kept in
        // registers (never written and re-read through global memory).  A
        // lane's 8 columns per k-block are contiguous: 16-byte loads, all of
        // one quantizer head issued together, the next head's code loading
        // meanwhile (one round trip per head, not one per element).
        float xv[MB][KB1][8];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const bool live = slot[i] >= 0;
            const int64_t sl = live ? slot[i] : 0;
            const float* x = io.x_in + sl * D;
            const int32_t* cd = io.codes + sl * m.H;
            float z[KB1][8], xin[KB1][8];
            int cnext = live ? cd[0] : 0;
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int k = kb * 32 + 8 * gq + 4 * h2;
                    const float4 xa = *reinterpret_cast<const float4*>(x + k);
                    const float4 ba = *reinterpret_cast<const float4*>(w.b_o + k);
                    xin[kb][4 * h2 + 0] = xa.x; xin[kb][4 * h2 + 1] = xa.y;
                    xin[kb][4 * h2 + 2] = xa.z; xin[kb][4 * h2 + 3] = xa.w;
                    z[kb][4 * h2 + 0] = ba.x; z[kb][4 * h2 + 1] = ba.y;
                    z[kb][4 * h2 + 2] = ba.z; z[kb][4 * h2 + 3] = ba.w;
                }
            for (int hq = 0; hq < m.H; ++hq) {
                const int c = cnext;
                if (hq + 1 < m.H) cnext = live ? cd[hq + 1] : 0;
                const float* tr = w.table + ((int64_t)hq * m.Q + c) * D;
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int k = kb * 32 + 8 * gq + 4 * h2;
                        const float4 ta = *reinterpret_cast<const float4*>(tr + k);
                        z[kb][4 * h2 + 0] += ta.x; z[kb][4 * h2 + 1] += ta.y;
                        z[kb][4 * h2 + 2] += ta.z; z[kb][4 * h2 + 3] += ta.w;
                    }
            }
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    xv[i][kb][j] = live ? xin[kb][j] + z[kb][j] : 0.0f;
        }
        bf16x8 ah[MB][KB1], al[MB][KB1];
        ln_frags_v<KB1, MB>(xv, w.ln2_g, w.ln2_b, ah, al);
        f32x4 out[MB][NBO];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int nb = 0; nb < NBO; ++nb) out[i][nb] = f32x4{0, 0, 0, 0};
        for (int hc = 0; hc < F / HC; ++hc) {
            __syncthreads();                       // stages free
            stage_store<PER1>(p1, s1);
            stage_store<PER2>(p2, s2);
            __syncthreads();
            // the next chunk's weights (chunk 0 again after the last: the
            // next tile's) load while this chunk is computed
            fetch_w(hc + 1 < F / HC ? hc + 1 : 0);
            // hidden chunk transposed: H^T = W1[:, chunk]^T LN2(x')^T; the K
            // loop is outermost so the NB1C accumulators are independent
            // MFMA chains
            f32x4 hacc[MB][NB1C];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int nb = 0; nb < NB1C; ++nb) hacc[i][nb] = f32x4{0, 0, 0, 0};
            // a k-block's W1 fragments are read from LDS while the previous
            // k-block is multiplied
            bf16x8 w1f[2][NB1C];
#pragma unroll
            for (int nb = 0; nb < NB1C; ++nb) w1f[0][nb] = s1[nb * KB1 * 64 + lane];
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) {
                if (kb + 1 < KB1) {
#pragma unroll
                    for (int nb = 0; nb < NB1C; ++nb)
                        w1f[(kb + 1) & 1][nb] = s1[(nb * KB1 + kb + 1) * 64 + lane];
                }
#pragma unroll
                for (int nb = 0; nb < NB1C; ++nb) {
                    const bf16x8 b = w1f[kb & 1][nb];
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        hacc[i][nb] = mfma(b, ah[i][kb], hacc[i][nb]);
                        hacc[i][nb] = mfma(b, al[i][kb], hacc[i][nb]);
                    }
                }
            }
            // GELU(. + b1) of hidden units nb*16 + 4 gq + r of row c16, split
            // hi/lo: blocks 2 kb and 2 kb + 1 form the A fragment of k-block kb
#pragma unroll
            for (int kb = 0; kb < KB2C; ++kb) {
                bf16x8 xh[MB], xl[MB];
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int nb = 2 * kb + half;
                    const float4 bq = *reinterpret_cast<const float4*>(
                        w.b1 + hc * HC + nb * 16 + 4 * gq);
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        bf16x2 h01, l01, h23, l23;
                        split2(gelu_as(hacc[i][nb][0] + bq.x),
                               gelu_as(hacc[i][nb][1] + bq.y), h01, l01);
                        split2(gelu_as(hacc[i][nb][2] + bq.z),
                               gelu_as(hacc[i][nb][3] + bq.w), h23, l23);
                        xh[i][4 * half + 0] = h01[0];
                        xh[i][4 * half + 1] = h01[1];
                        xh[i][4 * half + 2] = h23[0];
                        xh[i][4 * half + 3] = h23[1];
                        xl[i][4 * half + 0] = l01[0];
                        xl[i][4 * half + 1] = l01[1];
                        xl[i][4 * half + 2] = l23[0];
                        xl[i][4 * half + 3] = l23[1];
                    }
                }
#pragma unroll
                for (int nb = 0; nb < NBO; ++nb) {
                    const bf16x8 b = s2[(nb * KB2C + kb) * 64 + lane];
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        out[i][nb] = mfma(xh[i], b, out[i][nb]);
                        out[i][nb] = mfma(xl[i], b, out[i][nb]);
                    }
                }
            }
        }
        // x = x' + hidden W2 + b2, with x' recomputed for this lane's
        // elements in the prologue's addition order: every element is read
        // and written by one lane only, also when x_in and x coincide.  All
        // loads of a fragment's four rows are issued before its first store.
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            int64_t s4[4];
            bool v4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t sr = __shfl(slot[i], 4 * gq + r, 64);
                v4[r] = sr >= 0;
                s4[r] = v4[r] ? sr : 0;
            }
            float z[4][NBO], xin[4][NBO], b2v[NBO];
            int cn[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) cn[r] = v4[r] ? io.codes[s4[r] * m.H] : 0;
#pragma unroll
            for (int nb = 0; nb < NBO; ++nb) {
                const int col = nb * 16 + c16;
                const float bo = w.b_o[col];
                b2v[nb] = w.b2[col];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    z[r][nb] = bo;
                    xin[r][nb] = io.x_in[s4[r] * D + col];
                }
            }
            for (int hq = 0; hq < m.H; ++hq) {
                int c[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    c[r] = cn[r];
                    if (hq + 1 < m.H) cn[r] = v4[r] ? io.codes[s4[r] * m.H + hq + 1] : 0;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float* tr = w.table + ((int64_t)hq * m.Q + c[r]) * D;
#pragma unroll
                    for (int nb = 0; nb < NBO; ++nb) z[r][nb] += tr[nb * 16 + c16];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!v4[r]) continue;
                float* xo = io.x + s4[r] * D;
#pragma unroll
                for (int nb = 0; nb < NBO; ++nb) {
                    const float xp = xin[r][nb] + z[r][nb];
                    xo[nb * 16 + c16] = xp + (out[i][nb][r] + b2v[nb]);
                }
            }
        }
    }
}

// --------------------------------------------------------------- VQ search
// Running best / second-best (value, code) of g = a.w - |w|^2/2, which the
// nearest code maximises; equal values go to the lower code.
struct T2 {
    float b;
    int i;
    float s;
};
__device__ inline T2 t2_merge(T2 x, T2 y) {
    T2 r;
    if (y.b > x.b || (y.b == x.b && y.i < x.i)) {
        r.b = y.b;
        r.i = y.i;
        r.s = x.b > y.s ? x.b : y.s;
    } else {
        r.b = x.b;
        r.i = x.i;
        r.s = y.b > x.s ? y.b : x.s;
    }
    return r;
}

// Bound on the error of a computed score |w|^2 - 2 (hi + lo).w = -2 g for a
// row of norm na (g an FP32 sum, in any order, of n exact products and the
// exact -|w|^2/2), plus the representation error |a - (hi + lo)| <= 2^-16 |a|
// in both the product and the row norm that turns scores into distances.
__device__ inline float score_err_split(int n, float na, float wmax) {
    const float g = (float)(n + 4) * 5.9604645e-8f * 1.0625f;
    return g * (2.0f * na * wmax + wmax * wmax + na * na) +
           3.0517578e-5f * (na * wmax + na * na);
}

// Each wave owns 16*MB rows kept in registers as hi/lo fragments; the four
// waves of a workgroup stream the codes of the quantizer head through a
// double-buffered LDS stage (CBK code blocks of 16 codes per chunk, with
// -|w|^2/2 of every code: the accumulator input of the code's products, so
// the matrix core returns g = a.w - |w|^2/2 and the search only compares).
// The stages are filled by global-to-LDS loads (no registers, no store
// instructions), issued one chunk ahead: the next chunk of the head, or
// after a head's last chunk the first chunk of the next head (or of the
// next tile's first head) when the chunk count is even.  A chunk starts with
// this wave's loads complete and a barrier, after which every wave has also
// finished reading the other stage, which then takes the next chunk.  For
// a large codebook, eight code blocks per chunk (two workgroups per CU by
// LDS) took 10% less time than four (three per CU): the per-chunk wait and
// barrier cost more than the third workgroup hides.
// Every codebook fragment read from LDS feeds MB MFMAs, and MB more when
// the block gets its lo products.  The second-best value (for the
// certified-reuse margins) is tracked only when MARGIN, which searches
// every block in full; the chosen code is the same either way.
template <int KBS, int MB, bool MARGIN, int CBK, bool SEED>
__global__ void __launch_bounds__(kMT)
    __attribute__((amdgpu_waves_per_eu(MB <= 2 && !MARGIN ? 3 : 1)))
    k_vq_mfma(ModelDims m, LayerW<float> w, RowSet rows, BlockIO<PrecBF16> io,
              const bf16x8* __restrict__ cbp, VqSeed seed) {
    constexpr int DS = KBS * 32, WR = MB * 16;
    constexpr int CHUNK = CBK * KBS * 64;       // fragment lanes per chunk
    constexpr int PER = CHUNK / kMT;             // per thread
    constexpr int CN = CBK * 16;                 // code norms per chunk
    static_assert(CN % 64 == 0 && CN <= 256, "waves 0.. load a chunk's code norms");
    __shared__ bf16x8 stage0[CHUNK], stage1[CHUNK];
    __shared__ __align__(16) float cn0[CN], cn1[CN];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t n = rs_n(rows);
    const int64_t ntile = (n + 4 * WR - 1) / (4 * WR);
    const int QB = m.Q / 16;
    const int64_t cbtot = (int64_t)QB * KBS * 64;
    const int nchunk = (QB + CBK - 1) / CBK;
    const float inf = __builtin_inff();
    // chunk c of head hq into (st, cs): clamped addresses (entries past the
    // codebook are never read)
    auto fetch = [&](int hq, int c, bf16x8* st, float* cs) {
        const bf16x8* cbh = cbp + (int64_t)hq * cbtot;
        const int64_t e0 = (int64_t)c * CHUNK;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t e = e0 + threadIdx.x + k * kMT;
            lds_dma16(cbh + (e < cbtot ? e : cbtot - 1), st + wave * 64 + k * kMT);
        }
        if (wave < CN / 64) {
            const int code = c * CN + wave * 64 + lane;
            lds_dma4(w.cnh + (int64_t)hq * m.Q + (code < m.Q ? code : m.Q - 1),
                     cs + wave * 64);
        }
    };
    bool ahead = false;      // this head's first chunk is in stage0
    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        int64_t myslot[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int64_t r = t * 4 * WR + wave * WR + i * 16 + (lane & 15);
            myslot[i] = r < n ? rs_slot(rows, r) : -1;
        }
        for (int hq = 0; hq < m.H; ++hq) {
            bf16x8 ah[MB][KBS], al[MB][KBS];
            float nrm[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                float ss = 0.0f;
#pragma unroll
                for (int kb = 0; kb < KBS; ++kb) {
                    float v[8];
                    if (myslot[i] >= 0) {
                        const float4* p = reinterpret_cast<const float4*>(
                            io.a + myslot[i] * m.d + hq * DS + kb * 32 + 8 * (lane >> 4));
                        const float4 v0 = p[0], v1 = p[1];
                        v[0] = v0.x; v[1] = v0.y; v[2] = v0.z; v[3] = v0.w;
                        v[4] = v1.x; v[5] = v1.y; v[6] = v1.z; v[7] = v1.w;
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j) v[j] = 0.0f;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        __bf16 h, l;
                        split1(v[j], h, l);
                        ah[i][kb][j] = h;
                        al[i][kb][j] = l;
                        ss += v[j] * v[j];
                    }
                }
                ss += __shfl_xor(ss, 16, 64);
                ss += __shfl_xor(ss, 32, 64);
                nrm[i] = ss;                // |a|^2 of row i*16 + lane%16
            }
            // Seeded rows (a neighbour's row, whose sample has a code c0 for
            // the same row): with g0 = g(c0) from the vector unit, every
            // product of a code x lies within lo = 2^-8 |a| wmax of its hi
            // part alone (|a_lo| <= 2^-8 |a| per element after rounding to
            // nearest), and each FP32 sum within E of its real value.  So a
            // code whose hi-only value stays below g0 - lo - 4E has
            // g(x) < g(c0) and is not the nearest; a code block in which that
            // holds for every row of the wave skips its lo products and the
            // bookkeeping.  c0's own block always passes, so the chosen code
            // (the argmax of the same hi-then-lo sums, lowest index on equal
            // values) is the one the full search finds.  Unseeded: -inf.
            float ut[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i) ut[i] = -inf;
            if constexpr (SEED) {
                const float wmx = w.cnorm[(int64_t)m.H * m.Q + hq];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    float gp = 0.0f, cq0 = 0.0f;
                    const bool sd = seed.slot_nb != nullptr && myslot[i] >= 0;
                    if (sd) {
                        const int64_t sl = myslot[i];
                        const NbDesc D = seed.desc[seed.slot_nb[sl]];
                        const int row = first_row(D, m) + (int)(sl - D.ov);
                        const int c0 = seed.bcode[((int64_t)D.sigma * m.N + row) * m.H + hq];
                        const float* wc = w.codebook + ((int64_t)hq * m.Q + c0) * DS +
                                          8 * (lane >> 4);
                        cq0 = -0.5f * w.cnorm[(int64_t)hq * m.Q + c0];
#pragma unroll
                        for (int kb = 0; kb < KBS; ++kb) {
                            const float4 w0 = *reinterpret_cast<const float4*>(wc + kb * 32);
                            const float4 w1 = *reinterpret_cast<const float4*>(wc + kb * 32 + 4);
                            const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
                            for (int j = 0; j < 8; ++j)
                                gp = fmaf((float)ah[i][kb][j] + (float)al[i][kb][j], wv[j], gp);
                        }
                    }
                    gp += __shfl_xor(gp, 16, 64);
                    gp += __shfl_xor(gp, 32, 64);
                    float u = -inf;
                    if (sd) {
                        const float na = 1.001f * sqrtf(nrm[i]);
                        const float E = (float)(2 * DS + 8) * 5.9604645e-8f * 1.0625f *
                                        (0.5f * wmx * wmx + 1.01f * na * wmx);
                        const float lo = 3.90625e-3f * 1.004f * na * wmx;
                        u = (cq0 + gp) - lo - 4.0f * E;
                    }
                    ut[i] = u;
                }
            }
            // this lane's row i*16 + lane%16 against codes 4g..4g+3 of each
            // 16-code block (g = lane/16): the products are formed as
            // W A^T, so a lane's four results are one row's
            T2 best[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i) best[i] = T2{-inf, 0, -inf};
            if (!ahead) {
                // the first chunk was not fetched ahead (start, or odd
                // chunk count): both stages are free after the barrier
                __syncthreads();
                fetch(hq, 0, stage0, cn0);
            }
            // chunk c from (sb, cs), the next one into (nsb, ncs).  A head's
            // last chunk fetches the next head's first one (the next tile's
            // first head after the last) into stage0 when it reads stage1.
            auto chunk = [&](int c, const bf16x8* sb, const float* cs,
                             bf16x8* nsb, float* ncs, bool into0) {
                wait_vmem();
                __syncthreads();
                // in flight during this chunk's search
                if (c + 1 < nchunk) {
                    fetch(hq, c + 1, nsb, ncs);
                } else {
                    ahead = into0 && (hq + 1 < m.H || t + gridDim.x < ntile);
                    if (ahead) fetch(hq + 1 < m.H ? hq + 1 : 0, 0, nsb, ncs);
                }
                // code blocks of this chunk; each block's fragments (and
                // -|w|^2/2 of this lane's four codes) are read from LDS
                // while the previous block is searched
                const int ncb = min(CBK, QB - c * CBK);
                bf16x8 bf[2][KBS];
                f32x4 cqs[2];
                auto frags = [&](int cbl, bf16x8 (&b)[KBS], f32x4& cq) {
#pragma unroll
                    for (int kb = 0; kb < KBS; ++kb)
                        b[kb] = sb[(cbl * KBS + kb) * 64 + lane];
                    cq = *reinterpret_cast<const f32x4*>(cs + cbl * 16 + 4 * (lane >> 4));
                };
                frags(0, bf[0], cqs[0]);
#pragma unroll
                for (int cbl = 0; cbl < CBK; ++cbl) {
                    if (cbl >= ncb) break;
                    const int cb = c * CBK + cbl;
                    if (cbl + 1 < ncb) frags(cbl + 1, bf[(cbl + 1) & 1], cqs[(cbl + 1) & 1]);
                    // hi products first, then (for a block that may hold
                    // the nearest code of some row) the lo products: every
                    // search forms g in this order, seeded or not
                    f32x4 acc[MB];
#pragma unroll
                    for (int i = 0; i < MB; ++i) acc[i] = cqs[cbl & 1];
#pragma unroll
                    for (int kb = 0; kb < KBS; ++kb) {
                        const bf16x8 b = bf[cbl & 1][kb];
#pragma unroll
                        for (int i = 0; i < MB; ++i) acc[i] = mfma(b, ah[i][kb], acc[i]);
                    }
                    bool need = false;
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        const float mx = fmaxf(fmaxf(acc[i][0], acc[i][1]),
                                               fmaxf(acc[i][2], acc[i][3]));
                        need |= mx >= ut[i];
                    }
                    if (!MARGIN && __ballot(need) == 0) continue;
#pragma unroll
                    for (int kb = 0; kb < KBS; ++kb) {
                        const bf16x8 b = bf[cbl & 1][kb];
#pragma unroll
                        for (int i = 0; i < MB; ++i) acc[i] = mfma(b, al[i][kb], acc[i]);
                    }
                    const int code0 = cb * 16 + 4 * (lane >> 4);
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float g = acc[i][r];
                            if (MARGIN) {
                                if (g > best[i].b) {
                                    best[i].s = best[i].b;
                                    best[i].b = g;
                                    best[i].i = code0 + r;
                                } else if (g > best[i].s) {
                                    best[i].s = g;
                                }
                            } else {
                                const bool gt = g > best[i].b;
                                best[i].b = gt ? g : best[i].b;
                                best[i].i = gt ? code0 + r : best[i].i;
                            }
                        }
                }
            };
            // the two stages are distinct arrays, each named statically in
            // its copy of the chunk body: the compiler then sees that the
            // global-to-LDS loads into one never feed the reads of the other
            // and does not wait for them before the search
            for (int c = 0; c < nchunk; c += 2) {
                chunk(c, stage0, cn0, stage1, cn1, false);
                if (c + 1 < nchunk) chunk(c + 1, stage1, cn1, stage0, cn0, true);
            }
            // combine the four code groups of each row (lanes l, l^16,
            // l^32, l^48)
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                T2 v = best[i];
#pragma unroll
                for (int o = 16; o < 64; o <<= 1) {
                    T2 y;
                    y.b = __shfl_xor(v.b, o, 64);
                    y.i = __shfl_xor(v.i, o, 64);
                    y.s = MARGIN ? __shfl_xor(v.s, o, 64) : -inf;
                    v = t2_merge(v, y);
                }
                best[i] = v;
            }
            const float wmax = w.cnorm[(int64_t)m.H * m.Q + hq];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int64_t s = myslot[i];
                if ((lane >> 4) == 0 && s >= 0) {
                    io.codes[s * m.H + hq] = best[i].i;
                    if (MARGIN) {
                        const float a2 = nrm[i];
                        const float na = sqrtf(a2);
                        const float E = score_err_split(2 * DS, na, wmax);
                        // scores |w|^2 - 2 a.w = -2 g (exact scaling)
                        const float u1 = -2.0f * best[i].b + a2 + E;
                        const float l2 = -2.0f * best[i].s + a2 - E;
                        io.margin[(s * m.H + hq) * 2 + 0] = sqrtf(u1 > 0 ? u1 : 0.0f);
                        io.margin[(s * m.H + hq) * 2 + 1] = sqrtf(l2 > 0 ? l2 : 0.0f);
                    }
                }
            }
        }
    }
}

// ------------------------------------- half-block output projection
// out = x_in + (a W_o + b_o) for a set of rows (the attention-only block
// that ends the Table 1 networks): the attention output a, split hi/lo, is
// the A operand; W_o, packed like the QKV weights, streams through two LDS
// stages shared by the four waves (global-to-LDS loads one chunk ahead, as
// in k_qkv_mfma).  The matrix core sums the k-blocks of one row in a fixed
// order, so a row's result depends on that row only: full sequences,
// sampled rows and neighbour overlays give equal values for equal inputs.
// A row source gives, for the k-th row of the set, its residual input, its
// attention output and its destination (the destination may be the input:
// every element is read and written by one lane).
struct OprojRows {
    RowSet rows;
    const float* x_in;
    const float* a;
    float* x_out;
    int d;
    __device__ int64_t n() const { return rs_n(rows); }
    __device__ void at(int64_t k, const float*& xi, const float*& ar,
                       float*& o) const {
        const int64_t s = rs_slot(rows, k) * d;
        xi = x_in + s;
        ar = a + s;
        o = x_out + s;
    }
};
// Overlay rows of the neighbours (every row from p_min on): the input is
// the neighbour's row where it is in C_L, else the sample's.
struct OprojOverlay {
    const int32_t* n_rows;
    const int32_t* slot_nb;
    const NbDesc* desc;
    const uint64_t* mask;
    int W, N, d;
    const float* ox;
    const float* bx;
    const float* oa;
    float* out;
    __device__ int64_t n() const { return (int64_t)*n_rows; }
    __device__ void at(int64_t r, const float*& xi, const float*& ar,
                       float*& o) const {
        const int32_t nb = slot_nb[r];
        const NbDesc D = desc[nb];
        const int i = D.p1 + 1 + (int)(r - D.ov);
        const bool inC = (mask[(int64_t)nb * W + (i >> 6)] >> (i & 63)) & 1ull;
        xi = inC ? ox + r * d : bx + ((int64_t)D.sigma * N + i) * d;
        ar = oa + r * d;
        o = out + r * d;
    }
};

template <int KB, class Src>
__global__ void __launch_bounds__(kMT)
    __attribute__((amdgpu_waves_per_eu(KB <= 4 ? 3 : 2)))
    k_oproj_mfma(Src src, const float* __restrict__ bo,
                 const bf16x8* __restrict__ Bp) {
    constexpr int D = KB * 32, NBC = 4;
    constexpr int CHUNK = NBC * KB * 64, PER = CHUNK / kMT;
    constexpr int NBT = D / 16;
    constexpr int nchunk = NBT / NBC;
    static_assert(NBT % NBC == 0, "whole chunks");
    __shared__ bf16x8 stage0[CHUNK], stage1[CHUNK];
    __shared__ float bias0[NBC * 16], bias1[NBC * 16];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gq = lane >> 4, c16 = lane & 15;
    const int64_t n = src.n();
    const int64_t ntile = (n + 63) / 64;          // 16 rows per wave
    auto fetch = [&](int c, bf16x8* st, float* bs) {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            lds_dma16(Bp + (int64_t)c * CHUNK + threadIdx.x + k * kMT,
                      st + wave * 64 + k * kMT);
        if (wave == 0) lds_dma4(bo + c * NBC * 16 + lane, bs);
    };
    bool ahead = false;      // the tile's first chunk is in stage0
    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        // row c16 of the wave's 16: A fragments of its attention output
        const int64_t r = t * 64 + wave * 16 + c16;
        const float *xi = nullptr, *ar = nullptr;
        float* op = nullptr;
        if (r < n) src.at(r, xi, ar, op);
        bf16x8 ah[KB], al[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            float v[8];
            if (ar) {
                const float4* p = reinterpret_cast<const float4*>(ar + kb * 32 + 8 * gq);
                const float4 v0 = p[0], v1 = p[1];
                v[0] = v0.x; v[1] = v0.y; v[2] = v0.z; v[3] = v0.w;
                v[4] = v1.x; v[5] = v1.y; v[6] = v1.z; v[7] = v1.w;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                __bf16 h, l;
                split1(v[j], h, l);
                ah[kb][j] = h;
                al[kb][j] = l;
            }
        }
        // the result layout holds rows 4 gq + q (q = 0..3) of the 16
        int64_t oxi[4], oo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            oxi[q] = __shfl((int64_t)(uintptr_t)xi, 4 * gq + q, 64);
            oo[q] = __shfl((int64_t)(uintptr_t)op, 4 * gq + q, 64);
        }
        if (!ahead) {
            __syncthreads();                 // both stages free
            fetch(0, stage0, bias0);
        }
        float ov[NBC][4];                    // a W_o + b_o of the pending chunk
        float xv[NBC][4];                    // its residual inputs
        auto load_x = [&](int c) {
#pragma unroll
            for (int nbl = 0; nbl < NBC; ++nbl)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = (c * NBC + nbl) * 16 + c16;
                    xv[nbl][q] = oo[q] ? reinterpret_cast<const float*>(oxi[q])[col]
                                       : 0.0f;
                }
        };
        auto flush = [&](int c) {
#pragma unroll
            for (int nbl = 0; nbl < NBC; ++nbl)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = (c * NBC + nbl) * 16 + c16;
                    if (oo[q]) reinterpret_cast<float*>(oo[q])[col] = xv[nbl][q] + ov[nbl][q];
                }
        };
        auto chunk = [&](int c, const bf16x8* sb, const float* bs, bf16x8* nsb,
                         float* nbs, bool into0) {
            wait_vmem();
            __syncthreads();
            if (c + 1 < nchunk) {
                fetch(c + 1, nsb, nbs);
            } else {
                ahead = into0 && t + gridDim.x < ntile;
                if (ahead) fetch(0, nsb, nbs);
            }
            if (c > 0) flush(c - 1);
            load_x(c);
#pragma unroll
            for (int nbl = 0; nbl < NBC; ++nbl) {
                f32x4 acc = f32x4{0, 0, 0, 0};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const bf16x8 b = sb[(nbl * KB + kb) * 64 + lane];
                    acc = mfma(ah[kb], b, acc);
                    acc = mfma(al[kb], b, acc);
                }
                const float bias = bs[nbl * 16 + c16];
#pragma unroll
                for (int q = 0; q < 4; ++q) ov[nbl][q] = acc[q] + bias;
            }
        };
        for (int c = 0; c < nchunk; c += 2) {
            chunk(c, stage0, bias0, stage1, bias1, false);
            if (c + 1 < nchunk) chunk(c + 1, stage1, bias1, stage0, bias0, true);
        }
        flush(nchunk - 1);
    }
}

template <class Src>
static hipError_t oproj_go(const ModelDims& m, Src src, int64_t rows_max,
                           const float* bo, const bf16* Wo_p, hipStream_t st) {
    if (rows_max <= 0) return hipSuccess;
    const bf16x8* B = reinterpret_cast<const bf16x8*>(Wo_p);
    const dim3 g(mgrid((rows_max + 63) / 64));
    switch (m.d / 32) {
        case 2: hipLaunchKernelGGL((k_oproj_mfma<2, Src>), g, dim3(kMT), 0, st, src, bo, B); break;
        case 4: hipLaunchKernelGGL((k_oproj_mfma<4, Src>), g, dim3(kMT), 0, st, src, bo, B); break;
        case 8: hipLaunchKernelGGL((k_oproj_mfma<8, Src>), g, dim3(kMT), 0, st, src, bo, B); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_oproj_mfma(const ModelDims& m, const float* bo,
                             const bf16* Wo_p, RowSet rows, const float* x_in,
                             const float* a, float* x_out, hipStream_t st) {
    return oproj_go(m, OprojRows{rows, x_in, a, x_out, m.d}, rows.n_host, bo,
                    Wo_p, st);
}

hipError_t launch_oproj_overlay_mfma(const ModelDims& m, const float* bo,
                                     const bf16* Wo_p,
                                     const DedupIO<PrecBF16>& dd, float* out,
                                     hipStream_t st) {
    const OprojOverlay src{dd.n_rows, dd.slot_nb, dd.desc, dd.mask,
                           dd.mask_words, m.N, m.d, dd.ox, dd.bx, dd.oa, out};
    return oproj_go(m, src, dd.rows_max, bo, Wo_p, st);
}

hipError_t launch_pack_wo(const ModelDims& m, const float* W_o, bf16* out,
                          hipStream_t st) {
    const int d = m.d;
    const int64_t total = (int64_t)d * d;
    hipLaunchKernelGGL(k_pack_b, dim3(mgrid((total + 255) / 256)), dim3(256),
                       0, st, W_o, d, d, (int64_t)d, (int64_t)1, 0,
                       reinterpret_cast<__bf16*>(out));
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers
// Launch choices per model width (rows per wave of the three products).
// Every row's arithmetic is the same whichever is chosen: the choices trade
// register pressure against weight reuse, never results.
namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, int>, Tuning> g_tune;
}  // namespace

Tuning tuning_default(const ModelDims& m) {
    Tuning t;
    t.qkv_mb = m.d >= 256 ? 1 : 2;
    t.mlp_mb = m.d >= 256 ? 1 : 2;
    t.vq_mb = m.dseg >= 256 ? 1 : 2;
    return t;
}

Tuning tuning_get(const ModelDims& m) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({m.d, m.dseg});
    return it == g_tune.end() ? tuning_default(m) : it->second;
}

void tuning_set(const ModelDims& m, const Tuning& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{m.d, m.dseg}] = t;
}

bool tuning_valid(const ModelDims& m, const Tuning& t) {
    auto ok = [](int mb, int width) {
        return mb == 1 || (mb == 2 && width < 256);
    };
    const bool vq_ok = t.vq_mb == 1 || (t.vq_mb == 2 && m.dseg < 256) ||
                       (t.vq_mb == 4 && m.dseg <= 128);
    return ok(t.qkv_mb, m.d) && ok(t.mlp_mb, m.d) && vq_ok;
}

template <int KB, int MB>
static void qkv_go(const ModelDims& m, const LayerW<float>& w, RowSet rows,
                   const BlockIO<PrecBF16>& io, const bf16x8* B,
                   hipStream_t st) {
    constexpr int R = 64 * MB;    // rows per workgroup (4 waves)
    hipLaunchKernelGGL((k_qkv_mfma<KB, MB>), dim3(mgrid((rows.n_host + R - 1) / R)),
                       dim3(kMT), 0, st, m, w, rows, io, B);
}

hipError_t launch_qkv_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st) {
    const bf16x8* B = reinterpret_cast<const bf16x8*>(w.Wqkv_p);
    const int mb = tuning_get(m).qkv_mb;
    switch (m.d / 32 * 10 + mb) {
        case 21: qkv_go<2, 1>(m, w, rows, io, B, st); break;
        case 22: qkv_go<2, 2>(m, w, rows, io, B, st); break;
        case 41: qkv_go<4, 1>(m, w, rows, io, B, st); break;
        case 42: qkv_go<4, 2>(m, w, rows, io, B, st); break;
        case 81: qkv_go<8, 1>(m, w, rows, io, B, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KB, int MB>
static void mlp_go(const ModelDims& m, const LayerW<float>& w, RowSet rows,
                   const BlockIO<PrecBF16>& io, const bf16x8* B1,
                   const bf16x8* B2, hipStream_t st) {
    constexpr int R = 64 * MB;
    hipLaunchKernelGGL((k_mlp_mfma<KB, MB>), dim3(mgrid((rows.n_host + R - 1) / R)),
                       dim3(kMT), 0, st, m, w, rows, io, B1, B2);
}

hipError_t launch_mlp_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st) {
    const bf16x8* B1 = reinterpret_cast<const bf16x8*>(w.W1_p);
    const bf16x8* B2 = reinterpret_cast<const bf16x8*>(w.W2_p);
    const int mb = tuning_get(m).mlp_mb;
    switch (m.d / 32 * 10 + mb) {
        case 21: mlp_go<2, 1>(m, w, rows, io, B1, B2, st); break;
        case 22: mlp_go<2, 2>(m, w, rows, io, B1, B2, st); break;
        case 41: mlp_go<4, 1>(m, w, rows, io, B1, B2, st); break;
        case 42: mlp_go<4, 2>(m, w, rows, io, B1, B2, st); break;
        case 81: mlp_go<8, 1>(m, w, rows, io, B1, B2, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KBS, int MB>
static void vq_go(const ModelDims& m, const LayerW<float>& w, RowSet rows,
                  const BlockIO<PrecBF16>& io, const bf16x8* cb,
                  const VqSeed& seed, hipStream_t st) {
    constexpr int R = 64 * MB;    // 16*MB rows per wave, 4 waves
    const dim3 g(mgrid((rows.n_host + R - 1) / R));
    // Large codebooks with segments of up to 128: eight code blocks per LDS
    // chunk (32 KB per stage at 128) and, for neighbour rows, the search
    // seeded with the sample's code.  Small codebooks (fewer than 256 codes,
    // a handful of blocks) and segments of 256: four blocks per chunk and no
    // seed, whose set-up per row tile would cost more than it saves (and its
    // registers, at segment 256, a wave per SIMD).
    constexpr int CB8 = KBS <= 4 ? 8 : 4;
    const bool big = m.Q >= 256;
    if (io.margin) {
        if (big)
            hipLaunchKernelGGL((k_vq_mfma<KBS, MB, true, CB8, false>), g, dim3(kMT), 0,
                               st, m, w, rows, io, cb, VqSeed{});
        else
            hipLaunchKernelGGL((k_vq_mfma<KBS, MB, true, 4, false>), g, dim3(kMT), 0,
                               st, m, w, rows, io, cb, VqSeed{});
    } else if (big && KBS <= 4 && seed.slot_nb) {
        hipLaunchKernelGGL((k_vq_mfma<KBS, MB, false, CB8, KBS <= 4>), g, dim3(kMT), 0,
                           st, m, w, rows, io, cb, seed);
    } else if (big) {
        hipLaunchKernelGGL((k_vq_mfma<KBS, MB, false, CB8, false>), g, dim3(kMT), 0,
                           st, m, w, rows, io, cb, VqSeed{});
    } else {
        hipLaunchKernelGGL((k_vq_mfma<KBS, MB, false, 4, false>), g, dim3(kMT), 0, st,
                           m, w, rows, io, cb, VqSeed{});
    }
}

hipError_t launch_vq_mfma(const ModelDims& m, const LayerW<float>& w,
                          RowSet rows, const BlockIO<PrecBF16>& io,
                          hipStream_t st, const VqSeed& seed) {
    const bf16x8* cb = reinterpret_cast<const bf16x8*>(w.cb_p);
    const int mb = tuning_get(m).vq_mb;
    switch (m.dseg / 32 * 10 + mb) {
        case 11: vq_go<1, 1>(m, w, rows, io, cb, seed, st); break;
        case 12: vq_go<1, 2>(m, w, rows, io, cb, seed, st); break;
        case 21: vq_go<2, 1>(m, w, rows, io, cb, seed, st); break;
        case 22: vq_go<2, 2>(m, w, rows, io, cb, seed, st); break;
        case 14: vq_go<1, 4>(m, w, rows, io, cb, seed, st); break;
        case 24: vq_go<2, 4>(m, w, rows, io, cb, seed, st); break;
        case 41: vq_go<4, 1>(m, w, rows, io, cb, seed, st); break;
        case 42: vq_go<4, 2>(m, w, rows, io, cb, seed, st); break;
        case 44: vq_go<4, 4>(m, w, rows, io, cb, seed, st); break;
        case 81: vq_go<8, 1>(m, w, rows, io, cb, seed, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vq
