// Shared device/host definitions of the VQ-NQS HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "vqnqs.h"

#define VQ_WAVE 64
#define VQ_MAX_MASK_WORDS 16      // changed-row bitmask: N <= 1024 sites

// ---------------------------------------------------------------- bfloat16
struct bf16 {
    uint16_t u;
};

__host__ __device__ inline float bf2f(bf16 v) {
    uint32_t x = (uint32_t)v.u << 16;
    float f;
    memcpy(&f, &x, 4);
    return f;
}

// round to nearest even (NaN kept quiet)
__host__ __device__ inline bf16 f2bf(float f) {
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7f800000u) == 0x7f800000u && (x & 0x7fffffu)) {
        bf16 r;
        r.u = (uint16_t)((x >> 16) | 0x40u);
        return r;
    }
    uint32_t rnd = 0x7fffu + ((x >> 16) & 1u);
    bf16 r;
    r.u = (uint16_t)((x + rnd) >> 16);
    return r;
}

// --------------------------------------------------------- precision traits
// act: storage of activations (q, k, v, attention output)
// acc: arithmetic type and type of the residual stream and parameters
// The BF16 mode keeps activations in FP32; its products run on the matrix
// core with bfloat16 weights and activations split into hi + lo bfloat16.
struct PrecF64 {
    using act = double;
    using acc = double;
    static constexpr int id = VQNQS_F64;
};
struct PrecF32 {
    using act = float;
    using acc = float;
    static constexpr int id = VQNQS_F32;
};
struct PrecBF16 {
    using act = float;
    using acc = float;
    static constexpr int id = VQNQS_BF16;
};

template <typename To, typename From>
__device__ inline To cvt(From v) {
    return (To)v;
}
template <>
__device__ inline float cvt<float, bf16>(bf16 v) {
    return bf2f(v);
}
template <>
__device__ inline bf16 cvt<bf16, float>(float v) {
    return f2bf(v);
}
template <>
__device__ inline bf16 cvt<bf16, bf16>(bf16 v) {
    return v;
}
template <>
__device__ inline double cvt<double, bf16>(bf16 v) {
    return (double)bf2f(v);
}

__device__ inline float dexp(float x) { return expf(x); }
__device__ inline double dexp(double x) { return exp(x); }
__device__ inline float dlog(float x) { return logf(x); }
__device__ inline double dlog(double x) { return log(x); }
__device__ inline float dsqrt(float x) { return sqrtf(x); }
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float derf(float x) { return erff(x); }
__device__ inline double derf(double x) { return erf(x); }
template <typename T>
__device__ inline T gelu_exact(T x) {
    return (T)0.5 * x * ((T)1 + derf(x * (T)0.70710678118654752440));
}
template <typename T>
__device__ inline T neg_inf();
template <>
__device__ inline float neg_inf<float>() {
    return -__builtin_inff();
}
template <>
__device__ inline double neg_inf<double>() {
    return -__builtin_inf();
}

// ------------------------------------------------------ wave-level helpers
template <typename T>
__device__ inline T wave_sum(T v) {
    // fixed butterfly order: identical result on every lane, deterministic
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, VQ_WAVE);
    return v;
}

// ------------------------------------------------------ model description
namespace vq {

// Offsets (in elements) of every parameter tensor in the flat buffer.
struct LayerOffsets {
    int64_t ln1_g, ln1_b, W_qkv, b_qkv, codebook, W_o, b_o, ln2_g, ln2_b, W1,
        b1, W2, b2;
};

struct ModelDims {
    int L;         // lattice side (chain: sites)
    int N;         // sequence length: tokens per sample (T = S / K)
    int S, K;      // sites per sample, spins per token
    int enc;       // 1: bidirectional encoder with mean pooling as log psi
    int d, nl, nh, dh, dff, Q, H, dseg;
    int periodic, marshall, precision, flags;
    int mfma;      // BF16 products on the matrix core (split activations)
    int chain;     // 1: transverse-field Ising chain of N = L sites
    int tail;      // 1: an attention-only half-block ends the model
    double J;
    double gamma;  // transverse field (chain only)
};

// Per-layer view of the parameters handed to kernels (by value).
template <typename C>
struct LayerW {
    const C *ln1_g, *ln1_b, *W_qkv, *b_qkv, *codebook, *W_o, *b_o, *ln2_g,
        *ln2_b, *W1, *b1, *W2, *b2;
    const C* table;    // [H][Q][d]: codeword h,c times rows of W_o of segment h
    const C* cnorm;    // [H][Q]: squared norm of every codeword
    const float* cnh;  // BF16 packs: [H][Q], -cnorm/2
    const bf16* Wqkv_p;  // BF16 packs (MFMA fragment order); null otherwise
    const bf16* W1_p;
    const bf16* W2_p;
    const bf16* cb_p;
    const bf16* Wo_p;    // W_o pack of the attention-only half-block
};

template <typename C>
struct HeadW {
    const C *tok, *pos, *lnf_g, *lnf_b, *W_head, *b_head;
};

// One neighbour s' of sample `sigma`: the spins of sites s1 < s2
// exchanged, or site s1 flipped (s1 == s2), in the tokens p1 <= p2.  Token
// rows >= p1+1 are the only ones whose input can change; overlay rows of s'
// live at ov + (i - (p1+1)).
struct NbDesc {
    int32_t sigma;
    int16_t p1, p2;   // token positions of the changed sites (p1 <= p2;
                      // p1 == p2: one changed token)
    int64_t ov;
    int16_t s1, s2;   // the sites: exchange of s1 < s2, flip when s1 == s2
};

// First token row of neighbour D that can differ from the sample's: the
// decoder's rows before the first changed input see an unchanged prefix;
// every encoder row attends to the change.  (The changed input rows are
// p1 + 1 and p2 + 1 in both: the encoder's descriptors hold the changed
// tokens minus one.)
__device__ inline int first_row(const NbDesc& D, const ModelDims& m) {
    return m.enc ? 0 : D.p1 + 1;
}

// Value of token t of one sample's spins sp (sites tK .. tK+K-1):
// sum_k b_k 2^k with b_k = 1 for spin -1 at the token's k-th site.
__device__ inline int token_at(const int8_t* sp, int t, int K) {
    int v = 0;
    for (int k = 0; k < K; ++k) v |= (sp[t * K + k] < 0 ? 1 : 0) << k;
    return v;
}

// The same token of neighbour D of the sample with spins sp: the spins of
// sites s1, s2 exchanged, or of s1 flipped when s1 == s2.
__device__ inline int nb_token_at(const int8_t* sp, const NbDesc& D, int t,
                                  int K) {
    const bool flip = D.s1 == D.s2;
    int v = 0;
    for (int k = 0; k < K; ++k) {
        const int x = t * K + k;
        const int8_t s = x == D.s1 ? (flip ? (int8_t)-sp[x] : sp[D.s2])
                                   : (x == D.s2 ? sp[D.s1] : sp[x]);
        v |= (s < 0 ? 1 : 0) << k;
    }
    return v;
}

}  // namespace vq
