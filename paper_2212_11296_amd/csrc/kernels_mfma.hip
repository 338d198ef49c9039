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

// ---------------------------------------------------------------- packing
// out[((nb*KB + kb)*64 + l)*8 + j] = W[kb*32 + 8*(l/16) + j][nb*16 + l%16]
// with W[k][c] read at src[k*sk + c*sc] (K x Nout logical matrix).
__global__ void k_pack_b(const float* __restrict__ src, int K, int Nout,
                         int64_t sk, int64_t sc, __bf16* __restrict__ out) {
    const int64_t total = (int64_t)K * Nout;
    const int KB = K / 32;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e & 7);
        const int l = (int)((e >> 3) & 63);
        const int64_t f = e >> 9;             // fragment id nb*KB + kb
        const int kb = (int)(f % KB);
        const int nb = (int)(f / KB);
        const int k = kb * 32 + 8 * (l >> 4) + j;
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

hipError_t launch_pack_layer(const ModelDims& m, const LayerW<float>& w,
                             bf16* Wqkv_p, bf16* W1_p, bf16* W2_p, bf16* cb_p,
                             hipStream_t st) {
    const int d = m.d, F = m.dff;
    auto go = [&](const float* src, int K, int Nout, int64_t sk, int64_t sc,
                  bf16* out) {
        const int64_t total = (int64_t)K * Nout;
        hipLaunchKernelGGL(k_pack_b, dim3(mgrid((total + 255) / 256)),
                           dim3(256), 0, st, src, K, Nout, sk, sc,
                           reinterpret_cast<__bf16*>(out));
    };
    go(w.W_qkv, d, 3 * d, 3 * d, 1, Wqkv_p);
    go(w.W1, d, F, F, 1, W1_p);
    go(w.W2, F, d, d, 1, W2_p);
    // codebook head h as B[k][c] = cb[h][c][k]
    for (int h = 0; h < m.H; ++h)
        go(w.codebook + (int64_t)h * m.Q * m.dseg, m.dseg, m.Q, 1, m.dseg,
           cb_p + (int64_t)h * m.Q * m.dseg);
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

// --------------------------------------------------------------- LN1 + QKV
// Workgroup tile: 64 rows.  LN1 output is split into hi/lo bf16 in LDS; each
// wave computes a contiguous range of the 3d/16 output column blocks in
// groups of four, reusing every A fragment across the group.
template <int KB>
__global__ void __launch_bounds__(kMT) k_qkv_mfma(ModelDims m, LayerW<float> w,
                                                 RowSet rows, BlockIO<PrecBF16> io,
                                                 const bf16x8* __restrict__ Bp) {
    constexpr int D = KB * 32, LD = D + 8, TM = 64, MB = 4;
    __shared__ __align__(16) __bf16 Ahi[TM * LD];
    __shared__ __align__(16) __bf16 Alo[TM * LD];
    __shared__ int64_t slot[TM];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = rs_n(rows);
    const int64_t ntiles = (n + TM - 1) / TM;
    const int NBT = 3 * D / 16;
    const int nbs = wave * NBT / 4, nbe = (wave + 1) * NBT / 4;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int rr = wave * 16; rr < wave * 16 + 16; ++rr) {
            const int64_t r = t * TM + rr;
            if (r < n) {
                const int64_t s = rs_slot(rows, r);
                if (lane == 0) slot[rr] = s;
                const float* x = io.x + s * D;
                float mean, rstd;
                row_ln(x, D, mean, rstd);
                for (int k = lane; k < D; k += 64) {
                    const float y = (x[k] - mean) * rstd * w.ln1_g[k] + w.ln1_b[k];
                    split1(y, Ahi[rr * LD + k], Alo[rr * LD + k]);
                }
            } else {
                if (lane == 0) slot[rr] = -1;
                for (int k = lane; k < D; k += 64) {
                    Ahi[rr * LD + k] = (__bf16)0.0f;
                    Alo[rr * LD + k] = (__bf16)0.0f;
                }
            }
        }
        __syncthreads();
        for (int nb0 = nbs; nb0 < nbe; nb0 += 4) {
            f32x4 acc[MB][4];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                bf16x8 ah[MB], al[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    ah[i] = lds_frag(Ahi, LD, i, kb, lane);
                    al[i] = lds_frag(Alo, LD, i, kb, lane);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (nb0 + j < nbe) {
                        const bf16x8 b = Bp[((int64_t)(nb0 + j) * KB + kb) * 64 + lane];
#pragma unroll
                        for (int i = 0; i < MB; ++i) {
                            acc[i][j] = mfma(ah[i], b, acc[i][j]);
                            acc[i][j] = mfma(al[i], b, acc[i][j]);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (nb0 + j >= nbe) continue;
                const int col = (nb0 + j) * 16 + (lane & 15);
                float* dst = col < D ? io.q : (col < 2 * D ? io.k : io.v);
                const int cc = col < D ? col : (col < 2 * D ? col - D : col - 2 * D);
                const float bias = w.b_qkv[col];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = i * 16 + 4 * (lane >> 4) + r;
                        const int64_t s = slot[row];
                        if (s >= 0) dst[s * D + cc] = acc[i][j][r] + bias;
                    }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------ out-projection + residual + MLP
// x' = x_in + b_o + sum_h table[h][code_h]; hidden = GELU(LN2(x') W1 + b1)
// kept in LDS as hi/lo bf16; x = x' + hidden W2 + b2.
template <int KB1, int MB>
__global__ void __launch_bounds__(kMT) k_mlp_mfma(ModelDims m, LayerW<float> w,
                                                 RowSet rows, BlockIO<PrecBF16> io,
                                                 const bf16x8* __restrict__ B1,
                                                 const bf16x8* __restrict__ B2) {
    constexpr int D = KB1 * 32, F = 4 * D, KB2 = F / 32;
    constexpr int TM = MB * 16, LDA = D + 8, LDH = F + 8;
    __shared__ float xp[TM * D];
    __shared__ __align__(16) __bf16 Ahi[TM * LDA];
    __shared__ __align__(16) __bf16 Alo[TM * LDA];
    __shared__ __align__(16) __bf16 Hhi[TM * LDH];
    __shared__ __align__(16) __bf16 Hlo[TM * LDH];
    __shared__ int64_t slot[TM];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = rs_n(rows);
    const int64_t ntiles = (n + TM - 1) / TM;
    const int NB1 = F / 16, NB2 = D / 16;
    const int n1s = wave * NB1 / 4, n1e = (wave + 1) * NB1 / 4;
    const int n2s = wave * NB2 / 4, n2e = (wave + 1) * NB2 / 4;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int rr = wave; rr < TM; rr += 4) {
            const int64_t r = t * TM + rr;
            if (r < n) {
                const int64_t s = rs_slot(rows, r);
                if (lane == 0) slot[rr] = s;
                const float* x = io.x_in + s * D;
                const int32_t* cd = io.codes + s * m.H;
                for (int k = lane; k < D; k += 64) {
                    float z = w.b_o[k];
                    for (int hq = 0; hq < m.H; ++hq)
                        z += w.table[((int64_t)hq * m.Q + cd[hq]) * D + k];
                    xp[rr * D + k] = x[k] + z;
                }
                float mean, rstd;
                row_ln(xp + rr * D, D, mean, rstd);
                for (int k = lane; k < D; k += 64) {
                    const float y = (xp[rr * D + k] - mean) * rstd * w.ln2_g[k] + w.ln2_b[k];
                    split1(y, Ahi[rr * LDA + k], Alo[rr * LDA + k]);
                }
            } else {
                if (lane == 0) slot[rr] = -1;
                for (int k = lane; k < D; k += 64) {
                    xp[rr * D + k] = 0.0f;
                    Ahi[rr * LDA + k] = (__bf16)0.0f;
                    Alo[rr * LDA + k] = (__bf16)0.0f;
                }
            }
        }
        __syncthreads();
        // hidden = GELU(A W1 + b1)
        for (int nb0 = n1s; nb0 < n1e; nb0 += 4) {
            f32x4 acc[MB][4];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) {
                bf16x8 ah[MB], al[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    ah[i] = lds_frag(Ahi, LDA, i, kb, lane);
                    al[i] = lds_frag(Alo, LDA, i, kb, lane);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (nb0 + j < n1e) {
                        const bf16x8 b = B1[((int64_t)(nb0 + j) * KB1 + kb) * 64 + lane];
#pragma unroll
                        for (int i = 0; i < MB; ++i) {
                            acc[i][j] = mfma(ah[i], b, acc[i][j]);
                            acc[i][j] = mfma(al[i], b, acc[i][j]);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (nb0 + j >= n1e) continue;
                const int col = (nb0 + j) * 16 + (lane & 15);
                const float bias = w.b1[col];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = i * 16 + 4 * (lane >> 4) + r;
                        const float h = gelu_exact(acc[i][j][r] + bias);
                        split1(h, Hhi[row * LDH + col], Hlo[row * LDH + col]);
                    }
            }
        }
        __syncthreads();
        // x = x' + hidden W2 + b2
        for (int nb0 = n2s; nb0 < n2e; nb0 += 4) {
            f32x4 acc[MB][4];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
            for (int kb = 0; kb < KB2; ++kb) {
                bf16x8 ah[MB], al[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    ah[i] = lds_frag(Hhi, LDH, i, kb, lane);
                    al[i] = lds_frag(Hlo, LDH, i, kb, lane);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (nb0 + j < n2e) {
                        const bf16x8 b = B2[((int64_t)(nb0 + j) * KB2 + kb) * 64 + lane];
#pragma unroll
                        for (int i = 0; i < MB; ++i) {
                            acc[i][j] = mfma(ah[i], b, acc[i][j]);
                            acc[i][j] = mfma(al[i], b, acc[i][j]);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (nb0 + j >= n2e) continue;
                const int col = (nb0 + j) * 16 + (lane & 15);
                const float bias = w.b2[col];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = i * 16 + 4 * (lane >> 4) + r;
                        const int64_t s = slot[row];
                        if (s >= 0) io.x[s * D + col] = xp[row * D + col] + (acc[i][j][r] + bias);
                    }
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- VQ search
// Running best / second-best (score, code); ties go to the lower code.
struct T2 {
    float b;
    int i;
    float s;
};
__device__ inline T2 t2_merge(T2 x, T2 y) {
    T2 r;
    if (y.b < x.b || (y.b == x.b && y.i < x.i)) {
        r.b = y.b;
        r.i = y.i;
        r.s = x.b < y.s ? x.b : y.s;
    } else {
        r.b = x.b;
        r.i = x.i;
        r.s = y.b < x.s ? y.b : x.s;
    }
    return r;
}

// Bound on the error of a computed score |w|^2 - 2 (hi + lo).w for a row of
// norm na (length-n FP32 sums of exact products, any order), plus the
// representation error |a - (hi + lo)| <= 2^-16 |a| in both the product and
// the row norm that turns scores into distances.
__device__ inline float score_err_split(int n, float na, float wmax) {
    const float g = (float)(n + 4) * 5.9604645e-8f * 1.0625f;
    return g * (2.0f * na * wmax + wmax * wmax + na * na) +
           3.0517578e-5f * (na * wmax + na * na);
}

// One wave owns 16*MB rows kept in registers as hi/lo A fragments and
// streams all codes of the quantizer head through the matrix core.
template <int KBS, int MB>
__global__ void __launch_bounds__(kMT) k_vq_mfma(ModelDims m, LayerW<float> w,
                                                RowSet rows, BlockIO<PrecBF16> io,
                                                const bf16x8* __restrict__ cbp) {
    constexpr int DS = KBS * 32, WR = MB * 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = rs_n(rows);
    const int64_t nw = (n + WR - 1) / WR;       // wave tiles
    const int QB = m.Q / 16;
    const float inf = __builtin_inff();
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < nw;
         t += (int64_t)gridDim.x * 4) {
        int64_t myslot[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int64_t r = t * WR + i * 16 + (lane & 15);
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
            T2 best[MB][4];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) best[i][r] = T2{inf, 0x7fffffff, inf};
            const bf16x8* cbh = cbp + (int64_t)hq * QB * KBS * 64;
            const float* cn = w.cnorm + (int64_t)hq * m.Q;
            for (int cb = 0; cb < QB; ++cb) {
                f32x4 acc[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) acc[i] = f32x4{0, 0, 0, 0};
#pragma unroll
                for (int kb = 0; kb < KBS; ++kb) {
                    const bf16x8 b = cbh[((int64_t)cb * KBS + kb) * 64 + lane];
#pragma unroll
                    for (int i = 0; i < MB; ++i) {
                        acc[i] = mfma(ah[i][kb], b, acc[i]);
                        acc[i] = mfma(al[i][kb], b, acc[i]);
                    }
                }
                const int c = cb * 16 + (lane & 15);
                const float cnv = cn[c];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float sc = cnv - 2.0f * acc[i][r];
                        if (sc < best[i][r].b) {
                            best[i][r].s = best[i][r].b;
                            best[i][r].b = sc;
                            best[i][r].i = c;
                        } else if (sc < best[i][r].s) {
                            best[i][r].s = sc;
                        }
                    }
            }
            // combine the 16 column lanes of each row group
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T2 v = best[i][r];
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) {
                        T2 y;
                        y.b = __shfl_xor(v.b, o, 64);
                        y.i = __shfl_xor(v.i, o, 64);
                        y.s = __shfl_xor(v.s, o, 64);
                        v = t2_merge(v, y);
                    }
                    best[i][r] = v;
                }
            const float wmax = w.cnorm[(int64_t)m.H * m.Q + hq];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rw = 4 * (lane >> 4) + r;     // row within block
                    const float a2 = __shfl(nrm[i], rw, 64);
                    const int64_t s = __shfl(myslot[i], rw, 64);
                    if ((lane & 15) == 0 && s >= 0) {
                        io.codes[s * m.H + hq] = best[i][r].i;
                        if (io.margin) {
                            const float na = sqrtf(a2);
                            const float E = score_err_split(2 * DS, na, wmax);
                            const float u1 = best[i][r].b + a2 + E;
                            const float l2 = best[i][r].s + a2 - E;
                            io.margin[(s * m.H + hq) * 2 + 0] = sqrtf(u1 > 0 ? u1 : 0.0f);
                            io.margin[(s * m.H + hq) * 2 + 1] = sqrtf(l2 > 0 ? l2 : 0.0f);
                        }
                    }
                }
        }
    }
}

// ------------------------------------------------------------ launchers
hipError_t launch_qkv_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st) {
    const bf16x8* B = reinterpret_cast<const bf16x8*>(w.Wqkv_p);
    const unsigned g = mgrid((rows.n_host + 63) / 64);
    switch (m.d / 32) {
        case 2: hipLaunchKernelGGL((k_qkv_mfma<2>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, B); break;
        case 4: hipLaunchKernelGGL((k_qkv_mfma<4>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, B); break;
        case 8: hipLaunchKernelGGL((k_qkv_mfma<8>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, B); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mlp_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st) {
    const bf16x8* B1 = reinterpret_cast<const bf16x8*>(w.W1_p);
    const bf16x8* B2 = reinterpret_cast<const bf16x8*>(w.W2_p);
    switch (m.d / 32) {
        case 2: hipLaunchKernelGGL((k_mlp_mfma<2, 4>), dim3(mgrid((rows.n_host + 63) / 64)), dim3(kMT), 0, st, m, w, rows, io, B1, B2); break;
        case 4: hipLaunchKernelGGL((k_mlp_mfma<4, 2>), dim3(mgrid((rows.n_host + 31) / 32)), dim3(kMT), 0, st, m, w, rows, io, B1, B2); break;
        case 8: hipLaunchKernelGGL((k_mlp_mfma<8, 1>), dim3(mgrid((rows.n_host + 15) / 16)), dim3(kMT), 0, st, m, w, rows, io, B1, B2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_vq_mfma(const ModelDims& m, const LayerW<float>& w,
                          RowSet rows, const BlockIO<PrecBF16>& io,
                          hipStream_t st) {
    const bf16x8* cb = reinterpret_cast<const bf16x8*>(w.cb_p);
    const int KBS = m.dseg / 32;
    // waves of 64 rows (32 when the segment is 256 wide), 4 waves per group
    const int WR = KBS == 8 ? 32 : 64;
    const unsigned g = mgrid((rows.n_host + 4 * WR - 1) / (4 * WR));
    switch (KBS) {
        case 1: hipLaunchKernelGGL((k_vq_mfma<1, 4>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, cb); break;
        case 2: hipLaunchKernelGGL((k_vq_mfma<2, 4>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, cb); break;
        case 4: hipLaunchKernelGGL((k_vq_mfma<4, 4>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, cb); break;
        case 8: hipLaunchKernelGGL((k_vq_mfma<8, 2>), dim3(g), dim3(kMT), 0, st, m, w, rows, io, cb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vq
