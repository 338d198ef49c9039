// Backward pass of log psi with the straight-through quantizer (paper
// eqs. 7-8; chain-rule log psi of Sec. 2; network of Sec. 3.1).
//
// The forward of one layer is recomputed from its checkpointed input (layer
// checkpointing) and differentiated in reverse: output projection + MLP,
// the quantizer, causal attention, LN1 + QKV; then the head and the
// embeddings.  The quantizer passes the gradient through a softmax over the
// negative unsquared distances to all codewords (eq. 8):
//   p = softmax(-delta), delta_j = ||u - W_j||, e_j = g . W_j,
//   t_j = p_j (e_j - p.e),  G_j = t_j / delta_j,
//   dL/du   = -(sum_j G_j) u + sum_j G_j W_j,
//   dL/dW_j = [j == code] g + G_j u - G_j W_j,
// where g is the gradient reaching the quantized vector.  Eq. (8) writes
// the quantized vector as g(D)^T W with the stop gradient on the softmax
// output only: the codebook's own factor is the value of g(D), the one-hot
// vector, and the softmax reaches every codeword and u through D.
//
// Every parameter gradient is formed per sample (one group of N rows) into
// a [sample][P] array, so per-sample gradients need no extra pass and the
// weighted sum is a fixed-order reduction over samples (deterministic).
// Products are tiled VALU kernels in the arithmetic type T (double in the
// FP64 mode, float otherwise).
#include "kernels.h"

namespace vq {

constexpr int kGT = 256;          // threads per workgroup
constexpr int kGridMax = 65535;

static inline unsigned cap_grid(int64_t u) {
    if (u <= 0) return 1;
    return (unsigned)(u < 8192 ? u : 8192);
}

// ------------------------------------------------------------------- GEMM
// C[g] = beta * C[g] + op(A[g]) op(B[g]) for g < groups; op(A) is M x K
// (A[m*lda + k], or A[k*lda + m] when tA), op(B) is K x N (B[k*ldb + n],
// or B[n*ldb + k] when tB).  64 x 64 tiles, K steps of 16 through LDS.
template <typename T>
__global__ void __launch_bounds__(kGT) k_gemm(GemmDesc g) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];
    const int64_t grp = blockIdx.z;
    const T* A = static_cast<const T*>(g.A) + grp * g.sA;
    const T* B = static_cast<const T*>(g.B) + grp * g.sB;
    T* C = static_cast<T*>(g.C) + grp * g.sC;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + kGT * r;
            int mm, kk;
            if (g.tA) { kk = e >> 6; mm = e & 63; }
            else { mm = e >> 4; kk = e & 15; }
            const int64_t gm = m0 + mm, gk = k0 + kk;
            T v = 0;
            if (gm < g.M && gk < g.K)
                v = g.tA ? A[gk * g.lda + gm] : A[gm * g.lda + gk];
            As[kk][mm] = v;
            int nn;
            if (g.tB) { nn = e >> 4; kk = e & 15; }
            else { kk = e >> 6; nn = e & 63; }
            const int64_t gn = n0 + nn, gk2 = k0 + kk;
            T w = 0;
            if (gn < g.N && gk2 < g.K)
                w = g.tB ? B[gn * g.ldb + gk2] : B[gk2 * g.ldb + gn];
            Bs[kk][nn] = w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t gm = m0 + ty + 16 * i;
        if (gm >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gn = n0 + tx + 16 * j;
            if (gn >= g.N) continue;
            T* c = C + gm * g.ldc + gn;
            *c = g.beta ? *c + acc[i][j] : acc[i][j];
        }
    }
}

template <typename T>
hipError_t launch_gemm(const GemmDesc& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.groups <= 0) return hipSuccess;
    const int64_t gx = (g.N + 63) / 64, gy = (g.M + 63) / 64;
    if (gx > kGridMax || gy > kGridMax || g.groups > kGridMax)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gemm<T>), dim3((unsigned)gx, (unsigned)gy,
                                        (unsigned)g.groups),
                       dim3(kGT), 0, st, g);
    return hipGetLastError();
}

// ------------------------------------------------ GEMM on the matrix core
// FP32 operands enter the bf16 matrix core as hi + lo pairs; three passes
// hi.hi + hi.lo + lo.hi accumulate in FP32 (about 16 significant bits per
// product; the lo.lo term is below that).  When B is bf16-exact (the
// BF16 mode's weights) its lo part is zero and the hi.lo pass is skipped.
// Workgroup tile 128 x 128, each of the four waves 64 x 64 (4 x 4 tiles of
// 16 x 16), K steps of 32.  The operands are staged in LDS as [row][k] (A)
// and [col][k] (B), so every MFMA fragment is one 16-byte read per lane
// whatever the transposition.
typedef __attribute__((ext_vector_type(8))) __bf16 gbf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 gbf16x4;
typedef __attribute__((ext_vector_type(4))) float gf32x4;

// Four consecutive elements of one row of a matrix (0 past lim), one
// 16-byte load when vec (aligned rows) and all four are in range.
__device__ inline void load4(const float* base, int64_t lim, bool vec, float (&v)[4]) {
    if (vec && lim >= 4) {
        const float4 t = *reinterpret_cast<const float4*>(base);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = c < lim ? base[c] : 0.0f;
    }
}

// The 4 x 4 block (rows r0..r0+3, k k0..k0+3) of an operand read as
// X[row][k]: rows with k contiguous (kc) or k-major with rows contiguous.
__device__ inline void load_block(const float* X, int64_t ld, bool kc, bool vec,
                                  int64_t r0, int64_t nr, int64_t k0, int64_t nk,
                                  float (&v)[4][4]) {
    if (kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r0 + r < nr) {
                load4(X + (r0 + r) * ld + k0, nk - k0, vec, v[r]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) v[r][c] = 0.0f;
            }
        }
    } else {
        float w[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (k0 + c < nk) {
                load4(X + (k0 + c) * ld + r0, nr - r0, vec, w[c]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) w[c][r] = 0.0f;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[r][c] = w[c][r];
    }
}

__global__ void __launch_bounds__(kGT) k_gemm_mfma(GemmDesc g) {
    constexpr int BM = 128, BN = 128, BK = 32, LD = BK + 8;
    // two stages: a K step's MFMAs read one while the next step is
    // converted into the other
    __shared__ __align__(16) __bf16 Ah[2][BM * LD], Al[2][BM * LD];
    __shared__ __align__(16) __bf16 Bh[2][BN * LD], Bl[2][BN * LD];
    const int64_t grp = blockIdx.z;
    const float* A = static_cast<const float*>(g.A) + grp * g.sA;
    const float* B = static_cast<const float*>(g.B) + grp * g.sB;
    float* C = static_cast<float*>(g.C) + grp * g.sC;
    // Workgroups go to the 8 XCDs in turn, each with its own L2.  Where a
    // group's tile count is a multiple of 8, XCD x takes the x-th eighth of
    // the group's tiles in row-major order, so the column tiles of one row
    // tile run on one XCD and share its A rows in that L2 (otherwise every
    // XCD would fetch every A row tile from HBM).  A bijection on the tiles.
    int64_t bx = blockIdx.x, by = blockIdx.y;
    {
        const int64_t tiles = (int64_t)gridDim.x * gridDim.y;
        if (tiles % 8 == 0) {
            const int64_t L = bx + (int64_t)gridDim.x * by;
            const int64_t T = (L % 8) * (tiles / 8) + L / 8;
            bx = T % gridDim.x;
            by = T / gridDim.x;
        }
    }
    const int64_t m0 = by * BM, n0 = bx * BN;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    gf32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = gf32x4{0, 0, 0, 0};
    // Each thread converts one 4 x 4 block (4 rows x 4 k) of each operand
    // per K step.  Along a contiguous k the blocks of 8 consecutive threads
    // are consecutive in k (128 contiguous bytes per row); otherwise 4
    // consecutive threads take consecutive row blocks (64 contiguous bytes
    // per k) and the next ones the next k blocks, so that the 8-byte LDS
    // stores of 32 lanes fall on 64 distinct banks (consecutive row blocks
    // alone are 320 bytes apart, 8 lanes to a bank).
    const bool akc = !g.tA, bkc = g.tB != 0;
    const bool avec = g.lda % 4 == 0 && g.sA % 4 == 0 &&
                      (reinterpret_cast<uintptr_t>(g.A) & 15) == 0;
    const bool bvec = g.ldb % 4 == 0 && g.sB % 4 == 0 &&
                      (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;
    const int rr = (tid & 3) + 4 * (tid >> 5), rk = (tid >> 2) & 7;
    const int abr = akc ? tid >> 3 : rr, abk = akc ? tid & 7 : rk;
    const int bbr = bkc ? tid >> 3 : rr, bbk = bkc ? tid & 7 : rk;
    // two register sets: the loads for K step s + 2 are issued while step s
    // is multiplied and step s + 1 is converted into LDS
    float va0[4][4], vb0[4][4], va1[4][4], vb1[4][4];
    auto fetch = [&](int64_t k0, float (&va)[4][4], float (&vb)[4][4]) {
        load_block(A, g.lda, akc, avec, m0 + 4 * abr, g.M, k0 + 4 * abk, g.K, va);
        load_block(B, g.ldb, bkc, bvec, n0 + 4 * bbr, g.N, k0 + 4 * bbk, g.K, vb);
    };
    // hi = bf16(x), lo = bf16(x - hi); a row's four k go to LDS as 8 bytes
    auto stash = [&](int buf, const float (&va)[4][4], const float (&vb)[4][4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gbf16x4 h, l;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                h[c] = (__bf16)va[r][c];
                l[c] = (__bf16)(va[r][c] - (float)h[c]);
            }
            const int o = (4 * abr + r) * LD + 4 * abk;
            *reinterpret_cast<gbf16x4*>(&Ah[buf][o]) = h;
            *reinterpret_cast<gbf16x4*>(&Al[buf][o]) = l;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gbf16x4 h, l;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                h[c] = (__bf16)vb[r][c];
                l[c] = (__bf16)(vb[r][c] - (float)h[c]);
            }
            const int o = (4 * bbr + r) * LD + 4 * bbk;
            *reinterpret_cast<gbf16x4*>(&Bh[buf][o]) = h;
            if (!g.b_exact) *reinterpret_cast<gbf16x4*>(&Bl[buf][o]) = l;
        }
    };
    // K step k from LDS stage b: loads for k + 2 BK into (fa, fb), the
    // values of step k + BK from (sa, sb) into the other stage
    auto step = [&](int64_t k0, int b, float (&fa)[4][4], float (&fb)[4][4],
                    const float (&sa)[4][4], const float (&sb)[4][4]) {
        if (k0 + 2 * BK < g.K) fetch(k0 + 2 * BK, fa, fb);
        gbf16x8 bh[4], bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int nn = wn * 64 + j * 16 + (lane & 15);
            bh[j] = *reinterpret_cast<const gbf16x8*>(&Bh[b][nn * LD + 8 * (lane >> 4)]);
            if (!g.b_exact)
                bl[j] = *reinterpret_cast<const gbf16x8*>(&Bl[b][nn * LD + 8 * (lane >> 4)]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int mm = wm * 64 + i * 16 + (lane & 15);
            const gbf16x8 ah = *reinterpret_cast<const gbf16x8*>(&Ah[b][mm * LD + 8 * (lane >> 4)]);
            const gbf16x8 al = *reinterpret_cast<const gbf16x8*>(&Al[b][mm * LD + 8 * (lane >> 4)]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
                if (!g.b_exact)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
            }
        }
        if (k0 + BK < g.K) stash(b ^ 1, sa, sb);
        __syncthreads();
    };
    fetch(0, va0, vb0);
    stash(0, va0, vb0);
    if (BK < g.K) fetch(BK, va1, vb1);
    __syncthreads();
    // the two sets are named statically in two copies of the step
    for (int64_t k0 = 0; k0 < g.K; k0 += 2 * BK) {
        step(k0, 0, va0, vb0, va1, vb1);
        if (k0 + BK < g.K) step(k0 + BK, 1, va1, vb1, va0, vb0);
    }
    // D layout: lane holds rows 4*(lane/16) + r of column lane%16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
                const int64_t gn = n0 + wn * 64 + j * 16 + (lane & 15);
                if (gm < g.M && gn < g.N) {
                    float* c = C + gm * g.ldc + gn;
                    *c = g.beta ? *c + acc[i][j][r] : acc[i][j][r];
                }
            }
}

hipError_t launch_gemm_mfma(const GemmDesc& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.groups <= 0) return hipSuccess;
    const int64_t gx = (g.N + 127) / 128, gy = (g.M + 127) / 128;
    if (gx > kGridMax || gy > kGridMax || g.groups > kGridMax)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)gx, (unsigned)gy,
                                        (unsigned)g.groups),
                       dim3(kGT), 0, st, g);
    return hipGetLastError();
}

// ------------------------------------------------------- column reductions
// out[g*os + c] = beta*out + sum_{r < rows} A[(g*rows + r)*lda + c]
//                                         (* B[(g*rows + r)*ldb + c])
template <typename T>
__global__ void __launch_bounds__(kGT) k_colsum(int64_t groups, int64_t rows,
                                                int cols, const T* A,
                                                int64_t lda, const T* B,
                                                int64_t ldb, T* out,
                                                int64_t os, int beta) {
    const int64_t total = groups * cols;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t g = e / cols;
        const int c = (int)(e - g * cols);
        T s = 0;
        // eight rows' loads in flight together; the sum runs in row order
        int64_t r = 0;
        for (; r + 8 <= rows; r += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = A[(g * rows + r + u) * lda + c];
            if (B) {
                T w[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) w[u] = B[(g * rows + r + u) * ldb + c];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] *= w[u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; r < rows; ++r) {
            const int64_t row = g * rows + r;
            T v = A[row * lda + c];
            if (B) v *= B[row * ldb + c];
            s += v;
        }
        T* o = out + g * os + c;
        *o = beta ? *o + s : s;
    }
}

template <typename T>
hipError_t launch_colsum(int64_t groups, int64_t rows, int cols, const T* A,
                         int64_t lda, const T* B, int64_t ldb, T* out,
                         int64_t os, int beta, hipStream_t st) {
    const int64_t total = groups * cols;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_colsum<T>), dim3(cap_grid((total + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, groups, rows, cols, A, lda, B, ldb,
                       out, os, beta);
    return hipGetLastError();
}

// grad[p] = beta*grad[p] + sum_{s < n} part[s*P + p], samples in order.
template <typename T>
__global__ void __launch_bounds__(kGT) k_reduce_samples(int64_t n, int64_t P,
                                                        const T* part, T* grad,
                                                        int beta) {
    for (int64_t p = (int64_t)blockIdx.x * kGT + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * kGT) {
        T s = beta ? grad[p] : (T)0;
        // eight samples' loads in flight together, added in sample order
        int64_t i = 0;
        for (; i + 8 <= n; i += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(i + u) * P + p];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; i < n; ++i) s += part[i * P + p];
        grad[p] = s;
    }
}

template <typename T>
hipError_t launch_reduce_samples(int64_t n, int64_t P, const T* part, T* grad,
                                 int beta, hipStream_t st) {
    hipLaunchKernelGGL((k_reduce_samples<T>), dim3(cap_grid((P + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, n, P, part, grad, beta);
    return hipGetLastError();
}

// coef[s] = 1/2 * (w ? w[s] : 1): the upstream of every position's
// log-probability (log psi = 1/2 sum_i l_i).
template <typename T>
__global__ void k_coef(int64_t n, const double* w, T* coef) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) coef[s] = (T)(0.5 * (w ? w[s] : 1.0));
}

template <typename T>
hipError_t launch_coef(int64_t n, const double* w, T* coef, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_coef<T>), dim3((unsigned)((n + 255) / 256)), dim3(256),
                       0, st, n, w, coef);
    return hipGetLastError();
}

template <typename T>
__global__ void k_fill_t(T* p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kGT)
        p[i] = v;
}

template <typename T>
hipError_t launch_fill_t(T* p, int64_t n, T v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_t<T>), dim3(cap_grid((n + kGT - 1) / kGT)), dim3(kGT),
                       0, st, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------- LayerNorm
// One wave per row: y = xh * g + b with xh = (x - mean) * rstd (biased
// variance, eps 1e-5); xh and rstd are kept for the backward.
// Rows up to 64 kLnCols wide are held in registers by the LN kernels.
constexpr int kLnCols = 4;

template <typename T>
__global__ void __launch_bounds__(kGT) k_ln_save(int64_t R, int d, const T* x,
                                                 const T* g, const T* b, T* y,
                                                 T* xh, T* rstd) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        const T* xr = x + r * d;
        if (d <= 64 * kLnCols) {
            // the row in registers, read once; the same operations in the
            // same order as the general form below
            T xv[kLnCols];
#pragma unroll
            for (int u = 0; u < kLnCols; ++u)
                if (lane + 64 * u < d) xv[u] = xr[lane + 64 * u];
            T s = 0;
#pragma unroll
            for (int u = 0; u < kLnCols; ++u)
                if (lane + 64 * u < d) s += xv[u];
            const T mean = wave_sum(s) / (T)d;
            T v = 0;
#pragma unroll
            for (int u = 0; u < kLnCols; ++u)
                if (lane + 64 * u < d) {
                    const T t = xv[u] - mean;
                    v += t * t;
                }
            v = wave_sum(v) / (T)d;
            const T rs = (T)1 / dsqrt(v + (T)1e-5);
#pragma unroll
            for (int u = 0; u < kLnCols; ++u) {
                const int k = lane + 64 * u;
                if (k < d) {
                    const T h = (xv[u] - mean) * rs;
                    xh[r * d + k] = h;
                    y[r * d + k] = h * g[k] + b[k];
                }
            }
            if (lane == 0) rstd[r] = rs;
            continue;
        }
        T s = 0;
        for (int k = lane; k < d; k += 64) s += xr[k];
        const T mean = wave_sum(s) / (T)d;
        T v = 0;
        for (int k = lane; k < d; k += 64) {
            const T t = xr[k] - mean;
            v += t * t;
        }
        v = wave_sum(v) / (T)d;
        const T rs = (T)1 / dsqrt(v + (T)1e-5);
        for (int k = lane; k < d; k += 64) {
            const T h = (xr[k] - mean) * rs;
            xh[r * d + k] = h;
            y[r * d + k] = h * g[k] + b[k];
        }
        if (lane == 0) rstd[r] = rs;
    }
}

template <typename T>
hipError_t launch_ln_save(int64_t R, int d, const T* x, const T* g, const T* b,
                          T* y, T* xh, T* rstd, hipStream_t st) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ln_save<T>), dim3(cap_grid((R + 3) / 4)), dim3(kGT), 0, st,
                       R, d, x, g, b, y, xh, rstd);
    return hipGetLastError();
}

// out = (base ? base : 0) + LN backward of dy: with e = g * dy,
// dx = rstd * (e - mean(e) - xh * mean(e * xh)).
template <typename T>
__global__ void __launch_bounds__(kGT) k_ln_bwd(int64_t R, int d, const T* xh,
                                                const T* rstd, const T* g,
                                                const T* dy, const T* base,
                                                T* out) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        if (d <= 64 * kLnCols) {
            // e and xh of the row in registers, read once; the same
            // operations in the same order as the general form below
            T ev[kLnCols], hv[kLnCols];
            T s1 = 0, s2 = 0;
#pragma unroll
            for (int u = 0; u < kLnCols; ++u) {
                const int k = lane + 64 * u;
                if (k < d) {
                    ev[u] = g[k] * dy[r * d + k];
                    hv[u] = xh[r * d + k];
                }
            }
#pragma unroll
            for (int u = 0; u < kLnCols; ++u)
                if (lane + 64 * u < d) {
                    s1 += ev[u];
                    s2 += ev[u] * hv[u];
                }
            s1 = wave_sum(s1) / (T)d;
            s2 = wave_sum(s2) / (T)d;
            const T rs = rstd[r];
#pragma unroll
            for (int u = 0; u < kLnCols; ++u) {
                const int k = lane + 64 * u;
                if (k < d) {
                    const T v = rs * (ev[u] - s1 - hv[u] * s2);
                    out[r * d + k] = base ? base[r * d + k] + v : v;
                }
            }
            continue;
        }
        T s1 = 0, s2 = 0;
        for (int k = lane; k < d; k += 64) {
            const T e = g[k] * dy[r * d + k];
            s1 += e;
            s2 += e * xh[r * d + k];
        }
        s1 = wave_sum(s1) / (T)d;
        s2 = wave_sum(s2) / (T)d;
        const T rs = rstd[r];
        for (int k = lane; k < d; k += 64) {
            const T e = g[k] * dy[r * d + k];
            const T v = rs * (e - s1 - xh[r * d + k] * s2);
            out[r * d + k] = base ? base[r * d + k] + v : v;
        }
    }
}

template <typename T>
hipError_t launch_ln_bwd(int64_t R, int d, const T* xh, const T* rstd,
                         const T* g, const T* dy, const T* base, T* out,
                         hipStream_t st) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ln_bwd<T>), dim3(cap_grid((R + 3) / 4)), dim3(kGT), 0, st,
                       R, d, xh, rstd, g, dy, base, out);
    return hipGetLastError();
}

// ------------------------------------------------- recomputed block pieces
// x' = x + b_o + sum_h table[h][code_h] (the forward's order), and the
// quantized vector z = concat_h codebook[h][code_h].
template <typename T>
__global__ void __launch_bounds__(kGT) k_xprime(int64_t R, ModelDims m,
                                                const T* x, const int32_t* codes,
                                                const T* table, const T* b_o,
                                                const T* codebook, T* xp, T* z) {
    const int d = m.d;
    const int64_t total = R * d;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t r = e / d;
        const int k = (int)(e - r * d);
        const int32_t* cd = codes + r * m.H;
        T zz = b_o[k];
        for (int h = 0; h < m.H; ++h)
            zz += table[((int64_t)h * m.Q + cd[h]) * d + k];
        xp[e] = x[e] + zz;
        const int h = k / m.dseg;
        z[e] = codebook[((int64_t)h * m.Q + cd[h]) * m.dseg + (k - h * m.dseg)];
    }
}

template <typename T>
hipError_t launch_xprime(int64_t R, const ModelDims& m, const T* x,
                         const int32_t* codes, const T* table, const T* b_o,
                         const T* codebook, T* xp, T* z, hipStream_t st) {
    const int64_t total = R * m.d;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_xprime<T>), dim3(cap_grid((total + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, R, m, x, codes, table, b_o, codebook, xp, z);
    return hipGetLastError();
}

// u += b1 (in place), g = GELU(u) with the exact erf form.
template <typename T>
__global__ void __launch_bounds__(kGT) k_bias_gelu(int64_t R, int F, T* u,
                                                   const T* b1, T* g) {
    const int64_t total = R * F;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const T v = u[e] + b1[e % F];
        u[e] = v;
        g[e] = gelu_exact(v);
    }
}

template <typename T>
hipError_t launch_bias_gelu(int64_t R, int F, T* u, const T* b1, T* g,
                            hipStream_t st) {
    const int64_t total = R * F;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_bias_gelu<T>), dim3(cap_grid((total + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, R, F, u, b1, g);
    return hipGetLastError();
}

// dg *= GELU'(u) = Phi(u) + u phi(u).
template <typename T>
__global__ void __launch_bounds__(kGT) k_gelu_bwd(int64_t n, const T* u, T* dg) {
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kGT) {
        const T x = u[e];
        const T cdf = (T)0.5 * ((T)1 + derf(x * (T)0.70710678118654752440));
        const T pdf = dexp((T)-0.5 * x * x) * (T)0.39894228040143267794;
        dg[e] *= cdf + x * pdf;
    }
}

template <typename T>
hipError_t launch_gelu_bwd(int64_t n, const T* u, T* dg, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gelu_bwd<T>), dim3(cap_grid((n + kGT - 1) / kGT)), dim3(kGT),
                       0, st, n, u, dg);
    return hipGetLastError();
}

// ---------------------------------------------------------------- head
// One wave per row: f = LNf(x), logits = f W_head + b_head, target y from
// the spin; dlogit_c = coef * ([c == y] - softmax_c); df = W_head dlogit;
// dx = LN backward of df.  Keeps f, xh, rstd, dlogit, df for the parameter
// gradients.
template <typename T>
__global__ void __launch_bounds__(kGT) k_head_bwd(int64_t n, int N, int d,
                                                  HeadW<T> hw,
                                                  const int8_t* spins,
                                                  const T* x, const T* coef,
                                                  T* f, T* xh, T* rstd, T* dz,
                                                  T* df, T* dx) {
    const int lane = threadIdx.x & 63;
    const int64_t R = n * N, wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        const T* xr = x + r * d;
        T s = 0;
        for (int k = lane; k < d; k += 64) s += xr[k];
        const T mean = wave_sum(s) / (T)d;
        T v = 0;
        for (int k = lane; k < d; k += 64) {
            const T t = xr[k] - mean;
            v += t * t;
        }
        v = wave_sum(v) / (T)d;
        const T rs = (T)1 / dsqrt(v + (T)1e-5);
        T z0 = 0, z1 = 0;
        for (int k = lane; k < d; k += 64) {
            const T h = (xr[k] - mean) * rs;
            const T fk = h * hw.lnf_g[k] + hw.lnf_b[k];
            xh[r * d + k] = h;
            f[r * d + k] = fk;
            z0 += fk * hw.W_head[2 * k];
            z1 += fk * hw.W_head[2 * k + 1];
        }
        z0 = wave_sum(z0) + hw.b_head[0];
        z1 = wave_sum(z1) + hw.b_head[1];
        const T mx = z0 > z1 ? z0 : z1;
        const T e0 = dexp(z0 - mx), e1 = dexp(z1 - mx);
        const T p0 = e0 / (e0 + e1), p1 = e1 / (e0 + e1);
        const int y = spins[r] < 0 ? 1 : 0;
        const T c = coef[r / N];
        const T g0 = c * ((y == 0 ? (T)1 : (T)0) - p0);
        const T g1 = c * ((y == 1 ? (T)1 : (T)0) - p1);
        if (lane == 0) {
            dz[2 * r] = g0;
            dz[2 * r + 1] = g1;
            rstd[r] = rs;
        }
        T s1 = 0, s2 = 0;
        for (int k = lane; k < d; k += 64) {
            const T dfk = g0 * hw.W_head[2 * k] + g1 * hw.W_head[2 * k + 1];
            df[r * d + k] = dfk;
            const T e = hw.lnf_g[k] * dfk;
            s1 += e;
            s2 += e * xh[r * d + k];
        }
        s1 = wave_sum(s1) / (T)d;
        s2 = wave_sum(s2) / (T)d;
        for (int k = lane; k < d; k += 64) {
            const T e = hw.lnf_g[k] * df[r * d + k];
            dx[r * d + k] = rs * (e - s1 - xh[r * d + k] * s2);
        }
    }
}

// The same for tokens of K spins: V = 2^K values, logits z_c, target
// t = the token's value (sites iK .. iK+K-1 of the sample), dz[r][c] =
// coef (1[c == t] - p_c) and df = sum_c dz_c W[:, c] (values in order).
template <typename T, int V>
__global__ void __launch_bounds__(kGT) k_head_bwd_v(int64_t n, int N, int d,
                                                    int K, HeadW<T> hw,
                                                    const int8_t* spins,
                                                    const T* x, const T* coef,
                                                    T* f, T* xh, T* rstd, T* dz,
                                                    T* df, T* dx) {
    const int lane = threadIdx.x & 63;
    const int64_t R = n * N, wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        const T* xr = x + r * d;
        T s = 0;
        for (int k = lane; k < d; k += 64) s += xr[k];
        const T mean = wave_sum(s) / (T)d;
        T v = 0;
        for (int k = lane; k < d; k += 64) {
            const T t = xr[k] - mean;
            v += t * t;
        }
        v = wave_sum(v) / (T)d;
        const T rs = (T)1 / dsqrt(v + (T)1e-5);
        T z[V];
#pragma unroll
        for (int c = 0; c < V; ++c) z[c] = 0;
        for (int k = lane; k < d; k += 64) {
            const T h = (xr[k] - mean) * rs;
            const T fk = h * hw.lnf_g[k] + hw.lnf_b[k];
            xh[r * d + k] = h;
            f[r * d + k] = fk;
#pragma unroll
            for (int c = 0; c < V; ++c) z[c] += fk * hw.W_head[k * V + c];
        }
        T mx = neg_inf<T>();
#pragma unroll
        for (int c = 0; c < V; ++c) {
            z[c] = wave_sum(z[c]) + hw.b_head[c];
            mx = z[c] > mx ? z[c] : mx;
        }
        T sum = 0;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            z[c] = dexp(z[c] - mx);
            sum += z[c];
        }
        const int64_t smp = r / N;
        const int y = token_at(spins + smp * (int64_t)N * K, (int)(r - smp * N), K);
        const T cf = coef[smp];
        T g[V];
#pragma unroll
        for (int c = 0; c < V; ++c)
            g[c] = cf * ((c == y ? (T)1 : (T)0) - z[c] / sum);
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < V; ++c) dz[V * r + c] = g[c];
            rstd[r] = rs;
        }
        T s1 = 0, s2 = 0;
        for (int k = lane; k < d; k += 64) {
            T dfk = 0;
#pragma unroll
            for (int c = 0; c < V; ++c) dfk += g[c] * hw.W_head[k * V + c];
            df[r * d + k] = dfk;
            const T e = hw.lnf_g[k] * dfk;
            s1 += e;
            s2 += e * xh[r * d + k];
        }
        s1 = wave_sum(s1) / (T)d;
        s2 = wave_sum(s2) / (T)d;
        for (int k = lane; k < d; k += 64) {
            const T e = hw.lnf_g[k] * df[r * d + k];
            dx[r * d + k] = rs * (e - s1 - xh[r * d + k] * s2);
        }
    }
}

// The encoder's head: log psi = mean_i LN(x_i) . w + b, so the upstream of
// every row's term is 2 coef / N (coef holds half the weight, the
// decoder's factor), dz[r] = that value, df = dz w.
template <typename T>
__global__ void __launch_bounds__(kGT) k_head_bwd_enc(int64_t n, int N, int d,
                                                      HeadW<T> hw, const T* x,
                                                      const T* coef, T* f,
                                                      T* xh, T* rstd, T* dz,
                                                      T* df, T* dx) {
    const int lane = threadIdx.x & 63;
    const int64_t R = n * N, wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        const T* xr = x + r * d;
        T s = 0;
        for (int k = lane; k < d; k += 64) s += xr[k];
        const T mean = wave_sum(s) / (T)d;
        T v = 0;
        for (int k = lane; k < d; k += 64) {
            const T t = xr[k] - mean;
            v += t * t;
        }
        v = wave_sum(v) / (T)d;
        const T rs = (T)1 / dsqrt(v + (T)1e-5);
        for (int k = lane; k < d; k += 64) {
            const T h = (xr[k] - mean) * rs;
            xh[r * d + k] = h;
            f[r * d + k] = h * hw.lnf_g[k] + hw.lnf_b[k];
        }
        const T g0 = (T)2 * coef[r / N] / (T)N;
        if (lane == 0) {
            dz[r] = g0;
            rstd[r] = rs;
        }
        T s1 = 0, s2 = 0;
        for (int k = lane; k < d; k += 64) {
            const T dfk = g0 * hw.W_head[k];
            df[r * d + k] = dfk;
            const T e = hw.lnf_g[k] * dfk;
            s1 += e;
            s2 += e * xh[r * d + k];
        }
        s1 = wave_sum(s1) / (T)d;
        s2 = wave_sum(s2) / (T)d;
        for (int k = lane; k < d; k += 64) {
            const T e = hw.lnf_g[k] * df[r * d + k];
            dx[r * d + k] = rs * (e - s1 - xh[r * d + k] * s2);
        }
    }
}

template <typename T>
hipError_t launch_head_bwd(int64_t n, int N, int d, int K, int enc, const HeadW<T>& hw,
                           const int8_t* spins, const T* x, const T* coef, T* f,
                           T* xh, T* rstd, T* dz, T* df, T* dx, hipStream_t st) {
    const int64_t R = n * N;
    if (R <= 0) return hipSuccess;
    const dim3 g(cap_grid((R + 3) / 4)), b(kGT);
    if (enc) {
        hipLaunchKernelGGL((k_head_bwd_enc<T>), g, b, 0, st, n, N, d, hw, x, coef, f,
                           xh, rstd, dz, df, dx);
        return hipGetLastError();
    }
    switch (K) {
        case 1:
            hipLaunchKernelGGL((k_head_bwd<T>), g, b, 0, st, n, N, d, hw, spins, x,
                               coef, f, xh, rstd, dz, df, dx);
            break;
        case 2:
            hipLaunchKernelGGL((k_head_bwd_v<T, 4>), g, b, 0, st, n, N, d, K, hw,
                               spins, x, coef, f, xh, rstd, dz, df, dx);
            break;
        case 3:
            hipLaunchKernelGGL((k_head_bwd_v<T, 8>), g, b, 0, st, n, N, d, K, hw,
                               spins, x, coef, f, xh, rstd, dz, df, dx);
            break;
        case 4:
            hipLaunchKernelGGL((k_head_bwd_v<T, 16>), g, b, 0, st, n, N, d, K, hw,
                               spins, x, coef, f, xh, rstd, dz, df, dx);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- embedding
// x0_i = tok[u_i] + pos[i] with u_0 = BOS (2), u_i = token of spin i-1.
// Per sample s: dpos = dx0, dtok[t] = sum over positions with input t.
template <typename T>
__global__ void __launch_bounds__(kGT) k_embed_bwd(int64_t n, int N, int d,
                                                   const int8_t* spins,
                                                   const T* dx, T* grad,
                                                   int64_t P, int64_t tok_off,
                                                   int64_t pos_off) {
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t s = e / d;
        const int c = (int)(e - s * d);
        T t0 = 0, t1 = 0, t2 = 0;
        T* g = grad + s * P;
        for (int i = 0; i < N; ++i) {
            const T v = dx[(s * N + i) * d + c];
            g[pos_off + (int64_t)i * d + c] = v;
            if (i == 0) t2 += v;
            else if (spins[s * N + i - 1] < 0) t1 += v;
            else t0 += v;
        }
        g[tok_off + c] = t0;
        g[tok_off + d + c] = t1;
        g[tok_off + 2 * d + c] = t2;
    }
}

// The same for tokens of K spins: inputs u_0 = BOS (2^K), u_i = the value
// of token i-1; V + 1 token rows.
template <typename T, int V>
__global__ void __launch_bounds__(kGT) k_embed_bwd_v(int64_t n, int N, int d,
                                                     int K, int enc,
                                                     const int8_t* spins,
                                                     const T* dx, T* grad,
                                                     int64_t P, int64_t tok_off,
                                                     int64_t pos_off) {
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t s = e / d;
        const int c = (int)(e - s * d);
        T t[V + 1];
#pragma unroll
        for (int k = 0; k <= V; ++k) t[k] = 0;
        T* g = grad + s * P;
        const int8_t* sp = spins + s * (int64_t)N * K;
        for (int i = 0; i < N; ++i) {
            const T v = dx[(s * N + i) * d + c];
            g[pos_off + (int64_t)i * d + c] = v;
            // the encoder reads the token itself (V rows, no BOS)
            const int u = enc ? token_at(sp, i, K)
                              : (i == 0 ? V : token_at(sp, i - 1, K));
#pragma unroll
            for (int k = 0; k <= V; ++k)
                if (k == u) t[k] += v;
        }
        const int rows = enc ? V : V + 1;
#pragma unroll
        for (int k = 0; k <= V; ++k)
            if (k < rows) g[tok_off + (int64_t)k * d + c] = t[k];
    }
}

template <typename T>
hipError_t launch_embed_bwd(int64_t n, int N, int d, int K, int enc,
                            const int8_t* spins, const T* dx, T* grad, int64_t P,
                            int64_t tok_off, int64_t pos_off, hipStream_t st) {
    const int64_t total = n * d;
    if (total <= 0) return hipSuccess;
    const dim3 g(cap_grid((total + kGT - 1) / kGT)), b(kGT);
    switch (K) {
        case 1:
            if (enc)
                hipLaunchKernelGGL((k_embed_bwd_v<T, 2>), g, b, 0, st, n, N, d, K, enc,
                                   spins, dx, grad, P, tok_off, pos_off);
            else
                hipLaunchKernelGGL((k_embed_bwd<T>), g, b, 0, st, n, N, d, spins, dx,
                                   grad, P, tok_off, pos_off);
            break;
        case 2:
            hipLaunchKernelGGL((k_embed_bwd_v<T, 4>), g, b, 0, st, n, N, d, K, enc,
                               spins, dx, grad, P, tok_off, pos_off);
            break;
        case 3:
            hipLaunchKernelGGL((k_embed_bwd_v<T, 8>), g, b, 0, st, n, N, d, K, enc,
                               spins, dx, grad, P, tok_off, pos_off);
            break;
        case 4:
            hipLaunchKernelGGL((k_embed_bwd_v<T, 16>), g, b, 0, st, n, N, d, K, enc,
                               spins, dx, grad, P, tok_off, pos_off);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- quantizer
// One wave per row, quantizer head h: S holds a_h . W_j and E holds
// g_h . W_j on entry; on exit S holds G_j = t_j / delta_j and
// rowG[r] = sum_j G_j (E is left as it was).
// Codebooks up to 64 kVqBwdCols codes keep a row's values in registers.
constexpr int kVqBwdCols = 16;

template <typename T>
__global__ void __launch_bounds__(kGT) k_vq_bwd_rows(int64_t R, int Q, int dseg,
                                                     int H, int h, const T* a,
                                                     int lda,
                                                     const int32_t* codes,
                                                     const T* w2, T* S, T* E,
                                                     T* rowG) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = kGT / 64;
    for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < R;
         r += (int64_t)gridDim.x * wpb) {
        const T* ar = a + r * lda;
        T a2 = 0;
        for (int c = lane; c < dseg; c += 64) a2 += ar[c] * ar[c];
        a2 = wave_sum(a2);
        T* Sr = S + r * Q;
        T* Er = E + r * Q;
        const int code = codes[r * H + h];
        if (Q <= 64 * kVqBwdCols) {
            // the row's products and upstream values in registers: each is
            // read once and written once (the general form below reads S
            // three times), with the same operations in the same order
            constexpr int U = kVqBwdCols;
            T sv[U], ev[U], pt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = lane + 64 * u;
                if (j < Q) {
                    sv[u] = Sr[j];
                    ev[u] = Er[j];
                }
            }
            T dmin = -neg_inf<T>();
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = lane + 64 * u;
                if (j < Q) {
                    T q2 = a2 - (T)2 * sv[u] + w2[j];
                    q2 = q2 > (T)0 ? q2 : (T)0;
                    const T dl = dsqrt(q2);
                    sv[u] = dl;
                    dmin = dl < dmin ? dl : dmin;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const T other = __shfl_xor(dmin, o, 64);
                dmin = other < dmin ? other : dmin;
            }
            T l = 0, pe = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (lane + 64 * u < Q) {
                    pt[u] = dexp(dmin - sv[u]);
                    l += pt[u];
                    pe += pt[u] * ev[u];
                }
            }
            l = wave_sum(l);
            pe = wave_sum(pe) / l;
            T gs = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = lane + 64 * u;
                if (j < Q) {
                    const T dl = sv[u];
                    const T p = pt[u] / l;
                    const T t = p * (ev[u] - pe);
                    const T G = dl > (T)0 ? t / dl : (T)0;
                    Sr[j] = G;
                    gs += G;
                }
            }
            gs = wave_sum(gs);
            if (lane == 0) rowG[r] = gs;
            continue;
        }
        // distances (kept in S) and their minimum
        T dmin = -neg_inf<T>();
        for (int j = lane; j < Q; j += 64) {
            T q2 = a2 - (T)2 * Sr[j] + w2[j];
            q2 = q2 > (T)0 ? q2 : (T)0;
            const T dl = dsqrt(q2);
            Sr[j] = dl;
            dmin = dl < dmin ? dl : dmin;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const T other = __shfl_xor(dmin, o, 64);
            dmin = other < dmin ? other : dmin;
        }
        T l = 0, pe = 0;
        for (int j = lane; j < Q; j += 64) {
            const T pt = dexp(dmin - Sr[j]);
            l += pt;
            pe += pt * Er[j];
        }
        l = wave_sum(l);
        pe = wave_sum(pe) / l;
        T gs = 0;
        for (int j = lane; j < Q; j += 64) {
            const T dl = Sr[j];
            const T p = dexp(dmin - dl) / l;
            const T t = p * (Er[j] - pe);
            const T G = dl > (T)0 ? t / dl : (T)0;
            Sr[j] = G;
            gs += G;
        }
        gs = wave_sum(gs);
        if (lane == 0) rowG[r] = gs;
    }
}

template <typename T>
hipError_t launch_vq_bwd_rows(int64_t R, int Q, int dseg, int H, int h,
                              const T* a, int lda, const int32_t* codes,
                              const T* w2, T* S, T* E, T* rowG, hipStream_t st) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_vq_bwd_rows<T>), dim3(cap_grid((R + 3) / 4)), dim3(kGT), 0,
                       st, R, Q, dseg, H, h, a, lda, codes, w2, S, E, rowG);
    return hipGetLastError();
}

// da[r][c] -= rowG[r] * a[r][c] over the columns of one quantizer head.
template <typename T>
__global__ void __launch_bounds__(kGT) k_da_fix(int64_t R, int dseg, int ld,
                                                const T* a, const T* rowG,
                                                T* da) {
    const int64_t total = R * dseg;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t r = e / dseg;
        const int c = (int)(e - r * dseg);
        da[r * ld + c] -= rowG[r] * a[r * ld + c];
    }
}

template <typename T>
hipError_t launch_da_fix(int64_t R, int dseg, int ld, const T* a,
                         const T* rowG, T* da, hipStream_t st) {
    const int64_t total = R * dseg;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_da_fix<T>), dim3(cap_grid((total + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, R, dseg, ld, a, rowG, da);
    return hipGetLastError();
}

// dcb[g][j][c] -= colG[g][j] * cb[j][c] (per sample g; dcb stride P).
template <typename T>
__global__ void __launch_bounds__(kGT) k_cb_fix(int64_t n, int Q, int dseg,
                                                const T* colG, const T* cb,
                                                T* dcb, int64_t P) {
    const int64_t per = (int64_t)Q * dseg, total = n * per;
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kGT) {
        const int64_t g = e / per;
        const int64_t jc = e - g * per;
        const int j = (int)(jc / dseg);
        dcb[g * P + jc] -= colG[g * Q + j] * cb[jc];
    }
}

template <typename T>
hipError_t launch_cb_fix(int64_t n, int Q, int dseg, const T* colG, const T* cb,
                         T* dcb, int64_t P, hipStream_t st) {
    const int64_t total = n * (int64_t)Q * dseg;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_cb_fix<T>), dim3(cap_grid((total + kGT - 1) / kGT)),
                       dim3(kGT), 0, st, n, Q, dseg, colG, cb, dcb, P);
    return hipGetLastError();
}

// The one-hot factor of eq. (8): dcb[g][code_r][c] += g_r[c] over the rows
// r of sample g in row order (one workgroup per sample, a thread per
// column), so the codebook gradient needs no product with a one-hot matrix.
template <typename T>
__global__ void __launch_bounds__(kGT) k_onehot_scatter(int64_t n, int N,
                                                        int dseg, int ld, int H,
                                                        int h,
                                                        const int32_t* codes,
                                                        const T* g, T* dcb,
                                                        int64_t P) {
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        T* out = dcb + s * P;
        const int32_t* cs = codes + s * (int64_t)N * H + h;
        const T* gs = g + s * (int64_t)N * ld;
        for (int c = threadIdx.x; c < dseg; c += kGT)
            for (int r = 0; r < N; ++r)
                out[(int64_t)cs[(int64_t)r * H] * dseg + c] +=
                    gs[(int64_t)r * ld + c];
    }
}

template <typename T>
hipError_t launch_onehot_scatter(int64_t n, int N, int dseg, int ld, int H,
                                 int h, const int32_t* codes, const T* g,
                                 T* dcb, int64_t P, hipStream_t st) {
    if (n <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_onehot_scatter<T>), dim3(cap_grid(n)), dim3(kGT), 0,
                       st, n, N, dseg, ld, H, h, codes, g, dcb, P);
    return hipGetLastError();
}

// --------------------------------------------------------------- attention
// a . b over DH terms as four interleaved partial sums (c mod 4), added as
// (s0 + s1) + (s2 + s3): four independent FMA chains instead of one.
template <typename T, int DH>
__device__ inline T dot4(const T* a, const T* b) {
    static_assert(DH % 4 == 0, "head width a multiple of 4");
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int c = 0; c < DH; c += 4) {
        s0 += a[c] * b[c];
        s1 += a[c + 1] * b[c + 1];
        s2 += a[c + 2] * b[c + 2];
        s3 += a[c + 3] * b[c + 3];
    }
    return (s0 + s1) + (s2 + s3);
}

// Rows 0..N-1 of one head (DH columns at base + row * d) into an LDS tile
// [N][DH]: 16-byte loads, four per thread issued before their stores.
template <typename T, int DH, int NT>
__device__ inline void fill_tile(T* dst, const T* src, int64_t base, int N,
                                 int d) {
    constexpr int V = 16 / (int)sizeof(T);       // elements per 16 bytes
    static_assert(DH % V == 0, "whole 16-byte pieces per row");
    constexpr int G = DH / V, U = 4;
    typedef __attribute__((ext_vector_type(V))) T vec;
    const int tot = N * G;
    for (int e0 = 0; e0 < tot; e0 += NT * U) {
        vec v[U];
        int row[U], c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + NT * u + (int)threadIdx.x;
            const int ec = e < tot ? e : tot - 1;
            row[u] = ec / G;
            c[u] = (ec % G) * V;
            v[u] = *reinterpret_cast<const vec*>(src + base + (int64_t)row[u] * d + c[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + NT * u + (int)threadIdx.x < tot)
                *reinterpret_cast<vec*>(dst + row[u] * DH + c[u]) = v[u];
    }
}

// The dq pass holds the next key and value rows in registers (loaded from
// LDS while the current ones are used) where they fit beside a thread's
// other vectors.
template <typename T, int DH>
constexpr bool kPipeRows = sizeof(T) * DH <= 128 && (sizeof(T) == 4 || DH <= 8);

// Row j of an LDS tile [N][DH] into registers.
template <typename T, int DH>
__device__ inline void lds_row(const T* tile, int j, T (&r)[DH]) {
#pragma unroll
    for (int c = 0; c < DH; ++c) r[c] = tile[j * DH + c];
}

// One workgroup per (sample, head).  Scores s_ij = q_i . k_j / sqrt(d_head)
// for j <= i; P = softmax_j(s).  lse_i = log sum_j exp(s_ij), and
// Dd_i = dO_i . O_i (O = the forward attention output).
template <typename T, int DH, int NT>
__global__ void __launch_bounds__(NT) k_attn_stats(int64_t n, ModelDims m,
                                                    const T* q, const T* k,
                                                    const T* o, const T* dO,
                                                    T* lse, T* Dd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Ks = reinterpret_cast<T*>(smem_raw);
    const int N = m.N, d = m.d, nh = m.nh;
    const T scale = (T)1 / dsqrt((T)DH);
    for (int64_t u = blockIdx.x; u < n * nh; u += gridDim.x) {
        const int64_t s = u / nh;
        const int h = (int)(u - s * nh);
        const int64_t base = s * N * d + h * DH;
        __syncthreads();
        fill_tile<T, DH, NT>(Ks, k, base, N, d);
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += NT) {
            T qi[DH];
            T dd = 0;
#pragma unroll
            for (int c = 0; c < DH; ++c) {
                qi[c] = q[base + (int64_t)i * d + c];
                dd += dO[base + (int64_t)i * d + c] * o[base + (int64_t)i * d + c];
            }
            T mx = neg_inf<T>(), l = 0;
            const int jmax = m.enc ? N - 1 : i;   // the encoder sees every key
            for (int j = 0; j <= jmax; ++j) {
                T sc = dot4<T, DH>(qi, Ks + j * DH);
                sc *= scale;
                if (sc > mx) {
                    l = l * dexp(mx - sc) + (T)1;
                    mx = sc;
                } else {
                    l += dexp(sc - mx);
                }
            }
            lse[(s * N + i) * nh + h] = mx + dlog(l);
            Dd[(s * N + i) * nh + h] = dd;
        }
    }
}

// dq_i = scale * sum_{j <= i} dS_ij k_j with dS_ij = P_ij (dO_i . v_j - Dd_i).
template <typename T, int DH, int NT>
__global__ void __launch_bounds__(NT) k_attn_bwd_q(int64_t n, ModelDims m,
                                                    const T* q, const T* k,
                                                    const T* v, const T* dO,
                                                    const T* lse, const T* Dd,
                                                    T* dqkv) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Ks = reinterpret_cast<T*>(smem_raw);
    T* Vs = Ks + m.N * DH;
    const int N = m.N, d = m.d, nh = m.nh;
    const T scale = (T)1 / dsqrt((T)DH);
    for (int64_t u = blockIdx.x; u < n * nh; u += gridDim.x) {
        const int64_t s = u / nh;
        const int h = (int)(u - s * nh);
        const int64_t base = s * N * d + h * DH;
        __syncthreads();
        fill_tile<T, DH, NT>(Ks, k, base, N, d);
        fill_tile<T, DH, NT>(Vs, v, base, N, d);
        __syncthreads();
        // A wave walks the keys 0 .. (its last row) together; keys after a
        // lane's own row add exact zeros (p = 0), which leave its sums as
        // they are, so a lane's terms and their order are those of its row.
        for (int i0 = 0; i0 < N; i0 += NT) {
            const int wf = i0 + (int)(threadIdx.x & ~63);
            if (wf >= N) continue;
            const int i = i0 + (int)threadIdx.x;
            const int ir = i < N ? i : N - 1;
            const int jmax = m.enc ? N - 1 : min(wf + 63, N - 1);
            T qi[DH], gi[DH], acc[DH];
#pragma unroll
            for (int c = 0; c < DH; ++c) {
                qi[c] = q[base + (int64_t)ir * d + c];
                gi[c] = dO[base + (int64_t)ir * d + c];
                acc[c] = 0;
            }
            const T ls = lse[(s * N + ir) * nh + h], dd = Dd[(s * N + ir) * nh + h];
            auto term = [&](int j, const T* kc, const T* vc) {
                const T sc = dot4<T, DH>(qi, kc);
                const T dp = dot4<T, DH>(gi, vc);
                const T e = dexp(sc * scale - ls);
                const T p = (m.enc || j <= ir) ? e : (T)0;
                const T ds = p * (dp - dd);
#pragma unroll
                for (int c = 0; c < DH; ++c) acc[c] += ds * kc[c];
            };
            if constexpr (kPipeRows<T, DH>) {
                T ka[DH], va[DH], kb[DH], vb[DH];
                lds_row<T, DH>(Ks, 0, ka);
                lds_row<T, DH>(Vs, 0, va);
                for (int j = 0; j <= jmax; j += 2) {
                    if (j + 1 <= jmax) {
                        lds_row<T, DH>(Ks, j + 1, kb);
                        lds_row<T, DH>(Vs, j + 1, vb);
                    }
                    term(j, ka, va);
                    if (j + 1 > jmax) break;
                    if (j + 2 <= jmax) {
                        lds_row<T, DH>(Ks, j + 2, ka);
                        lds_row<T, DH>(Vs, j + 2, va);
                    }
                    term(j + 1, kb, vb);
                }
            } else {
                for (int j = 0; j <= jmax; ++j) term(j, Ks + j * DH, Vs + j * DH);
            }
            if (i < N) {
                T* out = dqkv + (s * N + i) * 3 * d + h * DH;
#pragma unroll
                for (int c = 0; c < DH; ++c) out[c] = acc[c] * scale;
            }
        }
    }
}

// dk_j = scale * sum_{i >= j} dS_ij q_i,  dv_j = sum_{i >= j} P_ij dO_i.
template <typename T, int DH, int NT>
__global__ void __launch_bounds__(NT) k_attn_bwd_kv(int64_t n, ModelDims m,
                                                     const T* q, const T* k,
                                                     const T* v, const T* dO,
                                                     const T* lse, const T* Dd,
                                                     T* dqkv) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Qs = reinterpret_cast<T*>(smem_raw);
    T* Gs = Qs + m.N * DH;
    T* Ls = Gs + m.N * DH;
    T* Ds = Ls + m.N;
    const int N = m.N, d = m.d, nh = m.nh;
    const T scale = (T)1 / dsqrt((T)DH);
    for (int64_t u = blockIdx.x; u < n * nh; u += gridDim.x) {
        const int64_t s = u / nh;
        const int h = (int)(u - s * nh);
        const int64_t base = s * N * d + h * DH;
        __syncthreads();
        fill_tile<T, DH, NT>(Qs, q, base, N, d);
        fill_tile<T, DH, NT>(Gs, dO, base, N, d);
        for (int i = threadIdx.x; i < N; i += NT) {
            Ls[i] = lse[(s * N + i) * nh + h];
            Ds[i] = Dd[(s * N + i) * nh + h];
        }
        __syncthreads();
        // The lanes of a wave walk the same query i from the wave's first
        // key, so every LDS read is a broadcast; a lane's terms for queries
        // before its own key are exact zeros, which leave its sums as they
        // would be without them.
        for (int jb = 0; jb < N; jb += NT) {
            const int jw = jb + (threadIdx.x & ~63);     // the wave's first key
            if (jw >= N) continue;
            const int j = jb + threadIdx.x;
            const bool live = j < N;
            const int jr = live ? j : N - 1;
            T kj[DH], vj[DH], dk[DH], dv[DH];
#pragma unroll
            for (int c = 0; c < DH; ++c) {
                kj[c] = k[base + (int64_t)jr * d + c];
                vj[c] = v[base + (int64_t)jr * d + c];
                dk[c] = 0;
                dv[c] = 0;
            }
            for (int i = m.enc ? 0 : jw; i < N; ++i) {
                const T sc = dot4<T, DH>(kj, Qs + i * DH);
                const T dp = dot4<T, DH>(vj, Gs + i * DH);
                const T p = (m.enc || i >= j) ? dexp(sc * scale - Ls[i]) : (T)0;
                const T ds = p * (dp - Ds[i]);
#pragma unroll
                for (int c = 0; c < DH; ++c) {
                    dv[c] += p * Gs[i * DH + c];
                    dk[c] += ds * Qs[i * DH + c];
                }
            }
            if (live) {
                T* out = dqkv + (s * N + j) * 3 * d + h * DH;
#pragma unroll
                for (int c = 0; c < DH; ++c) {
                    out[d + c] = dk[c] * scale;
                    out[2 * d + c] = dv[c];
                }
            }
        }
    }
}

// ------------------------------------ attention backward on the matrix core
// The dq pass and the key-side pass of the FP32 arithmetic on the matrix
// core: v_mfma_f32_16x16x4_f32, where lane l holds A[l%16][l/16] and
// B[l/16][l%16] of a 16x4 by 4x16 product and D[4(l/16)+r][l%16] (r < 4).
// The quantities are those of k_attn_bwd_q / k_attn_bwd_kv in FP32 (no
// operand splitting), summed in another order.  A wave owns a tile of 16
// queries (dq pass) or 16 keys (key-side pass) and walks the blocks of 16
// keys (queries) it attends to; the other side's rows sit in LDS as FP32
// rows of stride DH + 4.
//
// dq pass, per key block: S^T = K Q^T and dP^T = V dO^T leave lane
// (g, c) with keys 4g..4g+3 of query c; dS^T = P^T (dP^T - Dd) is then the
// B operand of dq^T += K^T dS^T when the contraction index of k-step kk in
// lane group g is key 4g + kk (the A operand reads K in the same order).
// The key-side pass is the mirror image: S = Q K^T and dP = dO V^T leave
// lane (g, c) with queries 4g..4g+3 of key c, the B operand of
// dv^T += dO^T P and dk^T += Q^T dS.
typedef __attribute__((ext_vector_type(4))) float f32x4b;

__device__ inline f32x4b mfma_f32(float a, float b, f32x4b c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int DH>
constexpr int kBwdLd = DH + 4;      // LDS row stride in floats

// Rows 0..Np-1 (Np = N rounded up to 16) of one head into an LDS tile of
// stride LD; rows from N on are zero (they enter products as exact zeros).
template <int DH, int LD, int NT>
__device__ inline void fill_rows(float* dst, const float* src, int64_t base,
                                 int N, int Np, int d) {
    constexpr int G = DH / 4, U = 4;
    const int tot = Np * G;
    for (int e0 = 0; e0 < tot; e0 += NT * U) {
        float4 v[U];
        int row[U], c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + NT * u + (int)threadIdx.x;
            const int ec = e < tot ? e : tot - 1;
            row[u] = ec / G;
            c[u] = (ec % G) * 4;
            const int rr = row[u] < N ? row[u] : N - 1;
            v[u] = *reinterpret_cast<const float4*>(src + base + (int64_t)rr * d + c[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + NT * u + (int)threadIdx.x < tot)
                *reinterpret_cast<float4*>(dst + row[u] * LD + c[u]) =
                    row[u] < N ? v[u] : float4{0.f, 0.f, 0.f, 0.f};
    }
}

// Whether tile i (tiles in falling order of cost) is this wave's: snake
// order over the waves, largest first.
template <int NW>
__device__ inline bool snake_mine(int i, int wave) {
    const int r = i % (2 * NW);
    return (r < NW ? r : 2 * NW - 1 - r) == wave;
}

template <int DH, int NT>
__global__ void __launch_bounds__(NT) k_attn_bwd_q_mfma(
    int64_t n, ModelDims m, const float* q, const float* k, const float* v,
    const float* dO, const float* lse, const float* Dd, float* dqkv) {
    constexpr int LD = kBwdLd<DH>, KS = DH / 4, MB = DH / 16, NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int N = m.N, d = m.d, nh = m.nh;
    const int Np = (N + 15) & ~15, NTQ = Np / 16;
    float* Ks = reinterpret_cast<float*>(smem_raw);
    float* Vs = Ks + Np * LD;
    const float scale = 1.0f / sqrtf((float)DH);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c16 = lane & 15;
    for (int64_t u = blockIdx.x; u < n * nh; u += gridDim.x) {
        const int64_t s = u / nh;
        const int h = (int)(u - s * nh);
        const int64_t base = s * N * d + h * DH;
        __syncthreads();
        fill_rows<DH, LD, NT>(Ks, k, base, N, Np, d);
        fill_rows<DH, LD, NT>(Vs, v, base, N, Np, d);
        __syncthreads();
        // query tile t has t + 1 key blocks: the largest first
        for (int i = 0; i < NTQ; ++i) {
            if (!snake_mine<NW>(i, wave)) continue;
            const int t = NTQ - 1 - i;
            const int iq = t * 16 + c16;              // this lane's query
            const int iqr = iq < N ? iq : N - 1;
            float qf[KS], gf[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                qf[ks] = q[base + (int64_t)iqr * d + 4 * ks + g];
                gf[ks] = dO[base + (int64_t)iqr * d + 4 * ks + g];
            }
            const float ls = lse[(s * N + iqr) * nh + h];
            const float dd = Dd[(s * N + iqr) * nh + h];
            f32x4b acc[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4b{0, 0, 0, 0};
            const int kbn = m.enc ? NTQ - 1 : t;      // the encoder: every key
            for (int kb = 0; kb <= kbn; ++kb) {
                const float* kr = Ks + (kb * 16 + c16) * LD + g;
                const float* vr = Vs + (kb * 16 + c16) * LD + g;
                f32x4b sc = f32x4b{0, 0, 0, 0}, dp = f32x4b{0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    sc = mfma_f32(kr[4 * ks], qf[ks], sc);
                    dp = mfma_f32(vr[4 * ks], gf[ks], dp);
                }
                float ds[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int key = kb * 16 + 4 * g + r;
                    const float p = (m.enc || key <= iq) && key < N
                                        ? dexp(sc[r] * scale - ls) : 0.0f;
                    ds[r] = p * (dp[r] - dd);
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const float* ka = Ks + (kb * 16 + 4 * g + kk) * LD + c16;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[mb] = mfma_f32(ka[16 * mb], ds[kk], acc[mb]);
                }
            }
            if (iq < N) {
                float* out = dqkv + (s * N + iq) * 3 * d + h * DH;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    *reinterpret_cast<float4*>(out + 16 * mb + 4 * g) =
                        float4{acc[mb][0] * scale, acc[mb][1] * scale,
                               acc[mb][2] * scale, acc[mb][3] * scale};
            }
        }
    }
}

template <int DH, int NT>
__global__ void __launch_bounds__(NT) k_attn_bwd_kv_mfma(
    int64_t n, ModelDims m, const float* q, const float* k, const float* v,
    const float* dO, const float* lse, const float* Dd, float* dqkv) {
    constexpr int LD = kBwdLd<DH>, KS = DH / 4, MB = DH / 16, NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int N = m.N, d = m.d, nh = m.nh;
    const int Np = (N + 15) & ~15, NTQ = Np / 16;
    float* Qs = reinterpret_cast<float*>(smem_raw);
    float* Gs = Qs + Np * LD;
    float* Ls = Gs + Np * LD;
    float* Ds = Ls + Np;
    const float scale = 1.0f / sqrtf((float)DH);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c16 = lane & 15;
    for (int64_t u = blockIdx.x; u < n * nh; u += gridDim.x) {
        const int64_t s = u / nh;
        const int h = (int)(u - s * nh);
        const int64_t base = s * N * d + h * DH;
        __syncthreads();
        fill_rows<DH, LD, NT>(Qs, q, base, N, Np, d);
        fill_rows<DH, LD, NT>(Gs, dO, base, N, Np, d);
        for (int i = threadIdx.x; i < Np; i += NT) {
            Ls[i] = i < N ? lse[(s * N + i) * nh + h] : 0.0f;
            Ds[i] = i < N ? Dd[(s * N + i) * nh + h] : 0.0f;
        }
        __syncthreads();
        // key tile t has NTQ - t query blocks: the largest first
        for (int i = 0; i < NTQ; ++i) {
            if (!snake_mine<NW>(i, wave)) continue;
            const int t = i;
            const int jk = t * 16 + c16;              // this lane's key
            const int jkr = jk < N ? jk : N - 1;
            float kf[KS], vf[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kf[ks] = k[base + (int64_t)jkr * d + 4 * ks + g];
                vf[ks] = v[base + (int64_t)jkr * d + 4 * ks + g];
            }
            f32x4b dk[MB], dv[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                dk[mb] = f32x4b{0, 0, 0, 0};
                dv[mb] = f32x4b{0, 0, 0, 0};
            }
            for (int qb = m.enc ? 0 : t; qb < NTQ; ++qb) {
                const float* qr = Qs + (qb * 16 + c16) * LD + g;
                const float* gr = Gs + (qb * 16 + c16) * LD + g;
                f32x4b sc = f32x4b{0, 0, 0, 0}, dp = f32x4b{0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    sc = mfma_f32(qr[4 * ks], kf[ks], sc);
                    dp = mfma_f32(gr[4 * ks], vf[ks], dp);
                }
                float p[4], ds[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int qi = qb * 16 + 4 * g + r;
                    p[r] = (m.enc || qi >= jk) && qi < N ? dexp(sc[r] * scale - Ls[qi])
                                                         : 0.0f;
                    ds[r] = p[r] * (dp[r] - Ds[qi]);
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int qrow = (qb * 16 + 4 * g + kk) * LD + c16;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        dv[mb] = mfma_f32(Gs[qrow + 16 * mb], p[kk], dv[mb]);
                        dk[mb] = mfma_f32(Qs[qrow + 16 * mb], ds[kk], dk[mb]);
                    }
                }
            }
            if (jk < N) {
                float* out = dqkv + (s * N + jk) * 3 * d + h * DH;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    *reinterpret_cast<float4*>(out + d + 16 * mb + 4 * g) =
                        float4{dk[mb][0] * scale, dk[mb][1] * scale,
                               dk[mb][2] * scale, dk[mb][3] * scale};
                    *reinterpret_cast<float4*>(out + 2 * d + 16 * mb + 4 * g) =
                        float4{dv[mb][0], dv[mb][1], dv[mb][2], dv[mb][3]};
                }
            }
        }
    }
}

template <int DH>
static size_t bwd_mfma_lds(const ModelDims& m, bool kv) {
    const size_t Np = (size_t)((m.N + 15) & ~15);
    return sizeof(float) * (2 * Np * kBwdLd<DH> + (kv ? 2 * Np : 0));
}

// Kernels whose dynamic LDS exceeds 64 KiB must opt in before launch.
template <typename F>
static hipError_t lds_attr(F f, size_t sm) {
    if (sm > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sm);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int DH, int NT>
static hipError_t attn_bwd_nt(int64_t n, const ModelDims& m, const T* q,
                              const T* k, const T* v, const T* o, const T* dO,
                              T* lse, T* Dd, T* dqkv, unsigned g, hipStream_t st) {
    const size_t s1 = sizeof(T) * (size_t)m.N * DH;
    const size_t s2 = 2 * s1;
    const size_t s3 = 2 * s1 + 2 * sizeof(T) * (size_t)m.N;
    hipError_t e;
    // the statistics pass keeps 256 threads: its tile leaves room for three
    // workgroups per CU, which its registers allow at that size only
    if ((e = lds_attr(k_attn_stats<T, DH, kGT>, s1))) return e;
    hipLaunchKernelGGL((k_attn_stats<T, DH, kGT>), dim3(g), dim3(kGT), s1, st, n, m, q, k,
                       o, dO, lse, Dd);
    if ((e = hipGetLastError())) return e;
    if ((e = lds_attr(k_attn_bwd_q<T, DH, NT>, s2))) return e;
    hipLaunchKernelGGL((k_attn_bwd_q<T, DH, NT>), dim3(g), dim3(NT), s2, st, n, m, q, k,
                       v, dO, lse, Dd, dqkv);
    if ((e = hipGetLastError())) return e;
    if ((e = lds_attr(k_attn_bwd_kv<T, DH, NT>, s3))) return e;
    hipLaunchKernelGGL((k_attn_bwd_kv<T, DH, NT>), dim3(g), dim3(NT), s3, st, n, m, q, k,
                       v, dO, lse, Dd, dqkv);
    return hipGetLastError();
}

// Statistics pass, then the dq and key-side passes on the matrix core.
template <int DH, int NT>
static hipError_t attn_bwd_mfma_nt(int64_t n, const ModelDims& m,
                                   const float* q, const float* k,
                                   const float* v, const float* o,
                                   const float* dO, float* lse, float* Dd,
                                   float* dqkv, unsigned g, hipStream_t st) {
    const size_t s1 = sizeof(float) * (size_t)m.N * DH;
    const size_t sq = bwd_mfma_lds<DH>(m, false), skv = bwd_mfma_lds<DH>(m, true);
    hipError_t e;
    if ((e = lds_attr(k_attn_stats<float, DH, kGT>, s1))) return e;
    hipLaunchKernelGGL((k_attn_stats<float, DH, kGT>), dim3(g), dim3(kGT), s1, st, n, m,
                       q, k, o, dO, lse, Dd);
    if ((e = hipGetLastError())) return e;
    if ((e = lds_attr(k_attn_bwd_q_mfma<DH, NT>, sq))) return e;
    hipLaunchKernelGGL((k_attn_bwd_q_mfma<DH, NT>), dim3(g), dim3(NT), sq, st, n, m, q,
                       k, v, dO, lse, Dd, dqkv);
    if ((e = hipGetLastError())) return e;
    if ((e = lds_attr(k_attn_bwd_kv_mfma<DH, NT>, skv))) return e;
    hipLaunchKernelGGL((k_attn_bwd_kv_mfma<DH, NT>), dim3(g), dim3(NT), skv, st, n, m,
                       q, k, v, dO, lse, Dd, dqkv);
    return hipGetLastError();
}

template <typename T, int DH>
static hipError_t attn_bwd_dh(int64_t n, const ModelDims& m, const T* q,
                              const T* k, const T* v, const T* o, const T* dO,
                              T* lse, T* Dd, T* dqkv, hipStream_t st) {
    const unsigned g = cap_grid(n * m.nh);
    // FP32: the matrix-core passes where the two row tiles fit the LDS
    // (1024 threads past 256 rows, whose tiles leave room for one workgroup
    // per CU only: four waves per SIMD)
    if constexpr (std::is_same<T, float>::value && DH % 16 == 0 && DH <= 64)
        if (bwd_mfma_lds<DH>(m, true) <= 160 * 1024)
            return m.N > kGT
                       ? attn_bwd_mfma_nt<DH, 4 * kGT>(n, m, q, k, v, o, dO, lse, Dd, dqkv, g, st)
                       : attn_bwd_mfma_nt<DH, kGT>(n, m, q, k, v, o, dO, lse, Dd, dqkv, g, st);
    // One thread per query (per key in the key-side pass).  Past 256 rows
    // the dq and key-side passes run 512 threads: up to 512 rows in one
    // round, two waves per SIMD where their tiles leave room for one
    // workgroup per CU only.  Only where a thread's row vectors fit the
    // registers of two waves per SIMD.
    if constexpr (sizeof(T) * DH <= 128)
        if (m.N > kGT)
            return attn_bwd_nt<T, DH, 2 * kGT>(n, m, q, k, v, o, dO, lse, Dd,
                                               dqkv, g, st);
    return attn_bwd_nt<T, DH, kGT>(n, m, q, k, v, o, dO, lse, Dd, dqkv, g, st);
}

template <typename T>
hipError_t launch_attn_bwd(int64_t n, const ModelDims& m, const T* q,
                           const T* k, const T* v, const T* o, const T* dO,
                           T* lse, T* Dd, T* dqkv, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (m.dh) {
        case 4: return attn_bwd_dh<T, 4>(n, m, q, k, v, o, dO, lse, Dd, dqkv, st);
        case 8: return attn_bwd_dh<T, 8>(n, m, q, k, v, o, dO, lse, Dd, dqkv, st);
        case 16: return attn_bwd_dh<T, 16>(n, m, q, k, v, o, dO, lse, Dd, dqkv, st);
        case 32: return attn_bwd_dh<T, 32>(n, m, q, k, v, o, dO, lse, Dd, dqkv, st);
        case 64: return attn_bwd_dh<T, 64>(n, m, q, k, v, o, dO, lse, Dd, dqkv, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------- instantiations
#define VQ_GRAD_INST(T)                                                          \
    template hipError_t launch_gemm<T>(const GemmDesc&, hipStream_t);           \
    template hipError_t launch_colsum<T>(int64_t, int64_t, int, const T*,       \
                                         int64_t, const T*, int64_t, T*,        \
                                         int64_t, int, hipStream_t);            \
    template hipError_t launch_reduce_samples<T>(int64_t, int64_t, const T*,    \
                                                 T*, int, hipStream_t);         \
    template hipError_t launch_coef<T>(int64_t, const double*, T*, hipStream_t); \
    template hipError_t launch_fill_t<T>(T*, int64_t, T, hipStream_t);          \
    template hipError_t launch_ln_save<T>(int64_t, int, const T*, const T*,     \
                                          const T*, T*, T*, T*, hipStream_t);   \
    template hipError_t launch_ln_bwd<T>(int64_t, int, const T*, const T*,      \
                                         const T*, const T*, const T*, T*,      \
                                         hipStream_t);                          \
    template hipError_t launch_xprime<T>(int64_t, const ModelDims&, const T*,   \
                                         const int32_t*, const T*, const T*,    \
                                         const T*, T*, T*, hipStream_t);        \
    template hipError_t launch_bias_gelu<T>(int64_t, int, T*, const T*, T*,     \
                                            hipStream_t);                       \
    template hipError_t launch_gelu_bwd<T>(int64_t, const T*, T*, hipStream_t); \
    template hipError_t launch_head_bwd<T>(int64_t, int, int, int, int,         \
                                           const HeadW<T>&,                     \
                                           const int8_t*, const T*, const T*,   \
                                           T*, T*, T*, T*, T*, T*, hipStream_t); \
    template hipError_t launch_embed_bwd<T>(int64_t, int, int, int, int,        \
                                            const int8_t*,                      \
                                            const T*, T*, int64_t, int64_t,     \
                                            int64_t, hipStream_t);              \
    template hipError_t launch_vq_bwd_rows<T>(int64_t, int, int, int, int,      \
                                              const T*, int, const int32_t*,    \
                                              const T*, T*, T*, T*,             \
                                              hipStream_t);                     \
    template hipError_t launch_da_fix<T>(int64_t, int, int, const T*, const T*, \
                                         T*, hipStream_t);                      \
    template hipError_t launch_cb_fix<T>(int64_t, int, int, const T*, const T*, \
                                         T*, int64_t, hipStream_t);             \
    template hipError_t launch_onehot_scatter<T>(int64_t, int, int, int, int,   \
                                                 int, const int32_t*, const T*, \
                                                 T*, int64_t, hipStream_t);     \
    template hipError_t launch_attn_bwd<T>(int64_t, const ModelDims&, const T*, \
                                           const T*, const T*, const T*,        \
                                           const T*, T*, T*, T*, hipStream_t);

VQ_GRAD_INST(double)
VQ_GRAD_INST(float)

}  // namespace vq
