// Transformer-block kernels of the VQ wave function (paper Sec. 3.1):
// embedding, LN1 + QKV projection, causal multi-head attention, the vector
// quantizer (eqs. 4-6), output projection + residual + MLP, output head.
// VALU implementations for every precision; each per-row result depends
// only on that row's inputs, so evaluating a row inside a full sequence or
// inside a neighbour's overlay gives bitwise identical values.
#include "kernels.h"

namespace vq {

constexpr int kThreads = 256;
constexpr int kGridCap = 8192;

static inline unsigned grid_for(int64_t units) {
    if (units <= 0) return 1;
    return (unsigned)(units < kGridCap ? units : kGridCap);
}

__device__ inline int64_t rowset_n(const RowSet& r) {
    return r.n_dev ? (int64_t)(*r.n_dev) * r.mult : r.n_host;
}
__device__ inline int64_t rowset_slot(const RowSet& r, int64_t k) {
    return r.idx ? r.idx[k] : k;
}
__device__ inline bool mask_bit(const uint64_t* m, int i) {
    return (m[i >> 6] >> (i & 63)) & 1ull;
}

// Wave computes LayerNorm statistics of a row of width d (biased variance,
// two passes, eps 1e-5); every lane gets the same values.
template <typename C, typename X>
__device__ inline void ln_stats(const X* x, int d, C& mean, C& rstd) {
    const int lane = threadIdx.x & 63;
    C s = 0;
    for (int k = lane; k < d; k += 64) s += cvt<C>(x[k]);
    mean = wave_sum(s) / (C)d;
    C v = 0;
    for (int k = lane; k < d; k += 64) {
        const C t = cvt<C>(x[k]) - mean;
        v += t * t;
    }
    v = wave_sum(v) / (C)d;
    rstd = (C)1 / dsqrt(v + (C)1e-5);
}

// ------------------------------------------------------------ preparation
// table[h][c][:] = codeword (h,c) times the rows of W_o of segment h;
// cnorm[h][c] = squared norm of the codeword as the distance kernel sees it
// (bfloat16-rounded in the BF16 mode); wmax[h] = max_c sqrt(cnorm).
template <class P>
__global__ void k_prepare_table(ModelDims m, LayerW<typename P::acc> w,
                                typename P::acc* table,
                                typename P::acc* cnorm) {
    using acc = typename P::acc;
    using act = typename P::act;
    const int hc = blockIdx.x;              // h*Q + c
    const int h = hc / m.Q;
    const acc* cw = w.codebook + (int64_t)hc * m.dseg;
    for (int col = threadIdx.x; col < m.d; col += blockDim.x) {
        acc s = 0;
        for (int k = 0; k < m.dseg; ++k)
            s += cw[k] * w.W_o[(int64_t)(h * m.dseg + k) * m.d + col];
        table[(int64_t)hc * m.d + col] = s;
    }
    if (threadIdx.x < 64) {
        acc s = 0;
        for (int k = threadIdx.x; k < m.dseg; k += 64) {
            const acc v = cvt<acc>(cvt<act>(cw[k]));
            s += v * v;
        }
        s = wave_sum(s);
        if (threadIdx.x == 0) cnorm[hc] = s;
    }
}

template <class P>
__global__ void k_prepare_wmax(ModelDims m, typename P::acc* cnorm) {
    using acc = typename P::acc;
    // cnorm holds H*Q norms followed by H slots for the per-head maximum
    const int h = blockIdx.x;
    if (threadIdx.x < 64) {
        acc mx = 0;
        for (int c = threadIdx.x; c < m.Q; c += 64) {
            const acc v = cnorm[(int64_t)h * m.Q + c];
            mx = v > mx ? v : mx;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const acc t = __shfl_xor(mx, o, 64);
            mx = t > mx ? t : mx;
        }
        if (threadIdx.x == 0) cnorm[(int64_t)m.H * m.Q + h] = dsqrt(mx);
    }
}

template <class P>
hipError_t launch_prepare(const ModelDims& m, const LayerW<typename P::acc>& w,
                          typename P::acc* table, typename P::acc* cnorm,
                          bf16*, bf16*, bf16*, bf16*, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare_table<P>, dim3(m.H * m.Q), dim3(128), 0, st,
                       m, w, table, cnorm);
    hipLaunchKernelGGL(k_prepare_wmax<P>, dim3(m.H), dim3(64), 0, st, m,
                       cnorm);
    return hipGetLastError();
}

// ------------------------------------------------------------- sequences
__global__ void k_materialise(const int8_t* __restrict__ spins,
                              const NbDesc* __restrict__ desc,
                              const int32_t* n_dev, int64_t n_max, int N,
                              int8_t* __restrict__ out) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    const int64_t total = n * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / N;
        const int i = (int)(e - k * N);
        const NbDesc dd = desc[k];
        // exchange of sites s1 < s2, or a flip of s1 when s1 == s2
        int src = i;
        if (i == dd.s1) src = dd.s2;
        else if (i == dd.s2) src = dd.s1;
        const int8_t v = spins[(int64_t)dd.sigma * N + src];
        out[e] = (dd.s1 == dd.s2 && i == dd.s1) ? (int8_t)-v : v;
    }
}

hipError_t launch_materialise(const int8_t* spins, const NbDesc* desc,
                              const int32_t* n_dev, int64_t n_max, int N,
                              int8_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_materialise, dim3(grid_for((n_max * N + 255) / 256)),
                       dim3(256), 0, st, spins, desc, n_dev, n_max, N, out);
    return hipGetLastError();
}

// x[s][i] = tok[u_i] + pos[i], u_0 = BOS (2), u_i = token of spin i-1.
template <class P>
__global__ void k_embed(ModelDims m, HeadW<typename P::acc> hw,
                        const int8_t* __restrict__ spins, const int32_t* n_dev,
                        int64_t n_seq, typename P::acc* __restrict__ x) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_seq;
    const int64_t total = n * m.N * m.d;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / m.d;
        const int col = (int)(e - row * m.d);
        const int64_t s = row / m.N;
        const int i = (int)(row - s * m.N);
        // input: the previous token, or the beginning-of-sequence token
        // 2^K (the encoder reads the token itself)
        const int u = m.enc ? token_at(spins + s * m.S, i, m.K)
                            : (i == 0 ? 1 << m.K : token_at(spins + s * m.S, i - 1, m.K));
        x[e] = hw.tok[u * m.d + col] + hw.pos[(int64_t)i * m.d + col];
    }
}

template <class P>
hipError_t launch_embed(const ModelDims& m, const HeadW<typename P::acc>& hw,
                        const int8_t* spins, const int32_t* n_dev,
                        int64_t n_seq, typename P::acc* x, hipStream_t st) {
    hipLaunchKernelGGL(k_embed<P>,
                       dim3(grid_for((n_seq * m.N * m.d + 255) / 256)),
                       dim3(256), 0, st, m, hw, spins, n_dev, n_seq, x);
    return hipGetLastError();
}

// ------------------------------------------------------------ LN1 + QKV
template <class P, int TR>
__global__ void __launch_bounds__(kThreads) k_qkv(ModelDims m,
                                                  LayerW<typename P::acc> w,
                                                  RowSet rows, BlockIO<P> io) {
    using acc = typename P::acc;
    using act = typename P::act;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    acc* hs = reinterpret_cast<acc*>(smem_raw);            // [TR][d]
    __shared__ int64_t slot[TR];
    const int64_t n = rowset_n(rows);
    const int64_t ntiles = (n + TR - 1) / TR;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int d = m.d, d3 = 3 * m.d;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int rr = wave; rr < TR; rr += kThreads / 64) {
            const int64_t r = t * TR + rr;
            if (r < n) {
                const int64_t s = rowset_slot(rows, r);
                if (lane == 0) slot[rr] = s;
                const acc* x = io.x + s * d;
                acc mean, rstd;
                ln_stats<acc>(x, d, mean, rstd);
                for (int k = lane; k < d; k += 64)
                    hs[rr * d + k] = (x[k] - mean) * rstd * w.ln1_g[k] + w.ln1_b[k];
            } else {
                if (lane == 0) slot[rr] = -1;
                for (int k = lane; k < d; k += 64) hs[rr * d + k] = 0;
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < d3; c += kThreads) {
            acc s[TR];
#pragma unroll
            for (int rr = 0; rr < TR; ++rr) s[rr] = 0;
            for (int k = 0; k < d; ++k) {
                const acc wv = cvt<acc>(cvt<act>(w.W_qkv[(int64_t)k * d3 + c]));
#pragma unroll
                for (int rr = 0; rr < TR; ++rr)
                    s[rr] += cvt<acc>(cvt<act>(hs[rr * d + k])) * wv;
            }
            act* dst = c < d ? io.q : (c < 2 * d ? io.k : io.v);
            const int cc = c < d ? c : (c < 2 * d ? c - d : c - 2 * d);
#pragma unroll
            for (int rr = 0; rr < TR; ++rr)
                if (slot[rr] >= 0)
                    dst[slot[rr] * d + cc] = cvt<act>(s[rr] + w.b_qkv[c]);
        }
        __syncthreads();
    }
}

template <class P>
hipError_t launch_qkv(const ModelDims& m, const LayerW<typename P::acc>& w,
                      RowSet rows, const BlockIO<P>& io, hipStream_t st) {
    constexpr int TR = 16;
    const size_t sm = sizeof(typename P::acc) * TR * m.d;
    hipLaunchKernelGGL((k_qkv<P, TR>), dim3(grid_for((rows.n_host + TR - 1) / TR)),
                       dim3(kThreads), sm, st, m, w, rows, io);
    return hipGetLastError();
}

// ------------------------------------------------------------- attention
// One query row against keys 0..i (online softmax), key j's vector at
// Ks + j * ld (LDS tiles: ld = DH).  Shared by the full-sequence, overlay
// and sampling kernels so all give identical bits.
template <typename C, int DH, typename A>
__device__ inline void attend_row(const C (&q)[DH], const A* __restrict__ Ks,
                                  const A* __restrict__ Vs, int i,
                                  C (&o)[DH], int64_t ld = DH,
                                  C* stat = nullptr) {
    C mx = neg_inf<C>(), l = 0;
#pragma unroll
    for (int c = 0; c < DH; ++c) o[c] = 0;
    for (int j = 0; j <= i; ++j) {
        C s = 0;
#pragma unroll
        for (int c = 0; c < DH; ++c) s += q[c] * cvt<C>(Ks[j * ld + c]);
        if (s > mx) {
            const C al = dexp(mx - s);
            l *= al;
#pragma unroll
            for (int c = 0; c < DH; ++c) o[c] *= al;
            mx = s;
        }
        const C p = dexp(s - mx);
        l += p;
#pragma unroll
        for (int c = 0; c < DH; ++c) o[c] += p * cvt<C>(Vs[j * ld + c]);
    }
    const C inv = (C)1 / l;
#pragma unroll
    for (int c = 0; c < DH; ++c) o[c] *= inv;
    // the softmax statistics: the largest score and sum_j exp(s_j - max)
    if (stat) {
        stat[0] = mx;
        stat[1] = l;
    }
}

template <class P, int DH>
__global__ void __launch_bounds__(kThreads) k_attn_seq(ModelDims m,
                                                       const int32_t* n_dev,
                                                       int64_t n_seq,
                                                       BlockIO<P> io,
                                                       int64_t* ctr) {
    using acc = typename P::acc;
    using act = typename P::act;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    act* Ks = reinterpret_cast<act*>(smem_raw);
    act* Vs = Ks + m.N * DH;
    const int64_t n = n_dev ? (int64_t)*n_dev : n_seq;
    const int64_t units = n * m.nh;
    const acc scale = (acc)1 / dsqrt((acc)DH);
    const int d = m.d, N = m.N;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t s = u / m.nh;
        const int h = (int)(u - s * m.nh);
        const int64_t base = s * N * d + h * DH;
        for (int e = threadIdx.x; e < N * DH; e += kThreads) {
            const int j = e / DH, c = e - (e / DH) * DH;
            Ks[e] = io.k[base + (int64_t)j * d + c];
            Vs[e] = io.v[base + (int64_t)j * d + c];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += kThreads) {
            acc q[DH], o[DH];
#pragma unroll
            for (int c = 0; c < DH; ++c)
                q[c] = cvt<acc>(io.q[base + (int64_t)i * d + c]) * scale;
            // keys 0..i (decoder) or all of them (encoder)
            attend_row<acc, DH, act>(
                q, Ks, Vs, m.enc ? N - 1 : i, o, DH,
                io.stat ? io.stat + ((s * N + i) * m.nh + h) * 2 : nullptr);
#pragma unroll
            for (int c = 0; c < DH; ++c)
                io.a[base + (int64_t)i * d + c] = cvt<act>(o[c]);
        }
        __syncthreads();
    }
    if (ctr && blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_ROWS),
                  (unsigned long long)(n * N));
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_PAIRS),
                  (unsigned long long)(n * (m.enc ? (int64_t)N * N
                                                  : (int64_t)N * (N + 1) / 2) * m.nh));
    }
}

template <class P, int DH>
static hipError_t attn_seq_dh(const ModelDims& m, const int32_t* n_dev,
                              int64_t n_seq, const BlockIO<P>& io,
                              int64_t* ctr, hipStream_t st) {
    const size_t sm = sizeof(typename P::act) * 2 * m.N * DH;
    if (sm > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)k_attn_seq<P, DH>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sm);
    hipLaunchKernelGGL((k_attn_seq<P, DH>), dim3(grid_for(n_seq * m.nh)),
                       dim3(kThreads), sm, st, m, n_dev, n_seq, io, ctr);
    return hipGetLastError();
}

template <class P>
hipError_t launch_attention_seq(const ModelDims& m, const int32_t* n_dev,
                                int64_t n_seq, const BlockIO<P>& io,
                                int64_t* ctr, hipStream_t st) {
    switch (m.dh) {
        case 4: return attn_seq_dh<P, 4>(m, n_dev, n_seq, io, ctr, st);
        case 8: return attn_seq_dh<P, 8>(m, n_dev, n_seq, io, ctr, st);
        case 16: return attn_seq_dh<P, 16>(m, n_dev, n_seq, io, ctr, st);
        case 32: return attn_seq_dh<P, 32>(m, n_dev, n_seq, io, ctr, st);
        case 64: return attn_seq_dh<P, 64>(m, n_dev, n_seq, io, ctr, st);
    }
    return hipErrorInvalidValue;
}

// Overlay attention of the neighbours: keys/values/queries of rows in the
// changed set C come from the neighbour's overlay rows, all others from the
// sample's cached rows.  Only query rows i >= p1 + 1 are evaluated.
template <class P, int DH>
__global__ void __launch_bounds__(kThreads) k_attn_dedup(ModelDims m,
                                                         DedupIO<P> dd,
                                                         int64_t* ctr) {
    using acc = typename P::acc;
    using act = typename P::act;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    act* Ks = reinterpret_cast<act*>(smem_raw);
    act* Vs = Ks + m.N * DH;
    const int64_t n = (int64_t)*dd.n_nb;
    const int64_t units = n * m.nh;
    const acc scale = (acc)1 / dsqrt((acc)DH);
    const int d = m.d, N = m.N, W = dd.mask_words;
    int64_t my_rows = 0, my_pairs = 0;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t nb = u / m.nh;
        const int h = (int)(u - nb * m.nh);
        const NbDesc D = dd.desc[nb];
        const int pmin = first_row(D, m);
        const uint64_t* mk = dd.mask + nb * W;
        const int64_t sb = (int64_t)D.sigma * N * d + h * DH;
        const int64_t ob = (D.ov - pmin) * (int64_t)d + h * DH;   // row i at ob + i*d
        for (int e = threadIdx.x; e < N * DH; e += kThreads) {
            const int j = e / DH, c = e - (e / DH) * DH;
            const bool ovl = j >= pmin && mask_bit(mk, j);
            const int64_t off = (ovl ? ob : sb) + (int64_t)j * d + c;
            Ks[e] = (ovl ? dd.ok : dd.bk)[off];
            Vs[e] = (ovl ? dd.ov : dd.bv)[off];
        }
        __syncthreads();
        for (int i = pmin + threadIdx.x; i < N; i += kThreads) {
            const bool ovl = mask_bit(mk, i);
            const act* qsrc = (ovl ? dd.oq + ob : dd.bq + sb) + (int64_t)i * d;
            acc q[DH], o[DH];
#pragma unroll
            for (int c = 0; c < DH; ++c) q[c] = cvt<acc>(qsrc[c]) * scale;
            attend_row<acc, DH, act>(q, Ks, Vs, m.enc ? N - 1 : i, o);
            act* dst = dd.oa + ob + (int64_t)i * d;
#pragma unroll
            for (int c = 0; c < DH; ++c) dst[c] = cvt<act>(o[c]);
        }
        if (h == 0 && threadIdx.x == 0) {
            my_rows += N - pmin;
            my_pairs += m.enc ? (int64_t)N * N
                              : ((int64_t)N * (N + 1) - (int64_t)pmin * (pmin + 1)) / 2;
        }
        __syncthreads();
    }
    if (ctr && threadIdx.x == 0 && my_rows) {
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_ROWS),
                  (unsigned long long)my_rows);
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_PAIRS),
                  (unsigned long long)(my_pairs * m.nh));
    }
}

template <class P, int DH>
static hipError_t attn_dedup_dh(const ModelDims& m, const DedupIO<P>& d,
                                int64_t* ctr, hipStream_t st) {
    const size_t sm = sizeof(typename P::act) * 2 * m.N * DH;
    if (sm > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)k_attn_dedup<P, DH>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sm);
    hipLaunchKernelGGL((k_attn_dedup<P, DH>), dim3(grid_for(d.n_nb_max * m.nh)),
                       dim3(kThreads), sm, st, m, d, ctr);
    return hipGetLastError();
}

template <class P>
hipError_t launch_attention_dedup(const ModelDims& m, const DedupIO<P>& d,
                                  int64_t* ctr, hipStream_t st) {
    switch (m.dh) {
        case 4: return attn_dedup_dh<P, 4>(m, d, ctr, st);
        case 8: return attn_dedup_dh<P, 8>(m, d, ctr, st);
        case 16: return attn_dedup_dh<P, 16>(m, d, ctr, st);
        case 32: return attn_dedup_dh<P, 32>(m, d, ctr, st);
        case 64: return attn_dedup_dh<P, 64>(m, d, ctr, st);
    }
    return hipErrorInvalidValue;
}

// Incremental attention of the neighbours: for a query row whose own input
// did not change (not in C), only the keys and values of the rows of C
// differ from the sample's, so its softmax sum is the sample's with those
// terms replaced (a rank-|C| update):
//   U' = f (l a - sum_C w_old v_old) + sum_C w_new v_new,
//   L' = f (l - sum_C w_old) + sum_C w_new,      a' = U' / L',
// with the sample's reference m and normaliser l of the row (cached by its
// forward pass), w_old = e^(s_old - m), w_new = e^(s_new - m'), m' the
// larger of m and the new scores, f = e^(m - m').  A row in C (changed
// query), a neighbour with more C rows
// than the LDS holds, or a row whose removed weight exceeds half its
// normaliser (cancellation) is evaluated in full over keys 0..i, in the
// order and arithmetic of attend_row.
template <class P, int DH>
__global__ void __launch_bounds__(kThreads) k_attn_incr(
    ModelDims m, DedupIO<P> dd, const typename P::acc* __restrict__ bstat,
    int64_t* ctr) {
    using acc = typename P::acc;
    using act = typename P::act;
    constexpr int CAP = 8192 / (DH * (int)sizeof(act));   // 32 KiB of rows
    __shared__ act Ko[CAP * DH], Vo[CAP * DH], Kn[CAP * DH], Vn[CAP * DH];
    __shared__ int jr[CAP];
    const int64_t n = (int64_t)*dd.n_nb;
    const int64_t units = n * m.nh;
    const acc scale = (acc)1 / dsqrt((acc)DH);
    const int d = m.d, N = m.N, W = dd.mask_words;
    auto ex = [](acc x) -> acc { return dexp(x); };
    int64_t my_rows = 0, my_pairs = 0;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t nb = u / m.nh;
        const int h = (int)(u - nb * m.nh);
        const NbDesc D = dd.desc[nb];
        const int pmin = first_row(D, m);
        const uint64_t* mk = dd.mask + nb * W;
        const int64_t sb = (int64_t)D.sigma * N * d + h * DH;
        const int64_t ob = (D.ov - pmin) * (int64_t)d + h * DH;
        const int cc = dd.ccnt[nb];
        const bool fits = cc <= CAP;
        __syncthreads();
        if (fits) {
            for (int e = threadIdx.x; e < cc * DH; e += kThreads) {
                const int c = e / DH, k = e - (e / DH) * DH;
                const int j = dd.crow[D.ov + c];
                Ko[e] = dd.bk[sb + (int64_t)j * d + k];
                Vo[e] = dd.bv[sb + (int64_t)j * d + k];
                Kn[e] = dd.ok[ob + (int64_t)j * d + k];
                Vn[e] = dd.ov[ob + (int64_t)j * d + k];
                if (k == 0) jr[c] = j;
            }
        }
        __syncthreads();
        for (int i = pmin + threadIdx.x; i < N; i += kThreads) {
            const bool qchg = mask_bit(mk, i);
            const act* qsrc = (qchg ? dd.oq + ob : dd.bq + sb) + (int64_t)i * d;
            acc q[DH], o[DH];
            bool done = false;
            if (!qchg && fits) {
                // the C rows at or before i
                int nc = 0;
                while (nc < cc && jr[nc] <= i) ++nc;
                const acc* st = bstat + (((int64_t)D.sigma * N + i) * m.nh + h) * 2;
                const acc m0 = st[0], l0 = st[1];
#pragma unroll
                for (int c = 0; c < DH; ++c) q[c] = cvt<acc>(qsrc[c]) * scale;
                acc mn = m0;
                for (int c = 0; c < nc; ++c) {
                    acc sn = 0;
#pragma unroll
                    for (int k = 0; k < DH; ++k) sn += q[k] * cvt<acc>(Kn[c * DH + k]);
                    mn = sn > mn ? sn : mn;
                }
                acc rw = 0, aw = 0, ro[DH], ao[DH];
#pragma unroll
                for (int k = 0; k < DH; ++k) ro[k] = ao[k] = 0;
                for (int c = 0; c < nc; ++c) {
                    acc so = 0, sn = 0;
#pragma unroll
                    for (int k = 0; k < DH; ++k) {
                        so += q[k] * cvt<acc>(Ko[c * DH + k]);
                        sn += q[k] * cvt<acc>(Kn[c * DH + k]);
                    }
                    const acc wo = ex(so - m0), wn = ex(sn - mn);
                    rw += wo;
                    aw += wn;
#pragma unroll
                    for (int k = 0; k < DH; ++k) {
                        ro[k] += wo * cvt<acc>(Vo[c * DH + k]);
                        ao[k] += wn * cvt<acc>(Vn[c * DH + k]);
                    }
                }
                if (rw <= (acc)0.5 * l0) {
                    const acc f = ex(m0 - mn);
                    const acc L = f * (l0 - rw) + aw;
                    const act* a0 = dd.ba + sb + (int64_t)i * d;
#pragma unroll
                    for (int k = 0; k < DH; ++k)
                        o[k] = (f * (l0 * cvt<acc>(a0[k]) - ro[k]) + ao[k]) / L;
                    done = true;
                    my_pairs += 2 * nc;
                }
            }
            if (!done) {
                // every key 0..i: the neighbour's overlay rows where they
                // changed, the sample's elsewhere (attend_row's arithmetic)
#pragma unroll
                for (int c = 0; c < DH; ++c) q[c] = cvt<acc>(qsrc[c]) * scale;
                acc mx = neg_inf<acc>(), l = 0;
#pragma unroll
                for (int c = 0; c < DH; ++c) o[c] = 0;
                for (int j = 0; j <= i; ++j) {
                    const bool ovl = j >= pmin && mask_bit(mk, j);
                    const int64_t off = (ovl ? ob : sb) + (int64_t)j * d;
                    const act* K = (ovl ? dd.ok : dd.bk) + off;
                    const act* V = (ovl ? dd.ov : dd.bv) + off;
                    acc sc = 0;
#pragma unroll
                    for (int c = 0; c < DH; ++c) sc += q[c] * cvt<acc>(K[c]);
                    if (sc > mx) {
                        const acc al = dexp(mx - sc);
                        l *= al;
#pragma unroll
                        for (int c = 0; c < DH; ++c) o[c] *= al;
                        mx = sc;
                    }
                    const acc pj = dexp(sc - mx);
                    l += pj;
#pragma unroll
                    for (int c = 0; c < DH; ++c) o[c] += pj * cvt<acc>(V[c]);
                }
                const acc inv = (acc)1 / l;
#pragma unroll
                for (int c = 0; c < DH; ++c) o[c] *= inv;
                my_pairs += i + 1;
            }
            act* dst = dd.oa + ob + (int64_t)i * d;
#pragma unroll
            for (int c = 0; c < DH; ++c) dst[c] = cvt<act>(o[c]);
        }
        if (h == 0 && threadIdx.x == 0) my_rows += N - pmin;
    }
    if (ctr) {
        // pairs summed over the block's threads (rows counted by thread 0)
        __shared__ unsigned long long red[kThreads / 64];
        const unsigned long long pw = wave_sum((unsigned long long)my_pairs);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pw;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long pt = 0;
            for (int w = 0; w < kThreads / 64; ++w) pt += red[w];
            if (my_rows)
                atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_ROWS),
                          (unsigned long long)my_rows);
            if (pt)
                atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_PAIRS), pt);
        }
    }
}

template <class P, int DH>
static hipError_t attn_incr_dh(const ModelDims& m, const DedupIO<P>& d,
                               const typename P::acc* bstat, int64_t* ctr,
                               hipStream_t st) {
    hipLaunchKernelGGL((k_attn_incr<P, DH>), dim3(grid_for(d.n_nb_max * m.nh)),
                       dim3(kThreads), 0, st, m, d, bstat, ctr);
    return hipGetLastError();
}

template <class P>
hipError_t launch_attention_incr(const ModelDims& m, const DedupIO<P>& d,
                                 const typename P::acc* bstat, int64_t* ctr,
                                 hipStream_t st) {
    switch (m.dh) {
        case 4: return attn_incr_dh<P, 4>(m, d, bstat, ctr, st);
        case 8: return attn_incr_dh<P, 8>(m, d, bstat, ctr, st);
        case 16: return attn_incr_dh<P, 16>(m, d, bstat, ctr, st);
        case 32: return attn_incr_dh<P, 32>(m, d, bstat, ctr, st);
        case 64: return attn_incr_dh<P, 64>(m, d, bstat, ctr, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------ attention-only half-block
// Output projection with residual of the half-block that ends the model
// (no quantizer, no MLP): out = x + a W_o + b_o for a set of rows.  Each
// wave takes four rows and every lane four output columns, so a row of W_o
// loaded once serves the four rows; sums over k in order, contraction off
// so that a row's result does not depend on the other rows of its wave.
// Rows are addressed through `src`: fn(k) gives (x_in row, a row, out row)
// of the k-th row of the set.
constexpr int kOpR = 4;
template <class P, class F>
__device__ inline void out_proj_rows(const ModelDims& m,
                                     const typename P::acc* __restrict__ Wo,
                                     const typename P::acc* __restrict__ bo,
                                     int64_t nrows, F fn) {
#pragma clang fp contract(off)
    using acc = typename P::acc;
    using act = typename P::act;
    const int lane = threadIdx.x & 63;
    const int d = m.d;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t r0 = (blockIdx.x * (int64_t)(kThreads / 64) + (threadIdx.x >> 6)) * kOpR;
         r0 < nrows; r0 += waves * kOpR) {
        const acc* xin[kOpR];
        const act* ar[kOpR];
        acc* out[kOpR];
        bool ok[kOpR];
#pragma unroll
        for (int r = 0; r < kOpR; ++r) {
            ok[r] = r0 + r < nrows;
            fn(ok[r] ? r0 + r : r0, xin[r], ar[r], out[r]);
        }
        // the rows' attention outputs, 8 columns per lane (d <= 512)
        acc av[kOpR][8];
#pragma unroll
        for (int r = 0; r < kOpR; ++r)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = lane + 64 * j;
                av[r][j] = k < d ? cvt<acc>(ar[r][k]) : (acc)0;
            }
        for (int c0 = 0; c0 < d; c0 += 256) {
            acc sum[kOpR][4];
#pragma unroll
            for (int r = 0; r < kOpR; ++r)
#pragma unroll
                for (int u = 0; u < 4; ++u) sum[r][u] = 0;
            for (int k = 0; k < d; ++k) {
                const int j = k >> 6, src = k & 63;
                acc w[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int col = c0 + lane + 64 * u;
                    w[u] = col < d ? Wo[(int64_t)k * d + col] : (acc)0;
                }
#pragma unroll
                for (int r = 0; r < kOpR; ++r) {
                    acc akv = 0;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        if (jj == j) akv = __shfl(av[r][jj], src, 64);
#pragma unroll
                    for (int u = 0; u < 4; ++u) sum[r][u] += akv * w[u];
                }
            }
#pragma unroll
            for (int r = 0; r < kOpR; ++r) {
                if (!ok[r]) continue;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int col = c0 + lane + 64 * u;
                    if (col < d) out[r][col] = xin[r][col] + (sum[r][u] + bo[col]);
                }
            }
        }
    }
}

// Rows of a RowSet (full sequences and sampling): in place or into x_out.
template <class P>
__global__ void __launch_bounds__(kThreads) k_out_proj(
    ModelDims m, const typename P::acc* Wo, const typename P::acc* bo,
    RowSet rows, const typename P::acc* x_in, const typename P::act* a,
    typename P::acc* x_out) {
    using acc = typename P::acc;
    using act = typename P::act;
    const int64_t n = rowset_n(rows);
    out_proj_rows<P>(m, Wo, bo, n,
                     [&](int64_t k, const acc*& xi, const act*& ar, acc*& o) {
                         const int64_t row = rowset_slot(rows, k);
                         xi = x_in + row * m.d;
                         ar = a + row * m.d;
                         o = x_out + row * m.d;
                     });
}

template <class P>
hipError_t launch_out_proj(const ModelDims& m, const typename P::acc* Wo,
                           const typename P::acc* bo, RowSet rows,
                           const typename P::acc* x_in,
                           const typename P::act* a, typename P::acc* x_out,
                           hipStream_t st) {
    const int64_t wv = (rows.n_host + kOpR - 1) / kOpR;
    hipLaunchKernelGGL(k_out_proj<P>, dim3(grid_for((wv + 3) / 4)),
                       dim3(kThreads), 0, st, m, Wo, bo, rows, x_in, a, x_out);
    return hipGetLastError();
}

// The overlay rows of every neighbour (all rows from p_min on): the
// half-block's input is the neighbour's row where it is in C_L, else the
// sample's; the output goes to `out` at the same slot.
template <class P>
__global__ void __launch_bounds__(kThreads) k_out_proj_overlay(
    ModelDims m, const typename P::acc* Wo, const typename P::acc* bo,
    DedupIO<P> dd, typename P::acc* out) {
    using acc = typename P::acc;
    using act = typename P::act;
    const int64_t n = (int64_t)*dd.n_rows;
    const int W = dd.mask_words;
    out_proj_rows<P>(m, Wo, bo, n,
                     [&](int64_t r, const acc*& xi, const act*& ar, acc*& o) {
                         const int32_t nb = dd.slot_nb[r];
                         const NbDesc D = dd.desc[nb];
                         const int i = first_row(D, m) + (int)(r - D.ov);
                         const bool inC = mask_bit(dd.mask + (int64_t)nb * W, i);
                         xi = inC ? dd.ox + r * m.d
                                  : dd.bx + ((int64_t)D.sigma * m.N + i) * m.d;
                         ar = dd.oa + r * m.d;
                         o = out + r * m.d;
                     });
}

template <class P>
hipError_t launch_out_proj_overlay(const ModelDims& m,
                                   const typename P::acc* Wo,
                                   const typename P::acc* bo,
                                   const DedupIO<P>& dd,
                                   typename P::acc* out, hipStream_t st) {
    const int64_t wv = (dd.rows_max + kOpR - 1) / kOpR;
    hipLaunchKernelGGL(k_out_proj_overlay<P>, dim3(grid_for((wv + 3) / 4)),
                       dim3(kThreads), 0, st, m, Wo, bo, dd, out);
    return hipGetLastError();
}

// Every row from p_min on is changed after the half-block: the row masks
// (read by the output head) become rows p_min .. N-1.
__global__ void k_mask_from_pmin(const NbDesc* __restrict__ desc,
                                 const int32_t* n_nb, int W, int N,
                                 uint64_t* __restrict__ mask) {
    const int64_t n = (int64_t)*n_nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < n * W; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t nb = e / W;
        const int wd = (int)(e - nb * W);
        const int pmin = desc[nb].p1 + 1;
        uint64_t v = 0;
        for (int b = 0; b < 64; ++b) {
            const int i = wd * 64 + b;
            if (i >= pmin && i < N) v |= 1ull << b;
        }
        mask[e] = v;
    }
}

hipError_t launch_mask_from_pmin(const NbDesc* desc, const int32_t* n_nb,
                                 int64_t n_max, int W, int N, uint64_t* mask,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_mask_from_pmin, dim3(grid_for((n_max * W + 255) / 256)),
                       dim3(256), 0, st, desc, n_nb, W, N, mask);
    return hipGetLastError();
}

// ------------------------------------------------------- vector quantizer
// Running best / second-best of (score, index); ties go to the lower index.
template <typename C>
struct Top2 {
    C b;
    int i;
    C s;
};
template <typename C>
__device__ inline Top2<C> top2_merge(Top2<C> x, Top2<C> y) {
    Top2<C> r;
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

// Unit roundoff of the distance arithmetic and a bound on the error of a
// computed score |w|^2 - 2 a.w (length-n sums, any summation order).
template <typename C>
__device__ inline C unit_roundoff();
template <>
__device__ inline float unit_roundoff<float>() {
    return 5.9604645e-8f;
}
template <>
__device__ inline double unit_roundoff<double>() {
    return 1.1102230246251565e-16;
}
template <typename C>
__device__ inline C score_err(int n, C na, C wmax) {
    const C g = (C)(n + 4) * unit_roundoff<C>() * (C)1.0625;
    return g * ((C)2 * na * wmax + wmax * wmax + na * na);
}

// Scores of TR rows against all Q codes of one quantizer head per pass; the
// result per row is the code, plus bounds U1 >= best distance and
// L2 <= second-best distance used by the certified-reuse test.
template <class P, int TR>
__global__ void __launch_bounds__(kThreads) k_vq(ModelDims m,
                                                 LayerW<typename P::acc> w,
                                                 RowSet rows, BlockIO<P> io) {
    using acc = typename P::acc;
    using act = typename P::act;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    acc* as = reinterpret_cast<acc*>(smem_raw);          // [TR][dseg]
    __shared__ acc a2[TR];
    __shared__ int64_t slot[TR];
    __shared__ Top2<acc> part[kThreads / 64][TR];
    const int64_t n = rowset_n(rows);
    const int64_t ntiles = (n + TR - 1) / TR;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ds = m.dseg;
    const acc inf = -neg_inf<acc>();
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int hq = 0; hq < m.H; ++hq) {
            for (int rr = wave; rr < TR; rr += kThreads / 64) {
                const int64_t r = t * TR + rr;
                acc s2 = 0;
                if (r < n) {
                    const int64_t s = rowset_slot(rows, r);
                    if (lane == 0) slot[rr] = s;
                    const act* a = io.a + s * m.d + hq * ds;
                    for (int k = lane; k < ds; k += 64) {
                        const acc v = cvt<acc>(a[k]);
                        as[rr * ds + k] = v;
                        s2 += v * v;
                    }
                } else {
                    if (lane == 0) slot[rr] = -1;
                    for (int k = lane; k < ds; k += 64) as[rr * ds + k] = 0;
                }
                s2 = wave_sum(s2);
                if (lane == 0) a2[rr] = s2;
            }
            __syncthreads();
            Top2<acc> best[TR];
#pragma unroll
            // start from code 0: any finite distance replaces it (so results
            // are unchanged), and a row whose distances are all non-finite
            // still gets a valid code for the table lookups that follow
            for (int rr = 0; rr < TR; ++rr) best[rr] = Top2<acc>{inf, 0, inf};
            const acc* cb = w.codebook + (int64_t)hq * m.Q * ds;
            const acc* cn = w.cnorm + (int64_t)hq * m.Q;
            for (int c = threadIdx.x; c < m.Q; c += kThreads) {
                acc dot[TR];
#pragma unroll
                for (int rr = 0; rr < TR; ++rr) dot[rr] = 0;
                for (int k = 0; k < ds; ++k) {
                    const acc wv = cvt<acc>(cvt<act>(cb[(int64_t)c * ds + k]));
#pragma unroll
                    for (int rr = 0; rr < TR; ++rr) dot[rr] += as[rr * ds + k] * wv;
                }
#pragma unroll
                for (int rr = 0; rr < TR; ++rr) {
                    const acc sc = cn[c] - (acc)2 * dot[rr];
                    best[rr] = top2_merge(best[rr], Top2<acc>{sc, c, inf});
                }
            }
#pragma unroll
            for (int rr = 0; rr < TR; ++rr) {
                Top2<acc> v = best[rr];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    Top2<acc> y;
                    y.b = __shfl_xor(v.b, o, 64);
                    y.i = __shfl_xor(v.i, o, 64);
                    y.s = __shfl_xor(v.s, o, 64);
                    // combine in lane order so every lane agrees
                    v = (lane & o) ? top2_merge(y, v) : top2_merge(v, y);
                }
                if (lane == 0) part[wave][rr] = v;
            }
            __syncthreads();
            if (threadIdx.x < TR) {
                const int rr = threadIdx.x;
                Top2<acc> v = part[0][rr];
                for (int wv = 1; wv < kThreads / 64; ++wv) v = top2_merge(v, part[wv][rr]);
                const int64_t s = slot[rr];
                if (s >= 0) {
                    io.codes[s * m.H + hq] = v.i;
                    if (io.margin) {
                        const acc wmax = w.cnorm[(int64_t)m.H * m.Q + hq];
                        const acc na = dsqrt(a2[rr]);
                        const acc E = score_err<acc>(ds, na, wmax);
                        const acc u1 = v.b + a2[rr] + E;
                        const acc l2 = v.s + a2[rr] - E;
                        io.margin[(s * m.H + hq) * 2 + 0] = dsqrt(u1 > 0 ? u1 : (acc)0);
                        io.margin[(s * m.H + hq) * 2 + 1] = dsqrt(l2 > 0 ? l2 : (acc)0);
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <class P>
hipError_t launch_vq(const ModelDims& m, const LayerW<typename P::acc>& w,
                     RowSet rows, const BlockIO<P>& io, hipStream_t st) {
    constexpr int TR = 8;
    const size_t sm = sizeof(typename P::acc) * TR * m.dseg;
    hipLaunchKernelGGL((k_vq<P, TR>), dim3(grid_for((rows.n_host + TR - 1) / TR)),
                       dim3(kThreads), sm, st, m, w, rows, io);
    return hipGetLastError();
}

// ---------------------------------------- output projection + residual + MLP
// x' = x_in + b_o + sum_h table[h][code_h];  x = x' + W2 GELU(LN2(x') W1 + b1) + b2
template <class P, int TR>
__global__ void __launch_bounds__(kThreads) k_mlp(ModelDims m,
                                                  LayerW<typename P::acc> w,
                                                  RowSet rows, BlockIO<P> io) {
    using acc = typename P::acc;
    using act = typename P::act;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    acc* xp = reinterpret_cast<acc*>(smem_raw);   // [TR][d]
    acc* hn = xp + TR * m.d;                      // [TR][d]
    acc* hid = hn + TR * m.d;                     // [TR][dff]
    __shared__ int64_t slot[TR];
    const int64_t n = rowset_n(rows);
    const int64_t ntiles = (n + TR - 1) / TR;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int d = m.d, F = m.dff;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int rr = wave; rr < TR; rr += kThreads / 64) {
            const int64_t r = t * TR + rr;
            if (r < n) {
                const int64_t s = rowset_slot(rows, r);
                if (lane == 0) slot[rr] = s;
                const acc* x = io.x_in + s * d;
                const int32_t* cd = io.codes + s * m.H;
                for (int k = lane; k < d; k += 64) {
                    acc z = w.b_o[k];
                    for (int hq = 0; hq < m.H; ++hq)
                        z += w.table[((int64_t)hq * m.Q + cd[hq]) * d + k];
                    xp[rr * d + k] = x[k] + z;
                }
                acc mean, rstd;
                ln_stats<acc>(xp + rr * d, d, mean, rstd);
                for (int k = lane; k < d; k += 64)
                    hn[rr * d + k] = (xp[rr * d + k] - mean) * rstd * w.ln2_g[k] + w.ln2_b[k];
            } else {
                if (lane == 0) slot[rr] = -1;
                for (int k = lane; k < d; k += 64) {
                    xp[rr * d + k] = 0;
                    hn[rr * d + k] = 0;
                }
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < F; c += kThreads) {
            acc s[TR];
#pragma unroll
            for (int rr = 0; rr < TR; ++rr) s[rr] = 0;
            for (int k = 0; k < d; ++k) {
                const acc wv = cvt<acc>(cvt<act>(w.W1[(int64_t)k * F + c]));
#pragma unroll
                for (int rr = 0; rr < TR; ++rr) s[rr] += cvt<acc>(cvt<act>(hn[rr * d + k])) * wv;
            }
#pragma unroll
            for (int rr = 0; rr < TR; ++rr) hid[rr * F + c] = gelu_exact(s[rr] + w.b1[c]);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < d; c += kThreads) {
            acc s[TR];
#pragma unroll
            for (int rr = 0; rr < TR; ++rr) s[rr] = 0;
            for (int k = 0; k < F; ++k) {
                const acc wv = cvt<acc>(cvt<act>(w.W2[(int64_t)k * d + c]));
#pragma unroll
                for (int rr = 0; rr < TR; ++rr) s[rr] += cvt<acc>(cvt<act>(hid[rr * F + k])) * wv;
            }
#pragma unroll
            for (int rr = 0; rr < TR; ++rr)
                if (slot[rr] >= 0) io.x[slot[rr] * d + c] = xp[rr * d + c] + (s[rr] + w.b2[c]);
        }
        __syncthreads();
    }
}

template <class P>
hipError_t launch_mlp(const ModelDims& m, const LayerW<typename P::acc>& w,
                      RowSet rows, const BlockIO<P>& io, hipStream_t st) {
    using acc = typename P::acc;
    int TR = 16;
    while (TR > 1 && sizeof(acc) * TR * (2 * m.d + m.dff) > 64 * 1024) TR >>= 1;
    const size_t sm = sizeof(acc) * TR * (2 * m.d + m.dff);
    const unsigned g = grid_for((rows.n_host + TR - 1) / TR);
    switch (TR) {
        case 16: hipLaunchKernelGGL((k_mlp<P, 16>), dim3(g), dim3(kThreads), sm, st, m, w, rows, io); break;
        case 8: hipLaunchKernelGGL((k_mlp<P, 8>), dim3(g), dim3(kThreads), sm, st, m, w, rows, io); break;
        case 4: hipLaunchKernelGGL((k_mlp<P, 4>), dim3(g), dim3(kThreads), sm, st, m, w, rows, io); break;
        case 2: hipLaunchKernelGGL((k_mlp<P, 2>), dim3(g), dim3(kThreads), sm, st, m, w, rows, io); break;
        default: hipLaunchKernelGGL((k_mlp<P, 1>), dim3(g), dim3(kThreads), sm, st, m, w, rows, io); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ head
// The three passes of head_rows over rows of any width, reading the rows
// and the head parameters from memory in each.
template <typename C, int R>
__device__ inline void head_passes(const C* const (&x)[R], int d,
                                   const HeadW<C>& hw, C (&s)[R], C (&v)[R],
                                   C (&mean)[R], C (&rstd)[R], C (&z0)[R],
                                   C (&z1)[R]) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    for (int k = lane; k < d; k += 64)
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] += x[r][k];
#pragma unroll
    for (int r = 0; r < R; ++r) mean[r] = wave_sum(s[r]) / (C)d;
    for (int k = lane; k < d; k += 64)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const C t = x[r][k] - mean[r];
            v[r] += t * t;
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
        rstd[r] = (C)1 / dsqrt(wave_sum(v[r]) / (C)d + (C)1e-5);
    for (int k = lane; k < d; k += 64) {
        const C g = hw.lnf_g[k], b = hw.lnf_b[k];
        const C w0 = hw.W_head[2 * k], w1 = hw.W_head[2 * k + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const C f = (x[r][k] - mean[r]) * rstd[r] * g + b;
            z0[r] += f * w0;
            z1[r] += f * w1;
        }
    }
}

// Final LN, linear d -> 2 and log-softmax of R rows, computed by one wave
// (all lanes return the same values).  The rows' chains are interleaved so
// their loads and reductions overlap; each row sees the same operations in
// the same order whatever R is, and contraction is off, so a row's result
// does not depend on which rows share the call.  Up to d = 64 kHeadCols a
// lane loads its columns of the rows and of the head parameters once, all
// before the first sum; wider rows are read in each of the three passes.
constexpr int kHeadCols = 4;
template <typename C, int R>
__device__ inline void head_rows(const C* const (&x)[R], int d,
                                 const HeadW<C>& hw, C (&lp0)[R], C (&lp1)[R]) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    C s[R], v[R], mean[R], rstd[R], z0[R], z1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = v[r] = z0[r] = z1[r] = 0;
    if (d <= 64 * kHeadCols) {
        constexpr int KH = kHeadCols;
        C xv[R][KH], g[KH], b[KH], w0[KH], w1[KH];
#pragma unroll
        for (int j = 0; j < KH; ++j) {
            const int k = lane + 64 * j;
            if (k < d) {
#pragma unroll
                for (int r = 0; r < R; ++r) xv[r][j] = x[r][k];
                g[j] = hw.lnf_g[k];
                b[j] = hw.lnf_b[k];
                w0[j] = hw.W_head[2 * k];
                w1[j] = hw.W_head[2 * k + 1];
            }
        }
        // the passes below take the columns k = lane, lane + 64, ... in
        // order, as the loops of the general form do
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (lane + 64 * j < d)
#pragma unroll
                for (int r = 0; r < R; ++r) s[r] += xv[r][j];
#pragma unroll
        for (int r = 0; r < R; ++r) mean[r] = wave_sum(s[r]) / (C)d;
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (lane + 64 * j < d)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const C t = xv[r][j] - mean[r];
                    v[r] += t * t;
                }
#pragma unroll
        for (int r = 0; r < R; ++r)
            rstd[r] = (C)1 / dsqrt(wave_sum(v[r]) / (C)d + (C)1e-5);
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (lane + 64 * j < d)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const C f = (xv[r][j] - mean[r]) * rstd[r] * g[j] + b[j];
                    z0[r] += f * w0[j];
                    z1[r] += f * w1[j];
                }
    } else {
        head_passes<C, R>(x, d, hw, s, v, mean, rstd, z0, z1);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const C a0 = wave_sum(z0[r]) + hw.b_head[0];
        const C a1 = wave_sum(z1[r]) + hw.b_head[1];
        const C mx = a0 > a1 ? a0 : a1;
        const C lse = mx + dlog(dexp(a0 - mx) + dexp(a1 - mx));
        lp0[r] = a0 - lse;
        lp1[r] = a1 - lse;
    }
}

// The same for tokens of V = 2^K values: log-probabilities lp[r][c] of
// every value.  V = 2 is head_rows itself; wider heads take the three
// passes over the columns (normalisation statistics, then the logits) with
// the values' sums kept per lane and reduced at the end, and the
// log-softmax sums the exponentials in value order.
template <typename C, int R, int V>
__device__ inline void head_rows_v(const C* const (&x)[R], int d,
                                   const HeadW<C>& hw, C (&lp)[R][V]) {
#pragma clang fp contract(off)
    if constexpr (V == 2) {
        C l0[R], l1[R];
        head_rows<C, R>(x, d, hw, l0, l1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            lp[r][0] = l0[r];
            lp[r][1] = l1[r];
        }
    } else {
        const int lane = threadIdx.x & 63;
        C s[R], v[R], mean[R], rstd[R], z[R][V];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s[r] = v[r] = 0;
#pragma unroll
            for (int c = 0; c < V; ++c) z[r][c] = 0;
        }
        for (int k = lane; k < d; k += 64)
#pragma unroll
            for (int r = 0; r < R; ++r) s[r] += x[r][k];
#pragma unroll
        for (int r = 0; r < R; ++r) mean[r] = wave_sum(s[r]) / (C)d;
        for (int k = lane; k < d; k += 64)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const C t = x[r][k] - mean[r];
                v[r] += t * t;
            }
#pragma unroll
        for (int r = 0; r < R; ++r)
            rstd[r] = (C)1 / dsqrt(wave_sum(v[r]) / (C)d + (C)1e-5);
        for (int k = lane; k < d; k += 64) {
            const C g = hw.lnf_g[k], b = hw.lnf_b[k];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const C f = (x[r][k] - mean[r]) * rstd[r] * g + b;
#pragma unroll
                for (int c = 0; c < V; ++c) z[r][c] += f * hw.W_head[k * V + c];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C a[V];
            C mx = neg_inf<C>();
#pragma unroll
            for (int c = 0; c < V; ++c) {
                a[c] = wave_sum(z[r][c]) + hw.b_head[c];
                mx = a[c] > mx ? a[c] : mx;
            }
            C sum = 0;
#pragma unroll
            for (int c = 0; c < V; ++c) sum += dexp(a[c] - mx);
            const C lse = mx + dlog(sum);
#pragma unroll
            for (int c = 0; c < V; ++c) lp[r][c] = a[c] - lse;
        }
    }
}

// Launch of a head kernel instantiated per token width: V = 2^K values.
#define VQ_BY_VALUES(K, CALL)        \
    switch (K) {                     \
        case 1: { constexpr int V = 2; CALL; break; }  \
        case 2: { constexpr int V = 4; CALL; break; }  \
        case 3: { constexpr int V = 8; CALL; break; }  \
        case 4: { constexpr int V = 16; CALL; break; } \
        default: return hipErrorInvalidValue;          \
    }

// Encoder head term of R rows (one wave): LN(x) . w with the final LN and
// the single-output head (the bias is added once, to the pooled mean);
// contraction off, each row's operations in one order.
template <typename C, int R>
__device__ inline void head_terms(const C* const (&x)[R], int d,
                                  const HeadW<C>& hw, C (&t)[R]) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    C s[R], v[R], mean[R], rstd[R], z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = v[r] = z[r] = 0;
    for (int k = lane; k < d; k += 64)
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] += x[r][k];
#pragma unroll
    for (int r = 0; r < R; ++r) mean[r] = wave_sum(s[r]) / (C)d;
    for (int k = lane; k < d; k += 64)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const C q = x[r][k] - mean[r];
            v[r] += q * q;
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
        rstd[r] = (C)1 / dsqrt(wave_sum(v[r]) / (C)d + (C)1e-5);
    for (int k = lane; k < d; k += 64) {
        const C g = hw.lnf_g[k], b = hw.lnf_b[k], w = hw.W_head[k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const C f = (x[r][k] - mean[r]) * rstd[r] * g + b;
            z[r] += f * w;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = wave_sum(z[r]);
}

// Encoder: log psi = (sum of the rows' terms in row order, FP64) / N + b;
// the terms are kept in lp when given (the samples' cache for the dedup).
template <class P>
__global__ void __launch_bounds__(kThreads) k_head_seq_enc(
    ModelDims m, HeadW<typename P::acc> hw, const int32_t* n_dev,
    int64_t n_seq, const typename P::acc* __restrict__ x,
    typename P::acc* __restrict__ lp, double* __restrict__ logpsi) {
    using acc = typename P::acc;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* ell = reinterpret_cast<double*>(smem_raw);   // [N]
    const int64_t n = n_dev ? (int64_t)*n_dev : n_seq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        for (int i = wave; i < m.N; i += kThreads / 64) {
            const int64_t row = s * m.N + i;
            const acc* xr[1] = {x + row * m.d};
            acc t[1];
            head_terms<acc, 1>(xr, m.d, hw, t);
            if (lane == 0) {
                ell[i] = (double)t[0];
                if (lp) lp[row] = t[0];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc64 = 0.0;
            for (int i = 0; i < m.N; ++i) acc64 += ell[i];
            logpsi[s] = acc64 / (double)m.N + (double)hw.b_head[0];
        }
        __syncthreads();
    }
}

template <class P, int V>
__global__ void __launch_bounds__(kThreads) k_head_seq(
    ModelDims m, HeadW<typename P::acc> hw, const int8_t* __restrict__ spins,
    const int32_t* n_dev, int64_t n_seq, const typename P::acc* __restrict__ x,
    typename P::acc* __restrict__ lp, double* __restrict__ logpsi) {
    using acc = typename P::acc;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* ell = reinterpret_cast<double*>(smem_raw);   // [N]
    const int64_t n = n_dev ? (int64_t)*n_dev : n_seq;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        for (int i = wave; i < m.N; i += kThreads / 64) {
            const int64_t row = s * m.N + i;
            const acc* xr[1] = {x + row * m.d};
            acc l[1][V];
            head_rows_v<acc, 1, V>(xr, m.d, hw, l);
            if (lane == 0) {
                ell[i] = (double)l[0][token_at(spins + s * m.S, i, m.K)];
                if (lp)
#pragma unroll
                    for (int c = 0; c < V; ++c) lp[row * V + c] = l[0][c];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc64 = 0.0;
            for (int i = 0; i < m.N; ++i) acc64 += ell[i];
            logpsi[s] = 0.5 * acc64;
        }
        __syncthreads();
    }
}

template <class P>
hipError_t launch_head_seq(const ModelDims& m, const HeadW<typename P::acc>& hw,
                           const int8_t* spins, const int32_t* n_dev,
                           int64_t n_seq, const typename P::acc* x,
                           typename P::acc* lp, double* logpsi,
                           hipStream_t st) {
    if (m.enc) {
        hipLaunchKernelGGL((k_head_seq_enc<P>), dim3(grid_for(n_seq)), dim3(kThreads),
                           sizeof(double) * m.N, st, m, hw, n_dev, n_seq, x, lp,
                           logpsi);
        return hipGetLastError();
    }
    VQ_BY_VALUES(m.K, hipLaunchKernelGGL((k_head_seq<P, V>), dim3(grid_for(n_seq)),
                                         dim3(kThreads), sizeof(double) * m.N, st,
                                         m, hw, spins, n_dev, n_seq, x, lp, logpsi));
    return hipGetLastError();
}

// ------------------------------------------------ autoregressive sampling
// Direct sampling from the chain rule P(s) = prod_i P(s_i | s_<i) (Sec. 2):
// position i of every sample is evaluated with the keys and values of
// positions < i kept per layer, and s_i is drawn from the head's
// conditional with the caller's uniform number u (s_i = +1 iff
// u < P(s_i = +1 | s_<i), in FP64).  Row i of every per-row kernel is the
// row a full forward pass of the finished sequence computes, with the same
// arithmetic in the same order.

// Step i: block input x of row i (embedding of the previous spin, as
// k_embed), the row list of step i, and at i = 0 the log-probability sums.
template <class P>
__global__ void k_sample_embed(ModelDims m, HeadW<typename P::acc> hw,
                               int64_t n, int i,
                               const int8_t* __restrict__ spins,
                               typename P::acc* __restrict__ x,
                               int64_t* __restrict__ list,
                               double* __restrict__ lpsum) {
    const int64_t total = n * m.d;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / m.d;
        const int col = (int)(e - s * m.d);
        const int64_t row = s * m.N + i;
        const int u = i == 0 ? 1 << m.K : token_at(spins + s * m.S, i - 1, m.K);
        x[row * m.d + col] = hw.tok[u * m.d + col] + hw.pos[(int64_t)i * m.d + col];
        if (col == 0) {
            list[s] = row;
            if (i == 0) lpsum[s] = 0.0;
        }
    }
}

template <class P>
hipError_t launch_sample_embed(const ModelDims& m,
                               const HeadW<typename P::acc>& hw, int64_t n,
                               int i, const int8_t* spins,
                               typename P::acc* x, int64_t* list,
                               double* lpsum, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_embed<P>, dim3(grid_for((n * m.d + 255) / 256)),
                       dim3(256), 0, st, m, hw, n, i, spins, x, list, lpsum);
    return hipGetLastError();
}

// Attention of query row i of every (sample, head) over its keys 0..i,
// one thread per (sample, head), keys read from the per-layer cache.
template <class P, int DH>
__global__ void __launch_bounds__(kThreads) k_attn_rows(ModelDims m, int64_t n,
                                                        int i, BlockIO<P> io) {
    using acc = typename P::acc;
    using act = typename P::act;
    const int64_t units = n * m.nh;
    const acc scale = (acc)1 / dsqrt((acc)DH);
    const int d = m.d, N = m.N;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = u / m.nh;
        const int h = (int)(u - s * m.nh);
        const int64_t base = s * N * d + h * DH;
        acc q[DH], o[DH];
#pragma unroll
        for (int c = 0; c < DH; ++c)
            q[c] = cvt<acc>(io.q[base + (int64_t)i * d + c]) * scale;
        attend_row<acc, DH, act>(q, io.k + base, io.v + base, i, o, d);
#pragma unroll
        for (int c = 0; c < DH; ++c)
            io.a[base + (int64_t)i * d + c] = cvt<act>(o[c]);
    }
}

template <class P>
hipError_t launch_attn_rows(const ModelDims& m, int64_t n, int i,
                            const BlockIO<P>& io, hipStream_t st) {
    const dim3 g(grid_for((n * m.nh + kThreads - 1) / kThreads)), b(kThreads);
    switch (m.dh) {
        case 4: hipLaunchKernelGGL((k_attn_rows<P, 4>), g, b, 0, st, m, n, i, io); break;
        case 8: hipLaunchKernelGGL((k_attn_rows<P, 8>), g, b, 0, st, m, n, i, io); break;
        case 16: hipLaunchKernelGGL((k_attn_rows<P, 16>), g, b, 0, st, m, n, i, io); break;
        case 32: hipLaunchKernelGGL((k_attn_rows<P, 32>), g, b, 0, st, m, n, i, io); break;
        case 64: hipLaunchKernelGGL((k_attn_rows<P, 64>), g, b, 0, st, m, n, i, io); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Head of row i of every sample (one wave each, as k_head_seq), the draw of
// token i, and the running sum of log P(t_i | t_<i) in position order (FP64,
// as k_head_seq sums it); at the last position log psi = sum / 2.  One
// spin per token: s_i = +1 iff u_i < P(+1).  Tokens of K spins: the
// smallest value c whose cumulative probability (exponentials of the
// log-probabilities summed in value order, FP64) exceeds the uniform
// number of the token's first site; the K spins are the bits of c.
template <class P, int V>
__global__ void __launch_bounds__(kThreads) k_sample_head(
    ModelDims m, HeadW<typename P::acc> hw, int64_t n, int i,
    const typename P::acc* __restrict__ x, const double* __restrict__ uni,
    int8_t* __restrict__ spins, double* __restrict__ lpsum,
    double* __restrict__ logpsi) {
    using acc = typename P::acc;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t s = blockIdx.x * (int64_t)(kThreads / 64) + (threadIdx.x >> 6);
         s < n; s += waves) {
        const int64_t row = s * m.N + i;
        const acc* xr[1] = {x + row * m.d};
        acc l[1][V];
        head_rows_v<acc, 1, V>(xr, m.d, hw, l);
        if (lane == 0) {
            const int64_t site = s * m.S + (int64_t)i * m.K;
            int c;
            if constexpr (V == 2) {
                c = uni[site] < exp((double)l[0][0]) ? 0 : 1;
            } else {
                const double u = uni[site];
                double cdf = 0.0;
                c = V - 1;
                for (int v = 0; v < V; ++v) {
                    cdf += exp((double)l[0][v]);
                    if (u < cdf) {
                        c = v;
                        break;
                    }
                }
            }
            for (int k = 0; k < m.K; ++k)
                spins[site + k] = ((c >> k) & 1) ? (int8_t)-1 : (int8_t)1;
            const double acc64 = lpsum[s] + (double)l[0][c];
            lpsum[s] = acc64;
            if (i == m.N - 1 && logpsi) logpsi[s] = 0.5 * acc64;
        }
    }
}

template <class P>
hipError_t launch_sample_head(const ModelDims& m,
                              const HeadW<typename P::acc>& hw, int64_t n,
                              int i, const typename P::acc* x,
                              const double* uni, int8_t* spins, double* lpsum,
                              double* logpsi, hipStream_t st) {
    VQ_BY_VALUES(m.K, hipLaunchKernelGGL((k_sample_head<P, V>),
                                         dim3(grid_for((n + kThreads / 64 - 1) / (kThreads / 64))),
                                         dim3(kThreads), 0, st, m, hw, n, i, x, uni,
                                         spins, lpsum, logpsi));
    return hipGetLastError();
}

// ratio = exp(log psi(s') - log psi(s)) for materialised neighbours (FP64)
__global__ void k_ratio_plain(const double* __restrict__ lnb,
                              const double* __restrict__ ls,
                              const NbDesc* __restrict__ desc,
                              const int32_t* n_dev, int64_t n_max,
                              double* __restrict__ ratio) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        ratio[k] = exp(lnb[k] - ls[desc[k].sigma]);
}

hipError_t launch_ratio_plain(const double* logpsi_nb, const double* logpsi_s,
                              const NbDesc* desc, const int32_t* n_dev,
                              int64_t n_max, double* ratio, hipStream_t st) {
    hipLaunchKernelGGL(k_ratio_plain, dim3(grid_for((n_max + 255) / 256)),
                       dim3(256), 0, st, logpsi_nb, logpsi_s, desc, n_dev,
                       n_max, ratio);
    return hipGetLastError();
}

// ------------------------------------------------------------ dedup steps
// C_0: the changed inputs p1+1 and p2+1 (when < N) get their new
// embeddings; every overlay row records its neighbour.  A wave reserves the
// list entries of kCdBatch neighbours with one atomic on the shared counter.
constexpr int kCdBatch = 8;

template <class P>
__global__ void __launch_bounds__(64) k_dedup_init(ModelDims m,
                                                   HeadW<typename P::acc> hw,
                                                   DedupIO<P> dd) {
    const int64_t n = (int64_t)*dd.n_nb;
    const int lane = threadIdx.x;
    const int N = m.N, d = m.d, W = dd.mask_words;
    const int64_t stride = gridDim.x;
    for (int64_t nb0 = blockIdx.x; nb0 < n; nb0 += stride * kCdBatch) {
        int all = 0;
#pragma unroll 1
        for (int g = 0; g < kCdBatch; ++g) {
            const int64_t nb = nb0 + g * stride;
            if (nb >= n) continue;
            const NbDesc D = dd.desc[nb];
            const int pmin = first_row(D, m);
            for (int i = lane; i < N - pmin; i += 64) dd.slot_nb[D.ov + i] = (int32_t)nb;
            uint64_t* mk = dd.mask + nb * W;
            const int8_t* sp = dd.spins + (int64_t)D.sigma * m.S;
            const int rowsC[2] = {D.p1 + 1, D.p2 + 1};
            // the neighbour's tokens p1 and p2 are the inputs of rows p1 + 1
            // and p2 + 1: two changed input tokens (p1 < p2 < N), or one at
            // p1 + 1, if there is one, when both changed sites (or the one
            // flipped site) lie in token p1 == p2
            const bool single = D.p1 == D.p2;
            // (the encoder reads token p + 1 itself at row p + 1)
            const int sh = m.enc ? 1 : 0;
            const int tokC[2] = {nb_token_at(sp, D, D.p1 + sh, m.K),
                                 nb_token_at(sp, D, D.p2 + sh, m.K)};
            const int nC = single ? (rowsC[0] < N ? 1 : 0) : (rowsC[1] < N ? 2 : 1);
            // every mask word written once, never read back within the kernel
            for (int wd = lane; wd < W; wd += 64) {
                uint64_t v = 0;
                for (int c = 0; c < nC; ++c)
                    if ((rowsC[c] >> 6) == wd) v |= 1ull << (rowsC[c] & 63);
                mk[wd] = v;
            }
            for (int c = 0; c < nC; ++c) {
                const int i = rowsC[c];
                const int64_t slot = D.ov + (i - pmin);
                for (int k = lane; k < d; k += 64)
                    dd.ox[slot * d + k] = hw.tok[tokC[c] * d + k] + hw.pos[(int64_t)i * d + k];
                if (lane == 0) dd.crow[D.ov + c] = (int16_t)i;
            }
            if (lane == 0) dd.ccnt[nb] = nC;
            all += nC;
        }
        int64_t pos = 0;
        if (lane == 0) pos = atomicAdd(dd.list_n, all);
        pos = __shfl(pos, 0, 64);
        if (lane == 0) {
#pragma unroll 1
            for (int g = 0; g < kCdBatch; ++g) {
                const int64_t nb = nb0 + g * stride;
                if (nb >= n) break;
                const NbDesc D = dd.desc[nb];
                const int pmin = first_row(D, m);
                const int nC = D.p1 == D.p2 ? (pmin < N ? 1 : 0)
                                            : (D.p2 + 1 < N ? 2 : 1);
                if (nC >= 1) dd.list[pos] = D.ov + (D.p1 + 1 - pmin);
                if (nC == 2) dd.list[pos + 1] = D.ov + (D.p2 + 1 - pmin);
                pos += nC;
            }
        }
    }
}

template <class P>
hipError_t launch_dedup_init(const ModelDims& m, const HeadW<typename P::acc>& hw,
                             const DedupIO<P>& d, hipStream_t st) {
    hipLaunchKernelGGL(k_dedup_init<P>, dim3(grid_for(d.n_nb_max)), dim3(64), 0,
                       st, m, hw, d);
    return hipGetLastError();
}

// Certified reuse test for every overlay row (or, without the flag, plain
// listing of every row for the codebook search).  One wave per row; rows
// that need the search collect in an LDS list of 64 and are appended to the
// shared list with one atomic per 64 rows.
template <class P>
__global__ void __launch_bounds__(64) k_certify(ModelDims m, DedupIO<P> dd,
                                                int certified, int64_t* ctr) {
    using acc = typename P::acc;
    __shared__ int64_t pend[64];
    const int64_t R = (int64_t)*dd.n_rows;
    const int lane = threadIdx.x;
    const int ds = m.dseg;
    int64_t n_cert = 0;
    int npend = 0;                 // the same in every lane
    auto flush = [&]() {
        __syncthreads();
        int64_t base = 0;
        if (lane == 0) base = atomicAdd(dd.vq_n, npend);
        base = __shfl(base, 0, 64);
        if (lane < npend) dd.vq_list[base + lane] = pend[lane];
        npend = 0;
        __syncthreads();
    };
    for (int64_t r = blockIdx.x; r < R; r += gridDim.x) {
        const int32_t nb = dd.slot_nb[r];
        const NbDesc D = dd.desc[nb];
        const int i = first_row(D, m) + (int)(r - D.ov);
        const int64_t brow = (int64_t)D.sigma * m.N + i;
        bool ok = certified != 0;
        for (int hq = 0; hq < m.H && ok; ++hq) {
            acc dl = 0, n1 = 0, n0 = 0;
            for (int k = lane; k < ds; k += 64) {
                const acc x1 = cvt<acc>(dd.oa[r * m.d + hq * ds + k]);
                const acc x0 = cvt<acc>(dd.ba[brow * m.d + hq * ds + k]);
                dl += (x1 - x0) * (x1 - x0);
                n1 += x1 * x1;
                n0 += x0 * x0;
            }
            dl = wave_sum(dl);
            n1 = dsqrt(wave_sum(n1));
            n0 = dsqrt(wave_sum(n0));
            const acc g = (acc)(ds + 4) * unit_roundoff<acc>() * (acc)2;
            acc delta = dsqrt(dl) * ((acc)1 + g) + unit_roundoff<acc>();
            // the matrix-core search sees hi + lo of each row, which moves a
            // row by at most 2^-16 of its norm
            if (m.mfma) delta += (acc)1.5258789e-5 * (n0 + n1);
            const acc U1 = dd.bmargin[(brow * m.H + hq) * 2];
            const acc L2 = dd.bmargin[(brow * m.H + hq) * 2 + 1];
            const acc lo = L2 - delta, hi = U1 + delta;
            const acc wmax = dd.wmax[hq];
            acc E = score_err<acc>(m.mfma ? 2 * ds : ds, n1, wmax);
            if (m.mfma) E += (acc)3.0517578e-5 * (n1 * wmax + n1 * n1);
            // lo bounds every other code's distance from below and hi the
            // kept code's from above; the computed scores then separate
            // strictly when the gap exceeds twice the score-error bound
            ok = lo > 0 && (lo * lo - hi * hi) > (acc)4 * E;
        }
        if (ok) {
            for (int hq = lane; hq < m.H; hq += 64)
                dd.ocode[r * m.H + hq] = dd.bcode[brow * m.H + hq];
            n_cert++;
        } else {
            if (lane == 0) pend[npend] = r;
            if (++npend == 64) flush();
        }
    }
    if (npend) flush();
    if (ctr && lane == 0 && n_cert)
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_VQ_CERTIFIED),
                  (unsigned long long)n_cert);
}

template <class P>
hipError_t launch_certify(const ModelDims& m, const DedupIO<P>& d,
                          int certified, int64_t* ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_certify<P>, dim3(grid_for(d.rows_max)), dim3(64), 0,
                       st, m, d, certified, ctr);
    return hipGetLastError();
}

// One wave copies rows sb + jl[p] of src to rows ob + jl[p] of dst
// (p < nj), V units of T per row: batches of 4 units per lane, the batch's
// loads issued before its stores (indices past the end are clamped; their
// values are not stored).
template <class T>
__device__ inline void copy_rows(const T* __restrict__ src, T* __restrict__ dst,
                                 int V, int64_t sb, int64_t ob, const int* jl,
                                 int nj) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const int tot = nj * V;
    for (int e0 = 0; e0 < tot; e0 += 64 * U) {
        T v[U];
        int64_t off[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + 64 * u + lane;
            const int ec = e < tot ? e : tot - 1;
            const int p = ec / V;
            off[u] = (int64_t)jl[p] * V + (ec - p * V);
            v[u] = src[sb * V + off[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + 64 * u + lane < tot) dst[ob * V + off[u]] = v[u];
    }
}

// C_l = C_{l-1} plus rows whose code differs from the sample's; rows that
// join C get the sample's block input copied into their overlay row, and
// all rows of C_l are listed for the MLP stage (and the next QKV stage).
// A wave takes kCdBatch of its neighbours at a time and reserves their list
// entries with one atomic on the shared counter (one per neighbour made the
// counter's atomics the bottleneck); the order of the list does not matter,
// every listed row is computed on its own.

template <class P>
__global__ void __launch_bounds__(64) k_code_diff(ModelDims m, DedupIO<P> dd) {
    using acc = typename P::acc;
    // The neighbours' mask words live in LDS while they change: global
    // memory is read once at the start and written once at the end, so no
    // lane ever reads back a word another lane stored in this kernel.
    __shared__ uint64_t smk[kCdBatch][VQ_MAX_MASK_WORDS];
    __shared__ int jl[64];
    const int64_t n = (int64_t)*dd.n_nb;
    const int lane = threadIdx.x;
    const int N = m.N, d = m.d, W = dd.mask_words;
    const int64_t stride = gridDim.x;
    for (int64_t nb0 = blockIdx.x; nb0 < n; nb0 += stride * kCdBatch) {
        int tot[kCdBatch];
        int all = 0;
#pragma unroll 1
        for (int g = 0; g < kCdBatch; ++g) {
            tot[g] = 0;
            const int64_t nb = nb0 + g * stride;
            if (nb >= n) continue;
            const NbDesc D = dd.desc[nb];
            const int pmin = first_row(D, m);
            const uint64_t* mk = dd.mask + nb * W;
            uint64_t* sm = smk[g];
            __syncthreads();
            for (int wd = lane; wd < W; wd += 64) sm[wd] = mk[wd];
            __syncthreads();
            for (int i0 = pmin; i0 < N; i0 += 64) {
                const int i = i0 + lane;
                bool joins = false;
                if (i < N && !mask_bit(sm, i)) {
                    const int64_t slot = D.ov + (i - pmin);
                    const int64_t brow = (int64_t)D.sigma * N + i;
                    for (int hq = 0; hq < m.H; ++hq)
                        joins |= dd.ocode[slot * m.H + hq] != dd.bcode[brow * m.H + hq];
                }
                const uint64_t jm = __ballot(joins);
                // copy the sample's block input into the overlay rows that
                // join: the group's joined rows are listed in LDS, then
                // copied in batches whose loads precede their stores
                if (jm) {
                    const uint64_t below = lane == 0 ? 0ull : (jm & (~0ull >> (64 - lane)));
                    if ((jm >> lane) & 1) jl[__popcll(below)] = lane;
                    __syncthreads();
                    const int nj = __popcll(jm);
                    const int64_t sb = (int64_t)D.sigma * N + i0;   // sample row i0
                    const int64_t ob = D.ov + (i0 - pmin);           // its overlay row
                    if ((d * (int)sizeof(acc)) % 16 == 0)
                        copy_rows<uint4>(reinterpret_cast<const uint4*>(dd.bx),
                                         reinterpret_cast<uint4*>(dd.ox),
                                         d * (int)sizeof(acc) / 16, sb, ob, jl, nj);
                    else
                        copy_rows<acc>(dd.bx, dd.ox, d, sb, ob, jl, nj);
                }
                // rows of this group occupy word i0/64 and possibly the next one
                __syncthreads();
                if (lane == 0 && jm) {
                    const int w0 = i0 >> 6, sh = i0 & 63;
                    sm[w0] |= jm << sh;
                    if (sh && w0 + 1 < W) sm[w0 + 1] |= jm >> (64 - sh);
                }
                __syncthreads();
            }
            for (int i0 = pmin; i0 < N; i0 += 64) {
                const int i = i0 + lane;
                tot[g] += __popcll(__ballot(i < N && mask_bit(sm, i)));
            }
            all += tot[g];
        }
        int64_t pos = 0;
        if (lane == 0 && all) pos = atomicAdd(dd.list_n, all);
        pos = __shfl(pos, 0, 64);
#pragma unroll 1
        for (int g = 0; g < kCdBatch; ++g) {
            const int64_t nb = nb0 + g * stride;
            if (nb >= n) continue;
            const NbDesc D = dd.desc[nb];
            const int pmin = first_row(D, m);
            const uint64_t* sm = smk[g];
            int k = 0;
            for (int i0 = pmin; i0 < N; i0 += 64) {
                const int i = i0 + lane;
                const bool inC = i < N && mask_bit(sm, i);
                const uint64_t cm = __ballot(inC);
                const uint64_t below = lane == 0 ? 0ull : (cm & (~0ull >> (64 - lane)));
                if (inC) {
                    dd.list[pos + k + __popcll(below)] = D.ov + (i - pmin);
                    dd.crow[D.ov + k + __popcll(below)] = (int16_t)i;
                }
                k += __popcll(cm);
            }
            pos += k;
            if (lane == 0) dd.ccnt[nb] = k;
            uint64_t* mk = dd.mask + nb * W;
            for (int wd = lane; wd < W; wd += 64) mk[wd] = sm[wd];
        }
    }
}

template <class P>
hipError_t launch_code_diff(const ModelDims& m, const DedupIO<P>& d,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_code_diff<P>, dim3(grid_for(d.n_nb_max)), dim3(64), 0,
                       st, m, d);
    return hipGetLastError();
}

// Delta log psi of each neighbour: rows of C_L get new head outputs, the
// exchanged sites p1, p2 (new targets) use the sample's cached log-probs
// when their hidden state is unchanged.  The rows of C_L are listed in LDS
// and evaluated four at a time, their new log-probs kept in LDS beside the
// sample's cached ones (loaded by all lanes at once); lane 0 sums the
// differences in FP64 in row order from LDS.
template <class P, int V>
__global__ void __launch_bounds__(64) k_head_dedup(
    ModelDims m, HeadW<typename P::acc> hw, DedupIO<P> dd,
    const typename P::acc* __restrict__ blp, double* __restrict__ ratio,
    int64_t* ctr) {
    using acc = typename P::acc;
    constexpr int R = 4;
    __shared__ uint64_t sm[VQ_MAX_MASK_WORDS];
    __shared__ int16_t rl[VQ_MAX_MASK_WORDS * 64];
    __shared__ typename P::acc lnw[VQ_MAX_MASK_WORDS * 64];   // by list position
    __shared__ typename P::acc lold[VQ_MAX_MASK_WORDS * 64];  // by list position
    const int64_t n = (int64_t)*dd.n_nb;
    const int lane = threadIdx.x;
    const int N = m.N, W = dd.mask_words;
    int64_t my_rows = 0;
    for (int64_t nb = blockIdx.x; nb < n; nb += gridDim.x) {
        const NbDesc D = dd.desc[nb];
        const int pmin = first_row(D, m);
        const uint64_t* mk = dd.mask + nb * W;
        const int8_t* sp = dd.spins + (int64_t)D.sigma * m.S;
        __syncthreads();
        for (int wd = lane; wd < W; wd += 64) sm[wd] = mk[wd];
        __syncthreads();
        // rows of C_L in order
        int nc = 0;
        for (int i0 = pmin; i0 < N; i0 += 64) {
            const int i = i0 + lane;
            const bool inC = i < N && mask_bit(sm, i);
            const uint64_t cm = __ballot(inC);
            const uint64_t below = lane == 0 ? 0ull : (cm & (~0ull >> (64 - lane)));
            if (inC) rl[nc + __popcll(below)] = (int16_t)i;
            nc += __popcll(cm);
        }
        __syncthreads();
        // target tokens of s' (exchanged sites swap spins, a flipped site
        // changes sign) and of s at row i; p1 == p2: one changed token
        const bool single = D.p1 == D.p2;
        auto tnew = [&](int i) { return nb_token_at(sp, D, i, m.K); };
        auto told = [&](int i) { return token_at(sp, i, m.K); };
        for (int c0 = 0; c0 < nc; c0 += R) {
            const acc* xr[R];
            int ir[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                ir[r] = rl[c0 + r < nc ? c0 + r : nc - 1];
                xr[r] = dd.ox + (D.ov + (ir[r] - pmin)) * (int64_t)m.d;
            }
            acc l[R][V];
            head_rows_v<acc, R, V>(xr, m.d, hw, l);
            if (lane < R && c0 + lane < nc) {
                // lane r takes row r of the group (no dynamic register index)
                int i = ir[0];
#pragma unroll
                for (int rr = 1; rr < R; ++rr)
                    if (lane == rr) i = ir[rr];
                const int t = tnew(i);
                acc a = l[0][0];
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int c = 0; c < V; ++c)
                        if (lane == rr && c == t) a = l[rr][c];
                lnw[c0 + lane] = a;
            }
        }
        my_rows += nc;
        __syncthreads();
        // the sample's log-prob of its own target at every listed row
        bool p2in = false;
        for (int c = lane; c < nc; c += 64) {
            const int i = rl[c];
            lold[c] = blp[((int64_t)D.sigma * N + i) * V + told(i)];
            p2in |= i == D.p2;
        }
        p2in = __ballot(p2in) != 0;
        __syncthreads();
        if (lane == 0) {
            // rows p1, then the listed rows (all after p1) with p2 in its
            // place: the rows and the order of a walk over i = p1 .. N-1
            auto unlisted = [&](int i) {
                const int64_t brow = (int64_t)D.sigma * N + i;
                return (double)blp[brow * V + tnew(i)] - (double)blp[brow * V + told(i)];
            };
            // one changed token has one changed target (p1); two changed
            // tokens a second one at p2 unless p2 is a listed row
            const double t2 = (p2in || single) ? 0.0 : unlisted(D.p2);
            double delta = 0.0;
            delta += unlisted(D.p1);
            bool p2done = p2in || single;
            for (int c = 0; c < nc; ++c) {
                if (!p2done && rl[c] > D.p2) {
                    delta += t2;
                    p2done = true;
                }
                delta += (double)lnw[c] - (double)lold[c];
            }
            if (!p2done) delta += t2;
            ratio[nb] = exp(0.5 * delta);
        }
    }
    if (ctr && lane == 0 && my_rows)
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_HEAD_ROWS),
                  (unsigned long long)my_rows);
}

// Encoder: log psi(s') - log psi(s) = (sum over the rows of C_L of the
// new term minus the sample's cached one, in row order, FP64) / N.  Rows
// of C_L are listed in LDS and evaluated four at a time.
template <class P>
__global__ void __launch_bounds__(64) k_head_dedup_enc(
    ModelDims m, HeadW<typename P::acc> hw, DedupIO<P> dd,
    const typename P::acc* __restrict__ bterm, double* __restrict__ ratio,
    int64_t* ctr) {
    using acc = typename P::acc;
    constexpr int R = 4;
    __shared__ uint64_t sm[VQ_MAX_MASK_WORDS];
    __shared__ int16_t rl[VQ_MAX_MASK_WORDS * 64];
    __shared__ typename P::acc tnw[VQ_MAX_MASK_WORDS * 64];
    const int64_t n = (int64_t)*dd.n_nb;
    const int lane = threadIdx.x;
    const int N = m.N, W = dd.mask_words;
    int64_t my_rows = 0;
    for (int64_t nb = blockIdx.x; nb < n; nb += gridDim.x) {
        const NbDesc D = dd.desc[nb];
        const int pmin = first_row(D, m);
        const uint64_t* mk = dd.mask + nb * W;
        __syncthreads();
        for (int wd = lane; wd < W; wd += 64) sm[wd] = mk[wd];
        __syncthreads();
        int nc = 0;
        for (int i0 = 0; i0 < N; i0 += 64) {
            const int i = i0 + lane;
            const bool inC = i < N && mask_bit(sm, i);
            const uint64_t cm = __ballot(inC);
            const uint64_t below = lane == 0 ? 0ull : (cm & (~0ull >> (64 - lane)));
            if (inC) rl[nc + __popcll(below)] = (int16_t)i;
            nc += __popcll(cm);
        }
        __syncthreads();
        for (int c0 = 0; c0 < nc; c0 += R) {
            const acc* xr[R];
            int ir[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                ir[r] = rl[c0 + r < nc ? c0 + r : nc - 1];
                xr[r] = dd.ox + (D.ov + (ir[r] - pmin)) * (int64_t)m.d;
            }
            acc t[R];
            head_terms<acc, R>(xr, m.d, hw, t);
            if (lane < R && c0 + lane < nc) {
                acc a = t[0];
#pragma unroll
                for (int r = 1; r < R; ++r)
                    if (lane == r) a = t[r];
                tnw[c0 + lane] = a;
            }
        }
        my_rows += nc;
        __syncthreads();
        if (lane == 0) {
            double delta = 0.0;
            for (int c = 0; c < nc; ++c)
                delta += (double)tnw[c] -
                         (double)bterm[(int64_t)D.sigma * N + rl[c]];
            ratio[nb] = exp(delta / (double)N);
        }
    }
    if (ctr && lane == 0 && my_rows)
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_HEAD_ROWS),
                  (unsigned long long)my_rows);
}

template <class P>
hipError_t launch_head_dedup(const ModelDims& m, const HeadW<typename P::acc>& hw,
                             const DedupIO<P>& d, const typename P::acc* blp,
                             const double*, double* ratio, int64_t* ctr,
                             hipStream_t st) {
    if (m.enc) {
        hipLaunchKernelGGL((k_head_dedup_enc<P>), dim3(grid_for(d.n_nb_max)), dim3(64),
                           0, st, m, hw, d, blp, ratio, ctr);
        return hipGetLastError();
    }
    VQ_BY_VALUES(m.K, hipLaunchKernelGGL((k_head_dedup<P, V>), dim3(grid_for(d.n_nb_max)),
                                         dim3(64), 0, st, m, hw, d, blp, ratio, ctr));
    return hipGetLastError();
}

// ------------------------------------------------------ instantiations
#define VQ_INST(P)                                                            \
    template hipError_t launch_prepare<P>(const ModelDims&,                   \
                                          const LayerW<P::acc>&, P::acc*,     \
                                          P::acc*, bf16*, bf16*, bf16*,       \
                                          bf16*, hipStream_t);                \
    template hipError_t launch_embed<P>(const ModelDims&,                     \
                                        const HeadW<P::acc>&, const int8_t*,  \
                                        const int32_t*, int64_t, P::acc*,     \
                                        hipStream_t);                         \
    template hipError_t launch_qkv<P>(const ModelDims&, const LayerW<P::acc>&, \
                                      RowSet, const BlockIO<P>&, hipStream_t); \
    template hipError_t launch_attention_seq<P>(const ModelDims&,             \
                                                const int32_t*, int64_t,      \
                                                const BlockIO<P>&, int64_t*,  \
                                                hipStream_t);                 \
    template hipError_t launch_vq<P>(const ModelDims&, const LayerW<P::acc>&,  \
                                     RowSet, const BlockIO<P>&, hipStream_t);  \
    template hipError_t launch_mlp<P>(const ModelDims&, const LayerW<P::acc>&, \
                                      RowSet, const BlockIO<P>&, hipStream_t); \
    template hipError_t launch_head_seq<P>(                                   \
        const ModelDims&, const HeadW<P::acc>&, const int8_t*,                \
        const int32_t*, int64_t, const P::acc*, P::acc*, double*,             \
        hipStream_t);                                                         \
    template hipError_t launch_dedup_init<P>(const ModelDims&,                \
                                             const HeadW<P::acc>&,            \
                                             const DedupIO<P>&, hipStream_t); \
    template hipError_t launch_attention_dedup<P>(                            \
        const ModelDims&, const DedupIO<P>&, int64_t*, hipStream_t);          \
    template hipError_t launch_certify<P>(const ModelDims&,                   \
                                          const DedupIO<P>&, int, int64_t*,   \
                                          hipStream_t);                       \
    template hipError_t launch_code_diff<P>(const ModelDims&,                 \
                                            const DedupIO<P>&, hipStream_t);  \
    template hipError_t launch_head_dedup<P>(                                 \
        const ModelDims&, const HeadW<P::acc>&, const DedupIO<P>&,            \
        const P::acc*, const double*, double*, int64_t*, hipStream_t);        \
    template hipError_t launch_out_proj<P>(                                   \
        const ModelDims&, const P::acc*, const P::acc*, RowSet,               \
        const P::acc*, const P::act*, P::acc*, hipStream_t);                  \
    template hipError_t launch_out_proj_overlay<P>(                           \
        const ModelDims&, const P::acc*, const P::acc*, const DedupIO<P>&,    \
        P::acc*, hipStream_t);                                                \
    template hipError_t launch_attention_incr<P>(                             \
        const ModelDims&, const DedupIO<P>&, const P::acc*, int64_t*,         \
        hipStream_t);                                                         \
    template hipError_t launch_sample_embed<P>(                               \
        const ModelDims&, const HeadW<P::acc>&, int64_t, int, const int8_t*,  \
        P::acc*, int64_t*, double*, hipStream_t);                             \
    template hipError_t launch_attn_rows<P>(const ModelDims&, int64_t, int,   \
                                            const BlockIO<P>&, hipStream_t);  \
    template hipError_t launch_sample_head<P>(                                \
        const ModelDims&, const HeadW<P::acc>&, int64_t, int, const P::acc*,  \
        const double*, int8_t*, double*, double*, hipStream_t);

VQ_INST(PrecF64)
VQ_INST(PrecF32)
VQ_INST(PrecBF16)

}  // namespace vq
