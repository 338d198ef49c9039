// Lattice-side kernels: spin validation, neighbour enumeration (ballot +
// prefix compaction), neighbour descriptors, local-energy assembly and the
// batch statistics.  Paper: eq. (2) local energy; k-local rows (Sec. 2);
// Heisenberg model with the Marshall sign rule and the transverse-field
// Ising chain (Sec. 4).
#include "kernels.h"

namespace vq {

// Bond b = 2*i + dir of site i = r*L + c; returns false when the bond does
// not exist (open boundaries).
__device__ inline bool bond_sites(int b, int L, int periodic, int& i, int& j) {
    i = b >> 1;
    const int r = i / L, c = i - (i / L) * L;
    if ((b & 1) == 0) {
        if (!periodic && c + 1 == L) return false;
        j = r * L + (c + 1 == L ? 0 : c + 1);
    } else {
        if (!periodic && r + 1 == L) return false;
        j = (r + 1 == L ? 0 : r + 1) * L + c;
    }
    return true;
}

// One wave per sample.  Anti-aligned bonds are found 64 at a time; a ballot
// and a popcount of the lanes below give each one its output slot, so the
// list comes out in increasing bond order without atomics.
__global__ void __launch_bounds__(64) k_neighbours(
    const int8_t* __restrict__ spins, int64_t batch, int L, int chain,
    int periodic, int K, int enc, double J, int16_t* __restrict__ bonds,
    int32_t* __restrict__ count,
    double* __restrict__ diag, int64_t* __restrict__ rows_cap,
    int32_t* __restrict__ status) {
    const int64_t s = blockIdx.x;
    if (s >= batch) return;
    const int lane = threadIdx.x;
    const int N = chain ? L : L * L;
    const int8_t* sp = spins + s * (int64_t)N;
    int bad = 0;
    for (int i = lane; i < N; i += 64) {
        const int8_t v = sp[i];
        bad |= (v != 1 && v != -1);
    }
    if (__any(bad) && lane == 0) atomicOr(status, 1);
    if (chain) {
        // transverse-field Ising chain: every site's flip is a neighbour
        // (listed by site), diagonal -J sum_<ij> s_i s_j over the bonds
        // (i, i+1) and, periodic, (N-1, 0); a flip of site i changes the
        // input tokens from token i/K + 1 on (T = N/K tokens: K rows of
        // T - t - 1 per token t, K T (T - 1) / 2 in all)
        int zz = 0;
        int16_t* out = bonds + s * (int64_t)(2 * N);
        for (int i = lane; i < N; i += 64) {
            out[i] = (int16_t)i;
            out[N + i] = -1;
            const int si = sp[i] < 0 ? -1 : 1;
            if (i + 1 < N) zz += si * (sp[i + 1] < 0 ? -1 : 1);
            else if (periodic && N > 2) zz += si * (sp[0] < 0 ? -1 : 1);
        }
        zz = wave_sum(zz);
        if (lane == 0) {
            count[s] = N;
            if (diag) diag[s] = -J * (double)zz;
            const int64_t T = N / K;
            if (rows_cap)
                rows_cap[s] = enc ? (int64_t)N * T : (int64_t)K * T * (T - 1) / 2;
        }
        return;
    }
    int total = 0;
    int zz = 0;          // sum of s_i s_j over existing bonds
    int64_t cap = 0;     // overlay rows: sum over anti bonds of T - t1 - 1,
                         // t1 = p1 / K the token of the first site
    const int T = N / K;
    int16_t* out = bonds + s * (int64_t)(2 * N);
    for (int b0 = 0; b0 < 2 * N; b0 += 64) {
        const int b = b0 + lane;
        int i = 0, j = 0;
        bool exists = (b < 2 * N) && bond_sites(b, L, periodic, i, j);
        bool anti = false;
        if (exists) {
            const int si = sp[i] < 0 ? -1 : 1, sj = sp[j] < 0 ? -1 : 1;
            zz += si * sj;
            anti = si != sj;
        }
        const uint64_t m = __ballot(anti);
        const uint64_t below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
        if (anti) {
            out[total + __popcll(below)] = (int16_t)b;
            const int p1 = i < j ? i : j;
            cap += enc ? T : T - p1 / K - 1;
        }
        total += __popcll(m);
    }
    for (int k = total + lane; k < 2 * N; k += 64) out[k] = -1;
    zz = wave_sum(zz);
    cap = wave_sum(cap);
    if (lane == 0) {
        count[s] = total;
        if (diag) diag[s] = 0.25 * J * (double)zz;
        if (rows_cap) rows_cap[s] = cap;
    }
}

// Exclusive prefix sums over the samples of a chunk (one workgroup; chunks
// hold at most a few thousand samples).
__global__ void __launch_bounds__(1024) k_scan_chunk(
    const int32_t* __restrict__ count, const int64_t* __restrict__ rows_cap,
    int n, int32_t* __restrict__ nb_off, int64_t* __restrict__ row_off,
    int32_t* __restrict__ n_nb_total, int32_t* __restrict__ n_rows_total) {
    __shared__ int32_t sc[1024];
    __shared__ int64_t sr[1024];
    __shared__ int32_t carry_c;
    __shared__ int64_t carry_r;
    if (threadIdx.x == 0) {
        carry_c = 0;
        carry_r = 0;
    }
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int t = threadIdx.x;
        const int k = base + t;
        sc[t] = k < n ? count[k] : 0;
        sr[t] = k < n ? rows_cap[k] : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {   // Hillis-Steele inclusive scan
            int32_t vc = t >= o ? sc[t - o] : 0;
            int64_t vr = t >= o ? sr[t - o] : 0;
            __syncthreads();
            sc[t] += vc;
            sr[t] += vr;
            __syncthreads();
        }
        if (k < n) {
            nb_off[k] = carry_c + (t ? sc[t - 1] : 0);
            row_off[k] = carry_r + (t ? sr[t - 1] : 0);
        }
        __syncthreads();
        if (t == 0) {
            carry_c += sc[1023];
            carry_r += sr[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nb_off[n] = carry_c;
        row_off[n] = carry_r;
        *n_nb_total = carry_c;
        *n_rows_total = (int32_t)carry_r;
    }
}

// Descriptors of every neighbour of a chunk: one wave per sample, a wave
// prefix-scan over its neighbours assigns overlay row offsets.
__global__ void __launch_bounds__(64) k_descriptors(
    const int16_t* __restrict__ bonds, const int32_t* __restrict__ count,
    const int32_t* __restrict__ nb_off, const int64_t* __restrict__ row_off,
    int n, int L, int chain, int K, int enc, NbDesc* __restrict__ desc) {
    const int s = blockIdx.x;
    if (s >= n) return;
    const int lane = threadIdx.x;
    const int N = chain ? L : L * L;
    const int cnt = count[s];
    const int16_t* bl = bonds + (int64_t)s * 2 * N;
    int64_t carry = row_off[s];
    for (int k0 = 0; k0 < cnt; k0 += 64) {
        const int k = k0 + lane;
        int p1 = 0, p2 = 0;
        int64_t rows = 0;
        if (k < cnt) {
            if (chain) {
                // a single flip: p1 == p2 is the flipped site
                p1 = p2 = bl[k];
            } else {
                int i, j;
                bond_sites(bl[k], L, 1, i, j);
                p1 = i < j ? i : j;
                p2 = i < j ? j : i;
            }
            // decoder: rows after the first changed token; encoder: all
            rows = enc ? N / K : N / K - p1 / K - 1;
        }
        int64_t incl = rows;   // inclusive wave scan
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int64_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (k < cnt) {
            NbDesc d;
            d.sigma = s;
            // tokens of the changed sites (the encoder's changed input
            // rows are the tokens themselves: held as token - 1, so that
            // rows p1 + 1 and p2 + 1 are the changed inputs in both)
            d.p1 = (int16_t)(p1 / K - enc);
            d.p2 = (int16_t)(p2 / K - enc);
            d.ov = carry + incl - rows;
            d.s1 = (int16_t)p1;
            d.s2 = (int16_t)p2;
            desc[nb_off[s] + k] = d;
        }
        carry += __shfl(incl, 63, 64);
    }
}

// E_loc(s) = diag(s) + h_off * sum_k r_k, summed in bond order (FP64).
__global__ void k_eloc(const double* __restrict__ diag,
                       const int32_t* __restrict__ count,
                       const int32_t* __restrict__ nb_off,
                       const double* __restrict__ r, int n, int N,
                       double h_off, double* __restrict__ eloc,
                       double* __restrict__ ratios_out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int c = count[s];
    const double* rs = r + nb_off[s];
    double acc = 0.0;
    for (int k = 0; k < c; ++k) acc += rs[k];
    eloc[s] = diag[s] + h_off * acc;
    if (ratios_out) {
        double* o = ratios_out + (int64_t)s * 2 * N;
        for (int k = 0; k < c; ++k) o[k] = rs[k];
        for (int k = c; k < 2 * N; ++k) o[k] = 0.0;
    }
}

// Batch mean and biased variance, two passes, fixed-order tree (FP64).
__global__ void __launch_bounds__(256) k_stats(const double* __restrict__ e,
                                               int64_t n,
                                               double* __restrict__ stats) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int64_t k = t; k < n; k += 256) a += e[k];
    red[t] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    const double mean = red[0] / (double)n;
    __syncthreads();
    double v = 0.0;
    for (int64_t k = t; k < n; k += 256) {
        const double dd = e[k] - mean;
        v += dd * dd;
    }
    red[t] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) {
        stats[0] = mean;
        stats[1] = red[0] / (double)n;
    }
}

__global__ void k_fill_i64(int64_t* p, int n, int64_t v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}
__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Copies a device-side count into a counter slot (integer, exact).
__global__ void k_counter_add(int64_t* ctr, int slot, const int32_t* v,
                              int64_t scale) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        atomicAdd((unsigned long long*)(ctr + slot),
                  (unsigned long long)((int64_t)(*v) * scale));
}

__global__ void k_counter_add_const(int64_t* ctr, int slot, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        atomicAdd((unsigned long long*)(ctr + slot), (unsigned long long)v);
}

// codes of layer l: [n][N][H] -> dst [n][nl][N][H]
__global__ void k_copy_codes(const int32_t* __restrict__ src, int64_t n, int N,
                             int H, int nl, int l, int32_t* __restrict__ dst) {
    const int64_t total = n * N * H;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / ((int64_t)N * H);
        const int64_t rest = e - s * N * H;
        dst[(s * nl + l) * (int64_t)N * H + rest] = src[e];
    }
}

// Slice l of a per-layer output: src [n][row] -> dst [n][nl][row].
template <typename T>
__global__ void k_copy_layer(const T* __restrict__ src, int64_t n,
                             int64_t row, int nl, int l, T* __restrict__ dst) {
    const int64_t total = n * row;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / row;
        dst[(s * nl + l) * row + (e - s * row)] = src[e];
    }
}

template <typename T>
hipError_t launch_copy_layer(const T* src, int64_t n, int64_t row, int nl,
                             int l, T* dst, hipStream_t st) {
    int64_t blocks = (n * row + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy_layer<T>, dim3((unsigned)blocks), dim3(256), 0,
                       st, src, n, row, nl, l, dst);
    return hipGetLastError();
}
template hipError_t launch_copy_layer<float>(const float*, int64_t, int64_t,
                                             int, int, float*, hipStream_t);
template hipError_t launch_copy_layer<double>(const double*, int64_t, int64_t,
                                              int, int, double*, hipStream_t);

// ------------------------------------------------------------ launchers
hipError_t launch_counter_add_const(int64_t* ctr, int slot, int64_t v,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_counter_add_const, dim3(1), dim3(64), 0, st, ctr,
                       slot, v);
    return hipGetLastError();
}

hipError_t launch_copy_codes(const int32_t* src, int64_t n, int N, int H,
                             int nl, int l, int32_t* dst, hipStream_t st) {
    int64_t blocks = (n * N * H + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy_codes, dim3((unsigned)blocks), dim3(256), 0, st,
                       src, n, N, H, nl, l, dst);
    return hipGetLastError();
}

hipError_t launch_neighbours(const int8_t* spins, int64_t batch,
                             const ModelDims& m, int16_t* bonds, int32_t* count,
                             double* diag, int64_t* rows_cap, int32_t* status,
                             hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_neighbours, dim3((unsigned)batch), dim3(64), 0, st,
                       spins, batch, m.L, m.chain, m.periodic, m.K, m.enc, m.J, bonds,
                       count, diag, rows_cap, status);
    return hipGetLastError();
}

hipError_t launch_scan_desc(const int16_t* bonds, const int32_t* count,
                            const int64_t* rows_cap, int n, int L, int chain,
                            int K, int enc, int32_t* nb_off, int64_t* row_off,
                            int32_t* n_nb_total, int32_t* n_rows_total,
                            NbDesc* desc, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_chunk, dim3(1), dim3(1024), 0, st, count,
                       rows_cap, n, nb_off, row_off, n_nb_total, n_rows_total);
    hipLaunchKernelGGL(k_descriptors, dim3(n), dim3(64), 0, st, bonds, count,
                       nb_off, row_off, n, L, chain, K, enc, desc);
    return hipGetLastError();
}

hipError_t launch_eloc(const double* diag, const int32_t* count,
                       const int32_t* nb_off, const double* r, int n, int N,
                       double h_off, double* eloc, double* ratios_out,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_eloc, dim3((n + 127) / 128), dim3(128), 0, st, diag,
                       count, nb_off, r, n, N, h_off, eloc, ratios_out);
    return hipGetLastError();
}

hipError_t launch_stats(const double* e, int64_t n, double* stats,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, st, e, n, stats);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i64, dim3((n + 255) / 256), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}

hipError_t launch_counter_add(int64_t* ctr, int slot, const int32_t* v,
                              int64_t scale, hipStream_t st) {
    hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, st, ctr, slot, v,
                       scale);
    return hipGetLastError();
}

// Status word of a multi-lattice call: the OR of its jobs' status words
// (each at the start of the job's workspace slice).
__global__ void k_or_status(char* base, StatusOffsets so) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int32_t v = 0;
        for (int i = 0; i < so.n; ++i)
            v |= *reinterpret_cast<const int32_t*>(base + so.off[i]);
        *reinterpret_cast<int32_t*>(base) = v;
    }
}

hipError_t launch_or_status(char* base, const StatusOffsets& so,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, st, base, so);
    return hipGetLastError();
}

}  // namespace vq
