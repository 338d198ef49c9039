// Causal multi-head self-attention on the matrix core (gfx950, BF16 mode),
// paper Sec. 3.1/3.2: the location-mixing operation, evaluated densely for
// every query row at or after the first changed input.
//
// Scores are computed transposed, S^T = K Q^T, with 16x16x32 MFMAs: lane l
// then holds the scores of query l%16 for keys 4g..4g+3 of each 16-key tile
// (g = l/16), i.e. 8 keys of a 32-key block, taken in the order
// pi(8g+j) = 4g+j (j<4), 16+4g+j-4 (j>=4).  The output is formed as
// O^T = V^T P^T: those 8 probabilities are then exactly the lane's B-operand
// fragment, V^T is read from LDS in the same key order, and the result
// O^T[dh][q] leaves every lane with one query column, so the online-softmax
// state of a query never leaves its lane.  FP32 operands enter as hi+lo
// bfloat16 pairs: q.k = qh.kh + qh.kl + ql.kh (+ ql.kl when the head width is
// 16, where it comes free), the terms laid end to end along the MFMA K
// dimension, and V^T P^T = vh.ph + vl.ph + vh.pl, accumulated in FP32.
// Softmax is online over 32-key blocks in base-2 exponentials, log2(e) and
// 1/sqrt(d_head) folded into the query; p = 2^(s - m) with the hardware
// exponential (results below the normal range flush to zero, a relative
// loss under 2^-126 of the row's largest term).
//
// One workgroup owns one (sequence, head): the sequence's K, Q (hi|lo rows)
// and V (hi/lo, transposed) stay in LDS.  In the overlay form the workgroup
// then walks all neighbours of its sample, rewriting only the rows changed
// by the previous or the current neighbour.  Query tiles sit at absolute
// 16-row positions and key blocks at absolute 32-key positions, so a row's
// result does not depend on which form evaluated it.
#include "kernels.h"

namespace vq {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kAT = 256;
constexpr int kAGridCap = 8192;
constexpr float kLog2e = 1.4426950408889634f;

__device__ inline f32x4 mfma_a(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline bool mbit(const uint64_t* m, int i) {
    return (m[i >> 6] >> (i & 63)) & 1ull;
}

__device__ inline int npad32(int N) { return (N + 31) & ~31; }
__device__ inline int ldv_of(int N) { return npad32(N) + 8; }

// LDS tiles of one (sequence, head).
template <int DH>
struct Tiles {
    __bf16* Kc;   // [Np][2DH]  k hi | k lo
    __bf16* Qc;   // [Np][2DH]  q hi | q lo (q pre-scaled)
    __bf16* Vt;   // [2DH][ldv] v hi rows then v lo rows, transposed
    int ldv;
    // Stores columns c4..c4+3 of row j: k, q*qs and v as hi+lo bfloat16
    // pairs (a row past the sequence, !live, stores zeros).  The scaling and
    // the split are kept free of FMA contraction so that a row gets the same
    // bits whichever loop stores it (the compiler decides contraction per
    // inlined copy otherwise).
    __device__ void put4(int j, int c4, bool live, float4 k, float4 qraw,
                         float qs, float4 v) const {
#pragma clang fp contract(off)
        const float kk[4] = {k.x, k.y, k.z, k.w};
        const float qq[4] = {qraw.x * qs, qraw.y * qs, qraw.z * qs, qraw.w * qs};
        const float vv[4] = {v.x, v.y, v.z, v.w};
        bf16x4 kh, kl, qh, ql;
        __bf16 vh[4], vl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float a = live ? kk[i] : 0.0f;
            const float b = live ? qq[i] : 0.0f;
            const float c = live ? vv[i] : 0.0f;
            kh[i] = (__bf16)a;
            kl[i] = (__bf16)(a - (float)kh[i]);
            qh[i] = (__bf16)b;
            ql[i] = (__bf16)(b - (float)qh[i]);
            vh[i] = (__bf16)c;
            vl[i] = (__bf16)(c - (float)vh[i]);
        }
        *reinterpret_cast<bf16x4*>(Kc + j * 2 * DH + c4) = kh;
        *reinterpret_cast<bf16x4*>(Kc + j * 2 * DH + DH + c4) = kl;
        *reinterpret_cast<bf16x4*>(Qc + j * 2 * DH + c4) = qh;
        *reinterpret_cast<bf16x4*>(Qc + j * 2 * DH + DH + c4) = ql;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Vt[(c4 + i) * ldv + j] = vh[i];
            Vt[(DH + c4 + i) * ldv + j] = vl[i];
        }
    }
};

template <int DH>
__device__ inline Tiles<DH> carve_tiles(unsigned char* smem, int N) {
    Tiles<DH> t;
    const int Np = npad32(N);
    t.Kc = reinterpret_cast<__bf16*>(smem);
    t.Qc = t.Kc + Np * 2 * DH;
    t.Vt = t.Qc + Np * 2 * DH;
    t.ldv = ldv_of(N);
    return t;
}

// All rows of the sequence at row offset sb (row j at sb + j*d), padded with
// zero rows to a multiple of 32.  Four columns per 16-byte load; each
// thread issues all its loads before the first store (rows past the
// sequence load row N-1 and store zeros), so the tile costs one round trip
// to HBM, not one per element.
template <int DH>
__device__ inline void load_all(const Tiles<DH>& T, int N, const float* Q,
                                const float* K, const float* V, int64_t sb,
                                int d, float qs) {
    constexpr int G = DH / 4;                 // 4-column groups per row
    constexpr int UNR = 4;
    const int tot = npad32(N) * G;
    for (int e0 = 0; e0 < tot; e0 += kAT * UNR) {
        float4 k[UNR], q[UNR], v[UNR];
#pragma unroll
        for (int i = 0; i < UNR; ++i) {
            const int e = e0 + kAT * i + threadIdx.x;
            const int j = e / G, c4 = (e % G) * 4;
            const int jr = j < N ? j : N - 1;
            const int64_t o = sb + (int64_t)jr * d + c4;
            k[i] = *reinterpret_cast<const float4*>(K + o);
            q[i] = *reinterpret_cast<const float4*>(Q + o);
            v[i] = *reinterpret_cast<const float4*>(V + o);
        }
#pragma unroll
        for (int i = 0; i < UNR; ++i) {
            const int e = e0 + kAT * i + threadIdx.x;
            if (e < tot) T.put4(e / G, (e % G) * 4, e / G < N, k[i], q[i], qs, v[i]);
        }
    }
}

// Probabilities are formed against a per-query reference that is raised
// lazily: only when a block's scores exceed it by more than kTau (base 2), so
// every p stays below 2^kTau and most blocks need no rescaling at all.  The
// reference enters the score MFMA as its accumulator input (the MFMA returns
// s - m directly), and the normaliser sum(p) comes out of the matrix core
// from an all-ones operand, so a block costs no cross-lane traffic unless it
// raises a reference.  The rescaling decision is taken per query, from that
// query's own scores, so a row's result depends on its own inputs only.
constexpr float kTau = 8.0f;

typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

// Maximum of two scores, NaN-propagating: it maps to v_maximum3_f32 and
// needs no quieting of the matrix-core results it reads (the maximum only
// decides when and by how much a reference is raised).
__device__ inline float vmax(float a, float b) {
    return __builtin_elementwise_maximum(a, b);
}

// x of lane l ^ 16 and of lane l ^ 32, by the gfx950 lane-swap instructions
// (VALU, no LDS round trip).  Given the same register twice, permlane16_swap
// returns rows (0,0,2,2) and (1,1,3,3) of 16 lanes, permlane32_swap the
// halves (lo,lo) and (hi,hi).
__device__ inline float lane_xor16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x),
                                                    __float_as_uint(x), false, false);
    return __uint_as_float(((threadIdx.x >> 4) & 1) ? r[0] : r[1]);
}
__device__ inline float lane_xor32(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x),
                                                    __float_as_uint(x), false, false);
    return __uint_as_float((threadIdx.x & 32) ? r[0] : r[1]);
}

// p as hi+lo bfloat16: hi is p truncated to its upper 16 bits, lo the exact
// remainder rounded to bfloat16 (relative error of hi+lo at most 2^-16).
__device__ inline void split_p(const float* p, bf16x8& ph, bf16x8& pl) {
    uint32_t u[8];
    float r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        u[k] = __float_as_uint(p[k]);
        r[k] = p[k] - __uint_as_float(u[k] & 0xffff0000u);
    }
    u32x4 hv;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        hv[i] = __builtin_amdgcn_perm(u[2 * i + 1], u[2 * i], 0x07060302u);
    ph = __builtin_bit_cast(bf16x8, hv);
#pragma unroll
    for (int k = 0; k < 8; ++k) pl[k] = (__bf16)r[k];
}

// Online-softmax state of one 16-query tile (this lane: query iq).
template <int DH>
struct QTile {
    bf16x8 b0, b1, b2;                // query fragments
    f32x4 o[DH / 16];                 // output accumulators
    f32x4 osum;                       // normaliser (all-ones operand)
    f32x4 negm;                       // -reference, the score MFMA's input
    float mref;
    int t, iq, nblk;
};

// CA: causal (keys 0..query); otherwise every key of the sequence.
template <int DH, bool CA = true>
__device__ inline void qtile_init(QTile<DH>& q, const Tiles<DH>& T, int t, int N) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c16 = lane & 15;
    q.t = t;
    q.iq = t * 16 + c16;
    q.nblk = CA ? (t * 16 + 15) / 32 + 1 : npad32(N) / 32;
    const __bf16* qr = T.Qc + q.iq * 2 * DH;
    if (DH == 16) {
        // [kh(16) | kl(16)] x [qh ; qh]  and  [kh | kl] x [ql ; ql]
        q.b0 = *reinterpret_cast<const bf16x8*>(qr + 8 * (g & 1));
        q.b1 = *reinterpret_cast<const bf16x8*>(qr + DH + 8 * (g & 1));
        q.b2 = q.b1;
    } else {
        // [kh(32)] x [qh], [kl(32)] x [qh], [kh(32)] x [ql]
        q.b0 = *reinterpret_cast<const bf16x8*>(qr + 8 * g);
        q.b1 = q.b0;
        q.b2 = *reinterpret_cast<const bf16x8*>(qr + DH + 8 * g);
    }
#pragma unroll
    for (int u = 0; u < DH / 16; ++u) q.o[u] = f32x4{0, 0, 0, 0};
    q.osum = f32x4{0, 0, 0, 0};
    q.negm = f32x4{0, 0, 0, 0};
    q.mref = 0.0f;
}

// One 32-key block (keys j0..j0+31) for NQ query tiles in lock step, from
// the block's K fragments ka/kb (per 16-key sub-tile) and V fragments
// vh/vl.  EDGE: the block may hold keys after a tile's queries or past the
// sequence (they are masked), or be the first block (it sets the
// references).  Otherwise the block is straight-line code apart from one
// wave-uniform branch, taken only when some reference must be raised; the
// tiles' chains are independent, so the scheduler interleaves one tile's
// exponentials with another's matrix-core work.  Per query the operations
// and their order do not depend on NQ or on which tiles share the block.
template <int DH, int NQ, bool EDGE, bool CA = true>
__device__ inline void qtiles_block(QTile<DH> (&q)[NQ], int N, int blk,
                                    const bf16x8 (&ka)[2], const bf16x8 (&kb)[2],
                                    const bf16x8 (&vh)[DH / 16],
                                    const bf16x8 (&vl)[DH / 16],
                                    const bf16x8& ones) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int j0 = blk * 32;
    float s[NQ][8], lm[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            f32x4 acc;
            if (DH == 16) {
                acc = mfma_a(ka[sub], q[i].b0, q[i].negm);
                acc = mfma_a(ka[sub], q[i].b1, acc);
            } else {
                acc = mfma_a(ka[sub], q[i].b0, q[i].negm);
                acc = mfma_a(kb[sub], q[i].b1, acc);
                acc = mfma_a(ka[sub], q[i].b2, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) s[i][sub * 4 + r] = acc[r];
        }
    }
    if (EDGE) {
        // keys beyond the query (causal) or the sequence
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            if ((CA && j0 + 31 > q[i].t * 16) || j0 + 31 >= N) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int key = j0 + (k >> 2) * 16 + 4 * g + (k & 3);
                    if ((CA && key > q[i].iq) || key >= N) s[i][k] = -__builtin_inff();
                }
            }
        }
    }
    const bool first = EDGE && blk == 0;
    bool raise = first;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        lm[i] = s[i][0];
#pragma unroll
        for (int k = 1; k < 8; ++k) lm[i] = vmax(lm[i], s[i][k]);
        raise = raise || lm[i] > kTau;
    }
    if (__builtin_amdgcn_ballot_w64(raise) != 0) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            float dm = vmax(lm[i], lane_xor16(lm[i]));
            dm = vmax(dm, lane_xor32(dm));
            // the first block sets the reference to its maximum; later
            // blocks raise it only past kTau
            const float delta = first ? dm : (dm > kTau ? dm : 0.0f);
            if (delta != 0.0f) {
                if (!first) {
                    const float alpha = __builtin_amdgcn_exp2f(-delta);
#pragma unroll
                    for (int u = 0; u < DH / 16; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) q[i].o[u][r] *= alpha;
#pragma unroll
                    for (int r = 0; r < 4; ++r) q[i].osum[r] *= alpha;
                }
                q[i].mref += delta;
#pragma unroll
                for (int k = 0; k < 8; ++k) s[i][k] -= delta;
                q[i].negm = f32x4{-q[i].mref, -q[i].mref, -q[i].mref, -q[i].mref};
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        float p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = __builtin_amdgcn_exp2f(s[i][k]);
        bf16x8 ph, pl;
        split_p(p, ph, pl);
        q[i].osum = mfma_a(ones, ph, q[i].osum);
        q[i].osum = mfma_a(ones, pl, q[i].osum);
#pragma unroll
        for (int u = 0; u < DH / 16; ++u) {
            q[i].o[u] = mfma_a(vh[u], ph, q[i].o[u]);
            q[i].o[u] = mfma_a(vl[u], ph, q[i].o[u]);
            q[i].o[u] = mfma_a(vh[u], pl, q[i].o[u]);
        }
    }
}

// K and V fragments of the 32-key block blk.
template <int DH>
__device__ inline void block_frags(const Tiles<DH>& T, int blk, bf16x8 (&ka)[2],
                                   bf16x8 (&kb)[2], bf16x8 (&vh)[DH / 16],
                                   bf16x8 (&vl)[DH / 16]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c16 = lane & 15;
    const int j0 = blk * 32;
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
        const __bf16* kr = T.Kc + (j0 + sub * 16 + c16) * 2 * DH;
        ka[sub] = *reinterpret_cast<const bf16x8*>(kr + 8 * g);
        kb[sub] = DH == 16 ? ka[sub]
                           : *reinterpret_cast<const bf16x8*>(kr + DH + 8 * g);
    }
#pragma unroll
    for (int u = 0; u < DH / 16; ++u) {
        const int vc = u * 16 + c16;
        const __bf16* vh_row = T.Vt + vc * T.ldv + j0 + 4 * g;
        const __bf16* vl_row = T.Vt + (DH + vc) * T.ldv + j0 + 4 * g;
        const bf16x4 h0 = *reinterpret_cast<const bf16x4*>(vh_row);
        const bf16x4 h1 = *reinterpret_cast<const bf16x4*>(vh_row + 16);
        const bf16x4 l0 = *reinterpret_cast<const bf16x4*>(vl_row);
        const bf16x4 l1 = *reinterpret_cast<const bf16x4*>(vl_row + 16);
        vh[u] = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
        vl[u] = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
    }
}

// Blocks [b0, b1) for NQ tiles, all of which have at least b1 blocks; the
// smallest tile is tq_min.  Blocks 1..last need no mask for any tile
// (32 blk + 31 <= 16 tq_min and 32 blk + 31 < N): they run the straight-line
// form, the others the edge form.
template <int DH, int NQ, bool CA = true>
__device__ inline void run_blocks(const Tiles<DH>& T, QTile<DH> (&q)[NQ], int N,
                                  int tq_min, int b0, int b1,
                                  const bf16x8& ones) {
    constexpr int NT = DH / 16;
    const int jl = CA ? min(16 * tq_min - 31, N - 32) : N - 32;
    const int last = jl >= 0 ? jl / 32 : 0;
    const int i0 = max(b0, 1), i1 = min(b1, last + 1);
    auto edge = [&](int blk) {
        bf16x8 ka[2], kb[2], vh[NT], vl[NT];
        block_frags<DH>(T, blk, ka, kb, vh, vl);
        qtiles_block<DH, NQ, true, CA>(q, N, blk, ka, kb, vh, vl, ones);
    };
    if (b0 == 0 && b1 > 0) edge(0);
    for (int blk = i0; blk < i1; ++blk) {
        bf16x8 ka[2], kb[2], vh[NT], vl[NT];
        block_frags<DH>(T, blk, ka, kb, vh, vl);
        qtiles_block<DH, NQ, false, CA>(q, N, blk, ka, kb, vh, vl, ones);
    }
    for (int blk = max(i0, i1); blk < b1; ++blk) edge(blk);
}

// Query tiles tq[0] >= tq[1] (NQ = 2) or tq[0] of one wave against the keys
// held in LDS.  The tiles advance in lock step, sharing every K and V
// fragment read, over the blocks they both have; the larger tile then runs
// its remaining blocks alone.  Writes rows i >= lo (and < N) through
// orow(i).
template <int DH, int NQ, bool CA = true, class OF>
__device__ inline void attn_tiles(const Tiles<DH>& T, int N, const int (&tq)[NQ],
                                  int lo, OF orow) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    constexpr int NT = DH / 16;
    QTile<DH> q[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) qtile_init<DH, CA>(q[i], T, tq[i], N);
    bf16x8 ones;
#pragma unroll
    for (int k = 0; k < 8; ++k) ones[k] = (__bf16)1.0f;
    QTile<DH>(&q0)[1] = *reinterpret_cast<QTile<DH>(*)[1]>(&q[0]);
    if (NQ == 2) {
        run_blocks<DH, NQ, CA>(T, q, N, tq[NQ - 1], 0, q[NQ - 1].nblk, ones);
        run_blocks<DH, 1, CA>(T, q0, N, tq[0], q[NQ - 1].nblk, q[0].nblk, ones);
    } else {
        run_blocks<DH, 1, CA>(T, q0, N, tq[0], 0, q[0].nblk, ones);
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        if (q[i].iq >= lo && q[i].iq < N) {
            float* dst = orow(q[i].iq);
            const float inv = 1.0f / q[i].osum[0];
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                float4 v;
                v.x = q[i].o[u][0] * inv;
                v.y = q[i].o[u][1] * inv;
                v.z = q[i].o[u][2] * inv;
                v.w = q[i].o[u][3] * inv;
                *reinterpret_cast<float4*>(dst + u * 16 + 4 * g) = v;
            }
        }
    }
}

// Active tiles (tmin..NTQ-1) from which adjacent tiles are paired.
constexpr int kPairTiles = 12;

// The query tiles of wave w (of 4), tiles below tmin not computed.  With at
// least kPairTiles active tiles, tiles are paired as (2k+1, 2k), which have
// the same k+1 key blocks, and the pairs, from the largest k down, are dealt
// to the waves in snake order (0 1 2 3 3 2 1 0 ...), which evens out the
// blocks per wave.  With fewer, wave w takes tiles NTQ-1-w, NTQ-5-w, ...,
// two at a time, so that every wave has work.
template <int DH, bool CA = true, class OF>
__device__ inline void wave_tiles(const Tiles<DH>& T, int N, int NTQ, int w,
                                  int tmin, int lo, OF orow) {
    if (NTQ - tmin >= kPairTiles) {
        const int K = (NTQ + 1) / 2;          // pairs
        const int kmin = tmin / 2;
        for (int i = 0; i < K - kmin; ++i) {
            const int r = i & 7;
            if ((r < 4 ? r : 7 - r) != w) continue;
            const int k = K - 1 - i;
            const int hi = 2 * k + 1, lo2 = 2 * k;
            if (hi < NTQ && lo2 >= tmin) {
                const int tq[2] = {hi, lo2};
                attn_tiles<DH, 2, CA>(T, N, tq, lo, orow);
            } else {
                const int tq[1] = {hi < NTQ ? hi : lo2};
                attn_tiles<DH, 1, CA>(T, N, tq, lo, orow);
            }
        }
        return;
    }
    int t = NTQ - 1 - w;
    for (; t - 4 >= tmin; t -= 8) {
        const int tq[2] = {t, t - 4};
        attn_tiles<DH, 2, CA>(T, N, tq, lo, orow);
    }
    if (t >= tmin) {
        const int tq[1] = {t};
        attn_tiles<DH, 1, CA>(T, N, tq, lo, orow);
    }
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD b % 8),
// and every XCD has its own L2.  A (sample, head) unit reads 64-byte pieces
// of rows whose 128-byte lines it shares with the other heads of the same
// sample, so unit indices are permuted to send the heads of one sample to
// consecutive workgroups of one XCD (the grid is a multiple of 8 whenever it
// strides).  Within each full block of 8 nh indices, index 8k + x maps to
// sample 8 blk + x, head k; a last partial block maps to itself, so the map
// is a bijection on [0, units).
__device__ inline int64_t xcd_unit(int64_t v, int64_t units, int nh) {
    const int64_t B = 8 * (int64_t)nh;
    const int64_t blk = v / B;
    if ((blk + 1) * B > units) return v;
    const int r = (int)(v - blk * B);
    return blk * B + (int64_t)(r & 7) * nh + (r >> 3);
}

// WPE: waves per SIMD the register allocation must allow (1: no cap).  Where
// the LDS tiles leave room for three workgroups per CU (head width 16 up to
// 16x16 lattices), the capped instance runs a third wave per SIMD, which
// hides much of the latency of the per-block chain (score MFMAs, maximum,
// exponentials, output MFMAs); the cap costs a few spills of loop-invariant
// values.  Elsewhere the uncapped instance runs.

// Full sequences (the samples themselves, or materialised neighbours).
template <int DH, int WPE, bool CA = true>
__global__ void __launch_bounds__(kAT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_attn_seq_mfma(ModelDims m,
                                                      const int32_t* n_dev,
                                                      int64_t n_seq,
                                                      BlockIO<PrecBF16> io,
                                                      int64_t* ctr) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int N = m.N, d = m.d;
    const Tiles<DH> T = carve_tiles<DH>(smem_raw, N);
    const float qs = kLog2e / sqrtf((float)DH);
    const int64_t n = n_dev ? (int64_t)*n_dev : n_seq;
    const int64_t units = n * m.nh;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NTQ = (N + 15) / 16;
    for (int64_t v = blockIdx.x; v < units; v += gridDim.x) {
        const int64_t u = xcd_unit(v, units, m.nh);
        const int64_t s = u / m.nh;
        const int h = (int)(u - s * m.nh);
        const int64_t sb = s * N * d + h * DH;
        __syncthreads();
        load_all<DH>(T, N, io.q, io.k, io.v, sb, d, qs);
        __syncthreads();
        wave_tiles<DH, CA>(T, N, NTQ, wave, 0, 0,
                           [&](int i) { return io.a + sb + (int64_t)i * d; });
    }
    if (ctr && blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_ROWS),
                  (unsigned long long)(n * N));
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_PAIRS),
                  (unsigned long long)(n * (CA ? (int64_t)N * (N + 1) / 2
                                                  : (int64_t)N * N) * m.nh));
    }
}

// Overlay form: one workgroup per (sample, head) walks the sample's
// neighbours.  Between two neighbours only rows in either changed set are
// rewritten: the previous neighbour's rows go back to the sample's values
// (unless the next one changes them too) and the next neighbour's rows take
// its overlay values.  The next neighbour's row mask is fetched during the
// current neighbour's compute and kept in LDS (two buffers by parity, so a
// neighbour costs two barriers); a step then waits for one batch of 16-byte
// value loads.
template <int DH, int WPE, bool CA = true>
__global__ void __launch_bounds__(kAT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_attn_dedup_mfma(ModelDims m,
                                                        DedupIO<PrecBF16> dd,
                                                        int64_t* ctr) {
    constexpr int G = DH / 4, UNR = 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ uint64_t msk[2][VQ_MAX_MASK_WORDS];   // by neighbour parity
    const int N = m.N, d = m.d, W = dd.mask_words;
    const Tiles<DH> T = carve_tiles<DH>(smem_raw, N);
    const float qs = kLog2e / sqrtf((float)DH);
    const int64_t units = dd.n_samples * m.nh;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NTQ = (N + 15) / 16;
    int64_t my_rows = 0, my_pairs = 0;
    for (int64_t v = blockIdx.x; v < units; v += gridDim.x) {
        const int64_t u = xcd_unit(v, units, m.nh);
        const int64_t sg = u / m.nh;
        const int h = (int)(u - sg * m.nh);
        const int64_t sb = sg * N * d + h * DH;
        const int k0 = dd.nb_off[sg], k1 = dd.nb_off[sg + 1];
        __syncthreads();
        load_all<DH>(T, N, dd.bq, dd.bk, dd.bv, sb, d, qs);
        // The next neighbour's mask words, descriptor, changed-row count and
        // first batch of row indices are loaded during the current one's
        // compute, so a step starts with only its value loads outstanding.
        uint64_t mnext = 0;
        NbDesc Dn{};
        int ccn = 0;
        int jjn[UNR];
        // row indices of the first batch of the step into the neighbour with
        // descriptor Dx and count ccx, after cpx rows of the one at povx
        auto first_rows = [&](int cpx, int64_t povx, const NbDesc& Dx, int ccx) {
            const int npx = cpx * G, totx = (cpx + ccx) * G;
            if (totx == 0) return;
#pragma unroll
            for (int i = 0; i < UNR; ++i) {
                const int e = kAT * i + threadIdx.x;
                const int ec = e < totx ? e : totx - 1;
                const int64_t ix = ec < npx ? povx + ec / G : Dx.ov + (ec - npx) / G;
                jjn[i] = dd.crow[ix];
            }
        };
        if (k0 < k1) {
            if (threadIdx.x < W) mnext = dd.mask[(int64_t)k0 * W + threadIdx.x];
            Dn = dd.desc[k0];
            ccn = dd.ccnt[k0];
            first_rows(0, 0, Dn, ccn);
        }
        int cp = 0;
        int64_t pov = 0;
        if (k0 < k1 && threadIdx.x < W) msk[0][threadIdx.x] = mnext;
        for (int k = k0; k < k1; ++k) {
            // LDS free (load_all or last compute done) and this neighbour's
            // mask words in msk[par], written after the previous compute
            const int par = (k - k0) & 1;
            __syncthreads();
            const uint64_t* mk = msk[par];
            // step (k-1 -> k): restore rows of C_{k-1} not in C_k, patch C_k
            const NbDesc D = Dn;
            const int pmin = CA ? D.p1 + 1 : 0;     // the encoder: every row
            const int cc = ccn;
            const int64_t ob0 = (D.ov - pmin) * (int64_t)d + h * DH;
            const int np = cp * G, tot = (cp + cc) * G;
            for (int e0 = 0; e0 < tot; e0 += kAT * UNR) {
                // a wave skips the elements none of its lanes has
                bool act[UNR];
#pragma unroll
                for (int i = 0; i < UNR; ++i) act[i] = e0 + kAT * i + 64 * wave < tot;
                int jj[UNR];
#pragma unroll
                for (int i = 0; i < UNR; ++i) {
                    if (!act[i]) continue;
                    if (e0 == 0) {
                        jj[i] = jjn[i];
                        continue;
                    }
                    const int e = e0 + kAT * i + threadIdx.x;
                    const int ec = e < tot ? e : tot - 1;
                    const int64_t ix = ec < np ? pov + ec / G : D.ov + (ec - np) / G;
                    jj[i] = dd.crow[ix];
                }
                float4 kv[UNR], qv[UNR], vv[UNR];
                bool use[UNR];
#pragma unroll
                for (int i = 0; i < UNR; ++i) {
                    if (!act[i]) continue;
                    const int e = e0 + kAT * i + threadIdx.x;
                    const int ec = e < tot ? e : tot - 1;
                    const bool restore = ec < np;
                    const int c4 = ((restore ? ec : ec - np) % G) * 4;
                    const int j = jj[i];
                    use[i] = e < tot && !(restore && mbit(mk, j));
                    const int64_t o = (restore ? sb : ob0) + (int64_t)j * d + c4;
                    const float* K = restore ? dd.bk : dd.ok;
                    const float* Q = restore ? dd.bq : dd.oq;
                    const float* V = restore ? dd.bv : dd.ov;
                    kv[i] = *reinterpret_cast<const float4*>(K + o);
                    qv[i] = *reinterpret_cast<const float4*>(Q + o);
                    vv[i] = *reinterpret_cast<const float4*>(V + o);
                }
#pragma unroll
                for (int i = 0; i < UNR; ++i) {
                    if (!act[i]) continue;
                    const int e = e0 + kAT * i + threadIdx.x;
                    const int ec = e < tot ? e : tot - 1;
                    const int c4 = ((ec < np ? ec : ec - np) % G) * 4;
                    if (use[i]) T.put4(jj[i], c4, true, kv[i], qv[i], qs, vv[i]);
                }
            }
            if (k + 1 < k1) {
                if (threadIdx.x < W) mnext = dd.mask[(int64_t)(k + 1) * W + threadIdx.x];
                Dn = dd.desc[k + 1];
                ccn = dd.ccnt[k + 1];
                first_rows(cc, D.ov, Dn, ccn);
            }
            cp = cc;
            pov = D.ov;
            __syncthreads();
            wave_tiles<DH, CA>(T, N, NTQ, wave, pmin / 16, pmin,
                           [&](int i) { return dd.oa + ob0 + (int64_t)i * d; });
            // the next neighbour's mask into the other buffer (last read by
            // the previous step, which every wave finished before this
            // neighbour's compute)
            if (k + 1 < k1 && threadIdx.x < W) msk[par ^ 1][threadIdx.x] = mnext;
            if (h == 0 && threadIdx.x == 0) {
                my_rows += N - pmin;
                my_pairs += CA ? ((int64_t)N * (N + 1) - (int64_t)pmin * (pmin + 1)) / 2
                               : (int64_t)N * N;
            }
        }
    }
    if (ctr && threadIdx.x == 0 && my_rows) {
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_ROWS),
                  (unsigned long long)my_rows);
        atomicAdd((unsigned long long*)(ctr + VQNQS_CTR_ATTN_PAIRS),
                  (unsigned long long)(my_pairs * m.nh));
    }
}

static size_t attn_lds(const ModelDims& m) {
    const int Np = (m.N + 31) & ~31;
    return sizeof(__bf16) *
           ((size_t)2 * Np * 2 * m.dh + (size_t)2 * m.dh * (Np + 8));
}

// The matrix-core kernels hold K, Q and V of a whole sequence in LDS; longer
// sequences use the vector-unit attention (K and V only).
bool attn_mfma_ok(const ModelDims& m) {
    return (m.dh == 16 || m.dh == 32) && attn_lds(m) <= 160 * 1024;
}

static unsigned agrid(int64_t units) {
    if (units <= 0) return 1;
    return (unsigned)(units < kAGridCap ? units : kAGridCap);
}

template <typename F>
static void big_lds(F f, size_t sm) {
    if (sm > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)f,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sm);
}

// Workgroups per CU that the LDS of one (sequence, head) allows.
static int attn_wg_per_cu(const ModelDims& m) {
    return (int)((160 * 1024) /
                 (attn_lds(m) + sizeof(uint64_t) * 2 * VQ_MAX_MASK_WORDS));
}

hipError_t launch_attn_seq_mfma(const ModelDims& m, const int32_t* n_dev,
                                int64_t n_seq, const BlockIO<PrecBF16>& io,
                                int64_t* ctr, hipStream_t st) {
    const size_t sm = attn_lds(m);
    const unsigned g = agrid(n_seq * m.nh);
    auto go = [&](auto kern) {
        big_lds(kern, sm);
        hipLaunchKernelGGL(kern, dim3(g), dim3(kAT), sm, st, m, n_dev, n_seq,
                           io, ctr);
    };
    if (m.enc) {                        // bidirectional encoder
        if (m.dh == 16 && attn_wg_per_cu(m) >= 3)
            go(k_attn_seq_mfma<16, 3, false>);
        else if (m.dh == 16)
            go(k_attn_seq_mfma<16, 1, false>);
        else if (m.dh == 32)
            go(k_attn_seq_mfma<32, 1, false>);
        else
            return hipErrorInvalidValue;
    } else if (m.dh == 16 && attn_wg_per_cu(m) >= 3)
        go(k_attn_seq_mfma<16, 3>);
    else if (m.dh == 16)
        go(k_attn_seq_mfma<16, 1>);
    else if (m.dh == 32)
        go(k_attn_seq_mfma<32, 1>);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_attn_dedup_mfma(const ModelDims& m,
                                  const DedupIO<PrecBF16>& d, int64_t* ctr,
                                  hipStream_t st) {
    const size_t sm = attn_lds(m);
    const unsigned g = agrid(d.n_samples * m.nh);
    auto go = [&](auto kern) {
        big_lds(kern, sm);
        hipLaunchKernelGGL(kern, dim3(g), dim3(kAT), sm, st, m, d, ctr);
    };
    if (m.enc) {                        // bidirectional encoder
        if (m.dh == 16 && attn_wg_per_cu(m) >= 3)
            go(k_attn_dedup_mfma<16, 3, false>);
        else if (m.dh == 16)
            go(k_attn_dedup_mfma<16, 1, false>);
        else if (m.dh == 32)
            go(k_attn_dedup_mfma<32, 1, false>);
        else
            return hipErrorInvalidValue;
    } else if (m.dh == 16 && attn_wg_per_cu(m) >= 3)
        go(k_attn_dedup_mfma<16, 3>);
    else if (m.dh == 16)
        go(k_attn_dedup_mfma<16, 1>);
    else if (m.dh == 32)
        go(k_attn_dedup_mfma<32, 1>);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace vq
