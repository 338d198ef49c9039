// Host orchestration: workspace planning and kernel sequencing for the
// forward pass, the plain and the deduplicated local energy.
#include "engine.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "profiler.h"

namespace vq {

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t param_count(const ModelDims& m);

// Token embedding rows: 2^K values plus the decoder's beginning-of-sequence
// token; head outputs: 2^K log-probabilities, or the encoder's one term.
static int64_t tok_rows(const ModelDims& m) {
    return ((int64_t)1 << m.K) + (m.enc ? 0 : 1);
}
static int64_t head_outputs(const ModelDims& m) {
    return m.enc ? 1 : (int64_t)1 << m.K;
}

// Worst case, over all configurations, of the overlay rows one sample needs:
// every bond anti-aligned, each neighbour keeping token rows p1+1 .. N-1
// (p1 the token of its first site).
static int64_t max_overlay_rows(const ModelDims& m) {
    int64_t tot = 0;
    const int L = m.L, N = m.N, S = m.S, K = m.K;
    // every encoder row attends to the change: N rows per neighbour
    if (m.enc) return (int64_t)(m.chain ? S : 2 * S) * N;
    // a chain's flip of site i keeps rows i/K+1 .. N-1
    if (m.chain) {
        for (int i = 0; i < S; ++i) tot += N - i / K - 1;
        return tot;
    }
    for (int b = 0; b < 2 * S; ++b) {
        const int i = b >> 1, r = i / L, c = i % L;
        int j;
        if ((b & 1) == 0) {
            if (!m.periodic && c + 1 == L) continue;
            j = r * L + (c + 1) % L;
        } else {
            if (!m.periodic && r + 1 == L) continue;
            j = ((r + 1) % L) * L + c;
        }
        tot += N - std::min(i, j) / K - 1;
    }
    return tot;
}

struct Carver {
    size_t off = 0;
    char* base = nullptr;
    template <typename T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = al256(off + sizeof(T) * (count ? count : 1));
        return p;
    }
};

// All workspace pointers of one call.  With base == nullptr only the size
// is computed.
template <class P>
struct Workspace {
    using acc = typename P::acc;
    using act = typename P::act;
    int32_t* status;
    // parameter preparation, per layer
    acc* table;   // [nl][H*Q*d]
    acc* cnorm;   // [nl][H*Q + H]
    float* prm;   // BF16 mode: parameters rounded to bfloat16
    bf16 *wqkv_p, *w1_p, *w2_p, *cb_p;   // [nl] matrix-core fragment packs
    bf16 *wqkv_tp, *wo_tp;               // the half-block's QKV and W_o packs
    float* cnh;                          // [nl][H*Q] -cnorm/2
    // chunk neighbour bookkeeping
    int16_t* bonds;
    int32_t *count, *nb_off, *n_nb, *n_rows, *list_n, *vq_n;
    double* diag;
    int64_t *rows_cap, *row_off;
    NbDesc* desc;
    double *ratio, *logpsi_s, *logpsi_nb;
    // sample (base) buffers
    acc* bx;      // [nlx][n][N][d]
    act *bq, *bk, *bv, *ba;   // [nlc][n][N][d]
    int32_t* bcode;           // [nlc][n][N][H]
    acc* bmargin;             // [nlc][n][N][H][2]
    acc* blp;                 // [n][N][2]
    acc* bstat;               // [nl][n][N][heads][2] softmax statistics
    // materialised neighbours (plain)
    int8_t* nspins;
    acc* nx;
    act *nq, *nk, *nv, *na;
    int32_t* ncode;
    // overlay (dedup)
    acc* ox;
    act *oq, *ok, *ov, *oa;
    int32_t *ocode, *slot_nb, *ccnt;
    int16_t* crow;
    uint64_t* mask;
    int64_t *list, *vq_list;
    // gradient of log psi: layer inputs (checkpoints), one layer's
    // recomputed activations and the backward's row buffers
    acc* gx;                  // [nl+1][n][N][d]
    act *gq, *gk, *gv, *ga;   // [n][N][d]
    int32_t* gcode;           // [n][N][H]
    double* glogpsi;          // [n]
    acc *h1, *xh1, *rs1, *xp, *zq, *h2, *xh2, *rs2;
    acc *gu, *gg, *dF;        // [n][N][d_ff]
    acc *dX, *dXp, *dT, *da;  // [n][N][d]
    acc* dqkv;                // [n][N][3d]
    acc *lse, *Dd;            // [n][N][heads]
    acc *S, *E;               // [n][N][Q]
    acc *rowG, *colG, *dz2, *coef;
    acc* part;                // [n][P] per-sample gradients (weighted form)
    size_t bytes;
};

enum class Job { Forward, Plain, Dedup, Neighbours, Grad, Sample };

template <class P>
static Workspace<P> carve(const ModelDims& m, Job job, int64_t chunk,
                          void* base) {
    using acc = typename P::acc;
    using act = typename P::act;
    Workspace<P> w{};
    Carver c;
    c.base = static_cast<char*>(base);
    // rows: N token positions per sample; spins and neighbour slots: S sites
    const int64_t n = chunk, N = m.N, S = m.S, d = m.d, H = m.H;
    const int64_t V = (int64_t)1 << m.K;
    const int64_t nbmax = n * 2 * S;
    w.status = c.take<int32_t>(64);
    if (job != Job::Neighbours) {
        w.table = c.take<acc>((size_t)m.nl * H * m.Q * d);
        w.cnorm = c.take<acc>((size_t)m.nl * (H * m.Q + H));
        if (m.precision == VQNQS_BF16) w.prm = c.take<float>(param_count(m));
        if (m.mfma) {
            w.wqkv_p = c.take<bf16>((size_t)m.nl * d * 3 * d);
            w.w1_p = c.take<bf16>((size_t)m.nl * d * m.dff);
            w.w2_p = c.take<bf16>((size_t)m.nl * m.dff * d);
            w.cb_p = c.take<bf16>((size_t)m.nl * m.Q * d);
            w.cnh = c.take<float>((size_t)m.nl * H * m.Q);
            if (m.tail) {
                w.wqkv_tp = c.take<bf16>((size_t)d * 3 * d);
                w.wo_tp = c.take<bf16>((size_t)d * d);
            }
        }
    }
    w.bonds = c.take<int16_t>(n * 2 * S);
    w.count = c.take<int32_t>(n);
    w.diag = c.take<double>(n);
    w.rows_cap = c.take<int64_t>(n);
    w.nb_off = c.take<int32_t>(n + 1);
    w.row_off = c.take<int64_t>(n + 1);
    w.n_nb = c.take<int32_t>(1);
    w.n_rows = c.take<int32_t>(1);
    w.list_n = c.take<int32_t>(1);
    w.vq_n = c.take<int32_t>(1);
    if (job == Job::Neighbours) {
        w.bytes = c.off;
        return w;
    }
    if (job == Job::Sample) {
        // one position of every sample at a time: the residual rows, query
        // and attention rows, the keys and values of every layer (the
        // positions drawn so far), codes, the row list and FP64 sums
        const int64_t R = n * N;
        w.bx = c.take<acc>(R * d);
        w.bq = c.take<act>(R * d);
        w.ba = c.take<act>(R * d);
        w.bk = c.take<act>((size_t)(m.nl + m.tail) * R * d);
        w.bv = c.take<act>((size_t)(m.nl + m.tail) * R * d);
        w.bcode = c.take<int32_t>(R * H);
        w.list = c.take<int64_t>(n);
        w.logpsi_s = c.take<double>(n);
        w.bytes = c.off;
        return w;
    }
    if (job == Job::Grad) {
        const int64_t R = n * N, F = m.dff, Q = m.Q;
        w.gx = c.take<acc>((size_t)(m.nl + 1 + m.tail) * R * d);
        w.gq = c.take<act>(R * d);
        w.gk = c.take<act>(R * d);
        w.gv = c.take<act>(R * d);
        w.ga = c.take<act>(R * d);
        w.gcode = c.take<int32_t>(R * H);
        w.glogpsi = c.take<double>(n);
        w.h1 = c.take<acc>(R * d);
        w.xh1 = c.take<acc>(R * d);
        w.rs1 = c.take<acc>(R);
        w.xp = c.take<acc>(R * d);
        w.zq = c.take<acc>(R * d);
        w.h2 = c.take<acc>(R * d);
        w.xh2 = c.take<acc>(R * d);
        w.rs2 = c.take<acc>(R);
        w.gu = c.take<acc>(R * F);
        w.gg = c.take<acc>(R * F);
        w.dF = c.take<acc>(R * F);
        w.dX = c.take<acc>(R * d);
        w.dXp = c.take<acc>(R * d);
        w.dT = c.take<acc>(R * d);
        w.da = c.take<acc>(R * d);
        w.dqkv = c.take<acc>(R * 3 * d);
        w.lse = c.take<acc>(R * m.nh);
        w.Dd = c.take<acc>(R * m.nh);
        w.S = c.take<acc>(R * Q);
        w.E = c.take<acc>(R * Q);
        w.rowG = c.take<acc>(R);
        w.colG = c.take<acc>(n * Q);
        w.dz2 = c.take<acc>(V * R);
        w.coef = c.take<acc>(n);
        w.part = c.take<acc>((size_t)n * param_count(m));
        w.bytes = c.off;
        return w;
    }
    w.desc = c.take<NbDesc>(nbmax);
    w.ratio = c.take<double>(nbmax);
    w.logpsi_s = c.take<double>(n);
    const bool dedup = job == Job::Dedup;
    // cached layers (and the half-block), block inputs + final output
    const int64_t nlc = dedup ? m.nl + m.tail : 1;
    const int64_t nlx = dedup ? m.nl + 1 + m.tail : 1;
    w.bx = c.take<acc>(nlx * n * N * d);
    w.bq = c.take<act>(nlc * n * N * d);
    w.bk = c.take<act>(nlc * n * N * d);
    w.bv = c.take<act>(nlc * n * N * d);
    w.ba = c.take<act>(nlc * n * N * d);
    w.bcode = c.take<int32_t>(nlc * n * N * H);
    if (dedup) {
        w.bmargin = c.take<acc>(nlc * n * N * H * 2);
        w.blp = c.take<acc>(n * N * V);
        if (m.flags & VQNQS_FLAG_INCREMENTAL_ATTN)
            w.bstat = c.take<acc>(nlc * n * N * m.nh * 2);
    }
    if (job == Job::Plain) {
        w.logpsi_nb = c.take<double>(nbmax);
        w.nspins = c.take<int8_t>(nbmax * S);
        w.nx = c.take<acc>(nbmax * N * d);
        w.nq = c.take<act>(nbmax * N * d);
        w.nk = c.take<act>(nbmax * N * d);
        w.nv = c.take<act>(nbmax * N * d);
        w.na = c.take<act>(nbmax * N * d);
        w.ncode = c.take<int32_t>(nbmax * N * H);
    }
    if (dedup) {
        const int64_t R = n * max_overlay_rows(m);
        const int W = (m.N + 63) / 64;
        w.ox = c.take<acc>(R * d);
        w.oq = c.take<act>(R * d);
        w.ok = c.take<act>(R * d);
        w.ov = c.take<act>(R * d);
        w.oa = c.take<act>(R * d);
        w.ocode = c.take<int32_t>(R * H);
        w.slot_nb = c.take<int32_t>(R);
        w.crow = c.take<int16_t>(R);
        w.ccnt = c.take<int32_t>(nbmax);
        w.list = c.take<int64_t>(R);
        w.vq_list = c.take<int64_t>(R);
        w.mask = c.take<uint64_t>(nbmax * W);
    }
    w.bytes = c.off;
    return w;
}

// Variational Monte Carlo step: the per-step buffers (samples, local
// energies, statistics, gradient weights, gradient) after the region the
// sampling, local-energy and gradient calls share in turn.
static size_t vmc_front_bytes(const ModelDims& m, int64_t B) {
    const size_t a = m.precision == VQNQS_F64 ? 8 : 4;
    return al256((size_t)B * m.S) + 3 * al256((size_t)B * 8) + 256 +
           al256((size_t)param_count(m) * a);
}

static size_t vmc_sub_bytes(const ModelDims& m, int64_t chunk) {
    return std::max(workspace_bytes(m, -4, chunk),
                    std::max(workspace_bytes(m, VQNQS_DEDUP, chunk),
                             workspace_bytes(m, -3, chunk)));
}

size_t vmc_workspace_bytes(const ModelDims& m, int64_t batch, int64_t chunk) {
    return al256(vmc_sub_bytes(m, chunk)) + vmc_front_bytes(m, batch);
}

size_t workspace_bytes(const ModelDims& m, int mode, int64_t chunk) {
    const Job job = mode == VQNQS_PLAIN   ? Job::Plain
                    : mode == VQNQS_DEDUP ? Job::Dedup
                    : mode == -2          ? Job::Neighbours
                    : mode == -3          ? Job::Grad
                    : mode == -4          ? Job::Sample
                                          : Job::Forward;
    switch (m.precision) {
        case VQNQS_F64: return carve<PrecF64>(m, job, chunk, nullptr).bytes;
        case VQNQS_F32: return carve<PrecF32>(m, job, chunk, nullptr).bytes;
        default: return carve<PrecBF16>(m, job, chunk, nullptr).bytes;
    }
}

int64_t max_overlay_rows_per_sample(const ModelDims& m) {
    return max_overlay_rows(m);
}

int64_t pick_chunk(const ModelDims& m, int mode, int64_t batch, size_t ws) {
    if (batch <= 0) return 0;
    const size_t one = workspace_bytes(m, mode, 1);
    if (one > ws) return 0;
    // the size is affine in the chunk up to 256-byte rounding: bisect
    int64_t lo = 1, hi = batch;
    // bound the chunk so overlay row counts and neighbour ids stay in int32
    const int64_t rows1 = std::max<int64_t>(1, max_overlay_rows(m));
    hi = std::min<int64_t>(hi, ((int64_t)1 << 30) / rows1);
    hi = std::min<int64_t>(hi, ((int64_t)1 << 30) / (2 * m.S));
    // gradient products tile rows by 64 with at most 65535 row tiles
    if (mode == -3) hi = std::min<int64_t>(hi, (int64_t)65535 * 64 / m.N);
    if (hi < 1) hi = 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes(m, mode, mid) <= ws) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------------- params
template <typename C>
static LayerW<C> layer_view(const ModelDims& m, const C* p, int l) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    const C* b = p + tok_rows(m) * d + N * d + per * l;
    LayerW<C> w{};
    w.ln1_g = b;
    w.ln1_b = b + d;
    w.W_qkv = b + 2 * d;
    w.b_qkv = w.W_qkv + d * 3 * d;
    w.codebook = w.b_qkv + 3 * d;
    w.W_o = w.codebook + Q * d;
    w.b_o = w.W_o + d * d;
    w.ln2_g = w.b_o + d;
    w.ln2_b = w.ln2_g + d;
    w.W1 = w.ln2_b + d;
    w.b1 = w.W1 + d * F;
    w.W2 = w.b1 + F;
    w.b2 = w.W2 + F * d;
    return w;
}

// Parameters of the attention-only half-block after the blocks (tail of
// the flat layout, before the final LayerNorm).
static int64_t tail_params(const ModelDims& m) {
    const int64_t d = m.d;
    return m.tail ? 2 * d + 3 * d * d + 3 * d + d * d + d : 0;
}

template <typename C>
static LayerW<C> tail_view(const ModelDims& m, const C* p) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    const C* b = p + tok_rows(m) * d + N * d + per * m.nl;
    LayerW<C> w{};
    w.ln1_g = b;
    w.ln1_b = b + d;
    w.W_qkv = b + 2 * d;
    w.b_qkv = w.W_qkv + d * 3 * d;
    w.W_o = w.b_qkv + 3 * d;
    w.b_o = w.W_o + d * d;
    return w;
}

template <typename C>
static HeadW<C> head_view(const ModelDims& m, const C* p) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    HeadW<C> h{};
    h.tok = p;
    const int64_t V = head_outputs(m);
    h.pos = p + tok_rows(m) * d;
    const C* t = p + tok_rows(m) * d + N * d + per * m.nl + tail_params(m);
    h.lnf_g = t;
    h.lnf_b = t + d;
    h.W_head = t + 2 * d;
    h.b_head = t + 2 * d + V * d;
    return h;
}

int64_t param_count(const ModelDims& m) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    const int64_t V = head_outputs(m);
    return tok_rows(m) * d + N * d + per * m.nl + tail_params(m) + 2 * d + V * d + V;
}

#define CK(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return VQNQS_ERR_HIP; \
    } while (0)

// Launch with optional per-kernel event timing on the launch stream.
#define LK(name, x)                                         \
    do {                                                    \
        Profiler& pf_ = Profiler::get();                    \
        if (pf_.enabled()) pf_.begin(name, st);             \
        hipError_t e_ = (x);                                \
        if (pf_.enabled()) pf_.end(st);                     \
        if (e_ != hipSuccess) return VQNQS_ERR_HIP;         \
    } while (0)

// Element offsets of every tensor of layer l (and of the head) in the flat
// parameter vector: the layout of include/vqnqs.h.
static LayerOffsets layer_offsets(const ModelDims& m, int l) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    LayerOffsets o;
    o.ln1_g = tok_rows(m) * d + N * d + per * l;
    o.ln1_b = o.ln1_g + d;
    o.W_qkv = o.ln1_b + d;
    o.b_qkv = o.W_qkv + d * 3 * d;
    o.codebook = o.b_qkv + 3 * d;
    o.W_o = o.codebook + Q * d;
    o.b_o = o.W_o + d * d;
    o.ln2_g = o.b_o + d;
    o.ln2_b = o.ln2_g + d;
    o.W1 = o.ln2_b + d;
    o.b1 = o.W1 + d * F;
    o.W2 = o.b1 + F;
    o.b2 = o.W2 + F * d;
    return o;
}

template <class P>
struct Runner {
    using acc = typename P::acc;
    using act = typename P::act;
    const ModelDims& m;
    const acc* params;     // replaced by the rounded copy in the BF16 mode
    Workspace<P> w;
    hipStream_t st;
    int64_t* ctr;

    LayerW<acc> layer(int l) const {
        LayerW<acc> lw = layer_view<acc>(m, params, l);
        lw.table = w.table + (int64_t)l * m.H * m.Q * m.d;
        lw.cnorm = w.cnorm + (int64_t)l * (m.H * m.Q + m.H);
        if (m.mfma) {
            lw.Wqkv_p = w.wqkv_p + (int64_t)l * m.d * 3 * m.d;
            lw.W1_p = w.w1_p + (int64_t)l * m.d * m.dff;
            lw.W2_p = w.w2_p + (int64_t)l * m.dff * m.d;
            lw.cb_p = w.cb_p + (int64_t)l * m.Q * m.d;
            lw.cnh = w.cnh + (int64_t)l * m.H * m.Q;
        }
        return lw;
    }

    // Products dispatch: matrix-core kernels for the BF16 mode.
    hipError_t qkv(const LayerW<acc>& lw, RowSet rs, const BlockIO<P>& io) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma) return launch_qkv_mfma(m, lw, rs, io, st);
        return launch_qkv<P>(m, lw, rs, io, st);
    }
    hipError_t mlp(const LayerW<acc>& lw, RowSet rs, const BlockIO<P>& io) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma) return launch_mlp_mfma(m, lw, rs, io, st);
        return launch_mlp<P>(m, lw, rs, io, st);
    }
    hipError_t attn_seq(const int32_t* n_dev, int64_t n, const BlockIO<P>& io,
                        int64_t* c) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma && attn_mfma_ok(m))
                return launch_attn_seq_mfma(m, n_dev, n, io, c, st);
        return launch_attention_seq<P>(m, n_dev, n, io, c, st);
    }
    hipError_t attn_dedup(const DedupIO<P>& dd) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma && attn_mfma_ok(m))
                return launch_attn_dedup_mfma(m, dd, ctr, st);
        return launch_attention_dedup<P>(m, dd, ctr, st);
    }
    hipError_t vqs(const LayerW<acc>& lw, RowSet rs, const BlockIO<P>& io,
                   const VqSeed& seed = VqSeed{}) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma) return launch_vq_mfma(m, lw, rs, io, st, seed);
        return launch_vq<P>(m, lw, rs, io, st);
    }
    HeadW<acc> head() const { return head_view<acc>(m, params); }
    LayerW<acc> tail() const {
        LayerW<acc> tw = tail_view<acc>(m, params);
        if (m.mfma) {
            tw.Wqkv_p = w.wqkv_tp;
            tw.Wo_p = w.wo_tp;
        }
        return tw;
    }
    // the half-block's output projection with residual, out = x + a W_o + b_o
    hipError_t tail_proj(const LayerW<acc>& tw, RowSet rs, const acc* x_in,
                         const act* a, acc* x_out) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma)
                return launch_oproj_mfma(m, tw.b_o, tw.Wo_p, rs, x_in, a, x_out, st);
        return launch_out_proj<P>(m, tw.W_o, tw.b_o, rs, x_in, a, x_out, st);
    }
    hipError_t tail_proj_overlay(const LayerW<acc>& tw, const DedupIO<P>& dd,
                                 acc* out) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma)
                return launch_oproj_overlay_mfma(m, tw.b_o, tw.Wo_p, dd, out, st);
        return launch_out_proj_overlay<P>(m, tw.W_o, tw.b_o, dd, out, st);
    }

    vqnqs_status prepare() {
        if constexpr (std::is_same<P, PrecBF16>::value) {
            // the BF16 mode evaluates the network at bf16-rounded parameters
            LK("round_bf16", launch_round_bf16(params, param_count(m), w.prm, st));
            params = w.prm;
        }
        for (int l = 0; l < m.nl; ++l) {
            LayerW<acc> lw = layer(l);
            LK("prepare", launch_prepare<P>(m, lw, const_cast<acc*>(lw.table),
                                 const_cast<acc*>(lw.cnorm), nullptr, nullptr,
                                 nullptr, nullptr, st));
            if constexpr (std::is_same<P, PrecBF16>::value)
                if (m.mfma)
                    LK("pack_layer", launch_pack_layer(m, lw, const_cast<bf16*>(lw.Wqkv_p),
                                         const_cast<bf16*>(lw.W1_p),
                                         const_cast<bf16*>(lw.W2_p),
                                         const_cast<bf16*>(lw.cb_p),
                                         const_cast<float*>(lw.cnh), st));
        }
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma && m.tail) {
                const LayerW<acc> tv = tail_view<acc>(m, params);
                LK("pack_layer", launch_pack_qkv(m, tv.W_qkv, w.wqkv_tp, st));
                LK("pack_layer", launch_pack_wo(m, tv.W_o, w.wo_tp, st));
            }
        return VQNQS_OK;
    }

    // Full forward of n sequences (count *n_dev if given, else n).  Layer
    // caches go to slice l of the cache arrays when `cache` is set.
    struct SeqBufs {
        const int8_t* spins;
        acc* x;           // [(nl+1 if cache else 1)][n][N][d]
        act *q, *k, *v, *a;
        int32_t* code;
        acc* margin;      // nullable
        acc* lp;          // nullable
        double* logpsi;
        bool cache;
        int32_t* codes_out;   // nullable [n][nl][N][H]
        bool keep_x = false;  // block inputs per layer only (checkpoints)
        act* attn_out = nullptr;  // nullable [n][nl][N][d] attention outputs
        acc* stat = nullptr;      // nullable [nl][n][N][heads][2] softmax stats
    };

    vqnqs_status forward(const SeqBufs& b, const int32_t* n_dev, int64_t n,
                         bool count_rows) {
        const int64_t rows = n * m.N, sd = rows * m.d, sh = rows * m.H;
        LK("embed", launch_embed<P>(m, head(), b.spins, n_dev, n, b.x, st));
        for (int l = 0; l < m.nl; ++l) {
            const int64_t cl = b.cache ? l : 0;
            const bool per_layer_x = b.cache || b.keep_x;
            BlockIO<P> io{};
            io.x = b.x + (per_layer_x ? (int64_t)(l + 1) * sd : 0);
            io.x_in = b.x + (per_layer_x ? (int64_t)l * sd : 0);
            io.q = b.q + cl * sd;
            io.k = b.k + cl * sd;
            io.v = b.v + cl * sd;
            io.a = b.a + cl * sd;
            io.codes = b.code + cl * sh;
            io.margin = b.margin ? b.margin + cl * sh * 2 : nullptr;
            io.stat = b.stat ? b.stat + (int64_t)l * rows * m.nh * 2 : nullptr;
            RowSet rs{nullptr, n_dev, rows, (int32_t)m.N};
            BlockIO<P> qio = io;
            qio.x = const_cast<acc*>(io.x_in);
            LK("qkv", qkv(layer(l), rs, qio));
            LK("attention_seq", attn_seq(n_dev, n, io, count_rows ? ctr : nullptr));
            if (b.attn_out)
                LK("copy_attn", launch_copy_layer<act>(io.a, n, (int64_t)m.N * m.d, m.nl, l,
                                                       b.attn_out, st));
            LK("vq", vqs(layer(l), rs, io));
            LK("mlp", mlp(layer(l), rs, io));
            if (b.codes_out)
                LK("copy_codes", launch_copy_codes(io.codes, n, m.N, m.H, m.nl, l, b.codes_out, st));
        }
        const bool per_layer_x = b.cache || b.keep_x;
        if (m.tail) {
            // attention-only half-block: input slice nl, output slice nl+1
            // when the layer inputs are kept (in place otherwise)
            const int64_t cl = b.cache ? m.nl : 0;
            BlockIO<P> io{};
            io.x_in = b.x + (per_layer_x ? (int64_t)m.nl * sd : 0);
            io.x = b.x + (per_layer_x ? (int64_t)(m.nl + 1) * sd : 0);
            io.q = b.q + cl * sd;
            io.k = b.k + cl * sd;
            io.v = b.v + cl * sd;
            io.a = b.a + cl * sd;
            io.codes = b.code;
            RowSet rs{nullptr, n_dev, rows, (int32_t)m.N};
            BlockIO<P> qio = io;
            qio.x = const_cast<acc*>(io.x_in);
            const LayerW<acc> tw = tail();
            LK("qkv", qkv(tw, rs, qio));
            LK("attention_seq", attn_seq(n_dev, n, io, count_rows ? ctr : nullptr));
            LK("tail_proj", tail_proj(tw, rs, io.x_in, io.a, io.x));
        }
        const acc* xf = b.x + (per_layer_x ? (int64_t)(m.nl + m.tail) * sd : 0);
        LK("head_seq", launch_head_seq<P>(m, head(), b.spins, n_dev, n, xf, b.lp, b.logpsi, st));
        if (count_rows && ctr) {
            if (n_dev) {
                CK(launch_counter_add(ctr, VQNQS_CTR_QKV_ROWS, n_dev, (int64_t)m.N * m.nl, st));
                CK(launch_counter_add(ctr, VQNQS_CTR_MLP_ROWS, n_dev, (int64_t)m.N * m.nl, st));
                CK(launch_counter_add(ctr, VQNQS_CTR_VQ_ROWS, n_dev, (int64_t)m.N * m.nl, st));
                CK(launch_counter_add(ctr, VQNQS_CTR_HEAD_ROWS, n_dev, (int64_t)m.N, st));
            } else {
                CK(launch_counter_add_const(ctr, VQNQS_CTR_QKV_ROWS, rows * m.nl, st));
                CK(launch_counter_add_const(ctr, VQNQS_CTR_MLP_ROWS, rows * m.nl, st));
                CK(launch_counter_add_const(ctr, VQNQS_CTR_VQ_ROWS, rows * m.nl, st));
                CK(launch_counter_add_const(ctr, VQNQS_CTR_HEAD_ROWS, rows, st));
            }
        }
        return VQNQS_OK;
    }

    // ------------------------------------------------ gradient of log psi
    hipError_t gemm(int64_t M, int64_t Nn, int64_t K, const acc* A, int64_t lda,
                    int64_t sA, int tA, const acc* B, int64_t ldb, int64_t sB,
                    int tB, acc* C, int64_t ldc, int64_t sC, int beta,
                    int64_t groups) {
        // B is bf16-exact when it is one of the (rounded) parameters
        const uintptr_t b = reinterpret_cast<uintptr_t>(B);
        const uintptr_t p0 = reinterpret_cast<uintptr_t>(params);
        const int b_exact =
            m.mfma && b >= p0 && b < p0 + sizeof(acc) * (uintptr_t)param_count(m);
        GemmDesc g{M, Nn, K, A, lda, sA, tA, B, ldb, sB, tB, C, ldc, sC, beta,
                   groups, b_exact};
        // the BF16 mode runs its products on the matrix core
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma) return launch_gemm_mfma(g, st);
        return launch_gemm<acc>(g, st);
    }
    hipError_t colsum(int64_t n, int cols, const acc* A, int64_t lda,
                      const acc* B, int64_t ldb, acc* out, int64_t os) {
        return launch_colsum<acc>(n, m.N, cols, A, lda, B, ldb, out, os, 0, st);
    }

    // Per-sample straight-through gradients of n samples into gout[n][P]
    // (upstream 1/2 * weight of every position's log-probability).  The
    // forward keeps only the layer inputs; each layer is recomputed with the
    // forward's own kernels (so its codes are the forward's) before its
    // backward.
    vqnqs_status grad_chunk(const int8_t* sp, int64_t n, const double* wts,
                            acc* gout, double* lp_out) {
        const int64_t N = m.N, d = m.d, F = m.dff, Q = m.Q, ds = m.dseg;
        const int64_t R = n * N, sd = R * d, NP = param_count(m);
        LK("neighbours", launch_neighbours(sp, n, m, w.bonds, w.count, nullptr,
                                           nullptr, w.status, st));
        SeqBufs sb{sp, w.gx, w.gq, w.gk, w.gv, w.ga, w.gcode, nullptr, nullptr,
                   lp_out ? lp_out : w.glogpsi, false, nullptr, true};
        vqnqs_status s = forward(sb, nullptr, n, false);
        if (s) return s;
        LK("grad_coef", launch_coef<acc>(n, wts, w.coef, st));
        const HeadW<acc> hw = head();
        const int64_t off_tail = layer_offsets(m, m.nl).ln1_g;
        const int64_t off_lnf = off_tail + tail_params(m);
        const int64_t off_Wh = off_lnf + 2 * d, off_bh = off_Wh + head_outputs(m) * d;
        // head: d log psi / d x_L (after the half-block, when there is one)
        const int64_t V = head_outputs(m);
        LK("grad_head", launch_head_bwd<acc>(n, (int)N, (int)d, m.K, m.enc, hw, sp,
                                             w.gx + (int64_t)(m.nl + m.tail) * sd,
                                             w.coef, w.h1, w.xh1, w.rs1, w.dz2,
                                             w.dT, w.dX, st));
        LK("grad_gemm", gemm(d, V, N, w.h1, d, N * d, 1, w.dz2, V, V * N, 0,
                             gout + off_Wh, V, NP, 0, n));
        LK("grad_colsum", colsum(n, (int)V, w.dz2, V, nullptr, 0, gout + off_bh, NP));
        LK("grad_colsum", colsum(n, d, w.dT, d, w.xh1, d, gout + off_lnf, NP));
        LK("grad_colsum", colsum(n, d, w.dT, d, nullptr, 0, gout + off_lnf + d, NP));
        if (m.tail) {
            // attention-only half-block, x = x_in + a W_o + b_o with
            // a = attention(LN(x_in) W_qkv + b_qkv): recompute, then
            // backward, the upstream dX at x turning into the one at x_in
            const LayerW<acc> tw = tail();
            const acc* xl = w.gx + (int64_t)m.nl * sd;
            const int64_t o_ln = off_tail, o_Wqkv = off_tail + 2 * d;
            const int64_t o_bqkv = o_Wqkv + 3 * d * d, o_Wo = o_bqkv + 3 * d;
            const int64_t o_bo = o_Wo + d * d;
            BlockIO<P> io{};
            io.x = const_cast<acc*>(xl);
            io.x_in = xl;
            io.q = w.gq;
            io.k = w.gk;
            io.v = w.gv;
            io.a = w.ga;
            io.codes = w.gcode;
            const RowSet rs{nullptr, nullptr, R, (int32_t)N};
            LK("qkv", qkv(tw, rs, io));
            LK("attention_seq", attn_seq(nullptr, n, io, nullptr));
            LK("grad_ln", launch_ln_save<acc>(R, (int)d, xl, tw.ln1_g, tw.ln1_b,
                                              w.h1, w.xh1, w.rs1, st));
            LK("grad_gemm", gemm(d, d, N, w.ga, d, N * d, 1, w.dX, d, N * d, 0,
                                 gout + o_Wo, d, NP, 0, n));
            LK("grad_colsum", colsum(n, d, w.dX, d, nullptr, 0, gout + o_bo, NP));
            LK("grad_gemm", gemm(R, d, d, w.dX, d, 0, 0, tw.W_o, d, 0, 1, w.da,
                                 d, 0, 0, 1));
            LK("grad_attention", launch_attn_bwd<acc>(n, m, w.gq, w.gk, w.gv,
                                                      w.ga, w.da, w.lse, w.Dd,
                                                      w.dqkv, st));
            LK("grad_gemm", gemm(d, 3 * d, N, w.h1, d, N * d, 1, w.dqkv, 3 * d,
                                 N * 3 * d, 0, gout + o_Wqkv, 3 * d, NP, 0, n));
            LK("grad_colsum", colsum(n, 3 * (int)d, w.dqkv, 3 * d, nullptr, 0,
                                     gout + o_bqkv, NP));
            LK("grad_gemm", gemm(R, d, 3 * d, w.dqkv, 3 * d, 0, 0, tw.W_qkv,
                                 3 * d, 0, 1, w.dT, d, 0, 0, 1));
            LK("grad_colsum", colsum(n, d, w.dT, d, w.xh1, d, gout + o_ln, NP));
            LK("grad_colsum", colsum(n, d, w.dT, d, nullptr, 0, gout + o_ln + d, NP));
            // the residual carries dX through; LN adds its part in place
            LK("grad_ln", launch_ln_bwd<acc>(R, (int)d, w.xh1, w.rs1, tw.ln1_g,
                                             w.dT, w.dX, w.dX, st));
        }
        for (int l = m.nl - 1; l >= 0; --l) {
            const LayerW<acc> lw = layer(l);
            const LayerOffsets o = layer_offsets(m, l);
            const acc* xl = w.gx + (int64_t)l * sd;
            // recompute q, k, v, a and the codes
            BlockIO<P> io{};
            io.x = const_cast<acc*>(xl);
            io.x_in = xl;
            io.q = w.gq;
            io.k = w.gk;
            io.v = w.gv;
            io.a = w.ga;
            io.codes = w.gcode;
            io.margin = nullptr;
            const RowSet rs{nullptr, nullptr, R, (int32_t)N};
            LK("qkv", qkv(lw, rs, io));
            LK("attention_seq", attn_seq(nullptr, n, io, nullptr));
            LK("vq", vqs(lw, rs, io));
            LK("grad_ln", launch_ln_save<acc>(R, (int)d, xl, lw.ln1_g, lw.ln1_b,
                                              w.h1, w.xh1, w.rs1, st));
            LK("grad_xprime", launch_xprime<acc>(R, m, xl, w.gcode, lw.table,
                                                 lw.b_o, lw.codebook, w.xp,
                                                 w.zq, st));
            LK("grad_ln", launch_ln_save<acc>(R, (int)d, w.xp, lw.ln2_g,
                                              lw.ln2_b, w.h2, w.xh2, w.rs2, st));
            LK("grad_gemm", gemm(R, F, d, w.h2, d, 0, 0, lw.W1, F, 0, 0, w.gu,
                                 F, 0, 0, 1));
            LK("grad_gelu", launch_bias_gelu<acc>(R, (int)F, w.gu, lw.b1, w.gg, st));
            // MLP: x = x' + GELU(LN2(x') W1 + b1) W2 + b2
            LK("grad_gemm", gemm(F, d, N, w.gg, F, N * F, 1, w.dX, d, N * d, 0,
                                 gout + o.W2, d, NP, 0, n));
            LK("grad_colsum", colsum(n, d, w.dX, d, nullptr, 0, gout + o.b2, NP));
            LK("grad_gemm", gemm(R, F, d, w.dX, d, 0, 0, lw.W2, d, 0, 1, w.dF,
                                 F, 0, 0, 1));
            LK("grad_gelu", launch_gelu_bwd<acc>(R * F, w.gu, w.dF, st));
            LK("grad_gemm", gemm(d, F, N, w.h2, d, N * d, 1, w.dF, F, N * F, 0,
                                 gout + o.W1, F, NP, 0, n));
            LK("grad_colsum", colsum(n, F, w.dF, F, nullptr, 0, gout + o.b1, NP));
            LK("grad_gemm", gemm(R, d, F, w.dF, F, 0, 0, lw.W1, F, 0, 1, w.dT,
                                 d, 0, 0, 1));
            LK("grad_colsum", colsum(n, d, w.dT, d, w.xh2, d, gout + o.ln2_g, NP));
            LK("grad_colsum", colsum(n, d, w.dT, d, nullptr, 0, gout + o.ln2_b, NP));
            LK("grad_ln", launch_ln_bwd<acc>(R, (int)d, w.xh2, w.rs2, lw.ln2_g,
                                             w.dT, w.dX, w.dXp, st));
            // output projection: x' = x + z W_o + b_o
            LK("grad_gemm", gemm(d, d, N, w.zq, d, N * d, 1, w.dXp, d, N * d, 0,
                                 gout + o.W_o, d, NP, 0, n));
            LK("grad_colsum", colsum(n, d, w.dXp, d, nullptr, 0, gout + o.b_o, NP));
            LK("grad_gemm", gemm(R, d, d, w.dXp, d, 0, 0, lw.W_o, d, 0, 1, w.dT,
                                 d, 0, 0, 1));
            // straight-through quantizer (eqs. 7-8), head by head
            for (int h = 0; h < m.H; ++h) {
                const acc* cb = lw.codebook + (int64_t)h * Q * ds;
                acc* dcb = gout + o.codebook + (int64_t)h * Q * ds;
                const acc* ah = w.ga + h * ds;
                LK("grad_gemm", gemm(R, Q, ds, ah, d, 0, 0, cb, ds, 0, 1, w.S,
                                     Q, 0, 0, 1));
                LK("grad_gemm", gemm(R, Q, ds, w.dT + h * ds, d, 0, 0, cb, ds,
                                     0, 1, w.E, Q, 0, 0, 1));
                LK("grad_vq", launch_vq_bwd_rows<acc>(R, (int)Q, (int)ds, m.H,
                                                      h, ah, (int)d, w.gcode,
                                                      lw.cnorm + (int64_t)h * Q,
                                                      w.S, w.E, w.rowG, st));
                LK("grad_gemm", gemm(R, ds, Q, w.S, Q, 0, 0, cb, ds, 0, 0,
                                     w.da + h * ds, d, 0, 0, 1));
                LK("grad_vq", launch_da_fix<acc>(R, (int)ds, (int)d, ah, w.rowG,
                                                 w.da + h * ds, st));
                // codebook: softmax path through the distances, then the
                // one-hot factor of eq. (8) (the upstream rows added to the
                // chosen codewords)
                LK("grad_gemm", gemm(Q, ds, N, w.S, Q, N * Q, 1, ah, d, N * d, 0,
                                     dcb, ds, NP, 0, n));
                LK("grad_vq", launch_onehot_scatter<acc>(n, (int)N, (int)ds,
                                                         (int)d, m.H, h, w.gcode,
                                                         w.dT + h * ds, dcb, NP,
                                                         st));
                LK("grad_colsum", colsum(n, (int)Q, w.S, Q, nullptr, 0, w.colG, Q));
                LK("grad_vq", launch_cb_fix<acc>(n, (int)Q, (int)ds, w.colG, cb,
                                                 dcb, NP, st));
            }
            // causal attention
            LK("grad_attention", launch_attn_bwd<acc>(n, m, w.gq, w.gk, w.gv,
                                                      w.ga, w.da, w.lse, w.Dd,
                                                      w.dqkv, st));
            // LN1 + QKV projection
            LK("grad_gemm", gemm(d, 3 * d, N, w.h1, d, N * d, 1, w.dqkv, 3 * d,
                                 N * 3 * d, 0, gout + o.W_qkv, 3 * d, NP, 0, n));
            LK("grad_colsum", colsum(n, 3 * (int)d, w.dqkv, 3 * d, nullptr, 0,
                                     gout + o.b_qkv, NP));
            LK("grad_gemm", gemm(R, d, 3 * d, w.dqkv, 3 * d, 0, 0, lw.W_qkv,
                                 3 * d, 0, 1, w.dT, d, 0, 0, 1));
            LK("grad_colsum", colsum(n, d, w.dT, d, w.xh1, d, gout + o.ln1_g, NP));
            LK("grad_colsum", colsum(n, d, w.dT, d, nullptr, 0, gout + o.ln1_b, NP));
            LK("grad_ln", launch_ln_bwd<acc>(R, (int)d, w.xh1, w.rs1, lw.ln1_g,
                                             w.dT, w.dXp, w.dX, st));
        }
        LK("grad_embed", launch_embed_bwd<acc>(n, (int)N, (int)d, m.K, m.enc, sp, w.dX,
                                               gout, NP, 0, tok_rows(m) * d, st));
        return VQNQS_OK;
    }

    vqnqs_status neighbours(const int8_t* spins, int64_t n) {
        LK("neighbours", launch_neighbours(spins, n, m, w.bonds, w.count, w.diag, w.rows_cap,
                             w.status, st));
        LK("scan_desc", launch_scan_desc(w.bonds, w.count, w.rows_cap, (int)n, m.L, m.chain, m.K, m.enc, w.nb_off,
                            w.row_off, w.n_nb, w.n_rows, w.desc, st));
        if (ctr) {
            CK(launch_counter_add_const(ctr, VQNQS_CTR_SAMPLES, n, st));
            CK(launch_counter_add(ctr, VQNQS_CTR_NEIGHBOURS, w.n_nb, 1, st));
        }
        return VQNQS_OK;
    }

    // Direct autoregressive sampling of n samples (chain rule, Sec. 2):
    // position by position, every layer's per-row kernels on row i of all
    // samples, attention of row i over the cached keys and values 0..i,
    // then the head draws s_i with the caller's uniform numbers.
    vqnqs_status sample_chunk(const double* uni, int64_t n, int8_t* spins,
                              double* logpsi) {
        const int64_t N = m.N, R = n * N, sd = R * m.d;
        RowSet rs{w.list, nullptr, n, 1};
        for (int i = 0; i < N; ++i) {
            LK("sample_embed", launch_sample_embed<P>(m, head(), n, i, spins, w.bx,
                                                      w.list, w.logpsi_s, st));
            for (int l = 0; l < m.nl; ++l) {
                BlockIO<P> io{};
                io.x = w.bx;
                io.x_in = w.bx;
                io.q = w.bq;
                io.k = w.bk + (int64_t)l * sd;
                io.v = w.bv + (int64_t)l * sd;
                io.a = w.ba;
                io.codes = w.bcode;
                io.margin = nullptr;
                LK("qkv", qkv(layer(l), rs, io));
                LK("attention_rows", launch_attn_rows<P>(m, n, i, io, st));
                LK("vq", vqs(layer(l), rs, io));
                LK("mlp", mlp(layer(l), rs, io));
            }
            if (m.tail) {
                BlockIO<P> io{};
                io.x = w.bx;
                io.x_in = w.bx;
                io.q = w.bq;
                io.k = w.bk + (int64_t)m.nl * sd;
                io.v = w.bv + (int64_t)m.nl * sd;
                io.a = w.ba;
                io.codes = w.bcode;
                const LayerW<acc> tw = tail();
                LK("qkv", qkv(tw, rs, io));
                LK("attention_rows", launch_attn_rows<P>(m, n, i, io, st));
                LK("tail_proj", tail_proj(tw, rs, w.bx, w.ba, w.bx));
            }
            LK("sample_head", launch_sample_head<P>(m, head(), n, i, w.bx,
                                                    uni + 0, spins, w.logpsi_s,
                                                    logpsi, st));
        }
        (void)R;
        return VQNQS_OK;
    }

    vqnqs_status plain_chunk(const int8_t* spins, int64_t n) {
        vqnqs_status s = neighbours(spins, n);
        if (s) return s;
        SeqBufs sb{spins, w.bx, w.bq, w.bk, w.bv, w.ba, w.bcode, nullptr,
                   nullptr, w.logpsi_s, false, nullptr};
        s = forward(sb, nullptr, n, true);
        if (s) return s;
        const int64_t nbmax = n * 2 * m.S;
        LK("materialise", launch_materialise(spins, w.desc, w.n_nb, nbmax, m.S, w.nspins, st));
        SeqBufs nbuf{w.nspins, w.nx, w.nq, w.nk, w.nv, w.na, w.ncode, nullptr,
                     nullptr, w.logpsi_nb, false, nullptr};
        s = forward(nbuf, w.n_nb, nbmax, true);
        if (s) return s;
        LK("ratio_plain", launch_ratio_plain(w.logpsi_nb, w.logpsi_s, w.desc, w.n_nb, nbmax,
                              w.ratio, st));
        return VQNQS_OK;
    }

    vqnqs_status dedup_chunk(const int8_t* spins, int64_t n) {
        vqnqs_status s = neighbours(spins, n);
        if (s) return s;
        const int64_t N = m.N, d = m.d, H = m.H;
        const int64_t sd = n * N * d, sh = n * N * H;
        // margins only feed the certified-reuse test
        const bool cert = (m.flags & VQNQS_FLAG_CERTIFIED_VQ) != 0;
        SeqBufs sb{spins, w.bx, w.bq, w.bk, w.bv, w.ba, w.bcode,
                   cert ? w.bmargin : nullptr,
                   w.blp, w.logpsi_s, true, nullptr};
        const bool incr = (m.flags & VQNQS_FLAG_INCREMENTAL_ATTN) != 0;
        // layers whose attention takes the rank-|C| update (the first ones,
        // where the changed sets are small)
        const int inc_layers = incr ? (VQNQS_INC_LAYERS_OF(m.flags) > 0
                                           ? VQNQS_INC_LAYERS_OF(m.flags)
                                           : 2)
                                    : 0;
        sb.stat = incr ? w.bstat : nullptr;
        s = forward(sb, nullptr, n, true);
        if (s) return s;
        const int64_t nbmax = n * 2 * m.S;
        const int64_t R = n * max_overlay_rows(m);
        DedupIO<P> dd{};
        dd.desc = w.desc;
        dd.n_nb = w.n_nb;
        dd.n_nb_max = nbmax;
        dd.nb_off = w.nb_off;
        dd.n_samples = n;
        dd.n_rows = w.n_rows;
        dd.rows_max = R;
        dd.spins = spins;
        dd.slot_nb = w.slot_nb;
        dd.crow = w.crow;
        dd.ccnt = w.ccnt;
        dd.ox = w.ox;
        dd.oq = w.oq;
        dd.ok = w.ok;
        dd.ov = w.ov;
        dd.oa = w.oa;
        dd.ocode = w.ocode;
        dd.mask = w.mask;
        dd.mask_words = (m.N + 63) / 64;
        dd.list = w.list;
        dd.list_n = w.list_n;
        dd.vq_list = w.vq_list;
        dd.vq_n = w.vq_n;
        CK(launch_fill_i32(w.list_n, 1, 0, st));
        LK("dedup_init", launch_dedup_init<P>(m, head(), dd, st));
        if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_CHANGED0, w.list_n, 1, st));
        const bool certified = (m.flags & VQNQS_FLAG_CERTIFIED_VQ) != 0;
        for (int l = 0; l < m.nl; ++l) {
            LayerW<acc> lw = layer(l);
            dd.bx = w.bx + (int64_t)l * sd;
            dd.bq = w.bq + (int64_t)l * sd;
            dd.bk = w.bk + (int64_t)l * sd;
            dd.bv = w.bv + (int64_t)l * sd;
            dd.ba = w.ba + (int64_t)l * sd;
            dd.bcode = w.bcode + (int64_t)l * sh;
            dd.bmargin = w.bmargin + (int64_t)l * sh * 2;
            dd.wmax = lw.cnorm + (int64_t)H * m.Q;
            // LN1 + QKV on the rows of C_{l-1}
            BlockIO<P> io{};
            io.x = w.ox;
            io.x_in = w.ox;
            io.q = w.oq;
            io.k = w.ok;
            io.v = w.ov;
            io.a = w.oa;
            io.codes = w.ocode;
            io.margin = nullptr;
            RowSet cl{w.list, w.list_n, R, 1};
            if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_QKV_ROWS, w.list_n, 1, st));
            LK("qkv", qkv(lw, cl, io));
            if (l < inc_layers) {
                LK("attention_incr",
                   launch_attention_incr<P>(m, dd, w.bstat + (int64_t)l * n * N * m.nh * 2,
                                            ctr, st));
            } else {
                LK("attention_dedup", attn_dedup(dd));
            }
            // the sample's codes of this layer seed the neighbours' searches
            VqSeed seed;
            seed.slot_nb = w.slot_nb;
            seed.desc = w.desc;
            seed.bcode = dd.bcode;
            if (certified) {
                CK(launch_fill_i32(w.vq_n, 1, 0, st));
                LK("certify", launch_certify<P>(m, dd, 1, ctr, st));
                RowSet vr{w.vq_list, w.vq_n, R, 1};
                LK("vq", vqs(lw, vr, io, seed));
                if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_VQ_ROWS, w.vq_n, 1, st));
            } else {
                RowSet vr{nullptr, w.n_rows, R, 1};
                LK("vq", vqs(lw, vr, io, seed));
                if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_VQ_ROWS, w.n_rows, 1, st));
            }
            CK(launch_fill_i32(w.list_n, 1, 0, st));
            LK("code_diff", launch_code_diff<P>(m, dd, st));
            if (ctr) {
                CK(launch_counter_add(ctr, VQNQS_CTR_CHANGED0 + l + 1, w.list_n, 1, st));
                CK(launch_counter_add(ctr, VQNQS_CTR_MLP_ROWS, w.list_n, 1, st));
            }
            LK("mlp", mlp(lw, cl, io));
        }
        if (m.tail) {
            // the half-block: LN + QKV on C_L, attention on every row from
            // p_min, its output projection on all of those rows (its input
            // the neighbour's row where in C_L, else the sample's), whose
            // results the head then reads for every row from p_min
            const int64_t lt = m.nl;
            dd.bx = w.bx + lt * sd;
            dd.bq = w.bq + lt * sd;
            dd.bk = w.bk + lt * sd;
            dd.bv = w.bv + lt * sd;
            dd.ba = w.ba + lt * sd;
            BlockIO<P> io{};
            io.x = w.ox;
            io.x_in = w.ox;
            io.q = w.oq;
            io.k = w.ok;
            io.v = w.ov;
            io.a = w.oa;
            io.codes = w.ocode;
            const LayerW<acc> tw = tail();
            RowSet cl{w.list, w.list_n, R, 1};
            if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_QKV_ROWS, w.list_n, 1, st));
            LK("qkv", qkv(tw, cl, io));
            LK("attention_dedup", attn_dedup(dd));
            LK("tail_proj", tail_proj_overlay(tw, dd, w.oq));
            LK("tail_mask", launch_mask_from_pmin(w.desc, w.n_nb, nbmax, dd.mask_words,
                                                  m.N, w.mask, st));
            dd.ox = w.oq;
            if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_TAIL_ROWS, w.n_rows, 1, st));
        }
        LK("head_dedup", launch_head_dedup<P>(m, head(), dd, w.blp, nullptr, w.ratio, ctr, st));
        return VQNQS_OK;
    }
};

template <class P>
static vqnqs_status run_local_energy(const ModelDims& m, const void* params,
                                     const int8_t* spins, int64_t batch,
                                     int mode, double* eloc, double* stats,
                                     double* ratios, int64_t* counters,
                                     void* ws, size_t ws_bytes,
                                     hipStream_t st) {
    // the rank-|C| attention update is built for the FP64 and FP32 modes
    if ((m.flags & VQNQS_FLAG_INCREMENTAL_ATTN) && m.precision == VQNQS_BF16)
        return VQNQS_ERR_UNSUPPORTED;
    const int64_t chunk = pick_chunk(m, mode, batch, ws_bytes);
    if (batch > 0 && chunk <= 0) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    Runner<P> r{m, static_cast<const typename P::acc*>(params),
                carve<P>(m, mode == VQNQS_PLAIN ? Job::Plain : Job::Dedup,
                         chunk, ws),
                st, counters};
    CK(launch_fill_i32(r.w.status, 1, 0, st));
    if (counters) CK(launch_fill_i64(counters, VQNQS_NCOUNTERS, 0, st));
    if (batch == 0) return VQNQS_OK;
    vqnqs_status s = r.prepare();
    if (s) return s;
    // off-diagonal element per neighbour: -Gamma per flip (chain),
    // -+J/2 per exchanged bond (Heisenberg, Marshall-rotated or not)
    const double h_off = m.chain ? -m.gamma : (m.marshall ? -0.5 * m.J : 0.5 * m.J);
    for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
        const int64_t n = std::min(chunk, batch - c0);
        const int8_t* sp = spins + c0 * m.S;
        s = mode == VQNQS_PLAIN ? r.plain_chunk(sp, n) : r.dedup_chunk(sp, n);
        if (s) return s;
        LK("eloc", launch_eloc(r.w.diag, r.w.count, r.w.nb_off, r.w.ratio, (int)n, m.S,
                       h_off, eloc + c0,
                       ratios ? ratios + c0 * 2 * m.S : nullptr, st));
    }
    if (stats) LK("stats", launch_stats(eloc, batch, stats, st));
    return VQNQS_OK;
}

vqnqs_status local_energy(const ModelDims& m, const void* params,
                          const int8_t* spins, int64_t batch, int mode,
                          double* eloc, double* stats, double* ratios,
                          int64_t* counters, void* ws, size_t ws_bytes,
                          hipStream_t st) {
    switch (m.precision) {
        case VQNQS_F64:
            return run_local_energy<PrecF64>(m, params, spins, batch, mode, eloc,
                                             stats, ratios, counters, ws,
                                             ws_bytes, st);
        case VQNQS_F32:
            return run_local_energy<PrecF32>(m, params, spins, batch, mode, eloc,
                                             stats, ratios, counters, ws,
                                             ws_bytes, st);
        default:
            return run_local_energy<PrecBF16>(m, params, spins, batch, mode,
                                              eloc, stats, ratios, counters, ws,
                                              ws_bytes, st);
    }
}

template <class P>
static vqnqs_status run_forward(const ModelDims& m, const void* params,
                                const int8_t* spins, int64_t batch,
                                double* logpsi, int32_t* codes, void* attn,
                                void* ws, size_t ws_bytes, hipStream_t st) {
    using act = typename P::act;
    const int64_t chunk = pick_chunk(m, -1, batch, ws_bytes);
    if (batch > 0 && chunk <= 0) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    Runner<P> r{m, static_cast<const typename P::acc*>(params),
                carve<P>(m, Job::Forward, chunk, ws), st, nullptr};
    CK(launch_fill_i32(r.w.status, 1, 0, st));
    if (batch == 0) return VQNQS_OK;
    vqnqs_status s = r.prepare();
    if (s) return s;
    for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
        const int64_t n = std::min(chunk, batch - c0);
        const int8_t* sp = spins + c0 * m.S;
        // spin validation shares the neighbour kernel
        LK("neighbours", launch_neighbours(sp, n, m, r.w.bonds, r.w.count, nullptr, nullptr,
                             r.w.status, st));
        typename Runner<P>::SeqBufs sb{
            sp, r.w.bx, r.w.bq, r.w.bk, r.w.bv, r.w.ba, r.w.bcode, nullptr,
            nullptr, logpsi + c0, false,
            codes ? codes + c0 * (int64_t)m.nl * m.N * m.H : nullptr};
        if (attn)
            sb.attn_out = static_cast<act*>(attn) + c0 * (int64_t)m.nl * m.N * m.d;
        s = r.forward(sb, nullptr, n, false);
        if (s) return s;
    }
    return VQNQS_OK;
}

vqnqs_status forward_logpsi(const ModelDims& m, const void* params,
                            const int8_t* spins, int64_t batch, double* logpsi,
                            int32_t* codes, void* attn, void* ws,
                            size_t ws_bytes, hipStream_t st) {
    switch (m.precision) {
        case VQNQS_F64:
            return run_forward<PrecF64>(m, params, spins, batch, logpsi, codes,
                                        attn, ws, ws_bytes, st);
        case VQNQS_F32:
            return run_forward<PrecF32>(m, params, spins, batch, logpsi, codes,
                                        attn, ws, ws_bytes, st);
        default:
            return run_forward<PrecBF16>(m, params, spins, batch, logpsi, codes,
                                         attn, ws, ws_bytes, st);
    }
}

template <class P>
static vqnqs_status run_sample(const ModelDims& m, const void* params,
                               const double* uniforms, int64_t batch,
                               int8_t* spins, double* logpsi, void* ws,
                               size_t ws_bytes, hipStream_t st) {
    const int64_t chunk = pick_chunk(m, -4, batch, ws_bytes);
    if (batch > 0 && chunk <= 0) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    Runner<P> r{m, static_cast<const typename P::acc*>(params),
                carve<P>(m, Job::Sample, chunk, ws), st, nullptr};
    CK(launch_fill_i32(r.w.status, 1, 0, st));
    if (batch == 0) return VQNQS_OK;
    vqnqs_status s = r.prepare();
    if (s) return s;
    for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
        const int64_t n = std::min(chunk, batch - c0);
        s = r.sample_chunk(uniforms + c0 * m.S, n, spins + c0 * m.S,
                           logpsi ? logpsi + c0 : nullptr);
        if (s) return s;
    }
    return VQNQS_OK;
}

vqnqs_status sample(const ModelDims& m, const void* params,
                    const double* uniforms, int64_t batch, int8_t* spins,
                    double* logpsi, void* ws, size_t ws_bytes,
                    hipStream_t st) {
    switch (m.precision) {
        case VQNQS_F64:
            return run_sample<PrecF64>(m, params, uniforms, batch, spins,
                                       logpsi, ws, ws_bytes, st);
        case VQNQS_F32:
            return run_sample<PrecF32>(m, params, uniforms, batch, spins,
                                       logpsi, ws, ws_bytes, st);
        default:
            return run_sample<PrecBF16>(m, params, uniforms, batch, spins,
                                        logpsi, ws, ws_bytes, st);
    }
}

vqnqs_status vmc_step(const ModelDims& m, void* params, void* opt_state,
                      int64_t step, double lr, const double* uniforms,
                      int64_t B, int8_t* spins_out, double* eloc_out,
                      double* stats_out, void* ws, size_t ws_bytes,
                      hipStream_t st) {
    const size_t front = vmc_front_bytes(m, B);
    if (ws_bytes <= front) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    const size_t sub = (ws_bytes - front) & ~(size_t)255;
    char* f = static_cast<char*>(ws) + sub;
    int8_t* spins = reinterpret_cast<int8_t*>(f);
    f += al256((size_t)B * m.S);
    double* eloc = reinterpret_cast<double*>(f);
    f += al256((size_t)B * 8);
    double* w = reinterpret_cast<double*>(f);
    f += al256((size_t)B * 8);
    double* stats = reinterpret_cast<double*>(f);
    f += 256;
    void* grad = f;
    if (spins_out) spins = spins_out;
    if (eloc_out) eloc = eloc_out;
    if (stats_out) stats = stats_out;
    // one sample's sub-call workspace must fit
    if (sub < vmc_sub_bytes(m, 1)) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    vqnqs_status s = sample(m, params, uniforms, B, spins, nullptr, ws, sub, st);
    if (s) return s;
    s = local_energy(m, params, spins, B, VQNQS_DEDUP, eloc, stats, nullptr,
                     nullptr, ws, sub, st);
    if (s) return s;
    LK("vmc_weights", launch_vmc_weights(eloc, stats, B, w, st));
    s = grad_logpsi(m, params, spins, B, w, grad, nullptr, ws, sub, st);
    if (s) return s;
    const int64_t P = param_count(m);
    if (m.precision == VQNQS_F64) {
        double* mo = static_cast<double*>(opt_state);
        LK("update", launch_update<double>(static_cast<double*>(params),
                                           static_cast<const double*>(grad),
                                           mo, mo ? mo + P : nullptr, P, lr,
                                           0.9, 0.999, 1e-8, step, st));
    } else {
        float* mo = static_cast<float*>(opt_state);
        LK("update", launch_update<float>(static_cast<float*>(params),
                                          static_cast<const float*>(grad),
                                          mo, mo ? mo + P : nullptr, P, lr,
                                          0.9, 0.999, 1e-8, step, st));
    }
    return VQNQS_OK;
}

template <class P>
static vqnqs_status run_grad(const ModelDims& m, const void* params,
                             const int8_t* spins, int64_t batch,
                             const double* weights, void* grad, double* logpsi,
                             void* ws, size_t ws_bytes, hipStream_t st) {
    using acc = typename P::acc;
    const int64_t chunk = pick_chunk(m, -3, batch, ws_bytes);
    if (batch > 0 && chunk <= 0) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    if (batch == 0 && ws_bytes < workspace_bytes(m, -3, 1))
        return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    Runner<P> r{m, static_cast<const acc*>(params),
                carve<P>(m, Job::Grad, std::max<int64_t>(chunk, 1), ws), st,
                nullptr};
    const int64_t Pn = param_count(m);
    acc* g = static_cast<acc*>(grad);
    CK(launch_fill_i32(r.w.status, 1, 0, st));
    if (batch == 0) {
        if (weights) CK(launch_fill_t<acc>(g, Pn, (acc)0, st));
        return VQNQS_OK;
    }
    vqnqs_status s = r.prepare();
    if (s) return s;
    for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
        const int64_t n = std::min(chunk, batch - c0);
        acc* gout = weights ? r.w.part : g + c0 * Pn;
        s = r.grad_chunk(spins + c0 * m.S, n, weights ? weights + c0 : nullptr,
                         gout, logpsi ? logpsi + c0 : nullptr);
        if (s) return s;
        if (weights)
            LK("grad_reduce", launch_reduce_samples<acc>(n, Pn, r.w.part, g,
                                                         c0 > 0 ? 1 : 0, st));
    }
    return VQNQS_OK;
}

vqnqs_status grad_logpsi(const ModelDims& m, const void* params,
                         const int8_t* spins, int64_t batch,
                         const double* weights, void* grad, double* logpsi,
                         void* ws, size_t ws_bytes, hipStream_t st) {
    switch (m.precision) {
        case VQNQS_F64:
            return run_grad<PrecF64>(m, params, spins, batch, weights, grad,
                                     logpsi, ws, ws_bytes, st);
        case VQNQS_F32:
            return run_grad<PrecF32>(m, params, spins, batch, weights, grad,
                                     logpsi, ws, ws_bytes, st);
        default:
            return run_grad<PrecBF16>(m, params, spins, batch, weights, grad,
                                      logpsi, ws, ws_bytes, st);
    }
}

vqnqs_status neighbours(const ModelDims& m, const int8_t* spins, int64_t batch,
                        int16_t* bonds, int32_t* count, double* diag, void* ws,
                        size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < workspace_bytes(m, -2, 0)) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    Workspace<PrecF64> w = carve<PrecF64>(m, Job::Neighbours, 0, ws);
    CK(launch_fill_i32(w.status, 1, 0, st));
    LK("neighbours", launch_neighbours(spins, batch, m, bonds, count, diag, nullptr, w.status,
                         st));
    return VQNQS_OK;
}

// ------------------------------------------------------------ autotuner
// Times the rows-per-wave variants of the three matrix-core products on the
// caller's inputs (one local-energy evaluation per variant, after a warm-up
// run) and keeps the fastest, per model width.  Results never depend on
// these choices; only speed does.
static double class_ms(const char* cls) {
    constexpr int kMax = 64, kLen = 48;
    static char names[kMax * kLen];
    double ms[kMax];
    long long cnt[kMax];
    const int n = std::min(Profiler::get().read(names, kLen, ms, cnt, kMax), kMax);
    for (int i = 0; i < n; ++i)
        if (std::strncmp(names + i * kLen, cls, kLen) == 0) return ms[i];
    return 0.0;
}

vqnqs_status autotune(const ModelDims& m, const void* params,
                      const int8_t* spins, int64_t batch, int mode, void* ws,
                      size_t ws_bytes, hipStream_t st, int32_t* choices) {
    Tuning best = tuning_get(m);
    if (m.mfma && batch > 0) {
        const size_t eb = al256((size_t)batch * sizeof(double));
        if (ws_bytes <= eb) return VQNQS_ERR_WORKSPACE_TOO_SMALL;
        double* eloc = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                                 ws_bytes - eb);
        const size_t usable = ws_bytes - eb;
        Profiler& pf = Profiler::get();
        const bool was_on = pf.enabled();
        pf.enable(false);
        auto run = [&]() {
            return local_energy(m, params, spins, batch, mode, eloc, nullptr,
                                nullptr, nullptr, ws, usable, st);
        };
        vqnqs_status s = run();                    // warm-up
        if (s) return s;
        const char* cls[3] = {"qkv", "mlp", "vq"};
        for (int c = 0; c < 3; ++c) {
            double best_ms = -1.0;
            Tuning pick = best;
            for (int mb = 1; mb <= 4; mb *= 2) {
                Tuning t = best;
                (c == 0 ? t.qkv_mb : c == 1 ? t.mlp_mb : t.vq_mb) = mb;
                if (!tuning_valid(m, t)) continue;
                tuning_set(m, t);
                pf.reset();
                pf.enable(true);
                s = run();
                pf.enable(false);
                if (s) return s;
                if (hipStreamSynchronize(st) != hipSuccess) return VQNQS_ERR_HIP;
                const double ms = class_ms(cls[c]);
                if (best_ms < 0 || ms < best_ms) {
                    best_ms = ms;
                    pick = t;
                }
            }
            best = pick;
        }
        tuning_set(m, best);
        pf.reset();
        pf.enable(was_on);
    }
    if (choices) {
        choices[0] = best.qkv_mb;
        choices[1] = best.mlp_mb;
        choices[2] = best.vq_mb;
    }
    return VQNQS_OK;
}

// ---------------------------------------------------- multi-lattice batch
// Several lattices (each its own model and parameters) in one call.  Each
// job's kernel sequence goes to an internal stream forked from the caller's
// stream, so small lattices run beside large ones, and the whole fork/join
// sequence is captured once into a HIP graph that later identical calls
// replay (one launch instead of thousands).
namespace {

constexpr int kMaxJobStreams = 8;
constexpr size_t kStatusBytes = 256;   // combined status word of the call
constexpr size_t kMaxGraphs = 16;

struct Pools {
    std::mutex mu;
    std::map<int, std::vector<hipStream_t>> streams;
    std::map<int, std::vector<hipEvent_t>> events;
    struct Graph {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
        hipEvent_t done;   // recorded after every launch of exec
    };
    std::vector<Graph> graphs;
};

Pools& pools() {
    static Pools p;
    return p;
}

// Internal streams (default priority, non-blocking) and events of the
// current device, created on first use and kept until the process ends.
hipError_t job_streams(int ns, std::vector<hipStream_t>& st,
                       std::vector<hipEvent_t>& ev) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Pools& p = pools();
    std::lock_guard<std::mutex> lk(p.mu);
    auto& sv = p.streams[dev];
    while ((int)sv.size() < ns) {
        hipStream_t s;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking))) return e;
        sv.push_back(s);
    }
    auto& evv = p.events[dev];
    while ((int)evv.size() < ns + 1) {
        hipEvent_t x;
        if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming))) return e;
        evv.push_back(x);
    }
    st.assign(sv.begin(), sv.begin() + ns);
    ev.assign(evv.begin(), evv.begin() + ns + 1);
    return hipSuccess;
}

}  // namespace

size_t workspace_bytes_multi(const ModelDims* ms, const vqnqs_job* jobs,
                             int njobs, int mode) {
    size_t tot = kStatusBytes;
    for (int i = 0; i < njobs; ++i)
        tot += al256(workspace_bytes(ms[i], mode, std::max<int64_t>(jobs[i].batch, 1)));
    return tot;
}

// Workspace slices: every job gets its full need when the total fits, else
// its minimum plus a share of the rest proportional to what it lacks.
static bool split_workspace(const ModelDims* ms, const vqnqs_job* jobs,
                            int njobs, int mode, size_t ws_bytes,
                            std::vector<size_t>& off, std::vector<size_t>& len) {
    std::vector<size_t> need(njobs), mn(njobs);
    size_t tn = 0, tm = 0;
    for (int i = 0; i < njobs; ++i) {
        const int64_t b = std::max<int64_t>(jobs[i].batch, 1);
        need[i] = al256(workspace_bytes(ms[i], mode, b));
        mn[i] = al256(workspace_bytes(ms[i], mode, 1));
        tn += need[i];
        tm += mn[i];
    }
    if (ws_bytes < kStatusBytes || tm > ws_bytes - kStatusBytes) return false;
    ws_bytes -= kStatusBytes;
    const size_t extra = ws_bytes - tm, want = tn - tm;
    off.assign(njobs, 0);
    len.assign(njobs, 0);
    size_t o = kStatusBytes;
    for (int i = 0; i < njobs; ++i) {
        size_t l = need[i];
        if (tn > ws_bytes) {
            const double frac = want ? (double)(need[i] - mn[i]) / (double)want : 0.0;
            l = mn[i] + ((size_t)(frac * (double)extra) & ~(size_t)255);
            l = std::min(l, need[i]);
        }
        off[i] = o;
        len[i] = l;
        o += l;
    }
    return true;
}

static vqnqs_status run_jobs(const ModelDims* ms, const vqnqs_job* jobs,
                             int njobs, int mode, void* ws,
                             const std::vector<size_t>& off,
                             const std::vector<size_t>& len, bool concurrent,
                             hipStream_t st) {
    char* base = static_cast<char*>(ws);
    StatusOffsets so{};
    so.n = njobs;
    for (int i = 0; i < njobs; ++i) so.off[i] = (int64_t)off[i];
    if (!concurrent || njobs == 1) {
        for (int i = 0; i < njobs; ++i) {
            const vqnqs_job& j = jobs[i];
            vqnqs_status s = local_energy(ms[i], j.params, j.spins, j.batch,
                                          mode, j.eloc, j.stats, j.ratios,
                                          j.counters, base + off[i], len[i], st);
            if (s) return s;
        }
        CK(launch_or_status(base, so, st));
        return VQNQS_OK;
    }
    const int ns = std::min(njobs, kMaxJobStreams);
    std::vector<hipStream_t> js;
    std::vector<hipEvent_t> ev;
    CK(job_streams(ns, js, ev));
    CK(hipEventRecord(ev[ns], st));                  // fork
    for (int k = 0; k < ns; ++k) CK(hipStreamWaitEvent(js[k], ev[ns], 0));
    for (int i = 0; i < njobs; ++i) {
        const vqnqs_job& j = jobs[i];
        vqnqs_status s = local_energy(ms[i], j.params, j.spins, j.batch, mode,
                                      j.eloc, j.stats, j.ratios, j.counters,
                                      base + off[i], len[i], js[i % ns]);
        if (s) return s;
    }
    for (int k = 0; k < ns; ++k) {                   // join
        CK(hipEventRecord(ev[k], js[k]));
        CK(hipStreamWaitEvent(st, ev[k], 0));
    }
    CK(launch_or_status(base, so, st));
    return VQNQS_OK;
}

static std::vector<int64_t> graph_key(const ModelDims* ms, const vqnqs_job* jobs,
                                      int njobs, int mode, int flags, void* ws,
                                      size_t ws_bytes, hipStream_t st) {
    std::vector<int64_t> k = {mode, flags, (int64_t)(intptr_t)ws,
                              (int64_t)ws_bytes, (int64_t)(intptr_t)st, njobs};
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.push_back(dev);
    for (int i = 0; i < njobs; ++i) {
        const vqnqs_job& j = jobs[i];
        const vqnqs_config& c = j.cfg;
        const Tuning t = tuning_get(ms[i]);
        int64_t jb, gb;
        std::memcpy(&jb, &c.J, sizeof jb);
        std::memcpy(&gb, &c.gamma, sizeof gb);
        const int64_t f[] = {c.L, c.periodic, c.marshall, jb, c.hamiltonian, gb,
                             c.attn_tail, c.d_model,
                             c.n_layers, c.n_heads, c.d_ff, c.codebook_size,
                             c.vq_heads, c.precision, c.flags,
                             (int64_t)(intptr_t)j.params,
                             (int64_t)(intptr_t)j.spins, j.batch,
                             (int64_t)(intptr_t)j.eloc, (int64_t)(intptr_t)j.stats,
                             (int64_t)(intptr_t)j.ratios,
                             (int64_t)(intptr_t)j.counters, t.qkv_mb, t.mlp_mb,
                             t.vq_mb};
        k.insert(k.end(), std::begin(f), std::end(f));
    }
    return k;
}

vqnqs_status local_energy_multi(const ModelDims* ms, const vqnqs_job* jobs,
                                int njobs, int mode, int flags, void* ws,
                                size_t ws_bytes, hipStream_t st) {
    std::vector<size_t> off, len;
    if (!split_workspace(ms, jobs, njobs, mode, ws_bytes, off, len))
        return VQNQS_ERR_WORKSPACE_TOO_SMALL;
    const bool concurrent = (flags & VQNQS_MULTI_CONCURRENT) != 0;
    // the legacy default stream cannot be captured
    if (!(flags & VQNQS_MULTI_GRAPH) || st == nullptr)
        return run_jobs(ms, jobs, njobs, mode, ws, off, len, concurrent, st);
    const std::vector<int64_t> key =
        graph_key(ms, jobs, njobs, mode, flags, ws, ws_bytes, st);
    Pools& p = pools();
    {
        std::lock_guard<std::mutex> lk(p.mu);
        for (auto& g : p.graphs)
            if (g.key == key) {
                CK(hipGraphLaunch(g.exec, st));
                CK(hipEventRecord(g.done, st));
                return VQNQS_OK;
            }
    }
    Profiler& pf = Profiler::get();
    const bool was_on = pf.enabled();
    pf.enable(false);                 // no timing events inside a graph
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        pf.enable(was_on);
        return VQNQS_ERR_HIP;
    }
    vqnqs_status s = run_jobs(ms, jobs, njobs, mode, ws, off, len, concurrent, st);
    e = hipStreamEndCapture(st, &graph);
    pf.enable(was_on);
    if (s) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess || !graph) return VQNQS_ERR_HIP;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return VQNQS_ERR_HIP;
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return VQNQS_ERR_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(p.mu);
        if (p.graphs.size() >= kMaxGraphs) {
            // the evicted graph may still run on some stream: wait for its
            // last launch before its resources go
            Pools::Graph& old = p.graphs.front();
            (void)hipEventSynchronize(old.done);
            (void)hipGraphExecDestroy(old.exec);
            (void)hipEventDestroy(old.done);
            p.graphs.erase(p.graphs.begin());
        }
        p.graphs.push_back({key, exec, done});
    }
    CK(hipGraphLaunch(exec, st));
    CK(hipEventRecord(done, st));
    return VQNQS_OK;
}

}  // namespace vq
