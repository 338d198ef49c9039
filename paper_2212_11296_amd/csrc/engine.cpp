// Host orchestration: workspace planning and kernel sequencing for the
// forward pass, the plain and the deduplicated local energy.
#include "engine.h"

#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "profiler.h"

namespace vq {

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t param_count(const ModelDims& m);

// Worst case, over all configurations, of the overlay rows one sample needs:
// every bond anti-aligned, each neighbour keeping rows p1+1 .. N-1.
static int64_t max_overlay_rows(const ModelDims& m) {
    int64_t tot = 0;
    const int L = m.L, N = m.N;
    for (int b = 0; b < 2 * N; ++b) {
        const int i = b >> 1, r = i / L, c = i % L;
        int j;
        if ((b & 1) == 0) {
            if (!m.periodic && c + 1 == L) continue;
            j = r * L + (c + 1) % L;
        } else {
            if (!m.periodic && r + 1 == L) continue;
            j = ((r + 1) % L) * L + c;
        }
        tot += N - std::min(i, j) - 1;
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
    size_t bytes;
};

enum class Job { Forward, Plain, Dedup, Neighbours };

template <class P>
static Workspace<P> carve(const ModelDims& m, Job job, int64_t chunk,
                          void* base) {
    using acc = typename P::acc;
    using act = typename P::act;
    Workspace<P> w{};
    Carver c;
    c.base = static_cast<char*>(base);
    const int64_t n = chunk, N = m.N, d = m.d, H = m.H;
    const int64_t nbmax = n * 2 * N;
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
        }
    }
    w.bonds = c.take<int16_t>(n * 2 * N);
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
    w.desc = c.take<NbDesc>(nbmax);
    w.ratio = c.take<double>(nbmax);
    w.logpsi_s = c.take<double>(n);
    const bool dedup = job == Job::Dedup;
    const int64_t nlc = dedup ? m.nl : 1;       // cached layers
    const int64_t nlx = dedup ? m.nl + 1 : 1;   // block inputs + final
    w.bx = c.take<acc>(nlx * n * N * d);
    w.bq = c.take<act>(nlc * n * N * d);
    w.bk = c.take<act>(nlc * n * N * d);
    w.bv = c.take<act>(nlc * n * N * d);
    w.ba = c.take<act>(nlc * n * N * d);
    w.bcode = c.take<int32_t>(nlc * n * N * H);
    if (dedup) {
        w.bmargin = c.take<acc>(nlc * n * N * H * 2);
        w.blp = c.take<acc>(n * N * 2);
    }
    if (job == Job::Plain) {
        w.logpsi_nb = c.take<double>(nbmax);
        w.nspins = c.take<int8_t>(nbmax * N);
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

size_t workspace_bytes(const ModelDims& m, int mode, int64_t chunk) {
    const Job job = mode == VQNQS_PLAIN   ? Job::Plain
                    : mode == VQNQS_DEDUP ? Job::Dedup
                    : mode == -2          ? Job::Neighbours
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
    hi = std::min<int64_t>(hi, ((int64_t)1 << 30) / (2 * m.N));
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
    const C* b = p + 3 * d + N * d + per * l;
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

template <typename C>
static HeadW<C> head_view(const ModelDims& m, const C* p) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    HeadW<C> h{};
    h.tok = p;
    h.pos = p + 3 * d;
    const C* t = p + 3 * d + N * d + per * m.nl;
    h.lnf_g = t;
    h.lnf_b = t + d;
    h.W_head = t + 2 * d;
    h.b_head = t + 2 * d + 2 * d;
    return h;
}

int64_t param_count(const ModelDims& m) {
    const int64_t d = m.d, N = m.N, Q = m.Q, F = m.dff;
    const int64_t per = 2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d +
                        d * F + F + F * d + d;
    return 3 * d + N * d + per * m.nl + 2 * d + 2 * d + 2;
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
    hipError_t vqs(const LayerW<acc>& lw, RowSet rs, const BlockIO<P>& io) {
        if constexpr (std::is_same<P, PrecBF16>::value)
            if (m.mfma) return launch_vq_mfma(m, lw, rs, io, st);
        return launch_vq<P>(m, lw, rs, io, st);
    }
    HeadW<acc> head() const { return head_view<acc>(m, params); }

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
                                         const_cast<bf16*>(lw.cb_p), st));
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
    };

    vqnqs_status forward(const SeqBufs& b, const int32_t* n_dev, int64_t n,
                         bool count_rows) {
        const int64_t rows = n * m.N, sd = rows * m.d, sh = rows * m.H;
        LK("embed", launch_embed<P>(m, head(), b.spins, n_dev, n, b.x, st));
        for (int l = 0; l < m.nl; ++l) {
            const int64_t cl = b.cache ? l : 0;
            BlockIO<P> io{};
            io.x = b.x + (b.cache ? (int64_t)(l + 1) * sd : 0);
            io.x_in = b.x + (b.cache ? (int64_t)l * sd : 0);
            io.q = b.q + cl * sd;
            io.k = b.k + cl * sd;
            io.v = b.v + cl * sd;
            io.a = b.a + cl * sd;
            io.codes = b.code + cl * sh;
            io.margin = b.margin ? b.margin + cl * sh * 2 : nullptr;
            RowSet rs{nullptr, n_dev, rows, (int32_t)m.N};
            BlockIO<P> qio = io;
            qio.x = const_cast<acc*>(io.x_in);
            LK("qkv", qkv(layer(l), rs, qio));
            LK("attention_seq", attn_seq(n_dev, n, io, count_rows ? ctr : nullptr));
            LK("vq", vqs(layer(l), rs, io));
            LK("mlp", mlp(layer(l), rs, io));
            if (b.codes_out)
                LK("copy_codes", launch_copy_codes(io.codes, n, m.N, m.H, m.nl, l, b.codes_out, st));
        }
        const acc* xf = b.x + (b.cache ? (int64_t)m.nl * sd : 0);
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

    vqnqs_status neighbours(const int8_t* spins, int64_t n) {
        LK("neighbours", launch_neighbours(spins, n, m, w.bonds, w.count, w.diag, w.rows_cap,
                             w.status, st));
        LK("scan_desc", launch_scan_desc(w.bonds, w.count, w.rows_cap, (int)n, m.L, w.nb_off,
                            w.row_off, w.n_nb, w.n_rows, w.desc, st));
        if (ctr) {
            CK(launch_counter_add_const(ctr, VQNQS_CTR_SAMPLES, n, st));
            CK(launch_counter_add(ctr, VQNQS_CTR_NEIGHBOURS, w.n_nb, 1, st));
        }
        return VQNQS_OK;
    }

    vqnqs_status plain_chunk(const int8_t* spins, int64_t n) {
        vqnqs_status s = neighbours(spins, n);
        if (s) return s;
        SeqBufs sb{spins, w.bx, w.bq, w.bk, w.bv, w.ba, w.bcode, nullptr,
                   nullptr, w.logpsi_s, false, nullptr};
        s = forward(sb, nullptr, n, true);
        if (s) return s;
        const int64_t nbmax = n * 2 * m.N;
        LK("materialise", launch_materialise(spins, w.desc, w.n_nb, nbmax, m.N, w.nspins, st));
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
        SeqBufs sb{spins, w.bx, w.bq, w.bk, w.bv, w.ba, w.bcode, w.bmargin,
                   w.blp, w.logpsi_s, true, nullptr};
        s = forward(sb, nullptr, n, true);
        if (s) return s;
        const int64_t nbmax = n * 2 * N;
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
            LK("attention_dedup", attn_dedup(dd));
            if (certified) {
                CK(launch_fill_i32(w.vq_n, 1, 0, st));
                LK("certify", launch_certify<P>(m, dd, 1, ctr, st));
                RowSet vr{w.vq_list, w.vq_n, R, 1};
                LK("vq", vqs(lw, vr, io));
                if (ctr) CK(launch_counter_add(ctr, VQNQS_CTR_VQ_ROWS, w.vq_n, 1, st));
            } else {
                RowSet vr{nullptr, w.n_rows, R, 1};
                LK("vq", vqs(lw, vr, io));
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
    const double h_off = m.marshall ? -0.5 * m.J : 0.5 * m.J;
    for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
        const int64_t n = std::min(chunk, batch - c0);
        const int8_t* sp = spins + c0 * m.N;
        s = mode == VQNQS_PLAIN ? r.plain_chunk(sp, n) : r.dedup_chunk(sp, n);
        if (s) return s;
        LK("eloc", launch_eloc(r.w.diag, r.w.count, r.w.nb_off, r.w.ratio, (int)n, m.N,
                       h_off, eloc + c0,
                       ratios ? ratios + c0 * 2 * m.N : nullptr, st));
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
                                double* logpsi, int32_t* codes, void* ws,
                                size_t ws_bytes, hipStream_t st) {
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
        const int8_t* sp = spins + c0 * m.N;
        // spin validation shares the neighbour kernel
        LK("neighbours", launch_neighbours(sp, n, m, r.w.bonds, r.w.count, nullptr, nullptr,
                             r.w.status, st));
        typename Runner<P>::SeqBufs sb{
            sp, r.w.bx, r.w.bq, r.w.bk, r.w.bv, r.w.ba, r.w.bcode, nullptr,
            nullptr, logpsi + c0, false,
            codes ? codes + c0 * (int64_t)m.nl * m.N * m.H : nullptr};
        s = r.forward(sb, nullptr, n, false);
        if (s) return s;
    }
    return VQNQS_OK;
}

vqnqs_status forward_logpsi(const ModelDims& m, const void* params,
                            const int8_t* spins, int64_t batch, double* logpsi,
                            int32_t* codes, void* ws, size_t ws_bytes,
                            hipStream_t st) {
    switch (m.precision) {
        case VQNQS_F64:
            return run_forward<PrecF64>(m, params, spins, batch, logpsi, codes,
                                        ws, ws_bytes, st);
        case VQNQS_F32:
            return run_forward<PrecF32>(m, params, spins, batch, logpsi, codes,
                                        ws, ws_bytes, st);
        default:
            return run_forward<PrecBF16>(m, params, spins, batch, logpsi, codes,
                                         ws, ws_bytes, st);
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

}  // namespace vq
