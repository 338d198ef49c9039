// Kernel launchers of the VQ-NQS library (internal header).
#pragma once
#include "common.h"

namespace vq {

// A set of rows of a row-major [rows][width] buffer: either the contiguous
// range [0, n) or the rows idx[0..n) of an index list, where n is the host
// value n_host or, when n_dev is set, the device value *n_dev (bounded above
// by n_host, which sizes the grid).
struct RowSet {
    const int64_t* idx;
    const int32_t* n_dev;
    int64_t n_host;
    int32_t mult;      // rows = (*n_dev) * mult when n_dev is set
};

// Per-row sources and destinations of one transformer block.
template <class P>
struct BlockIO {
    using act = typename P::act;
    using acc = typename P::acc;
    acc* x;            // residual rows (read, and written by the MLP stage)
    const acc* x_in;   // MLP-stage input rows (may equal x)
    act *q, *k, *v;    // projections
    act* a;            // attention output
    int32_t* codes;    // [row][H]
    acc* margin;       // [row][H] half gap of the two best distances, nullable
    acc* stat;         // [row][heads][2] softmax reference and normaliser of
                       // every attention row, nullable (full sequences only)
};

hipError_t launch_neighbours(const int8_t* spins, int64_t batch,
                             const ModelDims& m, int16_t* bonds,
                             int32_t* count, double* diag, int64_t* rows_cap,
                             int32_t* status, hipStream_t st);
hipError_t launch_scan_desc(const int16_t* bonds, const int32_t* count,
                            const int64_t* rows_cap, int n, int L, int chain,
                            int K, int enc,
                            int32_t* nb_off, int64_t* row_off,
                            int32_t* n_nb_total, int32_t* n_rows_total,
                            NbDesc* desc, hipStream_t st);
hipError_t launch_eloc(const double* diag, const int32_t* count,
                       const int32_t* nb_off, const double* r, int n, int N,
                       double h_off, double* eloc, double* ratios_out,
                       hipStream_t st);
hipError_t launch_stats(const double* e, int64_t n, double* stats,
                        hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st);
hipError_t launch_counter_add(int64_t* ctr, int slot, const int32_t* v,
                              int64_t scale, hipStream_t st);
hipError_t launch_counter_add_const(int64_t* ctr, int slot, int64_t v,
                                    hipStream_t st);
struct StatusOffsets {
    int n;
    int64_t off[64];
};
hipError_t launch_or_status(char* base, const StatusOffsets& so,
                            hipStream_t st);
hipError_t launch_copy_codes(const int32_t* src, int64_t n, int N, int H,
                             int nl, int l, int32_t* dst, hipStream_t st);
template <typename T>
hipError_t launch_copy_layer(const T* src, int64_t n, int64_t row, int nl,
                             int l, T* dst, hipStream_t st);

// ---- parameter preparation (tables, norms, BF16 packs)
template <class P>
hipError_t launch_prepare(const ModelDims& m, const LayerW<typename P::acc>& w,
                          typename P::acc* table, typename P::acc* cnorm,
                          bf16* Wqkv_p, bf16* W1_p, bf16* W2_p, bf16* cb_p,
                          hipStream_t st);

// ---- BF16 matrix-core path
// Rows per wave (16 * mb) of the QKV, MLP and quantizer products; results
// do not depend on them.  Process-wide, per model width.
struct Tuning {
    int qkv_mb, mlp_mb, vq_mb;
};
Tuning tuning_default(const ModelDims& m);
Tuning tuning_get(const ModelDims& m);
void tuning_set(const ModelDims& m, const Tuning& t);
bool tuning_valid(const ModelDims& m, const Tuning& t);
bool mfma_shapes_ok(const ModelDims& m);
hipError_t launch_round_bf16(const float* src, int64_t n, float* dst,
                             hipStream_t st);
hipError_t launch_pack_layer(const ModelDims& m, const LayerW<float>& w,
                             bf16* Wqkv_p, bf16* W1_p, bf16* W2_p, bf16* cb_p,
                             float* cnh, hipStream_t st);
hipError_t launch_qkv_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st);
hipError_t launch_mlp_mfma(const ModelDims& m, const LayerW<float>& w,
                           RowSet rows, const BlockIO<PrecBF16>& io,
                           hipStream_t st);
// Seed of a neighbour-row search: the sample's code of the same row and
// layer (codes [sample][N][H]), found through the row's owning neighbour.
struct VqSeed {
    const int32_t* slot_nb = nullptr;   // [rows] owning neighbour, or null
    const NbDesc* desc = nullptr;
    const int32_t* bcode = nullptr;
};
// y = GELU(x) by the matrix-core MLP's device function.
hipError_t launch_probe_gelu(const float* x, float* y, int64_t n, hipStream_t st);
hipError_t launch_vq_mfma(const ModelDims& m, const LayerW<float>& w,
                          RowSet rows, const BlockIO<PrecBF16>& io,
                          hipStream_t st, const VqSeed& seed = VqSeed{});
bool attn_mfma_ok(const ModelDims& m);
hipError_t launch_attn_seq_mfma(const ModelDims& m, const int32_t* n_dev,
                                int64_t n_seq, const BlockIO<PrecBF16>& io,
                                int64_t* ctr, hipStream_t st);

// ---- full-sequence forward pieces (samples or materialised neighbours)
hipError_t launch_materialise(const int8_t* spins, const NbDesc* desc,
                              const int32_t* n_dev, int64_t n_max, int N,
                              int8_t* out, hipStream_t st);
template <class P>
hipError_t launch_embed(const ModelDims& m, const HeadW<typename P::acc>& hw,
                        const int8_t* spins, const int32_t* n_dev,
                        int64_t n_seq, typename P::acc* x, hipStream_t st);
template <class P>
hipError_t launch_qkv(const ModelDims& m, const LayerW<typename P::acc>& w,
                      RowSet rows, const BlockIO<P>& io, hipStream_t st);
template <class P>
hipError_t launch_attention_seq(const ModelDims& m, const int32_t* n_dev,
                                int64_t n_seq, const BlockIO<P>& io,
                                int64_t* ctr, hipStream_t st);
template <class P>
hipError_t launch_vq(const ModelDims& m, const LayerW<typename P::acc>& w,
                     RowSet rows, const BlockIO<P>& io, hipStream_t st);
template <class P>
hipError_t launch_mlp(const ModelDims& m, const LayerW<typename P::acc>& w,
                      RowSet rows, const BlockIO<P>& io, hipStream_t st);
template <class P>
hipError_t launch_head_seq(const ModelDims& m, const HeadW<typename P::acc>& hw,
                           const int8_t* spins, const int32_t* n_dev,
                           int64_t n_seq, const typename P::acc* x,
                           typename P::acc* lp, double* logpsi,
                           hipStream_t st);

// ---- variational Monte Carlo step
hipError_t launch_vmc_weights(const double* eloc, const double* stats,
                              int64_t B, double* w, hipStream_t st);
template <typename T>
hipError_t launch_update(T* p, const T* g, T* m, T* v, int64_t n, double lr,
                         double b1, double b2, double eps, int64_t step,
                         hipStream_t st);

// ---- autoregressive sampling (one position of every sample per call)
template <class P>
hipError_t launch_sample_embed(const ModelDims& m,
                               const HeadW<typename P::acc>& hw, int64_t n,
                               int i, const int8_t* spins,
                               typename P::acc* x, int64_t* list,
                               double* lpsum, hipStream_t st);
template <class P>
hipError_t launch_attn_rows(const ModelDims& m, int64_t n, int i,
                            const BlockIO<P>& io, hipStream_t st);
template <class P>
hipError_t launch_sample_head(const ModelDims& m,
                              const HeadW<typename P::acc>& hw, int64_t n,
                              int i, const typename P::acc* x,
                              const double* uni, int8_t* spins, double* lpsum,
                              double* logpsi, hipStream_t st);

// ---- deduplicated neighbour evaluation
template <class P>
struct DedupIO {
    using act = typename P::act;
    using acc = typename P::acc;
    const NbDesc* desc;       // [n_nb]
    const int32_t* nb_off;    // [n+1] first neighbour of every sample
    int64_t n_samples;        // samples in the chunk
    const int32_t* n_nb;      // device count of neighbours in the chunk
    int64_t n_nb_max;
    const int32_t* n_rows;    // device: overlay rows of the chunk
    int64_t rows_max;
    const int8_t* spins;      // chunk samples [n][N]
    int32_t* slot_nb;         // [rows] owning neighbour of every overlay row
    int16_t* crow;            // [rows] rows of C of every neighbour, ascending,
                              // at the neighbour's overlay offset
    int32_t* ccnt;            // [n_nb] size of C of every neighbour
    // sample caches of the current layer: [n][N][...]
    const acc* bx;            // block input
    const act *bq, *bk, *bv, *ba;
    const int32_t* bcode;
    const acc* bmargin;       // [n][N][H][2] bounds on best / second distance
    const acc* wmax;          // [H] largest codeword norm per quantizer head
    // overlay rows of the neighbours: [rows][...]
    acc* ox;
    act *oq, *ok, *ov, *oa;
    int32_t* ocode;
    uint64_t* mask;           // [n_nb][W] rows in C (current layer)
    int mask_words;
    int64_t* list;            // rows of C (slots), capacity rows_max
    int32_t* list_n;          // device count
    int64_t* vq_list;         // rows needing a codebook search
    int32_t* vq_n;
};

template <class P>
hipError_t launch_dedup_init(const ModelDims& m, const HeadW<typename P::acc>& hw,
                             const DedupIO<P>& d, hipStream_t st);
template <class P>
hipError_t launch_attention_dedup(const ModelDims& m, const DedupIO<P>& d,
                                  int64_t* ctr, hipStream_t st);
// ---- attention-only half-block
template <class P>
hipError_t launch_out_proj(const ModelDims& m, const typename P::acc* Wo,
                           const typename P::acc* bo, RowSet rows,
                           const typename P::acc* x_in,
                           const typename P::act* a, typename P::acc* x_out,
                           hipStream_t st);
template <class P>
hipError_t launch_out_proj_overlay(const ModelDims& m,
                                   const typename P::acc* Wo,
                                   const typename P::acc* bo,
                                   const DedupIO<P>& dd,
                                   typename P::acc* out, hipStream_t st);
hipError_t launch_mask_from_pmin(const NbDesc* desc, const int32_t* n_nb,
                                 int64_t n_max, int W, int N, uint64_t* mask,
                                 hipStream_t st);
hipError_t launch_pack_qkv(const ModelDims& m, const float* W_qkv, bf16* out,
                           hipStream_t st);
hipError_t launch_pack_wo(const ModelDims& m, const float* W_o, bf16* out,
                          hipStream_t st);
// the half-block's output projection on the matrix core (BF16 mode)
hipError_t launch_oproj_mfma(const ModelDims& m, const float* bo,
                             const bf16* Wo_p, RowSet rows, const float* x_in,
                             const float* a, float* x_out, hipStream_t st);
hipError_t launch_oproj_overlay_mfma(const ModelDims& m, const float* bo,
                                     const bf16* Wo_p,
                                     const DedupIO<PrecBF16>& dd, float* out,
                                     hipStream_t st);
template <class P>
hipError_t launch_attention_incr(const ModelDims& m, const DedupIO<P>& d,
                                 const typename P::acc* bstat, int64_t* ctr,
                                 hipStream_t st);
template <class P>
hipError_t launch_certify(const ModelDims& m, const DedupIO<P>& d,
                          int certified, int64_t* ctr, hipStream_t st);
template <class P>
hipError_t launch_code_diff(const ModelDims& m, const DedupIO<P>& d,
                            hipStream_t st);
template <class P>
hipError_t launch_head_dedup(const ModelDims& m, const HeadW<typename P::acc>& hw,
                             const DedupIO<P>& d, const typename P::acc* blp,
                             const double* bell_unused, double* ratio,
                             int64_t* ctr, hipStream_t st);
hipError_t launch_attn_dedup_mfma(const ModelDims& m,
                                  const DedupIO<PrecBF16>& d, int64_t* ctr,
                                  hipStream_t st);
hipError_t launch_ratio_plain(const double* logpsi_nb, const double* logpsi_s,
                              const NbDesc* desc, const int32_t* n_dev,
                              int64_t n_max, double* ratio, hipStream_t st);

// ---- backward of log psi (straight-through quantizer, eqs. 7-8)
// C[g] = beta*C[g] + op(A[g]) op(B[g]), g < groups; op(A) M x K, op(B) K x N.
struct GemmDesc {
    int64_t M, N, K;
    const void* A;
    int64_t lda, sA;
    int tA;
    const void* B;
    int64_t ldb, sB;
    int tB;
    void* C;
    int64_t ldc, sC;
    int beta;
    int64_t groups;
    int b_exact;   // matrix-core form: B is bf16-exact (its lo part is zero)
};
template <typename T>
hipError_t launch_gemm(const GemmDesc& g, hipStream_t st);
// FP32 operands on the bf16 matrix core (hi/lo split, three passes)
hipError_t launch_gemm_mfma(const GemmDesc& g, hipStream_t st);
template <typename T>
hipError_t launch_colsum(int64_t groups, int64_t rows, int cols, const T* A,
                         int64_t lda, const T* B, int64_t ldb, T* out,
                         int64_t os, int beta, hipStream_t st);
template <typename T>
hipError_t launch_reduce_samples(int64_t n, int64_t P, const T* part, T* grad,
                                 int beta, hipStream_t st);
template <typename T>
hipError_t launch_coef(int64_t n, const double* w, T* coef, hipStream_t st);
template <typename T>
hipError_t launch_fill_t(T* p, int64_t n, T v, hipStream_t st);
template <typename T>
hipError_t launch_ln_save(int64_t R, int d, const T* x, const T* g, const T* b,
                          T* y, T* xh, T* rstd, hipStream_t st);
template <typename T>
hipError_t launch_ln_bwd(int64_t R, int d, const T* xh, const T* rstd,
                         const T* g, const T* dy, const T* base, T* out,
                         hipStream_t st);
template <typename T>
hipError_t launch_xprime(int64_t R, const ModelDims& m, const T* x,
                         const int32_t* codes, const T* table, const T* b_o,
                         const T* codebook, T* xp, T* z, hipStream_t st);
template <typename T>
hipError_t launch_bias_gelu(int64_t R, int F, T* u, const T* b1, T* g,
                            hipStream_t st);
template <typename T>
hipError_t launch_gelu_bwd(int64_t n, const T* u, T* dg, hipStream_t st);
template <typename T>
hipError_t launch_head_bwd(int64_t n, int N, int d, int K, int enc,
                           const HeadW<T>& hw,
                           const int8_t* spins, const T* x, const T* coef, T* f,
                           T* xh, T* rstd, T* dz, T* df, T* dx, hipStream_t st);
template <typename T>
hipError_t launch_embed_bwd(int64_t n, int N, int d, int K, int enc,
                            const int8_t* spins,
                            const T* dx, T* grad, int64_t P, int64_t tok_off,
                            int64_t pos_off, hipStream_t st);
template <typename T>
hipError_t launch_vq_bwd_rows(int64_t R, int Q, int dseg, int H, int h,
                              const T* a, int lda, const int32_t* codes,
                              const T* w2, T* S, T* E, T* rowG, hipStream_t st);
template <typename T>
hipError_t launch_da_fix(int64_t R, int dseg, int ld, const T* a,
                         const T* rowG, T* da, hipStream_t st);
template <typename T>
hipError_t launch_cb_fix(int64_t n, int Q, int dseg, const T* colG, const T* cb,
                         T* dcb, int64_t P, hipStream_t st);
template <typename T>
hipError_t launch_onehot_scatter(int64_t n, int N, int dseg, int ld, int H,
                                 int h, const int32_t* codes, const T* g,
                                 T* dcb, int64_t P, hipStream_t st);
template <typename T>
hipError_t launch_attn_bwd(int64_t n, const ModelDims& m, const T* q,
                           const T* k, const T* v, const T* o, const T* dO,
                           T* lse, T* Dd, T* dqkv, hipStream_t st);

}  // namespace vq
