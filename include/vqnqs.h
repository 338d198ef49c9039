/*
 * vqnqs.h - C ABI of the VQ-NQS local-energy library for MI355X (gfx950).
 *
 * The library evaluates a vector-quantized autoregressive transformer wave
 * function psi (Sharir, Chan, Anandkumar: "Towards Neural Variational Monte
 * Carlo That Scales Linearly with System Size", Sec. 3.1, eqs. 4-6) and the
 * variational Monte Carlo local energy of eq. (2),
 *
 *     E_loc(s) = sum_s' H_{s,s'} psi(s') / psi(s),
 *
 * for the spin-1/2 Heisenberg model H = J sum_<ij> S_i . S_j on an L x L
 * square lattice (Sec. 4), in the Marshall-rotated basis where the
 * off-diagonal element of every anti-aligned bond is -J/2 and psi > 0
 * (zero phase, Sec. 4).  The neighbours s' of a sample s are the
 * configurations with the two spins of one anti-aligned nearest-neighbour
 * bond exchanged (k-local rows, Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers marked DEVICE are device (HBM) addresses owned by the caller;
 * HOST pointers are ordinary host memory.  The library never allocates,
 * frees or keeps caller memory, and never synchronises the host: every
 * compute call only enqueues kernels on `stream` (a hipStream_t; NULL is the
 * legacy default stream) and returns.  Argument errors are detected on the
 * host before anything is enqueued and are returned as a status; a status of
 * VQNQS_ERR_HIP means a HIP runtime call failed while enqueueing.
 *
 * Spins: int8 array [batch][N], N = L*L, row-major sites i = r*L + c, values
 * +1 or -1.  Any other value sets VQNQS_ERR_BAD_SPIN in the device status
 * word of the workspace (read it with vqnqs_workspace_status); results for
 * such a batch are unspecified.
 *
 * Parameters: one flat DEVICE buffer in this order (row-major, every
 * matrix stored [in][out] and applied as x W; token 0 = spin +1, 1 = spin
 * -1, 2 = beginning of sequence):
 *     tok_emb[3][d]  pos_emb[N][d]
 *     per layer: ln1_g[d] ln1_b[d] W_qkv[d][3d] b_qkv[3d]
 *                codebook[H][Q][d/H] W_o[d][d] b_o[d] ln2_g[d] ln2_b[d]
 *                W1[d][d_ff] b1[d_ff] W2[d_ff][d] b2[d]
 *     with attn_tail = 1, the half-block: tail_ln_g[d] tail_ln_b[d]
 *         tail_W_qkv[d][3d] tail_b_qkv[3d] tail_W_o[d][d] tail_b_o[d]
 *     lnf_g[d] lnf_b[d] W_head[d][2] b_head[2]
 * The element type is double for VQNQS_F64 and float otherwise (FP32
 * master copy; the BF16 mode converts to bfloat16 inside the workspace).
 *
 * Network (Sec. 3.1): one token per spin, the input at position i is the
 * previous spin's token (beginning-of-sequence at i = 0); pre-LayerNorm
 * blocks  h = LN1(x), [q|k|v] = h W_qkv + b, a = causal MHSA(q,k,v),
 * z = VQ(a) (nearest codeword per quantizer head, lowest index on ties),
 * x' = x + z W_o + b_o, x = x' + W2 GELU(LN2(x') W1 + b1) + b2;  with
 * attn_tail = 1 an attention-only half-block follows (the networks of the
 * paper's Table 1 end with one; no quantizer, no MLP):
 * x = x + MHSA(LN(x) W_qkv + b) W_o + b_o;  final LN, head d->2,
 * log-softmax;  log psi(s) = 1/2 sum_i log P(s_i | s_<i).  In the dedup
 * form every row from the first changed input passes the half-block's
 * output projection.
 *
 * Workspace: a DEVICE buffer of ws_bytes bytes, 256-byte aligned.  The call
 * processes the batch in chunks of as many samples as fit; the minimum that
 * works is vqnqs_workspace_size(cfg, batch, mode, 1, &bytes).  Concurrent
 * calls must use distinct workspaces.  Identical inputs give bitwise
 * identical outputs.  (vqnqs_local_energy_static is the one entry point
 * without a workspace argument: it runs in a static device array of the
 * library's own.)
 */
#ifndef VQNQS_H
#define VQNQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VQNQS_OK = 0,
    VQNQS_ERR_NULL_POINTER = 1,      /* a required pointer is NULL            */
    VQNQS_ERR_INVALID_CONFIG = 2,    /* inconsistent vqnqs_config             */
    VQNQS_ERR_INVALID_SHAPE = 3,     /* batch < 0, or sizes out of range      */
    VQNQS_ERR_WORKSPACE_TOO_SMALL = 4,
    VQNQS_ERR_UNSUPPORTED = 5,       /* valid but not implemented (e.g. d/n_heads) */
    VQNQS_ERR_BAD_SPIN = 6,          /* a spin value other than +1/-1          */
    VQNQS_ERR_HIP = 7,               /* a HIP runtime call failed             */
    VQNQS_ERR_EXCEEDS_STATIC_SCRATCH = 8 /* one sample's workspace is larger
                                            than the library's static scratch */
} vqnqs_status;

typedef enum { VQNQS_F64 = 0, VQNQS_F32 = 1, VQNQS_BF16 = 2 } vqnqs_precision;

/* The two models of Sec. 4.  VQNQS_HEISENBERG_2D: H = J sum_<ij> S_i . S_j
 * on the L x L square lattice (N = L*L sites, neighbours = exchanges of
 * anti-aligned bonds, as described above).  VQNQS_TFIM_1D: the transverse-
 * field Ising chain H = -J sum_<ij> Z_i Z_j - Gamma sum_i X_i (Pauli
 * matrices) of N = L sites, bonds (i, i+1) and, periodic, (N-1, 0); the
 * neighbours of s are its N single-spin flips (k-local rows with k = 1,
 * Sec. 2) with element -Gamma, E_loc(s) = -J sum_<ij> s_i s_j
 * - Gamma sum_i psi(s^(i))/psi(s); marshall must be 0.  For the chain the
 * neighbour "bond" lists of vqnqs_neighbours hold the flipped sites. */
typedef enum { VQNQS_HEISENBERG_2D = 0, VQNQS_TFIM_1D = 1 } vqnqs_hamiltonian;

/* PLAIN re-evaluates psi from scratch on every neighbour (the definition of
 * eq. 2).  DEDUP reuses the sample's own evaluation and recomputes the
 * per-location operations only on rows whose input or VQ code differs
 * (Sec. 3.2); attention and the quantizer run on every row at or after the
 * first changed input, the rows before it being provably unchanged. */
typedef enum { VQNQS_PLAIN = 0, VQNQS_DEDUP = 1 } vqnqs_mode;

/* flags (DEDUP only): keep the sample's VQ code without a codebook search
 * when the attention output moved by less than half the gap between its
 * best and second-best code distances (exact by the triangle inequality,
 * with a floating-point allowance).  Results are unchanged by this flag. */
#define VQNQS_FLAG_CERTIFIED_VQ 1

/* flags (DEDUP only): the attention of the first layers by a rank-|C|
 * update of the sample's softmax instead of the dense overlay attention
 * (Sec. 3.2 names attention as the part that stays dense).  A query row
 * whose own input is unchanged sees the sample's keys except at the rows
 * C whose inputs changed, so its numerator and normaliser are the sample's
 * (kept by the sample's forward pass) with the terms of C replaced: cost
 * O(|C|) per row instead of O(i).  Changed query rows, and rows where the
 * removed weight exceeds half the normaliser (cancellation), are
 * evaluated in full.  VQNQS_INC_LAYERS(n) in the flags sets how many
 * leading layers use it (1..255; 0 means 2); deeper layers, whose changed
 * sets are larger, keep the dense attention.  Results agree with the dense
 * form to the rounding of the update; they are not bitwise equal to it.
 * FP64 and FP32 modes only (VQNQS_ERR_UNSUPPORTED in the BF16 mode, whose
 * matrix-core dense attention is faster than this vector-unit update). */
#define VQNQS_FLAG_INCREMENTAL_ATTN 2
#define VQNQS_INC_LAYERS(n) (((n) & 255) << 8)
#define VQNQS_INC_LAYERS_OF(flags) (((flags) >> 8) & 255)

typedef struct {
    int32_t L;             /* lattice side, N = L*L sites (3 <= L when periodic);
                              chain length N = L for VQNQS_TFIM_1D            */
    int32_t periodic;      /* 1 periodic, 0 open boundaries                      */
    int32_t marshall;      /* 1: off-diagonal -J/2 (needs a bipartite lattice)   */
    double  J;             /* exchange coupling                                  */
    int32_t d_model;       /* model width d                                      */
    int32_t n_layers;
    int32_t n_heads;       /* attention heads; d_model/n_heads in {4,8,16,32,64} */
    int32_t d_ff;          /* MLP width                                          */
    int32_t codebook_size; /* Q codes per quantizer head                         */
    int32_t vq_heads;      /* H quantizer heads; d_model % vq_heads == 0         */
    int32_t precision;     /* vqnqs_precision                                    */
    int32_t flags;         /* VQNQS_FLAG_*                                       */
    int32_t hamiltonian;   /* vqnqs_hamiltonian                                  */
    double  gamma;         /* transverse field Gamma (VQNQS_TFIM_1D)             */
    int32_t attn_tail;     /* 1: an attention-only half-block ends the model     */
    int32_t group;         /* K spins per token, 1..4 (0 reads as 1): tokens are
                              groups of K consecutive sites with 2^K values
                              (Sec. 3.1), T = N/K positions; N % K == 0.
                              Parameters: tok_emb [2^K + 1][d] (2^K = the
                              beginning-of-sequence token), pos_emb [T][d],
                              W_head [d][2^K], b_head [2^K].  Token value
                              sum_k b_k 2^k, b_k = 1 for spin -1 at the
                              token's k-th site.                            */
    int32_t encoder;       /* 1: the bidirectional encoder with mean pooling as
                              log psi (Sec. 3.1) in place of the decoder: the
                              tokens themselves as input (tok_emb [2^K][d], no
                              beginning-of-sequence token), attention over all
                              positions, log psi = mean_i LN(x_i) . w + b
                              (W_head [d][1], b_head [1]).  Not autoregressive:
                              vqnqs_sample and vqnqs_vmc_step return
                              VQNQS_ERR_UNSUPPORTED.  No half-block
                              (INVALID_CONFIG), no incremental attention
                              (UNSUPPORTED).                              */
} vqnqs_config;

/* Counters written by vqnqs_local_energy (int64, VQNQS_NCOUNTERS entries,
 * accumulated over the call; the call zeroes them first). */
#define VQNQS_NCOUNTERS 96
enum {
    VQNQS_CTR_SAMPLES = 0,      /* samples evaluated                        */
    VQNQS_CTR_NEIGHBOURS = 1,   /* sum of neighbour counts                  */
    VQNQS_CTR_ATTN_ROWS = 2,    /* query rows through attention, all layers */
    VQNQS_CTR_ATTN_PAIRS = 3,   /* (query, key) pairs through attention     */
    VQNQS_CTR_VQ_ROWS = 4,      /* rows with a full codebook search         */
    VQNQS_CTR_VQ_CERTIFIED = 5, /* rows whose code was certified unchanged  */
    VQNQS_CTR_QKV_ROWS = 6,     /* rows through LN1 + QKV projection        */
    VQNQS_CTR_MLP_ROWS = 7,     /* rows through out-projection + MLP        */
    VQNQS_CTR_HEAD_ROWS = 8,    /* rows through the output head             */
    VQNQS_CTR_TAIL_ROWS = 9,    /* rows through the half-block's projection */
    VQNQS_CTR_CHANGED0 = 16     /* [16 + l] = sum over neighbours of |C_l|,
                                   l = 0 (changed inputs) .. n_layers       */
};

/* Number of parameters of the flat buffer; < 0 for an invalid config. */
int64_t vqnqs_param_count(const vqnqs_config* cfg);

/* Workspace bytes needed to evaluate `batch` samples in `mode` processing
 * `chunk` samples at a time (chunk <= 0 means the whole batch at once).
 * mode is a vqnqs_mode for vqnqs_local_energy, VQNQS_WS_FORWARD for
 * vqnqs_forward_logpsi / vqnqs_neighbours, VQNQS_WS_GRAD for
 * vqnqs_grad_logpsi, VQNQS_WS_SAMPLE for vqnqs_sample, or VQNQS_WS_VMC
 * for vqnqs_vmc_step (its own per-step buffers hold the whole batch; the
 * calls inside the step run `chunk` samples at a time). */
#define VQNQS_WS_FORWARD (-1)
#define VQNQS_WS_GRAD (-3)
#define VQNQS_WS_SAMPLE (-4)
#define VQNQS_WS_VMC (-5)
vqnqs_status vqnqs_workspace_size(const vqnqs_config* cfg, int64_t batch,
                                  int32_t mode, int64_t chunk, size_t* bytes);

/* Neighbour enumeration (k-local rows, Sec. 2; Heisenberg bonds, Sec. 4).
 * Bonds are numbered b = 2*i + dir for site i = r*L + c, dir 0 linking
 * (r, c)-(r, c+1 mod L), dir 1 linking (r, c)-(r+1 mod L, c); open
 * boundaries drop the wrapping bonds.
 *   bonds [batch][2N] int16 DEVICE out: anti-aligned bond ids in increasing
 *         order, entries past count[b] set to -1
 *   count [batch]     int32 DEVICE out: number of anti-aligned bonds
 *   diag  [batch]     double DEVICE out, nullable: (J/4) sum_b s_i s_j      */
vqnqs_status vqnqs_neighbours(const vqnqs_config* cfg, const int8_t* spins,
                              int64_t batch, int16_t* bonds, int32_t* count,
                              double* diag, void* ws, size_t ws_bytes,
                              void* stream);

/* log psi(s) = 1/2 log P(s) for every sample (chain rule, Sec. 2; network
 * of Sec. 3.1).
 *   logpsi [batch] double DEVICE out
 *   codes  [batch][n_layers][N][vq_heads] int32 DEVICE out, nullable: the
 *          quantizer indices I_VQ of eq. (5) at every layer and position    */
vqnqs_status vqnqs_forward_logpsi(const vqnqs_config* cfg, const void* params,
                                  const int8_t* spins, int64_t batch,
                                  double* logpsi, int32_t* codes, void* ws,
                                  size_t ws_bytes, void* stream);

/* vqnqs_forward_logpsi that also returns every layer's attention output,
 * the vector the quantizer of eq. (5) receives (measurement support for
 * parity checks: a quantizer code is decided in floating point, and this
 * output lets a caller check a code against the input it was chosen for).
 *   attn [batch][n_layers][N][d] DEVICE out: double for VQNQS_F64, float
 *        otherwise (the BF16 mode keeps activations in FP32)
 *   logpsi, codes: as for vqnqs_forward_logpsi (codes nullable)
 * Workspace, errors and results otherwise as vqnqs_forward_logpsi. */
vqnqs_status vqnqs_forward_activations(const vqnqs_config* cfg,
                                       const void* params,
                                       const int8_t* spins, int64_t batch,
                                       double* logpsi, int32_t* codes,
                                       void* attn, void* ws, size_t ws_bytes,
                                       void* stream);

/* Local energy of eq. (2) for every sample, in `mode`.
 *   eloc     [batch] double DEVICE out
 *   stats    [2] double DEVICE out, nullable: batch mean and (biased)
 *            variance of E_loc (the estimator of eq. 1 for Born samples)
 *   ratios   [batch][2N] double DEVICE out, nullable: psi(s')/psi(s) per
 *            neighbour in bond order (entries past the count are 0)
 *   counters [VQNQS_NCOUNTERS] int64 DEVICE out, nullable: work counters   */
vqnqs_status vqnqs_local_energy(const vqnqs_config* cfg, const void* params,
                                const int8_t* spins, int64_t batch,
                                int32_t mode, double* eloc, double* stats,
                                double* ratios, int64_t* counters, void* ws,
                                size_t ws_bytes, void* stream);

/* Direct sampling of s ~ |psi(s)|^2 = P(s) through the chain rule
 * P(s) = prod_i P(s_i | s_<i) of the autoregressive network (Sec. 2: the
 * distribution supports exact sampling at the cost of evaluating it).
 * Position by position, row i of every sample goes through every layer
 * (the keys and values of positions < i are kept per layer), and the head's
 * conditional decides s_i = +1 iff uniforms[b][i] < P(s_i = +1 | s_<i),
 * compared in FP64.  The random numbers are the caller's, so a call is
 * deterministic.  No Sz = 0 constraint is imposed.
 *   uniforms [batch][N] double DEVICE in: numbers in [0, 1), one per site
 *   spins    [batch][N] int8 DEVICE out: the samples (+1 / -1)
 *   logpsi   [batch] double DEVICE out, nullable: log psi of every sample,
 *            1/2 the sum of the drawn conditionals' logs in site order
 *            (the same sum vqnqs_forward_logpsi forms)
 * Workspace: vqnqs_workspace_size(cfg, batch, VQNQS_WS_SAMPLE, chunk, ..). */
vqnqs_status vqnqs_sample(const vqnqs_config* cfg, const void* params,
                          const double* uniforms, int64_t batch,
                          int8_t* spins, double* logpsi, void* ws,
                          size_t ws_bytes, void* stream);

/* One variational Monte Carlo step (Sec. 2): direct samples s_i ~ psi^2
 * (vqnqs_sample with the caller's uniform numbers), their local energies
 * (eq. 2, deduplicated form), the energy gradient
 *     dE/dtheta = (2/B) sum_i (E_loc(s_i) - mean E_loc) d log psi(s_i)/dtheta
 * (eq. 3 for a real psi, as a batch mean; the straight-through gradient of
 * vqnqs_grad_logpsi), and the parameter update, all enqueued on `stream`.
 *   params    DEVICE in/out, the flat parameters (element type as for
 *             vqnqs_local_energy), updated in place
 *   opt_state DEVICE in/out, nullable: NULL = gradient descent,
 *             theta -= lr g; else Adam (b1 = 0.9, b2 = 0.999, eps = 1e-8)
 *             with its first and second moments [2][P] in the parameters'
 *             type (zero them before step 1)
 *   step      Adam step number t >= 1 (bias correction 1 - b^t)
 *   lr        learning rate
 *   uniforms  [batch][N] double DEVICE in, numbers in [0, 1)
 *   spins     [batch][N] int8 DEVICE out, nullable: this step's samples
 *   eloc      [batch] double DEVICE out, nullable: their local energies
 *   stats     [2] double DEVICE out, nullable: mean and variance of E_loc
 *             (the energy estimate of the parameters before the update)
 * Workspace: vqnqs_workspace_size(cfg, batch, VQNQS_WS_VMC, chunk, ..). */
vqnqs_status vqnqs_vmc_step(const vqnqs_config* cfg, void* params,
                            void* opt_state, int64_t step, double lr,
                            const double* uniforms, int64_t batch,
                            int8_t* spins, double* eloc, double* stats,
                            void* ws, size_t ws_bytes, void* stream);

/* Gradient of log psi with respect to the flat parameters, with the
 * straight-through quantizer of eqs. (7)-(8): the forward value is the
 * nearest codeword; the backward passes the gradient g reaching the
 * quantized vector to the chosen codeword (the codebook factor of
 * g(D)^T W, whose value is the one-hot vector: the stop gradient of eq. 8
 * acts on the softmax output only) and through the distances inside
 * p = softmax(-||u - W_j||) to every codeword of that quantizer head and
 * to the attention output u (softmax term).  Everything else
 * is differentiated exactly (log psi = 1/2 log P, Sec. 2).  The forward
 * keeps only every layer's input; each layer is recomputed with the forward
 * kernels (same codes) before its backward (layer checkpointing).
 *   weights [batch] double DEVICE in, nullable:
 *       non-NULL: grad[P] = sum_i weights[i] d log psi(s_i)/d theta
 *                 (the form a variational gradient step needs, Sec. 2)
 *       NULL:     grad[batch][P], one gradient per sample
 *   grad    DEVICE out, the parameters' element type (double for VQNQS_F64,
 *           float otherwise); P = vqnqs_param_count(cfg)
 *   logpsi  [batch] double DEVICE out, nullable: log psi of every sample
 * In the BF16 mode the forward and its recompute run on the matrix core at
 * the bfloat16-rounded parameters, the backward in FP32.  Workspace:
 * vqnqs_workspace_size(cfg, batch, VQNQS_WS_GRAD, chunk, &bytes); the
 * per-sample gradients of a chunk are held in it (P values per sample).
 * The weighted sum is accumulated over samples in a fixed order. */
vqnqs_status vqnqs_grad_logpsi(const vqnqs_config* cfg, const void* params,
                               const int8_t* spins, int64_t batch,
                               const double* weights, void* grad,
                               double* logpsi, void* ws, size_t ws_bytes,
                               void* stream);

/* Local energy (same arguments, results and errors as vqnqs_local_energy)
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops, harnesses that forbid allocation.  The workspace
 * is the library's own static device array of VQNQS_STATIC_SCRATCH_MIB MiB
 * (one per device, held from the first call on that device until the
 * process ends); the call allocates and frees nothing.  The batch is
 * processed in chunks of as many samples as the array holds, so any batch
 * size works as long as one sample's workspace,
 * vqnqs_workspace_size(cfg, 1, mode, 1, &bytes), fits; otherwise the call
 * returns VQNQS_ERR_EXCEEDS_STATIC_SCRATCH before enqueueing anything.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (several streams or threads) race and give undefined results;
 * calls ordered on one stream are safe.  The array keeps the last call's
 * contents; the call initialises everything it reads.
 *   status [1] int32 DEVICE out, nullable: the call's status word once the
 *          enqueued work has run (VQNQS_OK or VQNQS_ERR_BAD_SPIN), the value
 *          vqnqs_workspace_status reports for a caller's workspace      */
#define VQNQS_STATIC_SCRATCH_MIB 512
vqnqs_status vqnqs_local_energy_static(const vqnqs_config* cfg,
                                       const void* params,
                                       const int8_t* spins, int64_t batch,
                                       int32_t mode, double* eloc,
                                       double* stats, double* ratios,
                                       int64_t* counters, int32_t* status,
                                       void* stream);

/* One lattice of a multi-lattice batch: its own model, parameters and
 * samples, with the outputs of vqnqs_local_energy (same meanings). */
typedef struct {
    vqnqs_config cfg;
    const void* params;     /* DEVICE, flat parameters of this model        */
    const int8_t* spins;    /* DEVICE [batch][N]                            */
    int64_t batch;
    double* eloc;           /* DEVICE out [batch]                           */
    double* stats;          /* DEVICE out [2], nullable                     */
    double* ratios;         /* DEVICE out [batch][2N], nullable             */
    int64_t* counters;      /* DEVICE out [VQNQS_NCOUNTERS], nullable       */
} vqnqs_job;

/* flags of vqnqs_local_energy_multi */
#define VQNQS_MULTI_CONCURRENT 1   /* each job on its own internal stream   */
#define VQNQS_MULTI_GRAPH 2        /* capture once, replay as a HIP graph   */

/* Workspace for vqnqs_local_energy_multi to hold every job's whole batch;
 * any smaller workspace that holds every job's one-sample minimum also
 * works (the jobs are then chunked). */
vqnqs_status vqnqs_workspace_size_multi(const vqnqs_job* jobs, int32_t njobs,
                                        int32_t mode, size_t* bytes);

/* Local energies (eq. 2) of several lattices in one call: the batched
 * launch of a mixed-lattice sample set.  The workspace is split between
 * the jobs in proportion to their needs.  With VQNQS_MULTI_CONCURRENT every
 * job's kernels run on an internal stream (created on first use, default
 * priority, kept until the process ends) forked from and joined back to
 * `stream`, so small lattices fill the device beside large ones.  With
 * VQNQS_MULTI_GRAPH the whole sequence is captured into a HIP graph on the
 * first call and replayed by later calls with identical arguments (same
 * pointers, sizes, stream and tuning), one launch in place of thousands;
 * the graph reads the buffers' current contents at every replay.  The
 * legacy NULL stream cannot be captured: the call then runs directly.
 * The library keeps the 16 most recently captured graphs; capturing a 17th
 * drops the oldest once its last launch has finished (the host waits for
 * it: the one case in which this call synchronises).
 * Results equal those of one vqnqs_local_energy call per job, bit for bit.
 * Calls that overlap on one device must not share a workspace; the internal
 * streams are shared, so such calls also serialise. */
vqnqs_status vqnqs_local_energy_multi(const vqnqs_job* jobs, int32_t njobs,
                                      int32_t mode, int32_t flags, void* ws,
                                      size_t ws_bytes, void* stream);

/* Autotuner (measurement, not part of the method): times the rows-per-wave
 * variants of the BF16 matrix-core products (QKV projection, MLP, codebook
 * search) with one local-energy evaluation of the given samples per
 * variant, and keeps the fastest for every later call on a model of this
 * width (process-wide).  Results never depend on these choices.  The call
 * synchronises `stream` and clears the totals of vqnqs_profile_*.
 * Needs the workspace of vqnqs_local_energy plus 8 bytes per sample.
 *   choices [3] int32 HOST out, nullable: rows per wave / 16 of the QKV,
 *           MLP and codebook-search kernels now in force */
vqnqs_status vqnqs_autotune(const vqnqs_config* cfg, const void* params,
                            const int8_t* spins, int64_t batch, int32_t mode,
                            void* ws, size_t ws_bytes, void* stream,
                            int32_t* choices);

/* Sets the rows-per-wave choices (as returned by vqnqs_autotune) for
 * models of this width; VQNQS_ERR_INVALID_CONFIG for a choice the width
 * does not allow (QKV and MLP: 1 or 2 below model width 256, 1 at 256;
 * codebook search: 1, 2 or 4 up to segment width 128, 1 or 2 below 256,
 * 1 at 256). */
vqnqs_status vqnqs_set_tuning(const vqnqs_config* cfg, const int32_t* choices);

/* Reads the device status word of a workspace used by a previous call:
 * synchronises `stream`, then returns VQNQS_OK or VQNQS_ERR_BAD_SPIN. */
vqnqs_status vqnqs_workspace_status(const void* ws, void* stream);

const char* vqnqs_status_string(vqnqs_status s);

/* Measurement support (not part of the method).  When enabled, every kernel
 * launch of the library is bracketed by HIP events recorded on the launch
 * stream; vqnqs_profile_read waits for them and returns, per kernel class,
 * the summed device time in milliseconds and the number of launches.
 *   names [max][name_len] HOST out, nullable; total_ms [max], count [max]
 *   HOST out, nullable.  Returns the number of kernel classes (may exceed
 *   max).  Process-wide; not for concurrent use from several threads. */
void vqnqs_profile_enable(int on);
void vqnqs_profile_reset(void);
int  vqnqs_profile_read(char* names, int name_len, double* total_ms,
                        long long* count, int max);

/* Measurement support: the rate at which the device's vector units issue
 * the FP32 exponential (v_exp_f32), the operation that bounds attention
 * at small head widths (one exponential per query-key pair).  Runs
 * independent exponential chains on every SIMD (about 0.1 s), timed with
 * HIP events on `stream`; synchronises the stream.
 *   sink       DEVICE, one float the kernel writes (keeps the chains live)
 *   exps_per_s HOST out: exponentials per second over the whole device  */
vqnqs_status vqnqs_probe_exp_rate(float* sink, void* stream,
                                  double* exps_per_s);

/* Introspection: y[i] = GELU(x[i]) = x Phi(x) for FP32 values, by the same
 * device function the BF16 mode's matrix-core MLP applies to its hidden
 * layer (Sec. 3.1 block: MLP with a GELU; erf from Abramowitz & Stegun
 * 7.1.26, absolute error of erf at most 1.5e-7), so that tests can bound
 * its error against the exact erf form.  Asynchronous on `stream`.
 *   x  DEVICE [n] FP32 in;  y  DEVICE [n] FP32 out (may equal x)
 * Errors: NULL_POINTER for null x or y with n > 0, INVALID_SHAPE for n < 0. */
vqnqs_status vqnqs_probe_gelu(const float* x, float* y, int64_t n,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VQNQS_H */
