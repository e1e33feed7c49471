/*
 * tlda.h -- C ABI of the MI355X (gfx950) online tensor-LDA hot path.
 *
 * The method (arXiv 2511.07809, "Scalable Tensor LDA") streams batches of
 * bag-of-words documents through
 *   1. the first moment M1 and the centred second moment M2~ (section
 *      "Computing the Centered Cumulants"),
 *   2. a whitening matrix W with W^T M2~ W = I (section "Online Decomposition
 *      of the Second Moment"),
 *   3. the centred, whitened batch X = (F_B - 1 M1^T) W, and
 *   4. a stochastic gradient step on the CP factors Phi of the whitened third
 *      moment, eq. vec_deriv, without forming any D x D x D or V x V x V tensor
 *      (section "Online Learning of the Third Moment"),
 * and finally unwhitens and re-centres the factors into topics (section
 * "Recovering the Topic Model Parameters", Theorem 1).
 *
 * Conventions for every call
 *  - Every function returns a tlda_status; nothing throws, aborts or prints.
 *    tlda_last_error() returns a message for the last failed call on a context.
 *  - Argument and shape errors are detected on the host before any work is
 *    enqueued, so a failed call leaves the context unchanged.
 *  - Device pointers are HIP device (HBM) addresses; host pointers are plain
 *    process memory.  The caller owns every pointer it passes; the library keeps
 *    none of them after the call returns.  The context owns its own device
 *    state (moment accumulators, W, scratch).
 *  - Work is enqueued on the context's HIP stream (given at creation) and is
 *    asynchronous unless a call says otherwise: outputs are valid once that
 *    stream has been synchronised.
 *  - Arrays are row-major.  A context is not thread-safe: use one per stream.
 *  - Documents with fewer than three tokens are dropped (the paper's
 *    pre-processing rule): they are not counted in N, contribute nothing to the
 *    moments, and their rows of a whitened batch are written as zeros.
 *  - The frequency vector of a document is f = c / L, its counts over its
 *    length L (the paper's notation table).
 */
#ifndef TLDA_H
#define TLDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlda_ctx tlda_ctx;

typedef enum {
  TLDA_OK = 0,
  TLDA_ERR_ARG = 1,      /* a NULL pointer, a bad flag or an out-of-range scalar   */
  TLDA_ERR_SHAPE = 2,    /* sizes that do not fit the context's V, K, D or limits  */
  TLDA_ERR_CSR = 3,      /* CSR content rejected by validation                     */
  TLDA_ERR_STATE = 4,    /* call order: e.g. whitening before any W exists         */
  TLDA_ERR_NUMERIC = 5,  /* M2~ has fewer than D positive eigenvalues, N == 0 ...  */
  TLDA_ERR_OOM = 6,      /* device allocation failed                               */
  TLDA_ERR_DEVICE = 7    /* a HIP runtime error                                    */
} tlda_status;

/* Limits of this library. */
#define TLDA_MAX_D 256
#define TLDA_MAX_K 256
#define TLDA_MAX_DK 16384   /* D * K: Phi must fit in a 64 KiB LDS tile */

/* tlda_config.flags */
#define TLDA_VALIDATE_CSR 0x1u  /* check every batch's CSR content (synchronous);
                                 * a rejection (TLDA_ERR_CSR) names the global
                                 * index first_doc + row of the first bad row */
/* BF16 precision for the per-document work (requires D, K <= 128, else
 * TLDA_ERR_SHAPE): the whitening gathers read a BF16 copy W16 = bf16(fp32(W))
 * with its own mean projection W16^T M1 (FP64), so X = (F - 1 M1^T) W16 is
 * formed and centred in FP32; the CP contractions X Phi and X^T (X Phi)^2
 * take BF16 operands (X, Phi, S^2, round to nearest even) with FP32
 * accumulation.  The eigensolver, W, the penalty term, the 3 c3 / n scaling,
 * the update, unwhitening and inference stay FP64/FP32.  tlda_whiten_batch,
 * tlda_cp_step and tlda_whiten_cp_step switch; their interfaces do not. */
#define TLDA_BF16 0x2u
/* Classic moments (the appendix's alpha0-corrected cumulants, used as an
 * estimator rung of the same batched SGD; requires D, K <= 128, else
 * TLDA_ERR_SHAPE).  FP32 per-document arithmetic, or with TLDA_BF16: the
 * data term then reads the BF16 whitening copy W16 (and W16^T M1), Z16 =
 * bf16(W16 Phi), and its reduction rows are rounded to BF16 for the matrix
 * cores with FP32 accumulation; the per-document sums and coefficients, the
 * refresh, the penalty and the update stay FP64/FP32.
 *  - tlda_update_moments accumulates the unbiased pair piece
 *    P2 = (c c^T - diag c) / (L (L - 1)) per kept document in place of f f^T,
 *    and a refresh whitens M2 = (alpha0 + 1) sum P2 / N - alpha0 M1 M1^T.
 *  - tlda_whiten_cp_step takes the data term of the gradient from the
 *    per-document piece of the appendix's third moment,
 *    M3_d = c3 P3_d - c2 (P2_d x M1 + its two permutations) + alpha0^2 M1^3
 *    (P3_d: ordered distinct token triples over L (L - 1) (L - 2);
 *    c2 = alpha0 (alpha0 + 1) / 2, c3 = (alpha0 + 1)(alpha0 + 2) / 2),
 *    contracted with (W, phi_k, phi_k) per document without forming it:
 *      G = 3(1+theta) Phi (Phi^T Phi * Phi^T Phi)
 *          - (3 / n) sum_d M3_d(W, W, W)(I, phi_k, phi_k).
 *    tlda_cp_step (which sees only X) returns TLDA_ERR_STATE.
 *  - tlda_unwhiten returns the orthogonal recovery: lambda_i =
 *    (1+theta)|phi_i|^3, mu_i = lambda_i (W^T)^+ phi_i / |phi_i|, alpha_i
 *    proportional to lambda_i^-2 (a zero column gets mu 0 and weight 0).
 *  - tlda_whiten_batch and inference keep their definitions (X = W^T (f - M1)
 *    with this W). */
#define TLDA_CLASSIC 0x4u

typedef struct {
  int32_t V;            /* vocabulary size, 3 <= V <= 131072                       */
  int32_t K;            /* number of topics, 1 <= K <= TLDA_MAX_K                   */
  int32_t D;            /* whitening size, 1 <= D <= min(V, TLDA_MAX_D), D*K bound;
                         * an FP32 context (neither TLDA_BF16 nor TLDA_CLASSIC) also
                         * needs Dq Kq + 4 (Dq + Kq) <= 16384 with Dq, Kq = D, K
                         * rounded up to multiples of 4 (Phi and a 4-row tile in
                         * 64 KiB of LDS): D = K = 120 passes, 128 x 128 does not */
  int32_t flags;        /* TLDA_VALIDATE_CSR | TLDA_BF16 | TLDA_CLASSIC            */
  double alpha0;        /* topic mixing parameter, > 0                             */
  double theta;         /* orthogonality penalty of eq. full_vec_pb, >= 0          */
  int32_t eig_iters;    /* subspace iterations of a refresh, 0 = default (60)      */
  int32_t eig_block;    /* subspace width D <= p <= min(V, 512), 0 = default      */
  uint64_t eig_seed;    /* seed of the refresh's start block                       */
  int32_t eig_warm_iters; /* subspace iterations of a warm refresh, 0 = default (4) */
} tlda_config;

/* One CSR batch of documents (rows) over the vocabulary (columns): the rows
 * of the paper's N x V input matrix (package section "Input and Output") for
 * documents first_doc .. first_doc + n_rows - 1.  Counts are positive
 * integer-valued floats <= 2^24; column indices are strictly increasing
 * within a row.  row_ptr[0] == 0, row_ptr[n_rows] == nnz.
 * slot < 0: the arrays are caller-owned device memory.  slot >= 0: the arrays
 * are a staging slot filled by tlda_stage_batch; consuming calls then wait for
 * that copy and release the slot when their work is done.  (Host batches are
 * only read by the staging calls, which return the device view; no other
 * call reads host memory, so the batch carries no memory-kind field.)
 * first_doc: global index of row 0 in the corpus (>= 0); the library uses it
 * only to name documents in its messages (a CSR rejection names the global
 * index of the first rejected row), and the staging calls carry it over. */
typedef struct {
  int32_t n_rows;
  int32_t nnz;
  const int32_t* row_ptr;   /* [n_rows + 1] */
  const int32_t* col_idx;   /* [nnz]        */
  const float* val;         /* [nnz]        */
  int32_t slot;
  int64_t first_doc;
} tlda_csr_batch;

/* Create a context whose work runs on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  Validates the configuration (TLDA_ERR_ARG / TLDA_ERR_SHAPE).
 * Device memory for the second moment is allocated on the first
 * tlda_update_moments call: the exact accumulator of its upper triangle
 * (8 V (V + 1) bytes) and, at the first refresh, the FP64 V x V matrix the
 * refresh multiplies (8 V^2 bytes); about 16 V^2 bytes in all (40 GB at
 * V = 50 000; TLDA_ERR_OOM when the device cannot hold them). */
tlda_status tlda_create(const tlda_config* cfg, void* hip_stream, tlda_ctx** out);
void tlda_destroy(tlda_ctx* ctx);
const char* tlda_status_str(tlda_status s);
const char* tlda_last_error(const tlda_ctx* ctx);

/* tlda_update_moments flags */
#define TLDA_REFRESH_W 0x1u   /* after accumulating, recompute M1, M2~ and W       */
#define TLDA_RESET 0x2u       /* clear the accumulators before accumulating        */
#define TLDA_RELEASE 0x4u     /* last: free the V x V accumulator, clear the counts */
#define TLDA_REFRESH_WARM 0x8u  /* refresh W starting from the previous refresh    */

/* Section "Computing the Centered Cumulants" and the batched implementation:
 * accumulates, over the kept documents of `batch` (may be NULL when only
 * refreshing), the document count N, the dropped-document count, exact int64
 * token totals per word, sum f and the upper triangle of sum f f^T (exact,
 * see below).  With TLDA_REFRESH_W it then forms M1 = sum f / N and
 * M2~ = (alpha0 + 1)(sum f f^T / N - M1 M1^T) and recomputes
 * W = U diag(lambda)^(-1/2) from the top-D eigenpairs of M2~ by FP64 block
 * subspace iteration with Rayleigh-Ritz (section "Online Decomposition of the
 * Second Moment": W^T M2~ W = I).  Eigenvectors are ordered by decreasing
 * eigenvalue and signed so that their largest-magnitude entry is positive.
 * A refresh synchronises the stream; it returns TLDA_ERR_NUMERIC if N == 0 or
 * the D-th eigenvalue is not positive (the previous W is then kept).
 * TLDA_RELEASE (last, synchronous) frees the V x V accumulator and clears N,
 * the totals and sum f, keeping W: for contexts that only step after their
 * refresh (e.g. many time slices, whose accumulators could not all stay
 * resident).  A later update allocates the accumulator again.
 * The sums of f and of the pairs are accumulated exactly in 128-bit fixed
 * point (each FP64 term truncated to a multiple of 2^-64), so the moments,
 * and every W refreshed from them, are the same bits whatever the order or
 * the batching of the documents. */
tlda_status tlda_update_moments(tlda_ctx* ctx, const tlda_csr_batch* batch, uint32_t flags);

/* TLDA_REFRESH_WARM (fully online mode, section "Fully Online, Incremental
 * Tensor LDA": the incremental PCA update after each new batch) refreshes W
 * like TLDA_REFRESH_W but starts the block subspace iteration from the
 * orthonormal block that the previous refresh of this context converged to,
 * and runs cfg.eig_warm_iters iterations (default 4) before the Rayleigh-Ritz
 * step: the running M2~ changes little per batch, so its dominant subspace is
 * tracked at a fraction of a cold refresh's cost.  Without a previous refresh
 * (or after tlda_load_state) it is a cold refresh.  Every refresh and every
 * tlda_set_whitening keeps the whitening it replaces for tlda_rebase_phi. */

/* Fully online mode: carry Phi [D][K] (device float, in place) from the
 * whitened space of the previous whitening W_old into that of the current W,
 * Phi <- W^T (W_old^T)^+ Phi = diag(eig)^(-1/2) U^T U_old diag(eig_old)^(1/2) Phi
 * (the paper keeps Phi across whitening updates without saying how; this maps
 * the factors' centred word-space vectors (W_old^T)^+ phi into the new
 * whitened coordinates).  FP64 arithmetic; TLDA_ERR_STATE when the context
 * has not replaced a whitening since it was created or loaded. */
tlda_status tlda_rebase_phi(tlda_ctx* ctx, float* Phi);

/* Whitened counts of the centred data (online second-moment section):
 * X[d, :] = W^T (f_d - M1) for kept rows, 0 for dropped rows.
 * X: device float [n_rows][D].  n_kept: device int32 (may be NULL) that
 * receives the number of kept rows of the batch (overwritten, not added).
 * Requires a W (TLDA_ERR_STATE otherwise). */
tlda_status tlda_whiten_batch(tlda_ctx* ctx, const tlda_csr_batch* batch, float* X, int32_t* n_kept);

/* Batched stochastic tensor gradient step, eq. vec_deriv and the update rule:
 *   G = 3(1+theta) Phi (Phi^T Phi * Phi^T Phi)
 *       - 3 (alpha0+1)(alpha0+2) / (2 n) X^T (X Phi * X Phi)
 *   Phi <- Phi - beta G
 * X: device float [n_rows][D] (dropped rows are zero and add nothing).
 * n_kept: device int32 with the batch's kept-row count n (as written by
 * tlda_whiten_batch), or NULL for n = n_rows.  When n == 0 the step is skipped.
 * Phi: device float [D][K], updated in place.  grad: device float [D][K] or
 * NULL.  The reduction order is fixed: results are bit-reproducible. */
tlda_status tlda_cp_step(tlda_ctx* ctx, const float* X, int32_t n_rows, const int32_t* n_kept,
                         float beta, float* Phi, float* grad);

/* The two calls above as one step, for the CP passes of the batched method:
 * the whitened rows of `batch` are formed in on-chip memory and used at once
 * by the gradient step (same definitions and results, up to FP32 rounding,
 * as tlda_whiten_batch followed by tlda_cp_step with the batch's kept-row
 * count), so X does not travel through HBM.  Phi: device float [D][K],
 * updated in place.  grad: device float [D][K] or NULL.  X_out: device float
 * [n_rows][D] or NULL (written only if given).  n_kept_out: device int32 or
 * NULL.  Requires a W (TLDA_ERR_STATE).  FP32 shapes outside the fused
 * kernel's range (D or K above 128) run the two calls in sequence through a
 * whitened-batch buffer of the context. */
tlda_status tlda_whiten_cp_step(tlda_ctx* ctx, const tlda_csr_batch* batch, float beta, float* Phi,
                                float* grad, float* X_out, int32_t* n_kept_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same step as
 * tlda_whiten_cp_step, same arguments and results up to the order of the FP32
 * partial sums, calling no allocating routine.  The reduction's per-block
 * partials go to one 16 MiB device array per GPU (4 Mi floats), held by the
 * library until the process ends, instead of the context's buffer that
 * tlda_whiten_cp_step grows on demand; the grid is capped at
 * floor(4 Mi / (D K)) blocks so that they fit (every block writes its whole
 * partial, so nothing needs clearing between calls).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (contexts on different
 * streams) race and must be ordered by the caller.  Covers BF16 contexts and
 * FP32 contexts with D, K <= 128 (FP32 shapes with D or K above 128 run two
 * calls through a whitened-batch buffer: TLDA_ERR_SHAPE); TLDA_ERR_ARG for classic-moment
 * contexts; TLDA_ERR_DEVICE if the array's device address could not be
 * found (it is looked up once per device by tlda_create). */
tlda_status tlda_whiten_cp_step_noalloc(tlda_ctx* ctx, const tlda_csr_batch* batch, float beta,
                                        float* Phi, float* grad, float* X_out,
                                        int32_t* n_kept_out);

/* tlda_unwhiten flags */
#define TLDA_PROJECT_SIMPLEX 0x1u  /* clip negative entries of mu and renormalise */

/* Section "Recovering the Topic Model Parameters" with Theorem 1, in this
 * reading for centred moments: E[M2~] = sum a_i nu_i nu_i^T with
 * sum a_i nu_i = 0 makes the whitened factors a tight frame,
 * a_i |W^T nu_i|^2 = 1 - a_i.  With w_i = (1+theta)^(1/3) phi_i, a_i is the
 * root in (0, 1] of a^(1/3) |w_i|^2 + a = 1, nu_i = (W^T)^+ a_i^(-1/3) w_i,
 * mu_i = nu_i + M1, alpha_i = a_i / sum_j a_j.
 * Phi: device float [D][K].  mu: device double [V][K].  alpha: device double
 * [K].  lambda: device double [K] or NULL, receives (1+theta)|phi_i|^3. */
tlda_status tlda_unwhiten(tlda_ctx* ctx, const float* Phi, double* mu, double* alpha,
                          double* lambda, uint32_t flags);

/* Document-topic proportions (package section "Input and Output": the N x K
 * document-topic output), as the minimiser over the probability simplex of
 * |x_d - A theta|^2 with x_d = W^T (f_d - M1) the whitened document and
 * A = W^T (mu - M1 1^T): projected gradient from theta = 1/K with step
 * 1 / lambda_max(A^T A), at most max_iter steps, stopping early when the L1
 * change of an iterate is below tol (tol = 0: exactly max_iter steps).
 * batch: the documents (device or staged); each is whitened as by
 * tlda_whiten_batch into the context's own buffer (grown on demand, which
 * synchronises the stream), then solved.  Dropped documents (fewer than
 * three tokens) have x_d = 0 and get the solve's value at x = 0.
 * mu: device double [V][K], e.g. from tlda_unwhiten.  theta_out: device float
 * [n_rows][K], rows on the simplex.  TLDA_ERR_STATE without a W. */
tlda_status tlda_infer_doc_topics(tlda_ctx* ctx, const tlda_csr_batch* batch, const double* mu,
                                  int32_t max_iter, float tol, float* theta_out);
/* The same solve for rows already whitened: X device float [n_rows][D] from
 * tlda_whiten_batch (or tlda_whiten_cp_step's X_out). */
tlda_status tlda_infer_doc_topics_whitened(tlda_ctx* ctx, const float* X, int32_t n_rows,
                                           const double* mu, int32_t max_iter, float tol,
                                           float* theta_out);

/* Streaming (batched implementation over data larger than device memory):
 * copy a CSR batch from pinned host memory (hipHostMalloc) into staging slot
 * `slot` (0 or 1) on the context's copy stream and return a device view of it
 * in *dev_out (dev_out->slot == slot).  The copy waits until every earlier
 * consumer of that slot has finished, and consumers of *dev_out wait for the
 * copy, so staging batch i+1 before consuming batch i overlaps the copy with
 * compute.  Slots grow on demand (TLDA_ERR_OOM on failure). */
tlda_status tlda_stage_batch(tlda_ctx* ctx, const tlda_csr_batch* host_batch, int32_t slot,
                             tlda_csr_batch* dev_out);

/* The compact staging format: the same CSR batch with 16-bit column indices
 * (the context's V <= 65536) and 16-bit counts (1 .. 65535), about half the
 * bytes of the 32-bit form over PCIe.  All arrays are pinned host memory. */
typedef struct {
  int32_t n_rows;
  int32_t nnz;
  const int32_t* row_ptr;   /* [n_rows + 1] */
  const uint16_t* col_idx;  /* [nnz]        */
  const uint16_t* val;      /* [nnz] counts */
  int64_t first_doc;        /* as in tlda_csr_batch, carried to the device view */
} tlda_csr_batch_u16;

/* tlda_stage_batch for a compact host batch: the 16-bit arrays are copied
 * and then widened on the device (on the copy stream, before the slot's ready
 * event) into the slot's 32-bit arrays, so *dev_out is an ordinary staged
 * batch.  TLDA_ERR_SHAPE when the context's V exceeds 65536. */
tlda_status tlda_stage_batch_u16(tlda_ctx* ctx, const tlda_csr_batch_u16* host_batch,
                                 int32_t slot, tlda_csr_batch* dev_out);

/* Inspection and test hooks (all synchronous; they change nothing but the
 * context's last-error message). */
/* N, dropped documents and the int64 token totals [V] (token_totals may be NULL). */
tlda_status tlda_get_stats(const tlda_ctx* ctx, int64_t* N, int64_t* n_skipped,
                           int64_t* token_totals);
/* Host copies: W [V][D], eigenvalues [D], M1 [V]; any may be NULL. */
tlda_status tlda_get_whitening(const tlda_ctx* ctx, double* W, double* eig, double* M1);
/* Install a whitening matrix W [V][D] (mutually orthogonal columns, as any
 * U diag(lambda)^(-1/2) has) and M1 [V] from host memory, e.g. computed by an
 * independent implementation; the eigenvalues are taken as 1/|w_d|^2. */
tlda_status tlda_set_whitening(tlda_ctx* ctx, const double* W, const double* M1);
/* ------------------------------------------------------------------------
 * Document-topic encoder: a d_in -> hidden -> hidden -> k_out perceptron
 * (GELU hidden layers, softmax output) that maps a whitened document x to
 * topic proportions on the simplex, standing in for the per-document solve of
 * tlda_infer_doc_topics, which stays as its judge and fallback
 * (tlda_infer_doc_topics_mlp).  Layers are X W + b with W stored input-major;
 * the matrix products run on BF16 matrix cores with FP32 accumulation (BF16
 * copies of FP32 master weights, BF16 activations, FP32 pre-activations);
 * gelu(z) = z Phi(z) with the standard normal distribution function Phi.
 * Training minimises the mean row cross-entropy -sum_k t_k log p_k against
 * target proportions t (e.g. solve outputs) with Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8).  Parameters are packed as W1 [d_in][hidden], b1 [hidden],
 * W2 [hidden][hidden], b2 [hidden], W3 [hidden][k_out], b3 [k_out] (FP32).
 * An encoder is bound to one HIP stream; it is not thread-safe.
 * ------------------------------------------------------------------------ */
#define TLDA_MLP_MAX_WIDTH 1024
typedef struct tlda_mlp tlda_mlp;

/* Number of packed parameters, or 0 for a non-positive width. */
int64_t tlda_mlp_param_count(int32_t d_in, int32_t hidden, int32_t k_out);
/* Create an encoder whose work runs on `hip_stream`; max_batch bounds the rows
 * of one training step (device scratch grows with it).  Parameters start at
 * zero: set them with tlda_mlp_set_params (the caller draws the
 * initialisation).  TLDA_ERR_SHAPE for widths outside 1 .. TLDA_MLP_MAX_WIDTH
 * (k_out <= TLDA_MAX_K). */
tlda_status tlda_mlp_create(int32_t d_in, int32_t hidden, int32_t k_out, int32_t max_batch,
                            void* hip_stream, tlda_mlp** out);
void tlda_mlp_destroy(tlda_mlp* mlp);
const char* tlda_mlp_last_error(const tlda_mlp* mlp);
/* Host copies of the packed FP32 parameters (synchronous).  Setting them
 * refreshes the BF16 copies and resets Adam's state. */
tlda_status tlda_mlp_set_params(tlda_mlp* mlp, const float* host_params);
tlda_status tlda_mlp_get_params(tlda_mlp* mlp, float* host_params);
/* theta_out [n_rows][k_out] = softmax(...) of X [n_rows][d_in] (device
 * float), in chunks of max_batch rows. */
tlda_status tlda_mlp_forward(tlda_mlp* mlp, const float* X, int64_t n_rows, float* theta_out);
/* Gradients of the mean cross-entropy of X against T [n_rows][k_out] (device
 * float, rows on the simplex), 1 <= n_rows <= max_batch: grads_out (device
 * float, packed like the parameters) and loss_out (device float); either may
 * be NULL. */
tlda_status tlda_mlp_gradients(tlda_mlp* mlp, const float* X, const float* T, int32_t n_rows,
                               float* grads_out, float* loss_out);
/* One Adam step with step size lr on the gradients of (X, T). */
tlda_status tlda_mlp_train_step(tlda_mlp* mlp, const float* X, const float* T, int32_t n_rows,
                                float lr, float* loss_out);
/* Document-topic proportions through the encoder, judged by the solve of
 * tlda_infer_doc_topics: each row starts at the encoder's output t (or at
 * 1/K when mlp is NULL: the plain solve under the same rule), takes
 * min_steps projected-gradient steps (each sets the smallest entries of the
 * softmax output to zero), then continues until the duality gap of
 * h(t) = |x - A t|^2 / 2 over the simplex, g.t - min_k g_k with
 * g = A^T (A t - x), which bounds h(t) - min h, is at most gap_tol, or
 * max_iter steps have been taken.  Rows that needed more than min_steps
 * steps (their refined encoder output failed the judge) are counted in
 * *n_stepped_out (device int32, or NULL).  The encoder must have d_in == D
 * and k_out == K and share the context's stream.  X: device float
 * [n_rows][D]; mu: device double [V][K]; theta_out: device float
 * [n_rows][K]. */
tlda_status tlda_infer_doc_topics_mlp(tlda_ctx* ctx, tlda_mlp* mlp, const float* X, int32_t n_rows,
                                      const double* mu, float gap_tol, int32_t min_steps,
                                      int32_t max_iter, float* theta_out,
                                      int32_t* n_stepped_out);

/* ------------------------------------------------------------------------
 * Batched time slices: many independent corpora (slices), each with its own
 * context (its own moments, whitening, K and Phi), stepped together.  A plan
 * fixes one CSR batch per slice; tlda_multi_step runs the same work as
 * tlda_whiten_cp_step on every slice's batch with two launches in all: one
 * persistent reduction launch whose blocks are laid out over the slices in
 * proportion to their row tiles, and one finish launch.  A sequence of steps
 * (e.g. a pass over every batch index) can be captured once in a HIP graph
 * and replayed.
 * ------------------------------------------------------------------------ */
typedef struct tlda_multi tlda_multi;
typedef struct tlda_graph tlda_graph;
/* ctxs: n_slices distinct BF16 contexts (TLDA_BF16) with D, K <= 64, a
 * whitening matrix, and one shared non-null stream.  batches: one device
 * batch per slice (caller-owned arrays that must stay valid while the plan
 * is used; staging slots are not accepted; n_rows may be 0, which leaves
 * that slice's Phi unchanged and its gradient zero).  Phis: distinct device
 * float [D_i][K_i], updated in place by each step.  betas: host [n_slices]
 * step sizes.  n_kept_out: device int32 [n_slices] or NULL, receives the
 * kept-row counts at each step.  Batches of contexts created with
 * TLDA_VALIDATE_CSR are validated once, here.  TLDA_ERR_SHAPE for a context
 * that is not BF16 or has D or K above 64; TLDA_ERR_ARG for a classic-moment
 * context (TLDA_CLASSIC: the multi-slice step is the centred one);
 * TLDA_ERR_STATE without a whitening matrix. */
tlda_status tlda_multi_create(int32_t n_slices, tlda_ctx* const* ctxs,
                              const tlda_csr_batch* batches, float* const* Phis,
                              const float* betas, int32_t* n_kept_out, tlda_multi** out);
void tlda_multi_destroy(tlda_multi* plan);
const char* tlda_multi_last_error(const tlda_multi* plan);
/* Launch shape: total reduction blocks over all slices (0 = one round of
 * resident blocks on the device, the default).  Synchronous. */
tlda_status tlda_multi_set_blocks(tlda_multi* plan, int32_t total_blocks);
tlda_status tlda_multi_get_blocks(const tlda_multi* plan, int32_t* total_blocks);
/* Tile shape of the reduction launch: documents per row tile x waves per
 * block, one of 64 x 4 (the default), 32 x 4 and 64 x 8 (TLDA_ERR_ARG
 * otherwise).  Setting it lays the blocks out again with one round of
 * resident blocks of that shape.  Synchronous. */
tlda_status tlda_multi_set_tile(tlda_multi* plan, int32_t rows_per_tile, int32_t waves_per_block);
tlda_status tlda_multi_get_tile(const tlda_multi* plan, int32_t* rows_per_tile,
                                int32_t* waves_per_block);
/* One step of every slice: two launches, the reduction over every slice's
 * batch and the finish (asynchronous on the contexts' stream). */
tlda_status tlda_multi_step(tlda_multi* plan);
/* Autotuner: times `reps` steps for every tile shape with each candidate
 * launch size (1, 2, ... resident blocks per CU of that shape, and two
 * rounds), keeps the fastest pair (read it back with tlda_multi_get_tile and
 * tlda_multi_get_blocks) and restores every Phi to its value at entry.
 * Synchronous. */
tlda_status tlda_multi_autotune(tlda_multi* plan, int32_t reps, int32_t* total_blocks_out);
/* Capture the steps of n_plans plans, in order, as one HIP graph on their
 * shared stream; tlda_graph_launch replays it (asynchronous).  A plan's
 * launch shape is frozen into the graph when it is captured. */
tlda_status tlda_graph_capture(tlda_multi* const* plans, int32_t n_plans, tlda_graph** out);
/* Capture n fused steps of one context, tlda_whiten_cp_step(ctx,
 * &batches[i], beta, Phi, NULL, NULL, NULL) for i = 0 .. n-1 in order, as one
 * HIP graph on the context's stream (a launch-bound pass over resident
 * batches then costs one launch).  The batches must be device batches
 * (slot < 0) that stay allocated while the graph lives; with
 * TLDA_VALIDATE_CSR they are validated once, before the capture.  Supported
 * for BF16 contexts and FP32 contexts within the fused kernel's shapes (D, K
 * <= 128), not classic ones (TLDA_ERR_SHAPE / TLDA_ERR_ARG); TLDA_ERR_ARG for a
 * context on the null stream.  Synchronous; the timing hook does not apply
 * to the captured launches. */
tlda_status tlda_graph_capture_steps(tlda_ctx* ctx, const tlda_csr_batch* batches, int32_t n,
                                     float beta, float* Phi, tlda_graph** out);
tlda_status tlda_graph_launch(tlda_graph* graph);
void tlda_graph_destroy(tlda_graph* graph);

/* Timing hook for profilers and benchmarks: `start` and `stop` are arrays of
 * n hipEvent_t (created by the caller with timing enabled; the caller keeps
 * ownership).  While set, each tlda_whiten_batch, tlda_cp_step and
 * tlda_whiten_cp_step call attaches the next pair (round robin) to the
 * dispatch of its main kernel (the whitening, the CP reduction or the fused
 * kernel), which records them when that kernel starts and ends, so
 * hipEventElapsedTime gives the kernel's own execution time.  n == 0
 * (arrays may be NULL) turns the hook off.  Not synchronous. */
tlda_status tlda_set_timing_events(tlda_ctx* ctx, void* const* start, void* const* stop,
                                   int32_t n);
/* Checkpoint of the moment state and W.  buf == NULL: *len receives the size.
 * The checkpoint records whether the moments are classic (TLDA_CLASSIC) or
 * centred; loading into a context of the other kind, or of another V, K or
 * D, is refused (TLDA_ERR_ARG / TLDA_ERR_SHAPE) with the context unchanged. */
tlda_status tlda_save_state(const tlda_ctx* ctx, void* buf, size_t* len);
tlda_status tlda_load_state(tlda_ctx* ctx, const void* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* TLDA_H */
