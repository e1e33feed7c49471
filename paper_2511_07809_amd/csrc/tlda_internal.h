// Internal declarations shared by the translation units of libtlda.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/tlda.h"

namespace tlda {

// Floats of the allocation-free step's partial buffer (16 MiB per device).
constexpr size_t kNoAllocFloats = size_t(4) << 20;

// Per-block count scratch: the whitening and the moment kernels cap their
// grids at this many blocks (the moment kernel stores two counts per block).
constexpr int kWhitenBlockCounts = 2048;

// Row stride (floats) of the FP32 whitening copy used for the gathers of the
// whitening SpMM: rows are aligned to a 128-byte cache line once D >= 32, and
// to a power of two of at least one float4 below that.
inline int padded_d(int D) {
  if (D >= 32) return (D + 31) / 32 * 32;
  int p = 4;
  while (p < D) p <<= 1;
  return p;
}

struct StageSlot {
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;
  float* val = nullptr;
  size_t cap_rows = 0, cap_nnz = 0;
  uint16_t* col16 = nullptr;    // compact staging copies (tlda_stage_batch_u16)
  uint16_t* val16 = nullptr;
  size_t cap16 = 0;
  hipEvent_t ready = nullptr;   // recorded on the copy stream after the copy
  hipEvent_t free_ = nullptr;   // recorded on the compute stream after consumers
  bool used = false;
};

// Moment accumulators.  fsum and acc hold exact 128-bit fixed-point sums
// ({lo, hi} pairs of 64-bit words, value hi + lo 2^-64), so the moments do
// not depend on the order documents are added in; S2 is the FP64 symmetric
// matrix the refresh forms from acc (k_fx_symmetric) for its products.
struct Moments {
  unsigned long long* counts = nullptr;  // [0] N kept, [1] dropped
  unsigned long long* totals = nullptr;  // [V] token totals of kept documents
  unsigned long long* fsum = nullptr;    // [V][2] sum of f over kept documents
  unsigned long long* acc = nullptr;     // [V (V + 1) / 2][2] packed upper triangle of sum f f^T
  double* S2 = nullptr;                  // [V][V] FP64 symmetric copy, formed at each refresh
};
// 64-bit words of the packed fixed-point accumulator of a V-word vocabulary
inline size_t tri_words(int V) { return (size_t)V * (V + 1); }

struct Whitening {
  bool ready = false;
  double* W = nullptr;     // [V][D]
  double* U = nullptr;     // [V][D]
  double* eig = nullptr;   // [D]
  double* m = nullptr;     // [V]
  float* W32 = nullptr;    // [V][Dp]
  float* mw32 = nullptr;   // [Dp], W^T M1
  uint16_t* W16 = nullptr; // [V][Dh] BF16 bits of fp32(W) (BF16 contexts only)
  float* mw16 = nullptr;   // [Dh], W16^T M1 from the rounded values
  // the whitening this one replaced (for tlda_rebase_phi)
  bool prev_ready = false;
  double* Uprev = nullptr;   // [V][D]
  double* eigprev = nullptr; // [D]
  double* C = nullptr;       // [D][D] U^T Uprev
};

struct EigScratch {
  int p = 0;
  double* Q = nullptr;     // [V][p]
  double* Y = nullptr;     // [V][p]
  double* G = nullptr;     // [p][p]  Gram / projected matrix
  double* Z = nullptr;     // [p][p]  eigenvectors of the projected matrix
  double* ev = nullptr;    // [p]
  double* t = nullptr;     // [p]     M1^T Q
  double* Binv = nullptr;  // [p][p]  inverse-transpose Cholesky factor
  double* sel = nullptr;   // [D + p*D] selected Ritz values and vectors
  double* mcand = nullptr; // [V]     M1 of the refresh in progress
  int* info = nullptr;     // [4]     device status words
  double* warm = nullptr;  // Q or Y: the orthonormal block the last refresh converged to
  double* part = nullptr;  // [part_chunks][p][p] partial sums of the Gram products
  int part_chunks = 0;     // min(kSplitMax, ceil(V / 64)): the most row chunks gemm() uses
  double* ws = nullptr;    // [splits][V][p] K-split partials of the S2 product
  size_t ws_doubles = 0;
};

// Launch-shape knobs (0 = built-in choice).  Initialised from the
// environment (TLDA_TUNE_CP_BLOCKS, TLDA_TUNE_WHITEN_V4, TLDA_TUNE_WHITEN_CHUNKS)
// when a context is created (and TLDA_TUNE_FUSED_BLOCKS: grid of the fused
// whitening + CP kernel, default one full round of resident blocks;
// TLDA_TUNE_BF16_BLOCKS: the same for the BF16 kernels).  cp_max_blocks: grid of the CP reduction
// (default: one full round of resident blocks); whiten_v4: float4 columns
// per lane (1 or 2); whiten_chunks: XCD column chunks (1, 2, 4, 8; -1 = by
// W size); gemm_route (TLDA_TUNE_GEMM): 1 runs the refresh's dense products
// on the library's vector-ALU tile kernel instead of the FP64 matrix cores.
struct Tuning {
  int cp_max_blocks = 0;
  int fused_blocks = 0;
  int bf16_blocks = 0;
  int bf16_resident[3] = {0, 0, 0};   // cached occupancy rounds of the BF16 kernels
  int classic_resident = 0;           // the same for the classic-moment kernel
  int classic16_resident = 0;         // and its BF16 variant
  int whiten_v4 = 0;
  int whiten_chunks = 0;
  int gemm_route = 0;                 // refresh products: 0 built-in choice, 1 the vector kernel
};

struct CpScratch {
  size_t cap = 0;             // floats available in partial
  float* partial = nullptr;   // [nblk][D][K]
  double* R1 = nullptr;       // [D][K]
  float* phi0 = nullptr;      // [D][K] copy of Phi taken by the reduction kernels
  float* grad = nullptr;      // [D][K] used when the caller passes no gradient buffer
  float* X = nullptr;         // [cap_x] whitened batch for the unfused fallback
  size_t cap_x = 0;
  float* Z = nullptr;         // [V][Kp] W Phi of the classic-moment step
  float* rz = nullptr;        // [Kp]    Phi^T W^T M1 of the classic-moment step
  uint16_t* Z16 = nullptr;    // [V][Kh] bf16(W16 Phi) of the BF16 classic-moment step
  double* gsq = nullptr;      // [K][K] squared Gram entries of Phi (large D x K only)
};

}  // namespace tlda

struct tlda_ctx {
  tlda_config cfg;
  int Dp = 0;
  int Dt = 0;                 // columns of W32's tail copy (0: none)
  int Dh = 0;                 // row stride of the BF16 whitening copy
  hipStream_t stream = nullptr;
  hipStream_t copy_stream = nullptr;
  int device = 0;
  int num_cu = 0;
  tlda::Moments mom;
  tlda::Whitening wh;
  tlda::EigScratch eig;
  tlda::CpScratch cp;
  tlda::Tuning tune;
  tlda::StageSlot slots[2];
  double* post = nullptr;     // [K] scratch for unwhiten
  double* postA = nullptr;    // [D][K] inference matrix
  double* postG = nullptr;    // [K][K]
  double* postZ = nullptr;    // [K][K]
  double* postEv = nullptr;   // [K]
  float* A32 = nullptr;       // [D][K]
  float* G32 = nullptr;       // [K][K]
  float* step32 = nullptr;    // [1]
  int* dev_flags = nullptr;   // [4] CSR validation and inference status words
  int* block_counts = nullptr;  // [2 * kWhitenBlockCounts] per-block document counts
  // timing hook: event pairs recorded around the main kernel of each hot-path call
  hipEvent_t* t_start = nullptr;
  hipEvent_t* t_stop = nullptr;
  int t_n = 0, t_next = 0;
  bool in_capture = false;    // capturing a graph of steps: no validation, no timing hook
  mutable std::string last_error;   // also set by the const inspection calls
  // device address of the allocation-free step's partial buffer on this
  // context's device (null, with the runtime's message, if the lookup failed)
  float* noalloc = nullptr;
  std::string noalloc_error;
};

// Document-topic encoder: d_in -> hidden -> hidden -> k_out MLP (GELU,
// softmax), FP32 master parameters with BF16 copies for the matrix cores.
struct tlda_mlp {
  int d_in = 0, hidden = 0, k_out = 0, max_batch = 0;
  size_t n_params = 0;
  hipStream_t stream = nullptr;
  float* params = nullptr;     // [n_params] FP32 master, packed W1 b1 W2 b2 W3 b3
  uint16_t* wb = nullptr;      // BF16 copies of W1, W2, W3 (same offsets as in params)
  float* grads = nullptr;      // [n_params]
  float* adam_m = nullptr;     // [n_params]
  float* adam_v = nullptr;     // [n_params]
  long long adam_t = 0;
  float* Z1 = nullptr;         // [max_batch][hidden] FP32 pre-activations
  float* Z2 = nullptr;
  uint16_t* H1 = nullptr;      // [max_batch][hidden] BF16 activations
  uint16_t* H2 = nullptr;
  float* logits = nullptr;     // [max_batch][k_out]
  uint16_t* dZ3 = nullptr;     // [max_batch][k_out] BF16
  uint16_t* dZa = nullptr;     // [max_batch][hidden] BF16 (dZ2, then dZ1)
  uint16_t* dZb = nullptr;
  float* row_loss = nullptr;   // [max_batch]
  float* ws = nullptr;         // split partials of the weight and bias gradients
  std::string last_error;
};

namespace tlda {

// One slice's share of a multi-slice step (device-side table entry): its
// batch, BF16 whitening copy, shapes, Phi, scratch, and which blocks of the
// reduction launch (blk0 .. blk0 + nblk - 1) and of the finish launch
// (fin0 ..) serve it.
struct SliceStep {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  int n_rows;
  const uint16_t* W16;
  const float* mw16;
  int Dh, D, K, shape;
  float* Phi;            // read by the reduction (copied to phi_copy), written by the finish
  float* phi_copy;
  float* partial;        // [nblk][D][K]
  int* block_counts;     // [nblk]
  int nblk, blk0, fin0;
  float* grad;           // [D][K]
  double* R1;            // [D][K]
  int* n_kept_out;       // or null
  double alpha0, theta;
  float beta;
};
constexpr int multi_shape_id(int dq, int kq, int g) { return dq * 10000 + kq * 100 + g; }

// Timing hook of the main kernel of a hot-path call: the API stores a pair
// of events here right before launching it, and launch_main records them as
// part of that kernel's dispatch (hipExtLaunchKernelGGL), so their interval
// is the kernel's own execution.  The first launch_main consumes the pair.
struct KernelTimer {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local KernelTimer g_main_timer;

// Environment of the refresh's dense FP64 products, set by the API around a
// refresh or rebase (EigScope).  route 0: C = A B on the FP64 matrix cores
// (k_dgemm_mfma), with a K split over ws (splits x M x N doubles) when the
// grid would not fill the device; route 1: the vector-ALU tile kernel.
// The transposed products A^T B over many rows (the refresh's Gram products)
// split their rows into up to kSplitMax chunks, each writing its own M x N
// partial to `part`, added in chunk order afterwards (deterministic).
constexpr int kSplitMax = 256;
struct EigEnv {
  int route = 0;
  double* part = nullptr;     // part_chunks * part_mn doubles
  size_t part_mn = 0;         // largest M * N the scratch serves
  int part_chunks = 0;        // row chunks the scratch holds (at most kSplitMax)
  double* ws = nullptr;       // K-split workspace of the matrix-core product
  size_t ws_doubles = 0;
  int num_cu = 256;
};
extern thread_local EigEnv g_eig_env;
struct EigScope {
  EigEnv prev;
  explicit EigScope(const EigEnv& e) : prev(g_eig_env) { g_eig_env = e; }
  ~EigScope() { g_eig_env = prev; }
};
// K-split count of the matrix-core product C (M x N) = A (M x K) B: the count
// in 1 .. 8 (chunks of at least 1024) that fills the rounds of resident
// blocks best.
int dgemm_splits(int M, int N, int K, int num_cu);

template <typename... Params, typename... Args>
inline void launch_main(void (*kernel)(Params...), dim3 grid, dim3 block, unsigned shmem,
                        hipStream_t s, Args... args) {
  const KernelTimer t = g_main_timer;
  g_main_timer = KernelTimer{};
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u,
                        static_cast<Params>(args)...);
}

// ---- kernel launchers (one translation unit each) ----
// zero-fill with a kernel (no memset nodes, so callers may capture the work)
hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s);
// moments
// err[0] != 0 when some row is rejected; err[1] = n_rows - (first rejected
// row) then (err[0..1] zeroed by the caller)
hipError_t launch_validate_csr(const tlda_csr_batch& b, int V, int* err, hipStream_t s);
// block_counts: scratch for 2 * kWhitenBlockCounts ints
// classic: S2 takes the unbiased pair piece (c c^T - diag c) / (L (L - 1))
// instead of f f^T
hipError_t launch_accumulate(const tlda_csr_batch& b, int V, const Moments& m, int* block_counts,
                             bool classic, hipStream_t s);   // adds into m.acc, m.fsum, m.totals
// S2 (V x V, FP64, symmetric) from the packed fixed-point accumulator
hipError_t launch_fx_symmetric(const unsigned long long* acc, int V, double* S2, hipStream_t s);
// col[j] = col16[j], val[j] = val16[j] for j < nnz (compact staging)
hipError_t launch_widen_u16(const uint16_t* col16, const uint16_t* val16, size_t nnz,
                            int32_t* col, float* val, hipStream_t s);
hipError_t launch_mean(const unsigned long long* fsum, const unsigned long long* counts, double* m,
                       int V,
                       hipStream_t s);
// eigen-solver building blocks (FP64)
hipError_t launch_random_block(double* Q, int V, int p, uint64_t seed, hipStream_t s);
hipError_t launch_m2_apply(const double* S2, const double* m, const double* t, const double* Q,
                           double* Y, int V, int p, double scale_s, double scale_m,
                           hipStream_t s);
hipError_t launch_gram(const double* A, const double* B, double* G, int V, int p, hipStream_t s);
hipError_t launch_vecT_mat(const double* m, const double* Q, double* t, int V, int p,
                           hipStream_t s);
hipError_t launch_cholesky(double* G, int p, double shift_rel, int* info, hipStream_t s);
hipError_t launch_trsm_right_into(const double* Y, const double* G, double* Binv, double* Out, int V,
                                  int p, hipStream_t s);
hipError_t launch_jacobi(double* A, double* Z, double* ev, int p, int* info, hipStream_t s);
// Out (V x p) = Q (V x p) Z (p x p)
hipError_t launch_block_product(const double* Q, const double* Z, double* Out, int V, int p,
                                hipStream_t s);
hipError_t launch_ritz_vectors(const double* Q, const double* Z, const double* ev, int V, int p,
                               int D, double* U, double* eigD, hipStream_t s);
hipError_t launch_form_whitening(const double* U, const double* eig, const double* m, int V, int D,
                                 int Dp, double* W, float* W32, float* mw32, hipStream_t s);
hipError_t launch_from_injected(const double* W, int V, int D, double* U, double* eig,
                                hipStream_t s);
// whitening SpMM
// block_counts: scratch for kWhitenBlockCounts ints
hipError_t launch_whiten(const tlda_csr_batch& b, const float* W32, const float* mw32, int V, int D,
                         int Dp, float* X, int* n_kept, int* block_counts, const Tuning& t,
                         hipStream_t s);
int whiten_chunks(int V, int Dp);
// CP step
// The reduction kernels also copy Phi into phi_copy (D*K floats), which the
// finish kernel reads while it writes Phi.
hipError_t launch_cp_reduce(const float* X, int n_rows, const float* Phi, int D, int K, int nblk,
                            float* partial, float* phi_copy, hipStream_t s);
// n = sum of counts[0 .. ncounts), or n_default when counts is NULL; gsq
// (K x K squared Gram entries of Phi0 from launch_gram_sq) or NULL, in which
// case the finish forms the ones it needs itself
hipError_t launch_cp_finish(const float* partial, int nblk, const int* counts, int ncounts,
                            int n_default, const float* Phi0, int D, int K, double alpha0,
                            double theta, float beta, float* Phi, float* grad, double* R1,
                            int* n_out, const double* gsq, hipStream_t s);
// gsq[j][k] = (phi_j . phi_k)^2 in FP64 for Phi (D x K)
hipError_t launch_gram_sq(const float* Phi, int D, int K, double* gsq, hipStream_t s);
// From this many entries of Phi on, the squared Gram entries are formed once
// per step instead of by every finish block
constexpr int kGramOnceDK = 4096;
int cp_tile_rows(int D, int K);
int mfma_bucket(int n);
int cp_mfma_tile_rows(int D, int K);
// fused whitening + CP reduction
bool fused_supported(int D, int K, int Dp);
int fused_tile_rows(int D, int K);        // row tile of the fused kernel for this shape
// With partial == nullptr, launch_whiten_cp only stores in *block_counts how
// many blocks of the kernel it would launch can be resident on one CU.
// Dt > 0: W32 also holds, from element tail_base on, a [V][Dt] copy of the
// columns past the last whole 128-byte line of each row (w32_tail_cols).
// gsq != nullptr: the kernel also forms the K x K squared Gram entries of
// Phi for the finish (shapes where fused_forms_gram holds: the wide and the
// hybrid kernels; others ignore it).
hipError_t launch_whiten_cp(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                            int Dp, int Dt, uint32_t tail_base, const float* Phi, int K,
                            int nblk, float* partial, int* block_counts, float* Xout,
                            float* phi_copy, double* gsq, hipStream_t s);
bool fused_forms_gram(int D, int K);
// Columns of the tail copy that the wide FP32 fused kernels read instead of a
// row's last, mostly empty 128-byte line: D mod 32 rounded up to 4 when that
// is 1 to 8 and the shape takes a wide kernel, else 0 (no tail copy).
int w32_tail_cols(int D, int K);
// W32[tail_base + w Dt + j] = W32[w Dp + 32 floor(D / 32) + j], j < Dt.
hipError_t launch_w32_tail(float* W32, int V, int D, int Dp, int Dt, uint32_t tail_base,
                           hipStream_t s);
int cp_num_blocks(int n_rows, int D, int K, int max_blocks);
hipError_t launch_sum_counts(const int* block_counts, int n, int* out, hipStream_t s);
// multi-slice step: reduction over every slice's batch, then every slice's finish
// (sl: device table; blk_slice [n_blocks], fin_slice [n_fin]: slice of each block)
// v: tile shape of the multi-slice kernel, 0 .. kMultiTiles - 1 (rows per
// tile multi_tile_rows(v), waves per block multi_tile_waves(v))
constexpr int kMultiTiles = 3;
int multi_tile_rows(int v);
int multi_tile_waves(int v);
hipError_t launch_cp_bf16_multi(const SliceStep* sl, const int* blk_slice, int n_blocks, int v,
                                hipStream_t s);
hipError_t launch_cp_finish_multi(const SliceStep* sl, const int* fin_slice, int n_fin,
                                  int max_dk, hipStream_t s);
int multi_shape(int D, int K);            // shape id of the multi kernel for D, K <= 64, else -1
int cp_bf16_multi_per_cu(int v);          // resident blocks of the multi kernel per CU
constexpr int kFinishEntries = 16;        // entries of D x K per finish block
// BF16 path (D, K <= 128)
int bf16_cols(int D);
bool bf16_supported(int D, int K);
hipError_t launch_form_w16(const double* W, const double* m, int V, int D, int Dh, uint16_t* W16,
                           float* mw16, hipStream_t s);
// resident blocks of one round on the device; mode 0 fused, 1 from X, 2 whitening only
int bf16_resident_blocks(int mode, int D, int K, int Dh, int num_cu);
// gsq != nullptr: the kernel also forms the K x K squared Gram entries of
// Phi for the finish, as k_gram_sq does.
hipError_t launch_whiten_cp_bf16(const tlda_csr_batch& b, const uint16_t* W16, const float* mw16,
                                 int Dh, int D, const float* Phi, int K, int nblk, float* partial,
                                 int* block_counts, float* Xout, float* phi_copy, double* gsq,
                                 hipStream_t s);
hipError_t launch_cp_reduce_bf16(const float* X, int n_rows, const float* Phi, int D, int K,
                                 int nblk, float* partial, float* phi_copy, hipStream_t s);
hipError_t launch_whiten_bf16(const tlda_csr_batch& b, const uint16_t* W16, const float* mw16,
                              int Dh, int D, int nblk, float* X, int* block_counts, hipStream_t s);
// One full round of resident CP-reduction blocks on this device.
int cp_resident_blocks(int D, int K, int num_cu);
// classic-moment CP step (FP32, D, K <= 128): Z = W Phi, r = Phi^T mw32 and
// phi_copy = Phi, then the per-block data-term partials divided by c3 and the
// kept counts (block_counts[0 .. nblk)).  With partial == nullptr,
// launch_classic_cp only stores in *block_counts the resident blocks per CU.
bool classic_supported(int D, int K);
hipError_t launch_classic_z(const float* W32, int V, int D, int Dp, const float* Phi, int K,
                            int Kp, const float* mw32, float* Z, float* r, float* phi_copy,
                            int num_cu, hipStream_t s);
// BF16 variant: Z16 = bf16(W16 Phi) (V x Kh, Kh = bf16_cols(K)), r = Phi^T mw16
hipError_t launch_classic_z16(const uint16_t* W16, int V, int D, int Dh, const float* Phi, int K,
                              int Kh, const float* mw16, uint16_t* Z16, float* r, float* phi_copy,
                              int num_cu, hipStream_t s);
hipError_t launch_classic_cp16(const tlda_csr_batch& b, const uint16_t* W16, int Dh,
                               const uint16_t* Z16, int Kh, const float* mw16, const float* r,
                               int D, int K, double alpha0, int nblk, float* partial,
                               int* block_counts, hipStream_t s);
hipError_t launch_classic_cp(const tlda_csr_batch& b, const float* W32, int Dp, const float* Z,
                             int Kp, const float* mw32, const float* r, int D, int K,
                             double alpha0, int nblk, float* partial, int* block_counts,
                             hipStream_t s);
// document-topic encoder (MLP)
size_t mlp_param_count(int d_in, int hidden, int k_out);
// floats of the encoder's gradient workspace (split partials)
size_t mlp_workspace_floats(int d_in, int hidden, int k_out, int max_batch);
// offsets of W1, b1, W2, b2, W3, b3 in the packed parameter vector
void mlp_offsets(int d_in, int hidden, int k_out, size_t off[6]);
// forward pass of n <= max_batch rows: theta = softmax(...) (FP32 [n][k_out]);
// with train, also keeps the intermediates for mlp_backward
hipError_t mlp_forward(tlda_mlp& m, const float* X, int n, float* theta, bool train);
// loss and gradients of the mean cross-entropy against targets T [n][k_out]
// (needs a preceding mlp_forward(train) of the same rows); loss_out: device float or NULL
hipError_t mlp_backward(tlda_mlp& m, const float* X, const float* T, int n, float* loss_out);
hipError_t mlp_adam(tlda_mlp& m, float lr, float beta1, float beta2, float eps);
hipError_t mlp_refresh_bf16(tlda_mlp& m);
// post-processing
hipError_t launch_unwhiten(const float* Phi, const double* U, const double* eig, const double* m,
                           int V, int D, int K, double theta, uint32_t flags, double* mu,
                           double* alpha, double* lambda, double* scratch, hipStream_t s);
// classic recovery: lambda_k = (1+theta)|phi_k|^3, mu_k = lambda_k U diag(eig)^(1/2)
// phi_k / |phi_k|, alpha proportional to lambda^-2
hipError_t launch_unwhiten_classic(const float* Phi, const double* U, const double* eig, int V,
                                   int D, int K, double theta, uint32_t flags, double* mu,
                                   double* alpha, double* lambda, double* scratch, hipStream_t s);
// Phi[:, k] <- diag(eig)^(-1/2) C diag(eig_prev)^(1/2) Phi[:, k] (FP64 sums)
hipError_t launch_rebase(const double* C, const double* eig, const double* eig_prev, int D, int K,
                         float* Phi, hipStream_t s);
hipError_t launch_inference_setup(const double* W, const double* m, const double* mu, int V,
                                  int D, int K, double* A, double* G, double* Z, double* ev,
                                  float* A32, float* G32, float* step32, int* info,
                                  hipStream_t s);
hipError_t launch_infer(const float* X, int n_rows, const float* A32, const float* G32,
                        const float* step32, int D, int K, int max_iter, float tol,
                        float* theta, hipStream_t s);
// Projected gradient with a duality-gap stopping rule: from the start point
// held in theta (given_start) or from 1/K, at least min_steps steps, then
// until the gap of the iterate is at most gap_tol or max_iter steps; rows
// that need more than min_steps steps are counted in *n_stepped (which the
// caller zeroes).
hipError_t launch_infer_gap(const float* X, int n_rows, const float* A32, const float* G32,
                            const float* step32, int D, int K, bool given_start, float gap_tol,
                            int min_steps, int max_iter, float* theta, int* n_stepped,
                            hipStream_t s);

}  // namespace tlda
