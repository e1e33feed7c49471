// Host side of the C ABI declared in include/tlda.h: argument checks, device
// state, stream ordering, the whitening refresh driver and checkpoints.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "tlda_internal.h"

using tlda::launch_zero;

namespace {

struct Fail {
  tlda_status code;
};

void set_err(const tlda_ctx* c, const std::string& msg) {
  if (c) c->last_error = msg;
}

#define HIP_OK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_err(ctx, std::string(#expr) + ": " + hipGetErrorString(e_));             \
      return e_ == hipErrorOutOfMemory ? TLDA_ERR_OOM : TLDA_ERR_DEVICE;           \
    }                                                                              \
  } while (0)

#define CHECK_ARG(ctx, cond, code, msg) \
  do {                                  \
    if (!(cond)) {                      \
      set_err(ctx, msg);                \
      return code;                      \
    }                                   \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

namespace tlda {
thread_local KernelTimer g_main_timer;
}  // namespace tlda

namespace {

// Per-block partials of tlda_whiten_cp_step_noalloc: one array on every
// device the library runs on, held until the process ends.  Host code never
// passes this name to a kernel (on the host it is a stand-in, not a device
// address): it uses the address hipGetSymbolAddress returns for the device.
__device__ __align__(256) float scratch[tlda::kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_looked_up[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current; looked up
// once per device.
hipError_t scratch_address(int device, float** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_looked_up[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_addr[device] = e == hipSuccess ? static_cast<float*>(p) : nullptr;
    g_scratch_looked_up[device] = true;
  }
  *out = g_scratch_addr[device];
  return g_scratch_err[device];
}

}  // namespace

namespace {

bool is_bf16(const tlda_ctx* c) { return (c->cfg.flags & TLDA_BF16) != 0; }
bool is_classic(const tlda_ctx* c) { return (c->cfg.flags & TLDA_CLASSIC) != 0; }
// W32's tail copy starts right after its V x Dp rows.
uint32_t w32_tail_base(const tlda_ctx* c) { return (uint32_t)((size_t)c->cfg.V * c->Dp); }

// FP32 (and, in BF16 contexts, BF16) gather copies of W and their mean
// projections, from U, eig and M1.
hipError_t form_whitening(tlda_ctx* c) {
  const int V = c->cfg.V, D = c->cfg.D;
  hipError_t e = tlda::launch_form_whitening(c->wh.U, c->wh.eig, c->wh.m, V, D, c->Dp, c->wh.W,
                                             c->wh.W32, c->wh.mw32, c->stream);
  if (e == hipSuccess)
    e = tlda::launch_w32_tail(c->wh.W32, V, D, c->Dp, c->Dt, w32_tail_base(c), c->stream);
  if (e != hipSuccess || !is_bf16(c)) return e;
  return tlda::launch_form_w16(c->wh.W, c->wh.m, V, D, c->Dh, c->wh.W16, c->wh.mw16, c->stream);
}

// The next event pair of the timing hook goes to the next main-kernel launch.
// (Not while a graph is captured: events attached to a launch are not
// recorded in captured graphs.)
hipError_t timing_start(tlda_ctx* c) {
  tlda::g_main_timer = tlda::KernelTimer{};
  if (c->t_n <= 0 || c->in_capture) return hipSuccess;
  tlda::g_main_timer.start = c->t_start[c->t_next];
  tlda::g_main_timer.stop = c->t_stop[c->t_next];
  return hipSuccess;
}

hipError_t timing_stop(tlda_ctx* c) {
  tlda::g_main_timer = tlda::KernelTimer{};
  if (c->t_n <= 0 || c->in_capture) return hipSuccess;
  c->t_next = (c->t_next + 1) % c->t_n;
  return hipSuccess;
}

// Grid of the BF16 kernels: one full round of resident blocks (or the tuned
// size), at most one block per 64-document tile and per block-count slot.
int bf16_grid(tlda_ctx* c, int mode, int n_rows) {
  int cap = c->tune.bf16_blocks;
  if (cap <= 0) {
    if (c->tune.bf16_resident[mode] <= 0)
      c->tune.bf16_resident[mode] =
          tlda::bf16_resident_blocks(mode, c->cfg.D, c->cfg.K, c->Dh, c->num_cu);
    cap = c->tune.bf16_resident[mode];
  }
  const int ntiles = (n_rows + 63) / 64;
  int nblk = ntiles < cap ? ntiles : cap;
  if (nblk > 2 * tlda::kWhitenBlockCounts) nblk = 2 * tlda::kWhitenBlockCounts;
  return nblk < 1 ? 1 : nblk;
}

tlda_status ensure_partial(tlda_ctx* c, size_t need) {
  if (c->cp.cap < need) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    dfree(c->cp.partial);
    c->cp.cap = 0;
    HIP_OK(c, dalloc(&c->cp.partial, need));
    c->cp.cap = need;
  }
  return TLDA_OK;
}

// The context's own whitened-batch buffer, at least `need` floats.
tlda_status ensure_x(tlda_ctx* c, size_t need) {
  if (c->cp.cap_x < need) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    dfree(c->cp.X);
    c->cp.cap_x = 0;
    HIP_OK(c, dalloc(&c->cp.X, need));
    c->cp.cap_x = need;
  }
  return TLDA_OK;
}

// The finish of a step (gradient and update from the reduction's partials).
// From kGramOnceDK entries of Phi on, the squared Gram entries of Phi0 are
// formed once first rather than by every finish block.
// gram_ready: the reduction kernel already formed the squared Gram entries
// (also below kGramOnceDK: the BF16 fused kernel and the FP32 hybrid kernel
// form them at every shape they serve, so that their finish reads them
// instead of forming a column of Phi0^T Phi0 per entry from LDS; 62.0
// against 64.2 us per tweet-shaped FP32 step).
tlda_status finish_step(tlda_ctx* c, const float* partial, int nblk, const int* counts,
                        int ncounts, int n_default, float beta, float* Phi, float* grad,
                        int* n_out, bool gram_ready = false) {
  const int D = c->cfg.D, K = c->cfg.K;
  const double* gsq = nullptr;
  if (D * K >= tlda::kGramOnceDK || gram_ready) {
    if (!gram_ready) HIP_OK(c, tlda::launch_gram_sq(c->cp.phi0, D, K, c->cp.gsq, c->stream));
    gsq = c->cp.gsq;
  }
  HIP_OK(c, tlda::launch_cp_finish(partial, nblk, counts, ncounts, n_default, c->cp.phi0, D,
                                   K, c->cfg.alpha0, c->cfg.theta, beta, Phi, grad, c->cp.R1,
                                   n_out, gsq, c->stream));
  return TLDA_OK;
}

int default_block(const tlda_config& c) {
  int p = 2 * c.D;
  if (p < c.D + 16) p = c.D + 16;
  if (p > c.V) p = c.V;
  return p;
}

tlda_status check_batch(tlda_ctx* c, const tlda_csr_batch* b) {
  CHECK_ARG(c, b != nullptr, TLDA_ERR_ARG, "batch is NULL");
  CHECK_ARG(c, b->n_rows >= 0 && b->nnz >= 0, TLDA_ERR_SHAPE, "negative n_rows or nnz");
  CHECK_ARG(c, b->slot >= -1 && b->slot <= 1, TLDA_ERR_ARG, "slot must be -1, 0 or 1");
  CHECK_ARG(c, b->first_doc >= 0, TLDA_ERR_ARG, "first_doc must be >= 0");
  if (b->n_rows > 0) CHECK_ARG(c, b->row_ptr != nullptr, TLDA_ERR_ARG, "row_ptr is NULL");
  if (b->nnz > 0)
    CHECK_ARG(c, b->col_idx != nullptr && b->val != nullptr, TLDA_ERR_ARG,
              "col_idx or val is NULL");
  if (b->slot >= 0) {
    CHECK_ARG(c, c->slots[b->slot].used, TLDA_ERR_STATE, "staging slot was never filled");
    CHECK_ARG(c, b->row_ptr == c->slots[b->slot].row_ptr, TLDA_ERR_ARG,
              "batch does not view its staging slot");
  }
  return TLDA_OK;
}

// Optional CSR content validation: synchronous, before any state changes.
tlda_status validate_content(tlda_ctx* c, const tlda_csr_batch* b) {
  if (!(c->cfg.flags & TLDA_VALIDATE_CSR) || b->n_rows == 0 || c->in_capture) return TLDA_OK;
  if (b->slot >= 0) HIP_OK(c, hipStreamWaitEvent(c->stream, c->slots[b->slot].ready, 0));
  HIP_OK(c, launch_zero(c->dev_flags, 2 * sizeof(int), c->stream));
  HIP_OK(c, tlda::launch_validate_csr(*b, c->cfg.V, c->dev_flags, c->stream));
  int bad[2] = {0, 0};
  HIP_OK(c, hipMemcpyAsync(bad, c->dev_flags, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (bad[0] != 0) {
    const int row = b->n_rows - bad[1];
    set_err(c, "CSR content rejected at document " + std::to_string(b->first_doc + row) +
                   " (row " + std::to_string(row) +
                   " of the batch): row_ptr, column order/range or counts");
    return TLDA_ERR_CSR;
  }
  return TLDA_OK;
}

tlda_status begin_use(tlda_ctx* c, const tlda_csr_batch* b) {
  if (b->slot >= 0) HIP_OK(c, hipStreamWaitEvent(c->stream, c->slots[b->slot].ready, 0));
  return TLDA_OK;
}

tlda_status end_use(tlda_ctx* c, const tlda_csr_batch* b) {
  if (b->slot >= 0) HIP_OK(c, hipEventRecord(c->slots[b->slot].free_, c->stream));
  return TLDA_OK;
}

// The exact pair-sum accumulator (packed upper triangle, zeroed when made).
tlda_status ensure_acc(tlda_ctx* c) {
  if (c->mom.acc) return TLDA_OK;
  const size_t n = tlda::tri_words(c->cfg.V);
  HIP_OK(c, dalloc(&c->mom.acc, n));
  HIP_OK(c, launch_zero(c->mom.acc, n * sizeof(unsigned long long), c->stream));
  return TLDA_OK;
}

tlda_status ensure_eig(tlda_ctx* c, int p) {
  tlda::EigScratch& e = c->eig;
  if (e.p == p && e.Q) return TLDA_OK;
  dfree(e.Q); dfree(e.Y); dfree(e.G); dfree(e.Z); dfree(e.ev); dfree(e.t); dfree(e.Binv);
  dfree(e.sel); dfree(e.mcand); dfree(e.info); dfree(e.part); dfree(e.ws);
  e.p = 0;
  e.part_chunks = 0;
  e.ws_doubles = 0;
  e.warm = nullptr;
  const size_t V = c->cfg.V, D = c->cfg.D;
  HIP_OK(c, dalloc(&e.Q, V * p));
  HIP_OK(c, dalloc(&e.Y, V * p));
  HIP_OK(c, dalloc(&e.G, (size_t)p * p));
  HIP_OK(c, dalloc(&e.Z, (size_t)p * p));
  HIP_OK(c, dalloc(&e.Binv, (size_t)p * p));
  HIP_OK(c, dalloc(&e.ev, (size_t)p));
  HIP_OK(c, dalloc(&e.t, (size_t)p));
  HIP_OK(c, dalloc(&e.sel, D + (size_t)p * D));
  HIP_OK(c, dalloc(&e.mcand, V));
  HIP_OK(c, dalloc(&e.info, 4));
  // the Gram products split their V rows into chunks of at least 64 rows
  const int chunks = (int)std::min<size_t>(tlda::kSplitMax, (V + 63) / 64);
  HIP_OK(c, dalloc(&e.part, (size_t)chunks * p * p));
  e.part_chunks = chunks;
  // K-split partials of the S2 product on the matrix cores (V x p each)
  const int splits = tlda::dgemm_splits((int)V, p, (int)V, c->num_cu > 0 ? c->num_cu : 256);
  if (splits > 1) {
    HIP_OK(c, dalloc(&e.ws, (size_t)splits * V * p));
    e.ws_doubles = (size_t)splits * V * p;
  }
  e.p = p;
  return TLDA_OK;
}

// Two Cholesky-QR passes (the first with a small diagonal shift so that a
// rank-deficient block still factors): in -> out, using tmp as scratch.
tlda_status orthonormalise(tlda_ctx* c, const double* in, double* tmp, double* out) {
  tlda::EigScratch& e = c->eig;
  const int V = c->cfg.V, p = e.p;
  HIP_OK(c, tlda::launch_gram(in, in, e.G, V, p, c->stream));
  HIP_OK(c, tlda::launch_cholesky(e.G, p, 1e-12, e.info, c->stream));
  HIP_OK(c, tlda::launch_trsm_right_into(in, e.G, e.Binv, tmp, V, p, c->stream));
  HIP_OK(c, tlda::launch_gram(tmp, tmp, e.G, V, p, c->stream));
  HIP_OK(c, tlda::launch_cholesky(e.G, p, 0.0, e.info, c->stream));
  HIP_OK(c, tlda::launch_trsm_right_into(tmp, e.G, e.Binv, out, V, p, c->stream));
  return TLDA_OK;
}

// M2~ Q = (alpha0+1)(S2 Q / N - M1 (M1^T Q)) into Y; for classic-moment
// contexts M2 Q = (alpha0+1) S2 Q / N - alpha0 M1 (M1^T Q).
tlda_status apply_m2(tlda_ctx* c, const double* Q, double* Y, double N) {
  tlda::EigScratch& e = c->eig;
  const int V = c->cfg.V, p = e.p;
  const double a1 = c->cfg.alpha0 + 1.0;
  const double am = is_classic(c) ? c->cfg.alpha0 : a1;
  HIP_OK(c, tlda::launch_vecT_mat(e.mcand, Q, e.t, V, p, c->stream));
  HIP_OK(c, tlda::launch_m2_apply(c->mom.S2, e.mcand, e.t, Q, Y, V, p, a1 / N, am, c->stream));
  return TLDA_OK;
}

// Keeps the current whitening (if any) as the one tlda_rebase_phi maps from.
tlda_status save_prev(tlda_ctx* c) {
  if (!c->wh.ready) return TLDA_OK;
  const size_t V = c->cfg.V, D = c->cfg.D;
  if (c->wh.Uprev == nullptr) {
    HIP_OK(c, dalloc(&c->wh.Uprev, V * D));
    HIP_OK(c, dalloc(&c->wh.eigprev, D));
    HIP_OK(c, dalloc(&c->wh.C, D * D));
  }
  HIP_OK(c, hipMemcpyAsync(c->wh.Uprev, c->wh.U, sizeof(double) * V * D, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(c->wh.eigprev, c->wh.eig, sizeof(double) * D, hipMemcpyDeviceToDevice,
                           c->stream));
  c->wh.prev_ready = true;
  return TLDA_OK;
}

// The refresh's product environment: its matrix-core or vector route, the
// Gram-split and K-split scratch of this context.
tlda::EigEnv eig_env(const tlda_ctx* c) {
  tlda::EigEnv env;
  env.route = c->tune.gemm_route == 1 ? 1 : 0;
  env.part = c->eig.part;
  env.part_mn = c->eig.part ? (size_t)c->eig.p * c->eig.p : 0;
  env.part_chunks = c->eig.part_chunks;
  env.ws = c->eig.ws;
  env.ws_doubles = c->eig.ws_doubles;
  env.num_cu = c->num_cu > 0 ? c->num_cu : 256;
  return env;
}

// warm: start from the block the previous refresh converged to (if any) and
// run cfg.eig_warm_iters iterations instead of a seeded cold start.
tlda_status refresh(tlda_ctx* c, bool warm) {
  const int V = c->cfg.V, D = c->cfg.D;
  unsigned long long counts[2] = {0, 0};
  HIP_OK(c, hipMemcpyAsync(counts, c->mom.counts, sizeof(counts), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  CHECK_ARG(c, counts[0] > 0, TLDA_ERR_NUMERIC, "no kept documents: M1 and M2 are undefined");
  const int p = c->cfg.eig_block > 0 ? c->cfg.eig_block : default_block(c->cfg);
  tlda_status st = ensure_eig(c, p);
  if (st != TLDA_OK) return st;
  tlda::EigScratch& e = c->eig;
  tlda::EigScope scope(eig_env(c));
  warm = warm && e.warm != nullptr;
  const int iters = warm ? (c->cfg.eig_warm_iters > 0 ? c->cfg.eig_warm_iters : 4)
                         : (c->cfg.eig_iters > 0 ? c->cfg.eig_iters : 60);
  const double N = (double)counts[0];
  HIP_OK(c, launch_zero(e.info, 4 * sizeof(int), c->stream));
  if (c->mom.S2 == nullptr) HIP_OK(c, dalloc(&c->mom.S2, (size_t)V * V));
  HIP_OK(c, tlda::launch_mean(c->mom.fsum, c->mom.counts, e.mcand, V, c->stream));
  HIP_OK(c, tlda::launch_fx_symmetric(c->mom.acc, V, c->mom.S2, c->stream));
  double* q = e.Q;
  double* y = e.Y;
  if (warm) {
    // start block: the orthonormal block of the previous refresh
    if (e.warm != q) std::swap(q, y);
  }
  e.warm = nullptr;   // both buffers are overwritten below; set again on success
  if (!warm) {
    // start block: seeded uniform entries, orthonormalised (y -> tmp q -> y)
    HIP_OK(c, tlda::launch_random_block(y, V, p, c->cfg.eig_seed, c->stream));
    st = orthonormalise(c, y, q, y);
    if (st != TLDA_OK) return st;
    std::swap(q, y);   // q: orthonormal block
  }
  for (int it = 0; it < iters; ++it) {
    st = apply_m2(c, q, y, N);
    if (st != TLDA_OK) return st;
    st = orthonormalise(c, y, q, y);   // y -> tmp q -> y
    if (st != TLDA_OK) return st;
    std::swap(q, y);
  }
  // Rayleigh-Ritz: H = Q^T M2~ Q, eigenpairs by Jacobi, U = Q Z_top
  st = apply_m2(c, q, y, N);
  if (st != TLDA_OK) return st;
  HIP_OK(c, tlda::launch_gram(q, y, e.G, V, p, c->stream));
  HIP_OK(c, tlda::launch_jacobi(e.G, e.Z, e.ev, p, e.info, c->stream));
  HIP_OK(c, tlda::launch_ritz_vectors(q, e.Z, e.ev, V, p, D, y, e.sel, c->stream));
  int info[4] = {0, 0, 0, 0};
  std::vector<double> eigD(D);
  HIP_OK(c, hipMemcpyAsync(info, e.info, sizeof(info), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipMemcpyAsync(eigD.data(), e.sel, sizeof(double) * D, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  CHECK_ARG(c, (info[0] & 1) == 0, TLDA_ERR_NUMERIC,
            "Cholesky-QR of the subspace block failed (non-positive pivot)");
  CHECK_ARG(c, (info[0] & 2) == 0, TLDA_ERR_NUMERIC, "Jacobi eigen-solver did not converge");
  for (int d = 0; d < D; ++d)
    CHECK_ARG(c, std::isfinite(eigD[d]) && eigD[d] > 0.0, TLDA_ERR_NUMERIC,
              "M2~ has fewer than D positive eigenvalues; lower D");
  // commit
  st = save_prev(c);
  if (st != TLDA_OK) return st;
  HIP_OK(c, hipMemcpyAsync(c->wh.U, y, sizeof(double) * (size_t)V * D, hipMemcpyDeviceToDevice, c->stream));
  // the next warm start: the full Ritz basis Q Z (p columns), so that the
  // projected matrix of the next refresh starts close to diagonal
  HIP_OK(c, tlda::launch_block_product(q, e.Z, y, V, p, c->stream));
  e.warm = y;
  HIP_OK(c, hipMemcpyAsync(c->wh.eig, e.sel, sizeof(double) * D, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->wh.m, e.mcand, sizeof(double) * V, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, form_whitening(c));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->wh.ready = true;
  return TLDA_OK;
}

// The fused whitening + CP step of a BF16 context or of an FP32 context
// within the fused kernel's shapes (the batch is already checked).  The
// reduction's per-block partials go to `partial`, which holds part_cap
// floats: the grid is capped so that they fit (fewer blocks, each taking more
// row tiles).  partial == nullptr: the context's own buffer, grown to the
// grid's need.
tlda_status fused_step(tlda_ctx* c, const tlda_csr_batch* b, float beta, float* Phi, float* grad,
                       float* X_out, int32_t* n_kept_out, float* partial, size_t part_cap) {
  tlda_status st = validate_content(c, b);
  if (st != TLDA_OK) return st;
  if (b->n_rows == 0) {
    if (n_kept_out) HIP_OK(c, launch_zero(n_kept_out, sizeof(int32_t), c->stream));
    return TLDA_OK;
  }
  const int D = c->cfg.D, K = c->cfg.K;
  int nblk;
  if (is_bf16(c)) {
    nblk = bf16_grid(c, 0, b->n_rows);
  } else {
    const int T = tlda::fused_tile_rows(D, K);
    const int ntiles = (b->n_rows + T - 1) / T;
    if (c->tune.fused_blocks <= 0) {
      int per_cu = 0;
      HIP_OK(c, tlda::launch_whiten_cp(*b, c->wh.W32, c->wh.mw32, D, c->Dp, c->Dt,
                                       w32_tail_base(c), Phi, K, 0, nullptr,
                                       &per_cu, nullptr, nullptr, nullptr, c->stream));
      c->tune.fused_blocks = (per_cu > 0 ? per_cu : 1) * c->num_cu;
    }
    nblk = ntiles < c->tune.fused_blocks ? ntiles : c->tune.fused_blocks;
    if (nblk > 2 * tlda::kWhitenBlockCounts) nblk = 2 * tlda::kWhitenBlockCounts;
  }
  if (partial != nullptr) {
    const size_t fit = part_cap / ((size_t)D * K);
    if ((size_t)nblk > fit) nblk = (int)fit;
  } else {
    st = ensure_partial(c, (size_t)nblk * D * K);
    if (st != TLDA_OK) return st;
    partial = c->cp.partial;
  }
  float* g = grad ? grad : c->cp.grad;
  // the BF16 kernel and the FP32 wide and hybrid kernels form the finish's
  // squared Gram entries themselves (the BF16 and hybrid kernels also below
  // kGramOnceDK entries)
  const bool gram_in_kernel =
      is_bf16(c) || (tlda::fused_forms_gram(D, K) &&
                     (D * K >= tlda::kGramOnceDK || tlda::fused_tile_rows(D, K) == 48));
  st = begin_use(c, b);
  if (st != TLDA_OK) return st;
  HIP_OK(c, timing_start(c));
  if (is_bf16(c))
    HIP_OK(c, tlda::launch_whiten_cp_bf16(*b, c->wh.W16, c->wh.mw16, c->Dh, D, Phi, K, nblk,
                                          partial, c->block_counts, X_out, c->cp.phi0,
                                          c->cp.gsq, c->stream));
  else
    HIP_OK(c, tlda::launch_whiten_cp(*b, c->wh.W32, c->wh.mw32, D, c->Dp, c->Dt, w32_tail_base(c),
                                     Phi, K, nblk, partial, c->block_counts, X_out, c->cp.phi0,
                                     gram_in_kernel ? c->cp.gsq : nullptr, c->stream));
  HIP_OK(c, timing_stop(c));
  st = end_use(c, b);
  if (st != TLDA_OK) return st;
  return finish_step(c, partial, nblk, c->block_counts, nblk, 0, beta, Phi, g, n_kept_out,
                     gram_in_kernel);
}

// The CP step of a classic-moment context (the batch is already checked):
// Z = W Phi and r, the per-block data-term partials over the batch, then the
// shared finish kernel.  X_out, if given, receives the whitened batch first.
tlda_status classic_step(tlda_ctx* c, const tlda_csr_batch* b, float beta, float* Phi, float* grad,
                         float* X_out, int32_t* n_kept_out) {
  tlda_status st = validate_content(c, b);
  if (st != TLDA_OK) return st;
  if (X_out != nullptr) {
    st = tlda_whiten_batch(c, b, X_out, nullptr);
    if (st != TLDA_OK) return st;
  }
  if (b->n_rows == 0) {
    if (n_kept_out) HIP_OK(c, launch_zero(n_kept_out, sizeof(int32_t), c->stream));
    return TLDA_OK;
  }
  const int V = c->cfg.V, D = c->cfg.D, K = c->cfg.K;
  if (is_bf16(c)) {
    const int Kh = tlda::bf16_cols(K);
    if (c->cp.Z16 == nullptr) {
      HIP_OK(c, dalloc(&c->cp.Z16, (size_t)V * Kh));
      if (c->cp.rz == nullptr) HIP_OK(c, dalloc(&c->cp.rz, (size_t)Kh));
    }
    if (c->tune.classic16_resident <= 0) {
      int per_cu = 0;
      HIP_OK(c, tlda::launch_classic_cp16(*b, c->wh.W16, c->Dh, c->cp.Z16, Kh, c->wh.mw16,
                                          c->cp.rz, D, K, c->cfg.alpha0, 0, nullptr, &per_cu,
                                          c->stream));
      c->tune.classic16_resident = (per_cu > 0 ? per_cu : 1) * c->num_cu;
    }
    const int ntiles = (b->n_rows + 15) / 16;
    int nblk = ntiles < c->tune.classic16_resident ? ntiles : c->tune.classic16_resident;
    if (nblk > 2 * tlda::kWhitenBlockCounts) nblk = 2 * tlda::kWhitenBlockCounts;
    st = ensure_partial(c, (size_t)nblk * D * K);
    if (st != TLDA_OK) return st;
    float* g = grad ? grad : c->cp.grad;
    HIP_OK(c, tlda::launch_classic_z16(c->wh.W16, V, D, c->Dh, Phi, K, Kh, c->wh.mw16, c->cp.Z16,
                                       c->cp.rz, c->cp.phi0, c->num_cu, c->stream));
    st = begin_use(c, b);
    if (st != TLDA_OK) return st;
    HIP_OK(c, timing_start(c));
    HIP_OK(c, tlda::launch_classic_cp16(*b, c->wh.W16, c->Dh, c->cp.Z16, Kh, c->wh.mw16, c->cp.rz,
                                        D, K, c->cfg.alpha0, nblk, c->cp.partial, c->block_counts,
                                        c->stream));
    HIP_OK(c, timing_stop(c));
    st = end_use(c, b);
    if (st != TLDA_OK) return st;
    return finish_step(c, c->cp.partial, nblk, c->block_counts, nblk, 0, beta, Phi, g,
                     n_kept_out);
  }
  const int Kp = tlda::padded_d(K);
  if (c->cp.Z == nullptr) {
    HIP_OK(c, dalloc(&c->cp.Z, (size_t)V * Kp));
    HIP_OK(c, dalloc(&c->cp.rz, (size_t)Kp));
  }
  if (c->tune.classic_resident <= 0) {
    int per_cu = 0;
    HIP_OK(c, tlda::launch_classic_cp(*b, c->wh.W32, c->Dp, c->cp.Z, Kp, c->wh.mw32, c->cp.rz, D,
                                      K, c->cfg.alpha0, 0, nullptr, &per_cu, c->stream));
    c->tune.classic_resident = (per_cu > 0 ? per_cu : 1) * c->num_cu;
  }
  const int ntiles = (b->n_rows + 15) / 16;
  int nblk = ntiles < c->tune.classic_resident ? ntiles : c->tune.classic_resident;
  if (nblk > 2 * tlda::kWhitenBlockCounts) nblk = 2 * tlda::kWhitenBlockCounts;
  st = ensure_partial(c, (size_t)nblk * D * K);
  if (st != TLDA_OK) return st;
  float* g = grad ? grad : c->cp.grad;
  HIP_OK(c, tlda::launch_classic_z(c->wh.W32, V, D, c->Dp, Phi, K, Kp, c->wh.mw32, c->cp.Z,
                                   c->cp.rz, c->cp.phi0, c->num_cu, c->stream));
  st = begin_use(c, b);
  if (st != TLDA_OK) return st;
  HIP_OK(c, timing_start(c));
  HIP_OK(c, tlda::launch_classic_cp(*b, c->wh.W32, c->Dp, c->cp.Z, Kp, c->wh.mw32, c->cp.rz, D, K,
                                    c->cfg.alpha0, nblk, c->cp.partial, c->block_counts,
                                    c->stream));
  HIP_OK(c, timing_stop(c));
  st = end_use(c, b);
  if (st != TLDA_OK) return st;
  return finish_step(c, c->cp.partial, nblk, c->block_counts, nblk, 0, beta, Phi, g,
                     n_kept_out);
}

void destroy_all(tlda_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  dfree(c->mom.counts); dfree(c->mom.totals); dfree(c->mom.fsum); dfree(c->mom.acc);
  dfree(c->mom.S2);
  dfree(c->wh.W); dfree(c->wh.U); dfree(c->wh.eig); dfree(c->wh.m); dfree(c->wh.W32);
  dfree(c->wh.mw32); dfree(c->wh.W16); dfree(c->wh.mw16);
  dfree(c->wh.Uprev); dfree(c->wh.eigprev); dfree(c->wh.C);
  delete[] c->t_start;
  delete[] c->t_stop;
  tlda::EigScratch& e = c->eig;
  dfree(e.Q); dfree(e.Y); dfree(e.G); dfree(e.Z); dfree(e.ev); dfree(e.t); dfree(e.Binv);
  dfree(e.sel); dfree(e.mcand); dfree(e.info); dfree(e.part); dfree(e.ws);
  dfree(c->cp.partial); dfree(c->cp.R1); dfree(c->cp.phi0); dfree(c->cp.grad); dfree(c->cp.X);
  dfree(c->cp.gsq);
  dfree(c->cp.Z); dfree(c->cp.rz); dfree(c->cp.Z16);
  dfree(c->post); dfree(c->postA); dfree(c->postG); dfree(c->postZ); dfree(c->postEv);
  dfree(c->A32); dfree(c->G32); dfree(c->step32); dfree(c->dev_flags); dfree(c->block_counts);
  for (auto& s : c->slots) {
    if (s.free_) (void)hipEventSynchronize(s.free_);
    dfree(s.row_ptr); dfree(s.col_idx); dfree(s.val); dfree(s.col16); dfree(s.val16);
    if (s.ready) (void)hipEventDestroy(s.ready);
    if (s.free_) (void)hipEventDestroy(s.free_);
  }
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  delete c;
}

}  // namespace

extern "C" {

const char* tlda_status_str(tlda_status s) {
  // a C caller may pass any int: its bits are read as one (loading a value
  // outside the enumerators through the enum type is undefined in C++)
  static_assert(sizeof(tlda_status) == sizeof(int), "tlda_status is an int");
  int code;
  std::memcpy(&code, &s, sizeof(code));
  switch (code) {
    case TLDA_OK: return "ok";
    case TLDA_ERR_ARG: return "invalid argument";
    case TLDA_ERR_SHAPE: return "invalid shape";
    case TLDA_ERR_CSR: return "invalid CSR content";
    case TLDA_ERR_STATE: return "invalid call order";
    case TLDA_ERR_NUMERIC: return "numerical failure";
    case TLDA_ERR_OOM: return "device out of memory";
    case TLDA_ERR_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

const char* tlda_last_error(const tlda_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

tlda_status tlda_create(const tlda_config* cfg, void* hip_stream, tlda_ctx** out) {
  if (out == nullptr || cfg == nullptr) return TLDA_ERR_ARG;
  *out = nullptr;
  const tlda_config& c = *cfg;
  if (!(c.alpha0 > 0.0) || !std::isfinite(c.alpha0)) return TLDA_ERR_ARG;
  if (!(c.theta >= 0.0) || !std::isfinite(c.theta)) return TLDA_ERR_ARG;
  if (c.flags & ~(TLDA_VALIDATE_CSR | TLDA_BF16 | TLDA_CLASSIC)) return TLDA_ERR_ARG;
  if (c.eig_iters < 0 || c.eig_block < 0) return TLDA_ERR_ARG;
  if (c.V < 3 || c.V > 131072) return TLDA_ERR_SHAPE;
  if (c.K < 1 || c.K > TLDA_MAX_K || c.D < 1 || c.D > TLDA_MAX_D || c.D > c.V) return TLDA_ERR_SHAPE;
  if (c.D * c.K > TLDA_MAX_DK) return TLDA_ERR_SHAPE;
  if (!(c.flags & (TLDA_BF16 | TLDA_CLASSIC)) &&
      (((c.D + 3) / 4) * ((c.K + 3) / 4) > 1024 || tlda::cp_tile_rows(c.D, c.K) == 0))
    return TLDA_ERR_SHAPE;   // the FP32 reduction's shape limits (unused by BF16 and classic)
  if (c.eig_block != 0 && (c.eig_block < c.D || c.eig_block > c.V || c.eig_block > 512))
    return TLDA_ERR_SHAPE;
  if ((c.flags & TLDA_BF16) && !tlda::bf16_supported(c.D, c.K)) return TLDA_ERR_SHAPE;
  if ((c.flags & TLDA_CLASSIC) && !tlda::classic_supported(c.D, c.K)) return TLDA_ERR_SHAPE;
  tlda_ctx* ctx = new (std::nothrow) tlda_ctx();
  if (!ctx) return TLDA_ERR_OOM;
  ctx->cfg = c;
  ctx->Dp = tlda::padded_d(c.D);
  ctx->Dh = tlda::bf16_cols(c.D);
  if (!(c.flags & (TLDA_BF16 | TLDA_CLASSIC)) && std::getenv("TLDA_TUNE_NO_W32_TAIL") == nullptr)
    ctx->Dt = tlda::w32_tail_cols(c.D, c.K);
  auto env_int = [](const char* name) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : 0;
  };
  ctx->tune.cp_max_blocks = env_int("TLDA_TUNE_CP_BLOCKS");
  ctx->tune.whiten_v4 = env_int("TLDA_TUNE_WHITEN_V4");
  ctx->tune.whiten_chunks = env_int("TLDA_TUNE_WHITEN_CHUNKS");
  ctx->tune.fused_blocks = env_int("TLDA_TUNE_FUSED_BLOCKS");
  ctx->tune.bf16_blocks = env_int("TLDA_TUNE_BF16_BLOCKS");
  ctx->tune.gemm_route = env_int("TLDA_TUNE_GEMM");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  auto fail = [&](tlda_status s) {
    destroy_all(ctx);
    return s;
  };
  if (hipGetDevice(&ctx->device) != hipSuccess) return fail(TLDA_ERR_DEVICE);
  if (hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
      hipSuccess)
    return fail(TLDA_ERR_DEVICE);
  if (hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(TLDA_ERR_DEVICE);
  {
    // the allocation-free step's buffer on this device (its calls fail with
    // this message if the lookup did; every other call works without it)
    const hipError_t e = scratch_address(ctx->device, &ctx->noalloc);
    if (e != hipSuccess) ctx->noalloc_error = hipGetErrorString(e);
  }
  for (auto& s : ctx->slots) {
    if (hipEventCreateWithFlags(&s.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s.free_, hipEventDisableTiming) != hipSuccess)
      return fail(TLDA_ERR_DEVICE);
  }
  const size_t V = c.V, D = c.D, K = c.K;
  bool ok = dalloc(&ctx->mom.counts, 2) == hipSuccess && dalloc(&ctx->mom.totals, V) == hipSuccess &&
            dalloc(&ctx->mom.fsum, 2 * V) == hipSuccess && dalloc(&ctx->wh.W, V * D) == hipSuccess &&
            dalloc(&ctx->wh.U, V * D) == hipSuccess && dalloc(&ctx->wh.eig, D) == hipSuccess &&
            dalloc(&ctx->wh.m, V) == hipSuccess &&
            dalloc(&ctx->wh.W32, V * (size_t)(ctx->Dp + ctx->Dt)) == hipSuccess &&
            dalloc(&ctx->wh.mw32, (size_t)ctx->Dp) == hipSuccess &&
            dalloc(&ctx->cp.R1, D * K) == hipSuccess && dalloc(&ctx->cp.phi0, D * K) == hipSuccess &&
            dalloc(&ctx->cp.gsq, (size_t)K * K) == hipSuccess &&
            dalloc(&ctx->cp.grad, D * K) == hipSuccess && dalloc(&ctx->post, K) == hipSuccess &&
            dalloc(&ctx->postA, D * K) == hipSuccess && dalloc(&ctx->postG, K * K) == hipSuccess &&
            dalloc(&ctx->postZ, K * K) == hipSuccess && dalloc(&ctx->postEv, K) == hipSuccess &&
            dalloc(&ctx->A32, D * K) == hipSuccess && dalloc(&ctx->G32, K * K) == hipSuccess &&
            dalloc(&ctx->step32, 1) == hipSuccess && dalloc(&ctx->dev_flags, 4) == hipSuccess &&
            dalloc(&ctx->block_counts, 2 * tlda::kWhitenBlockCounts) == hipSuccess;
  if (ok && (c.flags & TLDA_BF16))
    ok = dalloc(&ctx->wh.W16, V * (size_t)ctx->Dh) == hipSuccess &&
         dalloc(&ctx->wh.mw16, (size_t)ctx->Dh) == hipSuccess;
  if (!ok) return fail(TLDA_ERR_OOM);
  if (launch_zero(ctx->mom.counts, 2 * sizeof(unsigned long long), ctx->stream) != hipSuccess ||
      launch_zero(ctx->mom.totals, V * sizeof(unsigned long long), ctx->stream) != hipSuccess ||
      launch_zero(ctx->mom.fsum, 2 * V * sizeof(unsigned long long), ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(TLDA_ERR_DEVICE);
  *out = ctx;
  return TLDA_OK;
}

void tlda_destroy(tlda_ctx* ctx) { destroy_all(ctx); }

tlda_status tlda_update_moments(tlda_ctx* c, const tlda_csr_batch* b, uint32_t flags) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c,
            (flags & ~(TLDA_REFRESH_W | TLDA_RESET | TLDA_RELEASE | TLDA_REFRESH_WARM)) == 0,
            TLDA_ERR_ARG, "unknown flags");
  if (flags & TLDA_REFRESH_WARM) flags |= TLDA_REFRESH_W;
  CHECK_ARG(c, b != nullptr || (flags & (TLDA_REFRESH_W | TLDA_RESET | TLDA_RELEASE)),
            TLDA_ERR_ARG,
            "batch is NULL and no refresh or reset was requested");
  if (b) {
    tlda_status st = check_batch(c, b);
    if (st != TLDA_OK) return st;
    st = validate_content(c, b);
    if (st != TLDA_OK) return st;
  }
  tlda_status st = TLDA_OK;
  if (b || (flags & (TLDA_REFRESH_W | TLDA_RESET))) {
    st = ensure_acc(c);
    if (st != TLDA_OK) return st;
  }
  const size_t V = c->cfg.V;
  if (flags & TLDA_RESET) {
    HIP_OK(c, launch_zero(c->mom.counts, 2 * sizeof(unsigned long long), c->stream));
    HIP_OK(c, launch_zero(c->mom.totals, V * sizeof(unsigned long long), c->stream));
    HIP_OK(c, launch_zero(c->mom.fsum, 2 * V * sizeof(unsigned long long), c->stream));
    HIP_OK(c, launch_zero(c->mom.acc, tlda::tri_words((int)V) * sizeof(unsigned long long),
                          c->stream));
  }
  if (b && b->n_rows > 0) {
    st = begin_use(c, b);
    if (st != TLDA_OK) return st;
    HIP_OK(c, tlda::launch_accumulate(*b, c->cfg.V, c->mom, c->block_counts, is_classic(c),
                                      c->stream));
    st = end_use(c, b);
    if (st != TLDA_OK) return st;
  }
  if (flags & TLDA_REFRESH_W) {
    st = refresh(c, (flags & TLDA_REFRESH_WARM) != 0);
    if (st != TLDA_OK) return st;
  }
  if (flags & TLDA_RELEASE) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    dfree(c->mom.S2);
    dfree(c->mom.acc);
    HIP_OK(c, launch_zero(c->mom.counts, 2 * sizeof(unsigned long long), c->stream));
    HIP_OK(c, launch_zero(c->mom.totals, V * sizeof(unsigned long long), c->stream));
    HIP_OK(c, launch_zero(c->mom.fsum, 2 * V * sizeof(unsigned long long), c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  return TLDA_OK;
}

tlda_status tlda_whiten_batch(tlda_ctx* c, const tlda_csr_batch* b, float* X, int32_t* n_kept) {
  if (!c) return TLDA_ERR_ARG;
  tlda_status st = check_batch(c, b);
  if (st != TLDA_OK) return st;
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet: refresh or set one first");
  CHECK_ARG(c, X != nullptr || b->n_rows == 0, TLDA_ERR_ARG, "X is NULL");
  st = validate_content(c, b);
  if (st != TLDA_OK) return st;
  st = begin_use(c, b);
  if (st != TLDA_OK) return st;
  if (is_bf16(c) && b->n_rows > 0) {
    int nblk = bf16_grid(c, 2, b->n_rows);
    if (nblk > tlda::kWhitenBlockCounts) nblk = tlda::kWhitenBlockCounts;
    HIP_OK(c, timing_start(c));
    HIP_OK(c, tlda::launch_whiten_bf16(*b, c->wh.W16, c->wh.mw16, c->Dh, c->cfg.D, nblk, X,
                                       c->block_counts, c->stream));
    HIP_OK(c, timing_stop(c));
    if (n_kept) HIP_OK(c, tlda::launch_sum_counts(c->block_counts, nblk, n_kept, c->stream));
  } else {
    HIP_OK(c, timing_start(c));
    HIP_OK(c, tlda::launch_whiten(*b, c->wh.W32, c->wh.mw32, c->cfg.V, c->cfg.D, c->Dp, X, n_kept,
                                  c->block_counts, c->tune, c->stream));
    HIP_OK(c, timing_stop(c));
  }
  return end_use(c, b);
}

tlda_status tlda_cp_step(tlda_ctx* c, const float* X, int32_t n_rows, const int32_t* n_kept,
                         float beta, float* Phi, float* grad) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, !is_classic(c), TLDA_ERR_STATE,
            "classic-moment contexts step from the batch (tlda_whiten_cp_step), not from X");
  CHECK_ARG(c, n_rows >= 0, TLDA_ERR_SHAPE, "negative n_rows");
  CHECK_ARG(c, Phi != nullptr, TLDA_ERR_ARG, "Phi is NULL");
  CHECK_ARG(c, X != nullptr || n_rows == 0, TLDA_ERR_ARG, "X is NULL");
  CHECK_ARG(c, std::isfinite(beta), TLDA_ERR_ARG, "beta is not finite");
  if (n_rows == 0) return TLDA_OK;
  const int D = c->cfg.D, K = c->cfg.K;
  int nblk;
  if (is_bf16(c)) {
    nblk = bf16_grid(c, 1, n_rows);
  } else {
    if (c->tune.cp_max_blocks <= 0)
      c->tune.cp_max_blocks = tlda::cp_resident_blocks(D, K, c->num_cu);
    nblk = tlda::cp_num_blocks(n_rows, D, K, c->tune.cp_max_blocks);
  }
  tlda_status st = ensure_partial(c, (size_t)nblk * D * K);
  if (st != TLDA_OK) return st;
  float* g = grad ? grad : c->cp.grad;
  HIP_OK(c, timing_start(c));
  if (is_bf16(c))
    HIP_OK(c, tlda::launch_cp_reduce_bf16(X, n_rows, Phi, D, K, nblk, c->cp.partial, c->cp.phi0,
                                          c->stream));
  else
    HIP_OK(c, tlda::launch_cp_reduce(X, n_rows, Phi, D, K, nblk, c->cp.partial, c->cp.phi0,
                                     c->stream));
  HIP_OK(c, timing_stop(c));
  return finish_step(c, c->cp.partial, nblk, n_kept, n_kept ? 1 : 0, n_rows, beta, Phi, g,
                     nullptr);
}

tlda_status tlda_whiten_cp_step(tlda_ctx* c, const tlda_csr_batch* b, float beta, float* Phi,
                                float* grad, float* X_out, int32_t* n_kept_out) {
  if (!c) return TLDA_ERR_ARG;
  tlda_status st = check_batch(c, b);
  if (st != TLDA_OK) return st;
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet: refresh or set one first");
  CHECK_ARG(c, Phi != nullptr, TLDA_ERR_ARG, "Phi is NULL");
  CHECK_ARG(c, std::isfinite(beta), TLDA_ERR_ARG, "beta is not finite");
  const int D = c->cfg.D, K = c->cfg.K;
  if (is_classic(c)) return classic_step(c, b, beta, Phi, grad, X_out, n_kept_out);
  if (!is_bf16(c) && !tlda::fused_supported(D, K, c->Dp)) {
    // two calls in sequence through the context's own X buffer
    const size_t need = (size_t)b->n_rows * D;
    float* X = X_out;
    if (X == nullptr) {
      st = ensure_x(c, need);
      if (st != TLDA_OK) return st;
      X = c->cp.X;
    }
    int32_t* nk = n_kept_out ? n_kept_out : c->dev_flags + 2;
    st = tlda_whiten_batch(c, b, X, nk);
    if (st != TLDA_OK) return st;
    return tlda_cp_step(c, X, b->n_rows, nk, beta, Phi, grad);
  }
  return fused_step(c, b, beta, Phi, grad, X_out, n_kept_out, nullptr, 0);
}

tlda_status tlda_whiten_cp_step_noalloc(tlda_ctx* c, const tlda_csr_batch* b, float beta,
                                        float* Phi, float* grad, float* X_out,
                                        int32_t* n_kept_out) {
  if (!c) return TLDA_ERR_ARG;
  tlda_status st = check_batch(c, b);
  if (st != TLDA_OK) return st;
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet: refresh or set one first");
  CHECK_ARG(c, Phi != nullptr, TLDA_ERR_ARG, "Phi is NULL");
  CHECK_ARG(c, std::isfinite(beta), TLDA_ERR_ARG, "beta is not finite");
  const int D = c->cfg.D, K = c->cfg.K;
  CHECK_ARG(c, !is_classic(c), TLDA_ERR_ARG,
            "classic-moment steps have no allocation-free variant (their Z buffers grow on "
            "first use)");
  CHECK_ARG(c, is_bf16(c) || tlda::fused_supported(D, K, c->Dp), TLDA_ERR_SHAPE,
            "this FP32 shape runs as two calls through a whitened-batch buffer; the "
            "allocation-free step covers BF16 contexts and FP32 contexts with D, K <= 128");
  CHECK_ARG(c, (size_t)D * K <= tlda::kNoAllocFloats, TLDA_ERR_SHAPE,
            "D * K exceeds the allocation-free step's partial buffer");
  CHECK_ARG(c, c->noalloc != nullptr, TLDA_ERR_DEVICE,
            "the allocation-free step's device buffer was not found on this device: " +
                c->noalloc_error);
  return fused_step(c, b, beta, Phi, grad, X_out, n_kept_out, c->noalloc, tlda::kNoAllocFloats);
}

tlda_status tlda_unwhiten(tlda_ctx* c, const float* Phi, double* mu, double* alpha, double* lambda,
                          uint32_t flags) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, Phi && mu && alpha, TLDA_ERR_ARG, "Phi, mu or alpha is NULL");
  CHECK_ARG(c, (flags & ~TLDA_PROJECT_SIMPLEX) == 0, TLDA_ERR_ARG, "unknown flags");
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  if (is_classic(c)) {
    HIP_OK(c, tlda::launch_unwhiten_classic(Phi, c->wh.U, c->wh.eig, c->cfg.V, c->cfg.D, c->cfg.K,
                                            c->cfg.theta, flags, mu, alpha, lambda, c->post,
                                            c->stream));
    return TLDA_OK;
  }
  HIP_OK(c, tlda::launch_unwhiten(Phi, c->wh.U, c->wh.eig, c->wh.m, c->cfg.V, c->cfg.D, c->cfg.K,
                                  c->cfg.theta, flags, mu, alpha, lambda, c->post, c->stream));
  return TLDA_OK;
}

tlda_status tlda_infer_doc_topics(tlda_ctx* c, const tlda_csr_batch* b, const double* mu,
                                  int32_t max_iter, float tol, float* theta_out) {
  if (!c) return TLDA_ERR_ARG;
  tlda_status st = check_batch(c, b);
  if (st != TLDA_OK) return st;
  CHECK_ARG(c, max_iter >= 0, TLDA_ERR_ARG, "negative max_iter");
  CHECK_ARG(c, tol >= 0.0f && std::isfinite(tol), TLDA_ERR_ARG, "tol must be finite and >= 0");
  CHECK_ARG(c, mu != nullptr, TLDA_ERR_ARG, "mu is NULL");
  CHECK_ARG(c, theta_out != nullptr || b->n_rows == 0, TLDA_ERR_ARG, "theta is NULL");
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  if (b->n_rows == 0) return TLDA_OK;
  st = ensure_x(c, (size_t)b->n_rows * c->cfg.D);
  if (st != TLDA_OK) return st;
  st = tlda_whiten_batch(c, b, c->cp.X, nullptr);
  if (st != TLDA_OK) return st;
  return tlda_infer_doc_topics_whitened(c, c->cp.X, b->n_rows, mu, max_iter, tol, theta_out);
}

tlda_status tlda_infer_doc_topics_whitened(tlda_ctx* c, const float* X, int32_t n_rows,
                                           const double* mu, int32_t max_iter, float tol,
                                           float* theta_out) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, n_rows >= 0 && max_iter >= 0, TLDA_ERR_ARG, "negative n_rows or max_iter");
  CHECK_ARG(c, tol >= 0.0f && std::isfinite(tol), TLDA_ERR_ARG, "tol must be finite and >= 0");
  CHECK_ARG(c, mu != nullptr, TLDA_ERR_ARG, "mu is NULL");
  CHECK_ARG(c, (X && theta_out) || n_rows == 0, TLDA_ERR_ARG, "X or theta is NULL");
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  if (n_rows == 0) return TLDA_OK;
  const int V = c->cfg.V, D = c->cfg.D, K = c->cfg.K;
  HIP_OK(c, launch_zero(c->dev_flags, 4 * sizeof(int), c->stream));
  HIP_OK(c, tlda::launch_inference_setup(c->wh.W, c->wh.m, mu, V, D, K, c->postA, c->postG,
                                         c->postZ, c->postEv, c->A32, c->G32, c->step32,
                                         c->dev_flags + 1, c->stream));
  HIP_OK(c, tlda::launch_infer(X, n_rows, c->A32, c->G32, c->step32, D, K, max_iter, tol,
                               theta_out, c->stream));
  return TLDA_OK;
}

tlda_status tlda_stage_batch(tlda_ctx* c, const tlda_csr_batch* h, int32_t slot,
                             tlda_csr_batch* dev_out) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, h && dev_out, TLDA_ERR_ARG, "host batch or output is NULL");
  CHECK_ARG(c, slot == 0 || slot == 1, TLDA_ERR_ARG, "slot must be 0 or 1");
  CHECK_ARG(c, h->n_rows >= 0 && h->nnz >= 0, TLDA_ERR_SHAPE, "negative n_rows or nnz");
  CHECK_ARG(c, h->row_ptr != nullptr, TLDA_ERR_ARG, "row_ptr is NULL");
  if (h->nnz > 0) CHECK_ARG(c, h->col_idx && h->val, TLDA_ERR_ARG, "col_idx or val is NULL");
  CHECK_ARG(c, h->first_doc >= 0, TLDA_ERR_ARG, "first_doc must be >= 0");
  tlda::StageSlot& s = c->slots[slot];
  const size_t rows = (size_t)h->n_rows + 1, nnz = (size_t)h->nnz;
  if (s.cap_rows < rows || s.cap_nnz < nnz) {
    if (s.used) HIP_OK(c, hipEventSynchronize(s.free_));
    dfree(s.row_ptr); dfree(s.col_idx); dfree(s.val);
    s.cap_rows = s.cap_nnz = 0;
    s.used = false;
    HIP_OK(c, dalloc(&s.row_ptr, rows));
    HIP_OK(c, dalloc(&s.col_idx, nnz));
    HIP_OK(c, dalloc(&s.val, nnz));
    s.cap_rows = rows;
    s.cap_nnz = nnz;
  }
  if (s.used) HIP_OK(c, hipStreamWaitEvent(c->copy_stream, s.free_, 0));
  HIP_OK(c, hipMemcpyAsync(s.row_ptr, h->row_ptr, rows * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->copy_stream));
  if (nnz) {
    HIP_OK(c, hipMemcpyAsync(s.col_idx, h->col_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice,
                             c->copy_stream));
    HIP_OK(c, hipMemcpyAsync(s.val, h->val, nnz * sizeof(float), hipMemcpyHostToDevice,
                             c->copy_stream));
  }
  HIP_OK(c, hipEventRecord(s.ready, c->copy_stream));
  // until a consumer records its own release, the slot is free once copied
  HIP_OK(c, hipEventRecord(s.free_, c->copy_stream));
  s.used = true;
  dev_out->n_rows = h->n_rows;
  dev_out->nnz = h->nnz;
  dev_out->row_ptr = s.row_ptr;
  dev_out->col_idx = s.col_idx;
  dev_out->val = s.val;
  dev_out->slot = slot;
  dev_out->first_doc = h->first_doc;
  return TLDA_OK;
}

tlda_status tlda_stage_batch_u16(tlda_ctx* c, const tlda_csr_batch_u16* h, int32_t slot,
                                 tlda_csr_batch* dev_out) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, h && dev_out, TLDA_ERR_ARG, "host batch or output is NULL");
  CHECK_ARG(c, slot == 0 || slot == 1, TLDA_ERR_ARG, "slot must be 0 or 1");
  CHECK_ARG(c, c->cfg.V <= 65536, TLDA_ERR_SHAPE, "16-bit column indices need V <= 65536");
  CHECK_ARG(c, h->n_rows >= 0 && h->nnz >= 0, TLDA_ERR_SHAPE, "negative n_rows or nnz");
  CHECK_ARG(c, h->row_ptr != nullptr, TLDA_ERR_ARG, "row_ptr is NULL");
  if (h->nnz > 0) CHECK_ARG(c, h->col_idx && h->val, TLDA_ERR_ARG, "col_idx or val is NULL");
  CHECK_ARG(c, h->first_doc >= 0, TLDA_ERR_ARG, "first_doc must be >= 0");
  tlda::StageSlot& s = c->slots[slot];
  const size_t rows = (size_t)h->n_rows + 1, nnz = (size_t)h->nnz;
  if (s.cap_rows < rows || s.cap_nnz < nnz || s.cap16 < nnz) {
    if (s.used) HIP_OK(c, hipEventSynchronize(s.free_));
    dfree(s.row_ptr); dfree(s.col_idx); dfree(s.val); dfree(s.col16); dfree(s.val16);
    s.cap_rows = s.cap_nnz = s.cap16 = 0;
    s.used = false;
    const size_t r = rows, z = std::max<size_t>(nnz, 1);
    HIP_OK(c, dalloc(&s.row_ptr, r));
    HIP_OK(c, dalloc(&s.col_idx, z));
    HIP_OK(c, dalloc(&s.val, z));
    HIP_OK(c, dalloc(&s.col16, z));
    HIP_OK(c, dalloc(&s.val16, z));
    s.cap_rows = r;
    s.cap_nnz = s.cap16 = z;
  }
  if (s.used) HIP_OK(c, hipStreamWaitEvent(c->copy_stream, s.free_, 0));
  HIP_OK(c, hipMemcpyAsync(s.row_ptr, h->row_ptr, rows * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->copy_stream));
  if (nnz) {
    HIP_OK(c, hipMemcpyAsync(s.col16, h->col_idx, nnz * sizeof(uint16_t), hipMemcpyHostToDevice,
                             c->copy_stream));
    HIP_OK(c, hipMemcpyAsync(s.val16, h->val, nnz * sizeof(uint16_t), hipMemcpyHostToDevice,
                             c->copy_stream));
    HIP_OK(c, tlda::launch_widen_u16(s.col16, s.val16, nnz, s.col_idx, s.val, c->copy_stream));
  }
  HIP_OK(c, hipEventRecord(s.ready, c->copy_stream));
  HIP_OK(c, hipEventRecord(s.free_, c->copy_stream));
  s.used = true;
  dev_out->n_rows = h->n_rows;
  dev_out->nnz = h->nnz;
  dev_out->row_ptr = s.row_ptr;
  dev_out->col_idx = s.col_idx;
  dev_out->val = s.val;
  dev_out->slot = slot;
  dev_out->first_doc = h->first_doc;
  return TLDA_OK;
}

tlda_status tlda_get_stats(const tlda_ctx* c, int64_t* N, int64_t* n_skipped, int64_t* totals) {
  if (!c) return TLDA_ERR_ARG;
  unsigned long long counts[2];
  HIP_OK(c, hipMemcpyAsync(counts, c->mom.counts, sizeof(counts), hipMemcpyDeviceToHost, c->stream));
  if (totals)
    HIP_OK(c, hipMemcpyAsync(totals, c->mom.totals, sizeof(int64_t) * c->cfg.V,
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (N) *N = (int64_t)counts[0];
  if (n_skipped) *n_skipped = (int64_t)counts[1];
  return TLDA_OK;
}

tlda_status tlda_get_whitening(const tlda_ctx* c, double* W, double* eig, double* M1) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  const size_t V = c->cfg.V, D = c->cfg.D;
  if (W) HIP_OK(c, hipMemcpyAsync(W, c->wh.W, sizeof(double) * V * D, hipMemcpyDeviceToHost, c->stream));
  if (eig) HIP_OK(c, hipMemcpyAsync(eig, c->wh.eig, sizeof(double) * D, hipMemcpyDeviceToHost, c->stream));
  if (M1) HIP_OK(c, hipMemcpyAsync(M1, c->wh.m, sizeof(double) * V, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return TLDA_OK;
}

tlda_status tlda_set_whitening(tlda_ctx* c, const double* W, const double* M1) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, W && M1, TLDA_ERR_ARG, "W or M1 is NULL");
  const int V = c->cfg.V, D = c->cfg.D;
  for (int i = 0; i < V * D; ++i)
    CHECK_ARG(c, std::isfinite(W[i]), TLDA_ERR_ARG, "W has a non-finite entry");
  for (int d = 0; d < D; ++d) {
    double s = 0.0;
    for (int i = 0; i < V; ++i) s += W[(size_t)i * D + d] * W[(size_t)i * D + d];
    CHECK_ARG(c, s > 0.0, TLDA_ERR_NUMERIC, "W has a zero column");
  }
  tlda_status st = save_prev(c);
  if (st != TLDA_OK) return st;
  HIP_OK(c, hipMemcpyAsync(c->wh.W, W, sizeof(double) * (size_t)V * D, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->wh.m, M1, sizeof(double) * V, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, tlda::launch_from_injected(c->wh.W, V, D, c->wh.U, c->wh.eig, c->stream));
  HIP_OK(c, form_whitening(c));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->wh.ready = true;
  return TLDA_OK;
}

tlda_status tlda_rebase_phi(tlda_ctx* c, float* Phi) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, Phi != nullptr, TLDA_ERR_ARG, "Phi is NULL");
  CHECK_ARG(c, c->wh.ready && c->wh.prev_ready, TLDA_ERR_STATE,
            "no previous whitening to rebase from");
  const int V = c->cfg.V, D = c->cfg.D, K = c->cfg.K;
  tlda::EigScope scope(eig_env(c));
  HIP_OK(c, tlda::launch_gram(c->wh.U, c->wh.Uprev, c->wh.C, V, D, c->stream));
  HIP_OK(c, tlda::launch_rebase(c->wh.C, c->wh.eig, c->wh.eigprev, D, K, Phi, c->stream));
  return TLDA_OK;
}

tlda_status tlda_set_timing_events(tlda_ctx* c, void* const* start, void* const* stop,
                                   int32_t n) {
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, n >= 0, TLDA_ERR_ARG, "negative event count");
  CHECK_ARG(c, n == 0 || (start && stop), TLDA_ERR_ARG, "event arrays are NULL");
  for (int i = 0; i < n; ++i)
    CHECK_ARG(c, start[i] && stop[i], TLDA_ERR_ARG, "an event is NULL");
  delete[] c->t_start;
  delete[] c->t_stop;
  c->t_start = c->t_stop = nullptr;
  c->t_n = c->t_next = 0;
  if (n == 0) return TLDA_OK;
  c->t_start = new (std::nothrow) hipEvent_t[n];
  c->t_stop = new (std::nothrow) hipEvent_t[n];
  if (!c->t_start || !c->t_stop) {
    delete[] c->t_start;
    delete[] c->t_stop;
    c->t_start = c->t_stop = nullptr;
    return TLDA_ERR_OOM;
  }
  for (int i = 0; i < n; ++i) {
    c->t_start[i] = static_cast<hipEvent_t>(start[i]);
    c->t_stop[i] = static_cast<hipEvent_t>(stop[i]);
  }
  c->t_n = n;
  return TLDA_OK;
}

// ---------------------------------------------------------------------------
// Document-topic encoder
// ---------------------------------------------------------------------------
namespace {

void mlp_free(tlda_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  dfree(m->params); dfree(m->wb); dfree(m->grads); dfree(m->adam_m); dfree(m->adam_v);
  dfree(m->Z1); dfree(m->Z2); dfree(m->H1); dfree(m->H2); dfree(m->logits); dfree(m->dZ3);
  dfree(m->dZa); dfree(m->dZb); dfree(m->row_loss); dfree(m->ws);
  delete m;
}

#define MLP_OK(m, expr)                                                            \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      (m)->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return e_ == hipErrorOutOfMemory ? TLDA_ERR_OOM : TLDA_ERR_DEVICE;           \
    }                                                                              \
  } while (0)

#define MLP_CHECK(m, cond, code, msg) \
  do {                                \
    if (!(cond)) {                    \
      (m)->last_error = msg;          \
      return code;                    \
    }                                 \
  } while (0)

}  // namespace

int64_t tlda_mlp_param_count(int32_t d_in, int32_t hidden, int32_t k_out) {
  if (d_in < 1 || hidden < 1 || k_out < 1) return 0;
  return (int64_t)tlda::mlp_param_count(d_in, hidden, k_out);
}

tlda_status tlda_mlp_create(int32_t d_in, int32_t hidden, int32_t k_out, int32_t max_batch,
                            void* hip_stream, tlda_mlp** out) {
  if (out == nullptr) return TLDA_ERR_ARG;
  *out = nullptr;
  if (d_in < 1 || d_in > TLDA_MLP_MAX_WIDTH || hidden < 1 || hidden > TLDA_MLP_MAX_WIDTH ||
      k_out < 1 || k_out > TLDA_MAX_K || max_batch < 1)
    return TLDA_ERR_SHAPE;
  tlda_mlp* m = new (std::nothrow) tlda_mlp();
  if (!m) return TLDA_ERR_OOM;
  m->d_in = d_in;
  m->hidden = hidden;
  m->k_out = k_out;
  m->max_batch = max_batch;
  m->n_params = tlda::mlp_param_count(d_in, hidden, k_out);
  m->stream = static_cast<hipStream_t>(hip_stream);
  const size_t P = m->n_params, B = (size_t)max_batch, H = hidden, K = k_out;
  bool ok = dalloc(&m->params, P) == hipSuccess && dalloc(&m->wb, P) == hipSuccess &&
            dalloc(&m->grads, P) == hipSuccess && dalloc(&m->adam_m, P) == hipSuccess &&
            dalloc(&m->adam_v, P) == hipSuccess && dalloc(&m->Z1, B * H) == hipSuccess &&
            dalloc(&m->Z2, B * H) == hipSuccess && dalloc(&m->H1, B * H) == hipSuccess &&
            dalloc(&m->H2, B * H) == hipSuccess && dalloc(&m->logits, B * K) == hipSuccess &&
            dalloc(&m->dZ3, B * K) == hipSuccess && dalloc(&m->dZa, B * H) == hipSuccess &&
            dalloc(&m->dZb, B * H) == hipSuccess && dalloc(&m->row_loss, B) == hipSuccess &&
            dalloc(&m->ws, tlda::mlp_workspace_floats(d_in, hidden, k_out, max_batch)) ==
                hipSuccess;
  if (!ok) {
    mlp_free(m);
    return TLDA_ERR_OOM;
  }
  if (launch_zero(m->params, P * sizeof(float), m->stream) != hipSuccess ||
      launch_zero(m->wb, P * sizeof(uint16_t), m->stream) != hipSuccess ||
      launch_zero(m->adam_m, P * sizeof(float), m->stream) != hipSuccess ||
      launch_zero(m->adam_v, P * sizeof(float), m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess) {
    mlp_free(m);
    return TLDA_ERR_DEVICE;
  }
  *out = m;
  return TLDA_OK;
}

void tlda_mlp_destroy(tlda_mlp* mlp) { mlp_free(mlp); }

const char* tlda_mlp_last_error(const tlda_mlp* mlp) { return mlp ? mlp->last_error.c_str() : ""; }

tlda_status tlda_mlp_set_params(tlda_mlp* m, const float* host_params) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, host_params != nullptr, TLDA_ERR_ARG, "params is NULL");
  for (size_t i = 0; i < m->n_params; ++i)
    MLP_CHECK(m, std::isfinite(host_params[i]), TLDA_ERR_ARG, "a parameter is not finite");
  MLP_OK(m, hipMemcpyAsync(m->params, host_params, m->n_params * sizeof(float),
                           hipMemcpyHostToDevice, m->stream));
  MLP_OK(m, tlda::mlp_refresh_bf16(*m));
  MLP_OK(m, launch_zero(m->adam_m, m->n_params * sizeof(float), m->stream));
  MLP_OK(m, launch_zero(m->adam_v, m->n_params * sizeof(float), m->stream));
  MLP_OK(m, hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  return TLDA_OK;
}

tlda_status tlda_mlp_get_params(tlda_mlp* m, float* host_params) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, host_params != nullptr, TLDA_ERR_ARG, "params is NULL");
  MLP_OK(m, hipMemcpyAsync(host_params, m->params, m->n_params * sizeof(float),
                           hipMemcpyDeviceToHost, m->stream));
  MLP_OK(m, hipStreamSynchronize(m->stream));
  return TLDA_OK;
}

tlda_status tlda_mlp_forward(tlda_mlp* m, const float* X, int64_t n_rows, float* theta_out) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, n_rows >= 0, TLDA_ERR_SHAPE, "negative n_rows");
  MLP_CHECK(m, (X && theta_out) || n_rows == 0, TLDA_ERR_ARG, "X or theta is NULL");
  for (int64_t r0 = 0; r0 < n_rows; r0 += m->max_batch) {
    const int n = (int)std::min<int64_t>(m->max_batch, n_rows - r0);
    MLP_OK(m, tlda::mlp_forward(*m, X + r0 * m->d_in, n, theta_out + r0 * m->k_out, false));
  }
  return TLDA_OK;
}

tlda_status tlda_mlp_gradients(tlda_mlp* m, const float* X, const float* T, int32_t n_rows,
                               float* grads_out, float* loss_out) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, n_rows >= 1 && n_rows <= m->max_batch, TLDA_ERR_SHAPE,
            "n_rows must be in 1 .. max_batch");
  MLP_CHECK(m, X && T, TLDA_ERR_ARG, "X or T is NULL");
  MLP_OK(m, tlda::mlp_forward(*m, X, n_rows, nullptr, true));
  MLP_OK(m, tlda::mlp_backward(*m, X, T, n_rows, loss_out));
  if (grads_out)
    MLP_OK(m, hipMemcpyAsync(grads_out, m->grads, m->n_params * sizeof(float),
                             hipMemcpyDeviceToDevice, m->stream));
  return TLDA_OK;
}

tlda_status tlda_mlp_train_step(tlda_mlp* m, const float* X, const float* T, int32_t n_rows,
                                float lr, float* loss_out) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, std::isfinite(lr) && lr > 0.f, TLDA_ERR_ARG, "lr must be finite and > 0");
  tlda_status st = tlda_mlp_gradients(m, X, T, n_rows, nullptr, loss_out);
  if (st != TLDA_OK) return st;
  MLP_OK(m, tlda::mlp_adam(*m, lr, 0.9f, 0.999f, 1e-8f));
  return TLDA_OK;
}

tlda_status tlda_infer_doc_topics_mlp(tlda_ctx* c, tlda_mlp* m, const float* X, int32_t n_rows,
                                      const double* mu, float gap_tol, int32_t min_steps,
                                      int32_t max_iter, float* theta_out,
                                      int32_t* n_stepped_out) {
  if (!c) return TLDA_ERR_ARG;
  if (m != nullptr) {
    CHECK_ARG(c, m->d_in == c->cfg.D && m->k_out == c->cfg.K, TLDA_ERR_SHAPE,
              "encoder widths do not match the context's D and K");
    CHECK_ARG(c, m->stream == c->stream, TLDA_ERR_ARG,
              "the encoder and the context must share a stream");
  }
  CHECK_ARG(c, n_rows >= 0 && max_iter >= 0 && min_steps >= 0, TLDA_ERR_ARG,
            "negative n_rows, min_steps or max_iter");
  CHECK_ARG(c, gap_tol >= 0.0f && std::isfinite(gap_tol), TLDA_ERR_ARG,
            "gap_tol must be finite and >= 0");
  CHECK_ARG(c, mu != nullptr, TLDA_ERR_ARG, "mu is NULL");
  CHECK_ARG(c, (X && theta_out) || n_rows == 0, TLDA_ERR_ARG, "X or theta is NULL");
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  int32_t* ns = n_stepped_out ? n_stepped_out : c->dev_flags + 3;
  HIP_OK(c, launch_zero(ns, sizeof(int32_t), c->stream));
  if (n_rows == 0) return TLDA_OK;
  const int V = c->cfg.V, D = c->cfg.D, K = c->cfg.K;
  HIP_OK(c, launch_zero(c->dev_flags + 1, sizeof(int), c->stream));
  HIP_OK(c, tlda::launch_inference_setup(c->wh.W, c->wh.m, mu, V, D, K, c->postA, c->postG,
                                         c->postZ, c->postEv, c->A32, c->G32, c->step32,
                                         c->dev_flags + 1, c->stream));
  if (m != nullptr) {
    tlda_status st = tlda_mlp_forward(m, X, n_rows, theta_out);
    if (st != TLDA_OK) {
      set_err(c, m->last_error);
      return st;
    }
  }
  HIP_OK(c, tlda::launch_infer_gap(X, n_rows, c->A32, c->G32, c->step32, D, K, m != nullptr,
                                   gap_tol, min_steps, max_iter, theta_out, ns, c->stream));
  return TLDA_OK;
}

// ---------------------------------------------------------------------------
// Batched time slices: one launch per step over many slices
// ---------------------------------------------------------------------------
struct tlda_multi {
  int n = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  std::vector<tlda_ctx*> ctxs;
  std::vector<tlda::SliceStep> host;   // table without the block layout
  std::vector<int> rows;               // documents of each slice's batch
  int tile = 0;                        // tile shape of the reduction (0 .. kMultiTiles - 1)
  tlda::SliceStep* d_table = nullptr;
  int* d_blk_slice = nullptr;
  int* d_fin_slice = nullptr;
  int n_blocks = 0, n_fin = 0, max_dk = 0, total_blocks = 0;
  float* partial = nullptr;
  int* counts = nullptr;
  size_t cap_partial = 0, cap_counts = 0, cap_blk = 0, cap_fin = 0;
  std::string last_error;
};

struct tlda_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
};

namespace {

void multi_free(tlda_multi* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  dfree(m->d_table); dfree(m->d_blk_slice); dfree(m->d_fin_slice); dfree(m->partial);
  dfree(m->counts);
  delete m;
}

// Lay out total_blocks reduction blocks over the slices in proportion to
// their row tiles of the plan's tile shape (at least one each, at most one
// per tile), and the finish blocks; upload the tables (synchronous, never
// inside a capture).
tlda_status multi_layout(tlda_multi* m, int total_blocks) {
  const int tr = tlda::multi_tile_rows(m->tile);
  std::vector<int> tiles(m->n);
  long long all_tiles = 0;
  for (int i = 0; i < m->n; ++i) {
    tiles[i] = (m->rows[i] + tr - 1) / tr;
    all_tiles += tiles[i];
  }
  if (total_blocks <= 0) total_blocks = tlda::cp_bf16_multi_per_cu(m->tile) * m->num_cu;
  std::vector<tlda::SliceStep> tab = m->host;
  std::vector<int> blk_slice, fin_slice;
  size_t need_p = 0, need_c = 0;
  int max_dk = 1;
  for (int i = 0; i < m->n; ++i) {
    tlda::SliceStep& d = tab[i];
    long long want = all_tiles > 0 ? (long long)((double)total_blocks * tiles[i] / all_tiles + 0.5) : 1;
    int nb = (int)std::max<long long>(1, std::min<long long>(want, std::max(1, tiles[i])));
    d.nblk = nb;
    d.blk0 = (int)blk_slice.size();
    for (int b = 0; b < nb; ++b) blk_slice.push_back(i);
    d.fin0 = (int)fin_slice.size();
    const int nf = (d.D * d.K + tlda::kFinishEntries - 1) / tlda::kFinishEntries;
    for (int b = 0; b < nf; ++b) fin_slice.push_back(i);
    need_p += (size_t)nb * d.D * d.K;
    need_c += (size_t)nb;
    max_dk = std::max(max_dk, d.D * d.K);
  }
  MLP_OK(m, hipStreamSynchronize(m->stream));
  if (m->cap_partial < need_p) {
    dfree(m->partial);
    m->cap_partial = 0;
    MLP_OK(m, dalloc(&m->partial, need_p));
    m->cap_partial = need_p;
  }
  if (m->cap_counts < need_c) {
    dfree(m->counts);
    m->cap_counts = 0;
    MLP_OK(m, dalloc(&m->counts, need_c));
    m->cap_counts = need_c;
  }
  if (m->cap_blk < blk_slice.size()) {
    dfree(m->d_blk_slice);
    m->cap_blk = 0;
    MLP_OK(m, dalloc(&m->d_blk_slice, blk_slice.size()));
    m->cap_blk = blk_slice.size();
  }
  if (m->cap_fin < fin_slice.size()) {
    dfree(m->d_fin_slice);
    m->cap_fin = 0;
    MLP_OK(m, dalloc(&m->d_fin_slice, fin_slice.size()));
    m->cap_fin = fin_slice.size();
  }
  size_t op = 0, oc = 0;
  for (auto& d : tab) {
    d.partial = m->partial + op;
    d.block_counts = m->counts + oc;
    op += (size_t)d.nblk * d.D * d.K;
    oc += (size_t)d.nblk;
  }
  MLP_OK(m, hipMemcpy(m->d_table, tab.data(), sizeof(tlda::SliceStep) * m->n,
                      hipMemcpyHostToDevice));
  MLP_OK(m, hipMemcpy(m->d_blk_slice, blk_slice.data(), sizeof(int) * blk_slice.size(),
                      hipMemcpyHostToDevice));
  MLP_OK(m, hipMemcpy(m->d_fin_slice, fin_slice.data(), sizeof(int) * fin_slice.size(),
                      hipMemcpyHostToDevice));
  m->n_blocks = (int)blk_slice.size();
  m->n_fin = (int)fin_slice.size();
  m->max_dk = max_dk;
  m->total_blocks = total_blocks;
  return TLDA_OK;
}

}  // namespace

tlda_status tlda_multi_create(int32_t n_slices, tlda_ctx* const* ctxs,
                              const tlda_csr_batch* batches, float* const* Phis,
                              const float* betas, int32_t* n_kept_out, tlda_multi** out) {
  if (out == nullptr) return TLDA_ERR_ARG;
  *out = nullptr;
  if (n_slices < 1 || !ctxs || !batches || !Phis || !betas) return TLDA_ERR_ARG;
  for (int i = 0; i < n_slices; ++i) {
    tlda_ctx* c = ctxs[i];
    if (!c || !Phis[i] || !std::isfinite(betas[i])) return TLDA_ERR_ARG;
    if (is_classic(c)) return TLDA_ERR_ARG;   // the multi-slice step is the centred one
    if (!is_bf16(c) || tlda::multi_shape(c->cfg.D, c->cfg.K) < 0) return TLDA_ERR_SHAPE;
    if (!c->wh.ready) return TLDA_ERR_STATE;
    if (c->stream != ctxs[0]->stream) return TLDA_ERR_ARG;
    const tlda_csr_batch& b = batches[i];
    if (b.slot >= 0 || b.n_rows < 0 || b.nnz < 0) return TLDA_ERR_ARG;
    if (b.n_rows > 0 && !b.row_ptr) return TLDA_ERR_ARG;
    if (b.nnz > 0 && (!b.col_idx || !b.val)) return TLDA_ERR_ARG;
  }
  tlda_multi* m = new (std::nothrow) tlda_multi();
  if (!m) return TLDA_ERR_OOM;
  m->n = n_slices;
  m->stream = ctxs[0]->stream;
  m->num_cu = ctxs[0]->num_cu;
  m->ctxs.assign(ctxs, ctxs + n_slices);
  for (int i = 0; i < n_slices; ++i) {
    tlda_ctx* c = ctxs[i];
    const tlda_csr_batch& b = batches[i];
    if (c->cfg.flags & TLDA_VALIDATE_CSR) {
      tlda_status st = validate_content(c, &b);
      if (st != TLDA_OK) {
        multi_free(m);
        return st;
      }
    }
    tlda::SliceStep d{};
    d.row_ptr = b.row_ptr;
    d.col_idx = b.col_idx;
    d.val = b.val;
    d.n_rows = b.n_rows;
    d.W16 = c->wh.W16;
    d.mw16 = c->wh.mw16;
    d.Dh = c->Dh;
    d.D = c->cfg.D;
    d.K = c->cfg.K;
    d.shape = tlda::multi_shape(d.D, d.K);
    d.Phi = Phis[i];
    d.phi_copy = c->cp.phi0;
    d.grad = c->cp.grad;
    d.R1 = c->cp.R1;
    d.n_kept_out = n_kept_out ? n_kept_out + i : nullptr;
    d.alpha0 = c->cfg.alpha0;
    d.theta = c->cfg.theta;
    d.beta = betas[i];
    m->host.push_back(d);
    m->rows.push_back(b.n_rows);
  }
  if (dalloc(&m->d_table, (size_t)n_slices) != hipSuccess) {
    multi_free(m);
    return TLDA_ERR_OOM;
  }
  tlda_status st = multi_layout(m, 0);
  if (st != TLDA_OK) {
    multi_free(m);
    return st;
  }
  *out = m;
  return TLDA_OK;
}

void tlda_multi_destroy(tlda_multi* plan) { multi_free(plan); }

const char* tlda_multi_last_error(const tlda_multi* plan) {
  return plan ? plan->last_error.c_str() : "";
}

tlda_status tlda_multi_set_blocks(tlda_multi* m, int32_t total_blocks) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, total_blocks >= 0 && total_blocks <= (1 << 20), TLDA_ERR_ARG,
            "total_blocks out of range");
  return multi_layout(m, total_blocks);
}

tlda_status tlda_multi_set_tile(tlda_multi* m, int32_t rows_per_tile, int32_t waves_per_block) {
  if (!m) return TLDA_ERR_ARG;
  int v = -1;
  for (int i = 0; i < tlda::kMultiTiles; ++i)
    if (tlda::multi_tile_rows(i) == rows_per_tile && tlda::multi_tile_waves(i) == waves_per_block)
      v = i;
  MLP_CHECK(m, v >= 0, TLDA_ERR_ARG, "tile shape must be 64 x 4, 32 x 4 or 64 x 8");
  const int prev = m->tile;
  m->tile = v;
  tlda_status st = multi_layout(m, 0);
  if (st != TLDA_OK) m->tile = prev;
  return st;
}

tlda_status tlda_multi_get_tile(const tlda_multi* m, int32_t* rows_per_tile,
                                int32_t* waves_per_block) {
  if (!m || !rows_per_tile || !waves_per_block) return TLDA_ERR_ARG;
  *rows_per_tile = tlda::multi_tile_rows(m->tile);
  *waves_per_block = tlda::multi_tile_waves(m->tile);
  return TLDA_OK;
}

tlda_status tlda_multi_get_blocks(const tlda_multi* m, int32_t* total_blocks) {
  if (!m || !total_blocks) return TLDA_ERR_ARG;
  *total_blocks = m->total_blocks;
  return TLDA_OK;
}

tlda_status tlda_multi_step(tlda_multi* m) {
  if (!m) return TLDA_ERR_ARG;
  MLP_OK(m, tlda::launch_cp_bf16_multi(m->d_table, m->d_blk_slice, m->n_blocks, m->tile,
                                       m->stream));
  MLP_OK(m, tlda::launch_cp_finish_multi(m->d_table, m->d_fin_slice, m->n_fin, m->max_dk,
                                         m->stream));
  return TLDA_OK;
}

tlda_status tlda_multi_autotune(tlda_multi* m, int32_t reps, int32_t* total_blocks_out) {
  if (!m) return TLDA_ERR_ARG;
  MLP_CHECK(m, reps >= 1 && reps <= 1000, TLDA_ERR_ARG, "reps must be in 1 .. 1000");
  // steps change Phi: keep each slice's Phi and restore it after every trial
  std::vector<float*> saved(m->n, nullptr);
  auto release = [&]() {
    for (auto& p : saved) dfree(p);
  };
  for (int i = 0; i < m->n; ++i) {
    const size_t dk = (size_t)m->host[i].D * m->host[i].K;
    if (dalloc(&saved[i], dk) != hipSuccess ||
        hipMemcpyAsync(saved[i], m->host[i].Phi, dk * sizeof(float), hipMemcpyDeviceToDevice,
                       m->stream) != hipSuccess) {
      release();
      m->last_error = "could not keep a copy of Phi";
      return TLDA_ERR_OOM;
    }
  }
  auto restore = [&]() -> hipError_t {
    for (int i = 0; i < m->n; ++i) {
      const size_t dk = (size_t)m->host[i].D * m->host[i].K;
      hipError_t e = hipMemcpyAsync(m->host[i].Phi, saved[i], dk * sizeof(float),
                                    hipMemcpyDeviceToDevice, m->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // candidates: every tile shape with 1, 2, ... resident blocks per CU and
  // two full rounds
  std::vector<std::pair<int, int>> cands;   // (tile shape, total blocks)
  for (int v = 0; v < tlda::kMultiTiles; ++v) {
    const int per_cu = tlda::cp_bf16_multi_per_cu(v);
    for (int b = 1; b <= per_cu; ++b) cands.push_back({v, b * m->num_cu});
    cands.push_back({v, 2 * per_cu * m->num_cu});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tlda_status st = TLDA_OK;
  std::pair<int, int> best = cands.front();
  float best_ms = 0.f;
  const int tile_entry = m->tile;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = TLDA_ERR_DEVICE;
  } else {
    for (const auto& cand : cands) {
      m->tile = cand.first;
      st = multi_layout(m, cand.second);
      if (st != TLDA_OK) break;
      if ((st = tlda_multi_step(m)) != TLDA_OK) break;   // warm-up
      hipEventRecord(e0, m->stream);
      for (int r = 0; r < reps && st == TLDA_OK; ++r) st = tlda_multi_step(m);
      hipEventRecord(e1, m->stream);
      if (st != TLDA_OK || hipEventSynchronize(e1) != hipSuccess) {
        if (st == TLDA_OK) st = TLDA_ERR_DEVICE;
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (best_ms == 0.f || ms < best_ms) {
        best_ms = ms;
        best = cand;
      }
      if (restore() != hipSuccess) {
        st = TLDA_ERR_DEVICE;
        break;
      }
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  m->tile = st == TLDA_OK ? best.first : tile_entry;
  if (st == TLDA_OK) st = multi_layout(m, best.second);
  if (restore() != hipSuccess || hipStreamSynchronize(m->stream) != hipSuccess)
    st = st == TLDA_OK ? TLDA_ERR_DEVICE : st;
  release();
  if (st == TLDA_OK && total_blocks_out) *total_blocks_out = best.second;
  return st;
}

tlda_status tlda_graph_capture(tlda_multi* const* plans, int32_t n_plans, tlda_graph** out) {
  if (!out) return TLDA_ERR_ARG;
  *out = nullptr;
  if (n_plans < 1 || !plans) return TLDA_ERR_ARG;
  for (int i = 0; i < n_plans; ++i)
    if (!plans[i] || plans[i]->stream != plans[0]->stream) return TLDA_ERR_ARG;
  hipStream_t s = plans[0]->stream;
  if (s == nullptr) return TLDA_ERR_ARG;      // the null stream cannot be captured
  if (hipStreamSynchronize(s) != hipSuccess) return TLDA_ERR_DEVICE;
  tlda_graph* g = new (std::nothrow) tlda_graph();
  if (!g) return TLDA_ERR_OOM;
  g->stream = s;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete g;
    return TLDA_ERR_DEVICE;
  }
  tlda_status st = TLDA_OK;
  for (int i = 0; i < n_plans && st == TLDA_OK; ++i) st = tlda_multi_step(plans[i]);
  hipError_t e = hipStreamEndCapture(s, &g->graph);
  if (st != TLDA_OK || e != hipSuccess ||
      hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
    return st != TLDA_OK ? st : TLDA_ERR_DEVICE;
  }
  *out = g;
  return TLDA_OK;
}

tlda_status tlda_graph_capture_steps(tlda_ctx* c, const tlda_csr_batch* batches, int32_t n,
                                     float beta, float* Phi, tlda_graph** out) {
  if (!out) return TLDA_ERR_ARG;
  *out = nullptr;
  if (!c) return TLDA_ERR_ARG;
  CHECK_ARG(c, n >= 1 && batches != nullptr && Phi != nullptr, TLDA_ERR_ARG,
            "need at least one batch, and Phi");
  CHECK_ARG(c, c->stream != nullptr, TLDA_ERR_ARG, "the null stream cannot be captured");
  CHECK_ARG(c, !is_classic(c), TLDA_ERR_ARG, "classic-moment steps are not captured");
  const int D = c->cfg.D, K = c->cfg.K;
  CHECK_ARG(c, is_bf16(c) || tlda::fused_supported(D, K, c->Dp), TLDA_ERR_SHAPE,
            "FP32 steps above the fused kernel's shapes are not captured");
  CHECK_ARG(c, c->wh.ready, TLDA_ERR_STATE, "no whitening matrix yet");
  CHECK_ARG(c, std::isfinite(beta), TLDA_ERR_ARG, "beta is not finite");
  // everything that may synchronise or allocate happens before the capture:
  // argument and content checks, and the largest partial buffer
  int max_rows = 0;
  for (int i = 0; i < n; ++i) {
    tlda_status st = check_batch(c, &batches[i]);
    if (st != TLDA_OK) return st;
    CHECK_ARG(c, batches[i].slot < 0, TLDA_ERR_ARG, "staged batches are not captured");
    st = validate_content(c, &batches[i]);
    if (st != TLDA_OK) return st;
    max_rows = std::max(max_rows, (int)batches[i].n_rows);
  }
  size_t need = 0;
  if (is_bf16(c)) {
    need = (size_t)bf16_grid(c, 0, max_rows) * D * K;
  } else {
    if (c->tune.fused_blocks <= 0) {
      int per_cu = 0;
      HIP_OK(c, tlda::launch_whiten_cp(batches[0], c->wh.W32, c->wh.mw32, D, c->Dp, c->Dt,
                                       w32_tail_base(c), Phi, K, 0,
                                       nullptr, &per_cu, nullptr, nullptr, nullptr, c->stream));
      c->tune.fused_blocks = (per_cu > 0 ? per_cu : 1) * c->num_cu;
    }
    int nblk = std::min(c->tune.fused_blocks, 2 * tlda::kWhitenBlockCounts);
    need = (size_t)nblk * D * K;
  }
  tlda_status st = ensure_partial(c, need);
  if (st != TLDA_OK) return st;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  tlda_graph* g = new (std::nothrow) tlda_graph();
  if (!g) return TLDA_ERR_OOM;
  g->stream = c->stream;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete g;
    CHECK_ARG(c, false, TLDA_ERR_DEVICE, "could not begin a capture on the context's stream");
  }
  c->in_capture = true;
  for (int i = 0; i < n && st == TLDA_OK; ++i)
    st = tlda_whiten_cp_step(c, &batches[i], beta, Phi, nullptr, nullptr, nullptr);
  c->in_capture = false;
  hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
  if (st != TLDA_OK || e != hipSuccess ||
      hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
    if (st != TLDA_OK) return st;
    CHECK_ARG(c, false, TLDA_ERR_DEVICE, "graph capture or instantiation failed");
  }
  *out = g;
  return TLDA_OK;
}

tlda_status tlda_graph_launch(tlda_graph* g) {
  if (!g) return TLDA_ERR_ARG;
  return hipGraphLaunch(g->exec, g->stream) == hipSuccess ? TLDA_OK : TLDA_ERR_DEVICE;
}

void tlda_graph_destroy(tlda_graph* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

// Checkpoint layout: header (magic, version, V, K, D, flags), the counts,
// token totals, the exact sum f, the exact pair-sum accumulator (when
// allocated), then W, U, eig and M1 (when ready).
namespace {
constexpr uint32_t kMagic = 0x41444c54u;   // "TLDA"
struct Header {
  uint32_t magic, version;
  int32_t V, K, D, has_acc, ready, moments;  // moments: 1 = classic (TLDA_CLASSIC), 0 = centred
};
constexpr uint32_t kVersion = 2u;           // 2: fixed-point moment accumulators
}  // namespace

tlda_status tlda_save_state(const tlda_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return TLDA_ERR_ARG;
  const size_t V = c->cfg.V, D = c->cfg.D;
  const bool has_acc = c->mom.acc != nullptr;
  const size_t acc_bytes = tlda::tri_words((int)V) * 8;
  size_t need = sizeof(Header) + 2 * 8 + V * 8 + V * 16;
  if (has_acc) need += acc_bytes;
  if (c->wh.ready) need += 2 * V * D * 8 + D * 8 + V * 8;
  if (!buf) {
    *len = need;
    return TLDA_OK;
  }
  CHECK_ARG(c, *len >= need, TLDA_ERR_SHAPE, "checkpoint buffer too small");
  char* p = static_cast<char*>(buf);
  Header h{kMagic, kVersion, (int32_t)V, c->cfg.K, (int32_t)D, has_acc ? 1 : 0, c->wh.ready ? 1 : 0,
           is_classic(c) ? 1 : 0};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  auto d2h = [&](const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMemcpyAsync(p, src, bytes, hipMemcpyDeviceToHost, c->stream);
    p += bytes;
    return e;
  };
  HIP_OK(c, d2h(c->mom.counts, 16));
  HIP_OK(c, d2h(c->mom.totals, V * 8));
  HIP_OK(c, d2h(c->mom.fsum, V * 16));
  if (has_acc) HIP_OK(c, d2h(c->mom.acc, acc_bytes));
  if (c->wh.ready) {
    HIP_OK(c, d2h(c->wh.W, V * D * 8));
    HIP_OK(c, d2h(c->wh.U, V * D * 8));
    HIP_OK(c, d2h(c->wh.eig, D * 8));
    HIP_OK(c, d2h(c->wh.m, V * 8));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  *len = need;
  return TLDA_OK;
}

tlda_status tlda_load_state(tlda_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return TLDA_ERR_ARG;
  CHECK_ARG(c, len >= sizeof(Header), TLDA_ERR_SHAPE, "checkpoint too short");
  Header h;
  std::memcpy(&h, buf, sizeof(h));
  CHECK_ARG(c, h.magic == kMagic && h.version == kVersion, TLDA_ERR_ARG,
            "not a checkpoint of this format");
  CHECK_ARG(c, h.V == c->cfg.V && h.K == c->cfg.K && h.D == c->cfg.D, TLDA_ERR_SHAPE,
            "checkpoint shape does not match the context");
  CHECK_ARG(c, (h.moments == 1) == is_classic(c), TLDA_ERR_ARG,
            "checkpoint moments (classic or centred) do not match the context");
  const size_t V = c->cfg.V, D = c->cfg.D;
  const size_t acc_bytes = tlda::tri_words((int)V) * 8;
  size_t need = sizeof(Header) + 16 + V * 8 + V * 16;
  if (h.has_acc) need += acc_bytes;
  if (h.ready) need += 2 * V * D * 8 + D * 8 + V * 8;
  CHECK_ARG(c, len >= need, TLDA_ERR_SHAPE, "checkpoint truncated");
  if (h.has_acc) {
    tlda_status st = ensure_acc(c);
    if (st != TLDA_OK) return st;
  }
  const char* p = static_cast<const char*>(buf) + sizeof(Header);
  auto h2d = [&](void* dst, size_t bytes) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, c->stream);
    p += bytes;
    return e;
  };
  HIP_OK(c, h2d(c->mom.counts, 16));
  HIP_OK(c, h2d(c->mom.totals, V * 8));
  HIP_OK(c, h2d(c->mom.fsum, V * 16));
  if (h.has_acc) HIP_OK(c, h2d(c->mom.acc, acc_bytes));
  else if (c->mom.acc) HIP_OK(c, launch_zero(c->mom.acc, acc_bytes, c->stream));
  if (h.ready) {
    HIP_OK(c, h2d(c->wh.W, V * D * 8));
    HIP_OK(c, h2d(c->wh.U, V * D * 8));
    HIP_OK(c, h2d(c->wh.eig, D * 8));
    HIP_OK(c, h2d(c->wh.m, V * 8));
    HIP_OK(c, form_whitening(c));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->wh.ready = h.ready != 0;
  c->wh.prev_ready = false;
  c->eig.warm = nullptr;
  return TLDA_OK;
}

}  // extern "C"
