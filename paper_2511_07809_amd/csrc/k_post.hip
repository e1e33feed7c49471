// Post-processing and document-topic inference (FP64 unless noted).
//
// Unwhitening (section "Recovering the Topic Model Parameters" and Theorem 1)
// in the tight-frame reading for centred moments: with
// w_k = (1+theta)^(1/3) phi_k, the topic weight a_k is the root in (0, 1] of
// a^(1/3) |w_k|^2 + a = 1, the centred topic is nu_k = (W^T)^+ a_k^(-1/3) w_k
// with (W^T)^+ = U diag(lambda)^(1/2), and mu_k = nu_k + M1.
//
// Inference: theta_d = argmin over the simplex of |x_d - A theta|^2 with
// A = W^T (mu - M1 1^T), by projected gradient with step 1 / lambda_max(A^T A).
#include "tlda_internal.h"

namespace tlda {
namespace {

// Per topic: scale[k] = (1+theta)^(1/3) a_k^(-1/3), alpha[k] = a_k / sum a,
// lambda[k] = (1+theta) |phi_k|^3.  One block; K <= 256.
__global__ void __launch_bounds__(256) k_frame_weights(const float* __restrict__ Phi, int D, int K,
                                                       double theta, double* __restrict__ scale,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ lambda) {
  __shared__ double a_sh[256];
  const int k = threadIdx.x;
  double a = 0.0;
  if (k < K) {
    double n2 = 0.0;
    for (int d = 0; d < D; ++d) {
      const double v = (double)Phi[d * K + k];
      n2 += v * v;
    }
    const double c = cbrt(1.0 + theta);
    const double r = c * c * n2;   // |w_k|^2
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (cbrt(mid) * r + mid < 1.0) lo = mid;
      else hi = mid;
    }
    a = 0.5 * (lo + hi);
    scale[k] = c / cbrt(a);
    if (lambda != nullptr) lambda[k] = (1.0 + theta) * n2 * sqrt(n2);
  }
  a_sh[k] = a;
  __syncthreads();
  if (k < K) {
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += a_sh[j];
    alpha[k] = a / s;
  }
}

// Classic recovery: lambda_k = (1+theta)|phi_k|^3, scale[k] = lambda_k / |phi_k|
// (so that mu_k = lambda_k (W^T)^+ phi_k / |phi_k|), alpha_k proportional to
// lambda_k^-2; a zero column gets scale 0 and weight 0.  One block; K <= 256.
__global__ void __launch_bounds__(256) k_classic_weights(const float* __restrict__ Phi, int D,
                                                         int K, double theta,
                                                         double* __restrict__ scale,
                                                         double* __restrict__ alpha,
                                                         double* __restrict__ lambda) {
  __shared__ double w_sh[256];
  const int k = threadIdx.x;
  double w = 0.0;
  if (k < K) {
    double n2 = 0.0;
    for (int d = 0; d < D; ++d) {
      const double v = (double)Phi[d * K + k];
      n2 += v * v;
    }
    const double lam = (1.0 + theta) * n2 * sqrt(n2);
    scale[k] = (1.0 + theta) * n2;
    w = lam > 0.0 ? 1.0 / (lam * lam) : 0.0;
    if (lambda != nullptr) lambda[k] = lam;
  }
  w_sh[k] = w;
  __syncthreads();
  if (k < K) {
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += w_sh[j];
    alpha[k] = s > 0.0 ? w / s : 0.0;
  }
}

// One block per column k of Phi (D <= 256): the column is read into LDS,
// then Phi[d][k] = eig[d]^(-1/2) sum_e C[d][e] eig_prev[e]^(1/2) phi[e].
__global__ void __launch_bounds__(256) k_rebase(const double* __restrict__ C,
                                                const double* __restrict__ eig,
                                                const double* __restrict__ eig_prev, int D, int K,
                                                float* __restrict__ Phi) {
  __shared__ double col[256];
  const int k = blockIdx.x, d = threadIdx.x;
  if (d < D) col[d] = (double)Phi[d * K + k] * sqrt(eig_prev[d]);
  __syncthreads();
  if (d < D) {
    double s = 0.0;
    for (int e = 0; e < D; ++e) s += C[d * D + e] * col[e];
    Phi[d * K + k] = (float)(s / sqrt(eig[d]));
  }
}

// mu[i][k] = sum_d U[i][d] sqrt(eig[d]) phi[d][k] scale[k] + m[i] (m may be NULL)
__global__ void k_mu(const float* __restrict__ Phi, const double* __restrict__ U,
                     const double* __restrict__ eig, const double* __restrict__ m,
                     const double* __restrict__ scale, int V, int D, int K,
                     double* __restrict__ mu) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)V * K) return;
  const int i = (int)(e / K), k = (int)(e % K);
  double s = 0.0;
  for (int d = 0; d < D; ++d) s += U[(size_t)i * D + d] * sqrt(eig[d]) * (double)Phi[d * K + k];
  mu[e] = s * scale[k] + (m != nullptr ? m[i] : 0.0);
}

// Clip negative entries and renormalise every column to sum one (a column
// with no positive entry is left at zero).  One block per column.
__global__ void __launch_bounds__(256) k_simplex_columns(double* __restrict__ mu, int V, int K) {
  __shared__ double red[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < V; i += blockDim.x) s += fmax(mu[(size_t)i * K + k], 0.0);
  red[tid] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double tot = red[0] > 0.0 ? red[0] : 1.0;
  for (int i = tid; i < V; i += blockDim.x) {
    const double v = fmax(mu[(size_t)i * K + k], 0.0);
    mu[(size_t)i * K + k] = v / tot;
  }
}

// A[d][k] = sum_i W[i][d] (mu[i][k] - m[i])
__global__ void k_infer_A(const double* __restrict__ W, const double* __restrict__ m,
                          const double* __restrict__ mu, int V, int D, int K,
                          double* __restrict__ A, float* __restrict__ A32) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * K) return;
  const int d = e / K, k = e % K;
  double s = 0.0;
  for (int i = 0; i < V; ++i) s += W[(size_t)i * D + d] * (mu[(size_t)i * K + k] - m[i]);
  A[e] = s;
  A32[e] = (float)s;
}

// G = A^T A (K x K) into the Jacobi work matrix Gw, plus an FP32 copy.
__global__ void k_infer_G(const double* __restrict__ A, int D, int K, double* __restrict__ Gw,
                          float* __restrict__ G32) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int j = e / K, k = e % K;
  double s = 0.0;
  for (int d = 0; d < D; ++d) s += A[d * K + j] * A[d * K + k];
  Gw[e] = s;
  G32[e] = (float)s;
}

// Orders this wave's LDS stores before its later LDS loads by other lanes.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ void k_infer_step(const double* __restrict__ ev, int K, float* __restrict__ step) {
  if (threadIdx.x != 0) return;
  double mx = 0.0;
  for (int k = 0; k < K; ++k) mx = fmax(mx, ev[k]);
  step[0] = mx > 0.0 ? (float)(1.0 / mx) : 0.0f;
}

// One wave per document; lane l owns topics l, l + 64, ... (TPL per lane).
// The simplex projection finds, for each topic, its rank in decreasing order
// (ties by index) and the sum of all values ranked at or above it; the
// largest rank r whose value exceeds (prefix_r - 1) / r sets the threshold.
//
// GIVEN: the start point is read from `out` (e.g. an encoder's output on the
// simplex) instead of the uniform 1/K.
// GAP_RULE: instead of stopping when the L1 change of an iterate falls below
// tol, stop at the first iterate after min_steps steps whose duality gap for
// h(t) = |x - A t|^2 / 2, g.t - min_k g_k with g = A^T (A t - x) = G t - b, is
// at most gap_tol (it bounds h(t) - min h); rows that need more than
// min_steps steps are counted in *n_stepped.
template <int TPL, bool GIVEN, bool GAP_RULE>
__global__ void __launch_bounds__(256) k_infer(const float* __restrict__ X, int n_rows,
                                               const float* __restrict__ A32,
                                               const float* __restrict__ G32,
                                               const float* __restrict__ step32, int D, int K,
                                               int max_iter, float tol, float* __restrict__ out,
                                               float gap_tol, int min_steps,
                                               int* __restrict__ n_stepped) {
  __shared__ float xs[4][TLDA_MAX_D];
  __shared__ float ys[4][64 * TPL];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wave;
  if (row >= n_rows) return;
  const float step = step32[0];
  for (int d = lane; d < D; d += 64) xs[wave][d] = X[(size_t)row * D + d];
  wave_sync();
  float b[TPL], t[TPL];
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    float s = 0.f;
    if (k < K)
      for (int d = 0; d < D; ++d) s = fmaf(A32[d * K + k], xs[wave][d], s);
    b[q] = s;
    if (GIVEN)
      t[q] = k < K ? out[(size_t)row * K + k] : 0.f;
    else
      t[q] = k < K ? 1.0f / (float)K : 0.f;
  }
  for (int it = 0; it < max_iter; ++it) {
#pragma unroll
    for (int q = 0; q < TPL; ++q) ys[wave][lane + 64 * q] = t[q];
    wave_sync();
    float y[TPL];
    float gt = 0.f, gmin = INFINITY;
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
      const int k = lane + 64 * q;
      float g = 0.f;
      if (k < K) {
        for (int j = 0; j < K; ++j) g = fmaf(G32[k * K + j], ys[wave][j], g);
        g -= b[q];
        gt = fmaf(g, t[q], gt);
        gmin = fminf(gmin, g);
      }
      y[q] = t[q] - step * g;
    }
    if (GAP_RULE) {
      for (int off = 32; off > 0; off >>= 1) {
        gt += __shfl_xor(gt, off, 64);
        gmin = fminf(gmin, __shfl_xor(gmin, off, 64));
      }
      if (it >= min_steps && gt - gmin <= gap_tol) break;   // within gap_tol of the minimum
      if (it == min_steps && lane == 0) atomicAdd(n_stepped, 1);
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < TPL; ++q) ys[wave][lane + 64 * q] = y[q];
    wave_sync();
    int best_rank = 0;
    float best_tau = 0.f;
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
      const int k = lane + 64 * q;
      if (k >= K) continue;
      int rank = 0;
      float pref = 0.f;
      for (int j = 0; j < K; ++j) {
        const float v = ys[wave][j];
        if (v > y[q] || (v == y[q] && j <= k)) {
          ++rank;
          pref += v;
        }
      }
      const float tau = (pref - 1.0f) / (float)rank;
      if (y[q] - tau > 0.f && rank > best_rank) {
        best_rank = rank;
        best_tau = tau;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const int orank = __shfl_xor(best_rank, off, 64);
      const float otau = __shfl_xor(best_tau, off, 64);
      if (orank > best_rank) {
        best_rank = orank;
        best_tau = otau;
      }
    }
    float change = 0.f;
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
      const int k = lane + 64 * q;
      const float tn = k < K ? fmaxf(y[q] - best_tau, 0.f) : 0.f;
      change += fabsf(tn - t[q]);
      t[q] = tn;
    }
    for (int off = 32; off > 0; off >>= 1) change += __shfl_xor(change, off, 64);
    wave_sync();
    if (!GAP_RULE && change < tol) break;
  }
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const int k = lane + 64 * q;
    if (k < K) out[(size_t)row * K + k] = t[q];
  }
}

}  // namespace

hipError_t launch_unwhiten(const float* Phi, const double* U, const double* eig, const double* m,
                           int V, int D, int K, double theta, uint32_t flags, double* mu,
                           double* alpha, double* lambda, double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_weights, dim3(1), dim3(256), 0, s, Phi, D, K, theta, scratch, alpha,
                     lambda);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t n = (size_t)V * K;
  hipLaunchKernelGGL(k_mu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Phi, U, eig, m,
                     scratch, V, D, K, mu);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (flags & TLDA_PROJECT_SIMPLEX) {
    hipLaunchKernelGGL(k_simplex_columns, dim3(K), dim3(256), 0, s, mu, V, K);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_rebase(const double* C, const double* eig, const double* eig_prev, int D, int K,
                         float* Phi, hipStream_t s) {
  hipLaunchKernelGGL(k_rebase, dim3(K), dim3(256), 0, s, C, eig, eig_prev, D, K, Phi);
  return hipGetLastError();
}

hipError_t launch_unwhiten_classic(const float* Phi, const double* U, const double* eig, int V,
                                   int D, int K, double theta, uint32_t flags, double* mu,
                                   double* alpha, double* lambda, double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_classic_weights, dim3(1), dim3(256), 0, s, Phi, D, K, theta, scratch,
                     alpha, lambda);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t n = (size_t)V * K;
  hipLaunchKernelGGL(k_mu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Phi, U, eig,
                     static_cast<const double*>(nullptr), scratch, V, D, K, mu);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (flags & TLDA_PROJECT_SIMPLEX) {
    hipLaunchKernelGGL(k_simplex_columns, dim3(K), dim3(256), 0, s, mu, V, K);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_inference_setup(const double* W, const double* m, const double* mu, int V,
                                  int D, int K, double* A, double* G, double* Z, double* ev,
                                  float* A32, float* G32, float* step32, int* info,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_infer_A, dim3((D * K + 255) / 256), dim3(256), 0, s, W, m, mu, V, D, K, A,
                     A32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_infer_G, dim3((K * K + 255) / 256), dim3(256), 0, s, A, D, K, G, G32);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_jacobi(G, Z, ev, K, info, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_infer_step, dim3(1), dim3(64), 0, s, ev, K, step32);
  return hipGetLastError();
}

template <bool GIVEN, bool GAP_RULE>
hipError_t launch_infer_t(const float* X, int n_rows, const float* A32, const float* G32,
                          const float* step32, int D, int K, int max_iter, float tol, float* theta,
                          float gap_tol, int min_steps, int* n_stepped, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  const dim3 grid((n_rows + 3) / 4);
  if (K <= 64)
    hipLaunchKernelGGL((k_infer<1, GIVEN, GAP_RULE>), grid, dim3(256), 0, s, X, n_rows, A32, G32,
                       step32, D, K, max_iter, tol, theta, gap_tol, min_steps,
                       n_stepped);
  else if (K <= 128)
    hipLaunchKernelGGL((k_infer<2, GIVEN, GAP_RULE>), grid, dim3(256), 0, s, X, n_rows, A32, G32,
                       step32, D, K, max_iter, tol, theta, gap_tol, min_steps,
                       n_stepped);
  else
    hipLaunchKernelGGL((k_infer<4, GIVEN, GAP_RULE>), grid, dim3(256), 0, s, X, n_rows, A32, G32,
                       step32, D, K, max_iter, tol, theta, gap_tol, min_steps,
                       n_stepped);
  return hipGetLastError();
}

hipError_t launch_infer(const float* X, int n_rows, const float* A32, const float* G32,
                        const float* step32, int D, int K, int max_iter, float tol,
                        float* theta, hipStream_t s) {
  return launch_infer_t<false, false>(X, n_rows, A32, G32, step32, D, K, max_iter, tol, theta,
                                      0.f, 0, nullptr, s);
}

hipError_t launch_infer_gap(const float* X, int n_rows, const float* A32, const float* G32,
                            const float* step32, int D, int K, bool given_start, float gap_tol,
                            int min_steps, int max_iter, float* theta, int* n_stepped,
                            hipStream_t s) {
  return given_start
             ? launch_infer_t<true, true>(X, n_rows, A32, G32, step32, D, K, max_iter, 0.f, theta,
                                          gap_tol, min_steps, n_stepped, s)
             : launch_infer_t<false, true>(X, n_rows, A32, G32, step32, D, K, max_iter, 0.f,
                                           theta, gap_tol, min_steps, n_stepped, s);
}

}  // namespace tlda
