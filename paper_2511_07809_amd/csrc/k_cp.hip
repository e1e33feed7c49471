// Batched stochastic tensor gradient step on the CP factors of the whitened,
// centred third moment (eq. vec_deriv and the update rule):
//   G = 3(1+theta) Phi (Phi^T Phi * Phi^T Phi) - 3 c3 / n X^T (X Phi * X Phi),
//   Phi <- Phi - beta G,   c3 = (alpha0 + 1)(alpha0 + 2) / 2.
// The data term R1 = X^T (X Phi)^2 is the only part that touches the batch;
// the D x D x D tensor is never formed.
//
// k_cp_reduce: each block walks a fixed set of row tiles (tile b, b + nblk,
// ...).  Per tile, Phi (D x K, resident in LDS for the whole block) and the
// X tile give S = X_t Phi with 4 x 4 register blocking, S is squared in LDS,
// and R1 += X_t^T S^2 accumulates in registers (each thread owns up to four
// 4 x 4 blocks of R1).  Each block writes its R1 partial; the row partition
// depends only on n_rows, so the reduction order is fixed.
#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRBlocks = 4;   // (D/4)*(K/4) <= 1024 for D*K <= 16384

__global__ void __launch_bounds__(kThreads) k_cp_reduce(const float* __restrict__ X, int n_rows,
                                                        const float* __restrict__ Phi, int D,
                                                        int K, int T, int nblk,
                                                        float* __restrict__ partial) {
  extern __shared__ float smem[];
  const int Dq = (D + 3) & ~3, Kq = (K + 3) & ~3;
  float* Ps = smem;                 // [Dq][Kq]
  float* Xs = Ps + Dq * Kq;         // [T][Dq]
  float* Ss = Xs + T * Dq;          // [T][Kq]
  const int tid = threadIdx.x;
  for (int e = tid; e < Dq * Kq; e += kThreads) {
    const int d = e / Kq, k = e % Kq;
    Ps[e] = (d < D && k < K) ? Phi[d * K + k] : 0.f;
  }
  const int nkb = Kq / 4, ndb = Dq / 4;
  const int nSb = (T / 4) * nkb;     // 4x4 blocks of S
  const int nRb = ndb * nkb;         // 4x4 blocks of R1
  float acc[kMaxRBlocks][4][4];
#pragma unroll
  for (int q = 0; q < kMaxRBlocks; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[q][i][j] = 0.f;

  const int ntiles = (n_rows + T - 1) / T;
  for (int tile = blockIdx.x; tile < ntiles; tile += nblk) {
    __syncthreads();
    const int r0 = tile * T;
    for (int e = tid; e < T * Dq; e += kThreads) {
      const int r = e / Dq, d = e % Dq;
      const int gr = r0 + r;
      Xs[e] = (gr < n_rows && d < D) ? X[(size_t)gr * D + d] : 0.f;
    }
    __syncthreads();
    // S = X_t Phi, squared
    for (int bidx = tid; bidx < nSb; bidx += kThreads) {
      const int rb = bidx / nkb, kb = bidx % nkb;
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) s[i][j] = 0.f;
      const float* x0 = Xs + (rb * 4) * Dq;
      for (int d = 0; d < Dq; ++d) {
        const float4 p = *reinterpret_cast<const float4*>(Ps + d * Kq + kb * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float xv = x0[i * Dq + d];
          s[i][0] = fmaf(xv, p.x, s[i][0]);
          s[i][1] = fmaf(xv, p.y, s[i][1]);
          s[i][2] = fmaf(xv, p.z, s[i][2]);
          s[i][3] = fmaf(xv, p.w, s[i][3]);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float4 o;
        o.x = s[i][0] * s[i][0];
        o.y = s[i][1] * s[i][1];
        o.z = s[i][2] * s[i][2];
        o.w = s[i][3] * s[i][3];
        *reinterpret_cast<float4*>(Ss + (rb * 4 + i) * Kq + kb * 4) = o;
      }
    }
    __syncthreads();
    // R1 += X_t^T S^2
#pragma unroll
    for (int q = 0; q < kMaxRBlocks; ++q) {
      const int bidx = tid + q * kThreads;
      if (bidx >= nRb) break;
      const int db = bidx / nkb, kb = bidx % nkb;
      for (int r = 0; r < T; ++r) {
        const float4 xv = *reinterpret_cast<const float4*>(Xs + r * Dq + db * 4);
        const float4 sv = *reinterpret_cast<const float4*>(Ss + r * Kq + kb * 4);
        const float xa[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[q][i][0] = fmaf(xa[i], sv.x, acc[q][i][0]);
          acc[q][i][1] = fmaf(xa[i], sv.y, acc[q][i][1]);
          acc[q][i][2] = fmaf(xa[i], sv.z, acc[q][i][2]);
          acc[q][i][3] = fmaf(xa[i], sv.w, acc[q][i][3]);
        }
      }
    }
  }
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < kMaxRBlocks; ++q) {
    const int bidx = tid + q * kThreads;
    if (bidx >= nRb) break;
    const int db = bidx / nkb, kb = bidx % nkb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int d = db * 4 + i;
      if (d >= D) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kb * 4 + j;
        if (k < K) out[d * K + k] = acc[q][i][j];
      }
    }
  }
}

// Gradient and update.  Thread (d, k) sums the partials of R1[d][k] in block
// order (FP64), forms its row of the penalty term
// 3(1+theta) sum_j Phi[d][j] (phi_j . phi_k)^2 from Phi (a few KB, cached),
// and writes grad[d][k].  Phi cannot be updated in place by the same threads
// (others still read it), so every block counts itself done and the last one
// applies Phi <- Phi - beta grad to all entries and re-arms the counter.
// n == 0 gives a zero gradient and leaves Phi unchanged.
__global__ void __launch_bounds__(256) k_cp_finalize(const float* __restrict__ partial, int nblk,
                                                     const int* __restrict__ n_kept, int n_rows,
                                                     float* __restrict__ Phi, int D, int K,
                                                     double alpha0, double theta, float beta,
                                                     float* __restrict__ grad,
                                                     double* __restrict__ R1,
                                                     int* __restrict__ sync) {
  __shared__ int is_last;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = n_kept != nullptr ? *n_kept : n_rows;
  if (e < D * K) {
    const int d = e / K, k = e % K;
    double r = 0.0;
    for (int b = 0; b < nblk; ++b) r += (double)partial[(size_t)b * D * K + e];
    R1[e] = r;
    if (n <= 0) {
      grad[e] = 0.f;
    } else {
      double pen = 0.0;
      for (int j = 0; j < K; ++j) {
        double g = 0.0;
        for (int q = 0; q < D; ++q) g += (double)Phi[q * K + j] * (double)Phi[q * K + k];
        pen += (double)Phi[d * K + j] * g * g;
      }
      const double c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0;
      grad[e] = (float)(3.0 * (1.0 + theta) * pen - 3.0 * c3 / (double)n * r);
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = (atomicAdd(sync, 1) == (int)gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (n > 0)
    for (int i = threadIdx.x; i < D * K; i += blockDim.x)
      Phi[i] = fmaf(-beta, __builtin_nontemporal_load(grad + i), Phi[i]);
  if (threadIdx.x == 0) atomicExch(sync, 0);
}

}  // namespace

// Row-tile height for the reduction: the largest of 64, 32, 16, 8, 4 whose
// LDS footprint (Phi + X tile + S tile) stays within 64 KiB.
int cp_tile_rows(int D, int K) {
  const int Dq = (D + 3) & ~3, Kq = (K + 3) & ~3;
  for (int T = 64; T >= 4; T >>= 1) {
    const size_t bytes = sizeof(float) * ((size_t)Dq * Kq + (size_t)T * (Dq + Kq));
    if (bytes <= 65536) return T;
  }
  return 0;
}

int cp_num_blocks(int n_rows, int D, int K) {
  const int T = cp_tile_rows(D, K);
  const int ntiles = (n_rows + T - 1) / T;
  return ntiles < 1024 ? (ntiles < 1 ? 1 : ntiles) : 1024;
}

hipError_t launch_cp_reduce(const float* X, int n_rows, const float* Phi, int D, int K, int nblk,
                            float* partial, hipStream_t s) {
  const int T = cp_tile_rows(D, K);
  const int Dq = (D + 3) & ~3, Kq = (K + 3) & ~3;
  const size_t bytes = sizeof(float) * ((size_t)Dq * Kq + (size_t)T * (Dq + Kq));
  hipLaunchKernelGGL(k_cp_reduce, dim3(nblk), dim3(kThreads), bytes, s, X, n_rows, Phi, D, K, T,
                     nblk, partial);
  return hipGetLastError();
}

hipError_t launch_cp_finalize(const float* partial, int nblk, const int* n_kept, int n_rows,
                              float* Phi, float* grad, int D, int K, double alpha0, double theta,
                              float beta, double* R1, int* sync, hipStream_t s) {
  hipLaunchKernelGGL(k_cp_finalize, dim3((D * K + 255) / 256), dim3(256), 0, s, partial, nblk,
                     n_kept, n_rows, Phi, D, K, alpha0, theta, beta, grad, R1, sync);
  return hipGetLastError();
}

}  // namespace tlda
