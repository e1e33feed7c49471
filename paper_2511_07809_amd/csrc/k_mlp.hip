// Document-topic encoder: a d_in -> hidden -> hidden -> k_out perceptron that
// maps a whitened document to topic proportions (GELU hidden layers, softmax
// output), standing in for the per-document simplex-constrained solve of the
// inference step, which stays as its judge and fallback.
//
// Every layer is one tiled GEMM on BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation) with the bias, activation or activation-derivative
// applied in its epilogue; weights are FP32 masters with BF16 copies,
// activations are stored in BF16 and pre-activations in FP32 (for GELU').
// Training minimises the mean cross-entropy against solve outputs by Adam.
//   forward : Z1 = X W1 + b1, H1 = gelu(Z1), Z2 = H1 W2 + b2, H2 = gelu(Z2),
//             Z3 = H2 W3 + b3, P = softmax(Z3)
//   backward: dZ3 = (P - T)/B, dW3 = H2^T dZ3, dZ2 = (dZ3 W3^T) gelu'(Z2),
//             dW2 = H1^T dZ2, dZ1 = (dZ2 W2^T) gelu'(Z1), dW1 = X^T dZ1,
//             db = column sums of dZ
// gelu(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2, from the device
// math library's erff and expf.
#include <algorithm>
#include <cmath>

#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kThreads = 256;
constexpr int kTileM = 64, kTileN = 64, kTileK = 32, kLdsK = kTileK + 8;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

enum { kEpiBiasGelu = 0, kEpiBias = 1, kEpiStore = 2, kEpiDGelu = 3 };

__device__ __forceinline__ uint16_t to_bf16(float f) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
  const b16x2 h = __builtin_convertvector((f32x2{f, 0.f}), b16x2);
  return (uint16_t)(__builtin_bit_cast(uint32_t, h) & 0xffffu);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C[M][N] = op(A) op(B) with op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k]
// (A in FP32 when AF32, else BF16) and op(B)[k][n] = TB ? B[n*ldb + k] :
// B[k*ldb + n] (BF16).  One 64 x 64 tile per block; each wave owns a 32 x 32
// quarter (2 x 2 matrix-core tiles).  Operand tiles go through LDS with the
// reduction index contiguous, which is what the matrix core's A and B
// fragments need.
// grid.z splits the reduction (kEpiStore only): block z takes rows
// z k_chunk .. of the reduction index and writes its partial to
// Cf + z c_stride_z (k_sum_slices then adds the partials in order).
template <bool TA, bool TB, bool AF32, int EPI>
__global__ void __launch_bounds__(kThreads) k_gemm(int M, int N, int Kd, const void* __restrict__ Av,
                                                  int lda, const uint16_t* __restrict__ B, int ldb,
                                                  const float* __restrict__ bias,
                                                  float* __restrict__ Cf, uint16_t* __restrict__ Cb,
                                                  int ldc, const float* __restrict__ Zaux,
                                                  int k_chunk, size_t c_stride_z) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kTileM * kLdsK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kTileN * kLdsK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * kTileM, n0 = blockIdx.x * kTileN;
  const float* Af = static_cast<const float*>(Av);
  const uint16_t* Ab = static_cast<const uint16_t*>(Av);
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int kbeg = blockIdx.z * k_chunk;
  Kd = min(Kd, kbeg + k_chunk);              // this block's end of the reduction index
  if (EPI == kEpiStore) Cf += blockIdx.z * c_stride_z;
  for (int k0 = kbeg; k0 < Kd; k0 += kTileK) {
    __syncthreads();
    // ---- A tile: As[m][k] = op(A)[m0 + m][k0 + k] ----
    if (!TA) {
      const int m = tid >> 2, kc = (tid & 3) * 8;
      const int gm = m0 + m;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gk = k0 + kc + i;
        uint16_t v = 0;
        if (gm < M && gk < Kd)
          v = AF32 ? to_bf16(Af[(size_t)gm * lda + gk]) : Ab[(size_t)gm * lda + gk];
        As[m * kLdsK + kc + i] = v;
      }
    } else {
      const int kk = tid >> 3, mc = (tid & 7) * 8;
      const int gk = k0 + kk;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gm = m0 + mc + i;
        uint16_t v = 0;
        if (gm < M && gk < Kd)
          v = AF32 ? to_bf16(Af[(size_t)gk * lda + gm]) : Ab[(size_t)gk * lda + gm];
        As[(mc + i) * kLdsK + kk] = v;
      }
    }
    // ---- B tile: Bs[n][k] = op(B)[k0 + k][n0 + n] ----
    if (TB) {
      const int n = tid >> 2, kc = (tid & 3) * 8;
      const int gn = n0 + n;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gk = k0 + kc + i;
        Bs[n * kLdsK + kc + i] = (gn < N && gk < Kd) ? B[(size_t)gn * ldb + gk] : (uint16_t)0;
      }
    } else {
      const int kk = tid >> 3, nc = (tid & 7) * 8;
      const int gk = k0 + kk;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gn = n0 + nc + i;
        Bs[(nc + i) * kLdsK + kk] = (gn < N && gk < Kd) ? B[(size_t)gk * ldb + gn] : (uint16_t)0;
      }
    }
    __syncthreads();
    u32x4 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      af[i] = *reinterpret_cast<const u32x4*>(As + (wm * 32 + i * 16 + l16) * kLdsK + 8 * l4);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      bfr[j] = *reinterpret_cast<const u32x4*>(Bs + (wn * 32 + j * 16 + l16) * kLdsK + 8 * l4);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                            __builtin_bit_cast(bf16x8, bfr[j]),
                                                            acc[i][j], 0, 0, 0);
  }
  // ---- epilogue: lane holds rows 4 l4 + r, column l16 of each 16 x 16 tile ----
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + l16;
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * l4 + r;
        if (m >= M) continue;
        const size_t o = (size_t)m * ldc + n;
        const float a = acc[i][j][r];
        if (EPI == kEpiBiasGelu) {
          const float z = a + bias[n];
          if (Cf) Cf[o] = z;
          Cb[o] = to_bf16(gelu(z));
        } else if (EPI == kEpiBias) {
          Cf[o] = a + bias[n];
        } else if (EPI == kEpiStore) {
          Cf[o] = a;
        } else {
          Cb[o] = to_bf16(a * gelu_grad(Zaux[o]));
        }
      }
    }
}

// Row-wise softmax of the logits (one wave per row, K <= 256): P to `theta`
// when given; with targets T, also the row's cross-entropy -sum t log p and
// dZ3 = (P - T) * inv_b in BF16.
__global__ void __launch_bounds__(kThreads) k_softmax(const float* __restrict__ Z, int n, int K,
                                                      float* __restrict__ theta,
                                                      const float* __restrict__ T, float inv_b,
                                                      uint16_t* __restrict__ dZ,
                                                      float* __restrict__ row_loss) {
  const int lane = threadIdx.x & 63, row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* z = Z + (size_t)row * K;
  float v[4];
  float mx = -INFINITY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = lane + 64 * q;
    v[q] = k < K ? z[k] : -INFINITY;
    mx = fmaxf(mx, v[q]);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  float sum = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = lane + 64 * q;
    v[q] = k < K ? expf(v[q] - mx) : 0.f;
    sum += v[q];
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  const float inv = 1.0f / sum;
  const float lse = mx + logf(sum);
  float ce = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = lane + 64 * q;
    if (k >= K) continue;
    const float p = v[q] * inv;
    if (theta) theta[(size_t)row * K + k] = p;
    if (T) {
      const float t = T[(size_t)row * K + k];
      ce += t * (lse - z[k]);   // -t log p with log p = z - logsumexp
      dZ[(size_t)row * K + k] = to_bf16((p - t) * inv_b);
    }
  }
  if (T) {
    for (int off = 32; off > 0; off >>= 1) ce += __shfl_xor(ce, off, 64);
    if (lane == 0) row_loss[row] = ce;
  }
}

// part[y][c] = sum over rows r of chunk y (rows y rchunk ..) of M[r][c] (BF16
// input, FP32 sum in a fixed order): block (x, y) takes 64 columns of row
// chunk y, 4 row phases per column combined in LDS; k_sum_slices then adds
// the chunks in order (the bias gradients: column sums of dZ).
__global__ void __launch_bounds__(kThreads) k_colsum(const uint16_t* __restrict__ Mx, int rows,
                                                     int cols, int rchunk,
                                                     float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rchunk, r1 = min(rows, r0 + rchunk);
  float s = 0.f;
  if (c < cols)
    for (int r = r0 + ph; r < r1; r += 4) s += from_bf16(Mx[(size_t)r * cols + c]);
  red[ph][threadIdx.x & 63] = s;
  __syncthreads();
  if (ph == 0 && c < cols)
    part[(size_t)blockIdx.y * cols + c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                          (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// out[e] = sum_z ws[z][e] for z = 0 .. nz - 1 in order (e < n)
__global__ void k_sum_slices(const float* __restrict__ ws, int nz, size_t n,
                             float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += ws[(size_t)z * n + e];
  out[e] = s;
}

// loss = sum of the row losses / n (fixed order, one block)
__global__ void __launch_bounds__(kThreads) k_loss(const float* __restrict__ row_loss, int n,
                                                   float* __restrict__ out) {
  __shared__ float red[kThreads];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += kThreads) s += row_loss[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / (float)n;
}

// Adam (Kingma & Ba, Algorithm 1) on every parameter; c1 = 1 - beta1^t and
// c2 = 1 - beta2^t are the bias corrections.  The BF16 copies of the weight
// matrices follow.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, uint16_t* __restrict__ wb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  wb[i] = to_bf16(pi);
}

__global__ void k_to_bf16(const float* __restrict__ p, size_t n, uint16_t* __restrict__ wb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = to_bf16(p[i]);
}

template <bool TA, bool TB, bool AF32, int EPI>
hipError_t gemm(int M, int N, int Kd, const void* A, int lda, const uint16_t* B, int ldb,
                const float* bias, float* Cf, uint16_t* Cb, int ldc, const float* Zaux,
                hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((N + kTileN - 1) / kTileN, (M + kTileM - 1) / kTileM);
  hipLaunchKernelGGL((k_gemm<TA, TB, AF32, EPI>), grid, dim3(kThreads), 0, s, M, N, Kd, A, lda, B,
                     ldb, bias, Cf, Cb, ldc, Zaux, Kd, (size_t)0);
  return hipGetLastError();
}

// Weight gradient C (M x N, FP32, ldc = N) = op(A) B over Kd rows, the rows
// split into chunks of at least kGradChunk so that the grid has up to
// kGradSplits times the output tiles; the chunk partials (in the encoder's
// workspace) are added in chunk order.
constexpr int kGradChunk = 128, kGradSplits = 32;
template <bool AF32>
hipError_t grad_gemm(tlda_mlp& m, int M, int N, int Kd, const void* A, int lda, const uint16_t* B,
                     int ldb, float* C) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int splits = std::min(kGradSplits, std::max(1, Kd / kGradChunk));
  const int chunk = (Kd + splits - 1) / splits;
  splits = (Kd + chunk - 1) / chunk;
  const size_t mn = (size_t)M * N;
  float* out = splits > 1 ? m.ws : C;
  const dim3 grid((N + kTileN - 1) / kTileN, (M + kTileM - 1) / kTileM, splits);
  hipLaunchKernelGGL((k_gemm<true, false, AF32, kEpiStore>), grid, dim3(kThreads), 0, m.stream, M,
                     N, Kd, A, lda, B, ldb, nullptr, out, nullptr, N, nullptr, chunk, mn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, m.stream,
                     m.ws, splits, mn, C);
  return hipGetLastError();
}

// Bias gradient out[c] = sum over the n rows of dZ[r][c]: row chunks of 64
// in parallel, then their sums in chunk order.
hipError_t bias_grad(tlda_mlp& m, const uint16_t* dZ, int n, int cols, float* out) {
  const int rchunk = 64;
  const int nch = (n + rchunk - 1) / rchunk;
  hipLaunchKernelGGL(k_colsum, dim3((cols + 63) / 64, nch), dim3(kThreads), 0, m.stream, dZ, n,
                     cols, rchunk, m.ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_slices, dim3((cols + 255) / 256), dim3(256), 0, m.stream, m.ws, nch,
                     (size_t)cols, out);
  return hipGetLastError();
}

}  // namespace

size_t mlp_workspace_floats(int d_in, int hidden, int k_out, int max_batch) {
  const size_t mn = std::max({(size_t)d_in * hidden, (size_t)hidden * hidden,
                              (size_t)hidden * k_out});
  const size_t chunks = ((size_t)max_batch + 63) / 64;
  return std::max((size_t)kGradSplits * mn, chunks * (size_t)std::max(hidden, k_out));
}

size_t mlp_param_count(int d_in, int hidden, int k_out) {
  return (size_t)d_in * hidden + hidden + (size_t)hidden * hidden + hidden +
         (size_t)hidden * k_out + k_out;
}

void mlp_offsets(int d_in, int hidden, int k_out, size_t off[6]) {
  off[0] = 0;                                     // W1 [d_in][hidden]
  off[1] = off[0] + (size_t)d_in * hidden;        // b1 [hidden]
  off[2] = off[1] + hidden;                       // W2 [hidden][hidden]
  off[3] = off[2] + (size_t)hidden * hidden;      // b2
  off[4] = off[3] + hidden;                       // W3 [hidden][k_out]
  off[5] = off[4] + (size_t)hidden * k_out;       // b3 [k_out]
}

hipError_t mlp_forward(tlda_mlp& m, const float* X, int n, float* theta, bool train) {
  size_t o[6];
  mlp_offsets(m.d_in, m.hidden, m.k_out, o);
  const int H = m.hidden, K = m.k_out;
  hipError_t e = gemm<false, false, true, kEpiBiasGelu>(n, H, m.d_in, X, m.d_in, m.wb + o[0], H,
                                                         m.params + o[1], train ? m.Z1 : nullptr,
                                                         m.H1, H, nullptr, m.stream);
  if (e != hipSuccess) return e;
  e = gemm<false, false, false, kEpiBiasGelu>(n, H, H, m.H1, H, m.wb + o[2], H, m.params + o[3],
                                               train ? m.Z2 : nullptr, m.H2, H, nullptr, m.stream);
  if (e != hipSuccess) return e;
  e = gemm<false, false, false, kEpiBias>(n, K, H, m.H2, H, m.wb + o[4], K, m.params + o[5],
                                          m.logits, nullptr, K, nullptr, m.stream);
  if (e != hipSuccess) return e;
  if (theta != nullptr) {
    hipLaunchKernelGGL(k_softmax, dim3((n + 3) / 4), dim3(kThreads), 0, m.stream, m.logits, n, K,
                       theta, nullptr, 0.f, nullptr, nullptr);
    e = hipGetLastError();
  }
  return e;
}

hipError_t mlp_backward(tlda_mlp& m, const float* X, const float* T, int n, float* loss_out) {
  size_t o[6];
  mlp_offsets(m.d_in, m.hidden, m.k_out, o);
  const int H = m.hidden, K = m.k_out, Din = m.d_in;
  float* g = m.grads;
  hipLaunchKernelGGL(k_softmax, dim3((n + 3) / 4), dim3(kThreads), 0, m.stream, m.logits, n, K,
                     nullptr, T, 1.0f / (float)n, m.dZ3, m.row_loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss_out != nullptr) {
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kThreads), 0, m.stream, m.row_loss, n, loss_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // layer 3
  if ((e = grad_gemm<false>(m, H, K, n, m.H2, H, m.dZ3, K, g + o[4])) != hipSuccess) return e;
  if ((e = bias_grad(m, m.dZ3, n, K, g + o[5])) != hipSuccess) return e;
  if ((e = gemm<false, true, false, kEpiDGelu>(n, H, K, m.dZ3, K, m.wb + o[4], K, nullptr, nullptr,
                                               m.dZa, H, m.Z2, m.stream)) != hipSuccess)
    return e;
  // layer 2
  if ((e = grad_gemm<false>(m, H, H, n, m.H1, H, m.dZa, H, g + o[2])) != hipSuccess) return e;
  if ((e = bias_grad(m, m.dZa, n, H, g + o[3])) != hipSuccess) return e;
  if ((e = gemm<false, true, false, kEpiDGelu>(n, H, H, m.dZa, H, m.wb + o[2], H, nullptr, nullptr,
                                               m.dZb, H, m.Z1, m.stream)) != hipSuccess)
    return e;
  // layer 1
  if ((e = grad_gemm<true>(m, Din, H, n, X, Din, m.dZb, H, g + o[0])) != hipSuccess) return e;
  return bias_grad(m, m.dZb, n, H, g + o[1]);
}

hipError_t mlp_adam(tlda_mlp& m, float lr, float beta1, float beta2, float eps) {
  m.adam_t += 1;
  const float c1 = 1.0f - (float)std::pow((double)beta1, (double)m.adam_t);
  const float c2 = 1.0f - (float)std::pow((double)beta2, (double)m.adam_t);
  const size_t n = m.n_params;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m.stream, m.params,
                     m.grads, m.adam_m, m.adam_v, n, lr, beta1, beta2, eps, c1, c2, m.wb);
  return hipGetLastError();
}

hipError_t mlp_refresh_bf16(tlda_mlp& m) {
  const size_t n = m.n_params;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m.stream,
                     m.params, n, m.wb);
  return hipGetLastError();
}

}  // namespace tlda
