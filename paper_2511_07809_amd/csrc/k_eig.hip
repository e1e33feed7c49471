// FP64 building blocks of the whitening refresh: the top-D eigenpairs of
// M2~ = (alpha0 + 1)(S2 / N - M1 M1^T) by block subspace iteration with
// Cholesky-QR orthonormalisation and a final Rayleigh-Ritz step solved by
// parallel-order cyclic Jacobi (section "Online Decomposition of the Second
// Moment": W = U diag(lambda)^(-1/2) so that W^T M2~ W = I).
#include <algorithm>

#include "tlda_internal.h"

namespace tlda {

thread_local EigEnv g_eig_env;

namespace {

// ---------------------------------------------------------------------------
// Dense FP64 GEMM: C = alpha * op(A) * B (+ C when accumulating through
// atomics for split-K).  op(A) is A (M x Kd, row-major, lda) or A^T where A is
// stored Kd x M.  B is Kd x N row-major (ldb), C is M x N row-major (ldc).
// 64 x 64 output tile per 256-thread block, 4 x 4 register tile per thread,
// K step 16 staged through LDS.  grid.z splits Kd into chunks of k_chunk
// rows; with more than one chunk the tile is added to C with FP64 atomics.
// ---------------------------------------------------------------------------
// (c_stride_z != 0: chunk z writes its own tile to C + z * c_stride_z.)
template <bool TRANS_A>
__global__ void __launch_bounds__(256) k_gemm64(int M, int N, int Kd, const double* __restrict__ A,
                                                int lda, const double* __restrict__ B, int ldb,
                                                double* __restrict__ C, int ldc, double alpha,
                                                int k_chunk, int atomic_out, size_t c_stride_z) {
  C += blockIdx.z * c_stride_z;
  __shared__ double As[16][64 + 2];
  __shared__ double Bs[16][64 + 2];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * k_chunk;
  const int kend = min(Kd, kbeg + k_chunk);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    // A tile: 64 rows x 16 k  ->  As[k][row]
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      int r, kk;
      if (TRANS_A) { kk = idx >> 6; r = idx & 63; }   // consecutive threads along M
      else { r = idx >> 4; kk = idx & 15; }           // consecutive threads along K
      const int gr = row0 + r, gk = k0 + kk;
      double v = 0.0;
      if (gr < M && gk < kend) v = TRANS_A ? A[(size_t)gk * lda + gr] : A[(size_t)gr * lda + gk];
      As[kk][r] = v;
    }
    // B tile: 16 k x 64 cols
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx >> 6, c = idx & 63;
      const int gk = k0 + kk, gc = col0 + c;
      Bs[kk][c] = (gk < kend && gc < N) ? B[(size_t)gk * ldb + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gr = row0 + ty + 16 * i;
    if (gr >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + tx + 16 * j;
      if (gc >= N) continue;
      if (atomic_out) unsafeAtomicAdd(&C[(size_t)gr * ldc + gc], alpha * acc[i][j]);
      else C[(size_t)gr * ldc + gc] = alpha * acc[i][j];
    }
  }
}

// ---------------------------------------------------------------------------
// Dense FP64 GEMM on the matrix cores: C = alpha * A * B (row-major; A is
// M x K, B is K x N), v_mfma_f64_16x16x4f64 with FP64 accumulation.
// Block: 8 waves over a 128-row x 16 NT-column tile of C (NT 16-column
// tiles, at most 8: wider products take several column blocks, and two
// blocks fit on a CU); wave (wr, wc) owns rows 32 wr .. 32 wr + 31 (two
// 16-row MFMA tiles) and column half wc (tiles 0 .. NT0 - 1 or NT0 .. NT - 1).
// K advances 16 at a time through double-buffered LDS: the next K tile is
// loaded into registers while the current one is multiplied (loads are
// unconditional, from clamped addresses, with out-of-range entries zeroed by
// selects, so none of them waits on another).  For the tall products (C = S2
// times the subspace block, V rows) the 128-row tile reads each row block of
// B once per 128 rows of A: B's traffic is N / 128 of A's.  grid.z splits K
// into chunks whose C tiles go to their own slice of a workspace
// (c_stride_z apart); k_sum_splits adds the slices in order.
// Operand layout of the instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 r + l / 16][l % 16].
// ---------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kDgBM = 128, kDgBK = 16, kDgThreads = 512;

template <int NT>
__global__ void __launch_bounds__(kDgThreads, 4) k_dgemm_mfma(
    int M, int N, int K, int k_chunk, const double* __restrict__ A, int lda,
    const double* __restrict__ B, int ldb, double* __restrict__ C, int ldc, size_t c_stride_z,
    double alpha) {
  constexpr int BNC = 16 * NT, LDA_S = kDgBK + 1, LDB_S = BNC + 2;
  constexpr int NT0 = (NT + 1) / 2;
  constexpr int A_PER = kDgBM * kDgBK / kDgThreads;
  constexpr int B_PER = (kDgBK * BNC + kDgThreads - 1) / kDgThreads;
  __shared__ double As[2][kDgBM * LDA_S];
  __shared__ double Bs[2][kDgBK * LDB_S];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 3, wc = wave >> 2;
  const int ct0 = wc ? NT0 : 0;
  const int nct = wc ? NT - NT0 : NT0;
  const int row0 = blockIdx.y * kDgBM, col0 = blockIdx.x * BNC;
  const int kbeg = blockIdx.z * k_chunk;
  const int kend = min(K, kbeg + k_chunk);
  C += blockIdx.z * c_stride_z;
  doublex4 acc[2][NT0];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < NT0; ++j) acc[t][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  // raw loaded values and which of them are in range: the selects happen
  // when the tile is stored to LDS, after the matrix work, so nothing waits
  // for the loads before then
  double ra[A_PER], rb[B_PER];
  unsigned am = 0, bm = 0;
  auto load = [&](int k0) {
    am = bm = 0;
#pragma unroll
    for (int i = 0; i < A_PER; ++i) {
      const int e = tid + i * kDgThreads;
      const int gr = row0 + e / kDgBK, gk = k0 + e % kDgBK;
      const bool in = gr < M && gk < kend;
      ra[i] = A[in ? (size_t)gr * lda + gk : 0];
      am |= (in ? 1u : 0u) << i;
    }
#pragma unroll
    for (int i = 0; i < B_PER; ++i) {
      const int e = tid + i * kDgThreads;
      const int gk = k0 + e / BNC, gc = col0 + e % BNC;
      const bool in = e < kDgBK * BNC && gk < kend && gc < N;
      rb[i] = B[in ? (size_t)gk * ldb + gc : 0];
      bm |= (in ? 1u : 0u) << i;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_PER; ++i) {
      const int e = tid + i * kDgThreads;
      As[buf][(e / kDgBK) * LDA_S + e % kDgBK] = ((am >> i) & 1u) ? ra[i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < B_PER; ++i) {
      const int e = tid + i * kDgThreads;
      if (e < kDgBK * BNC) Bs[buf][(e / BNC) * LDB_S + e % BNC] = ((bm >> i) & 1u) ? rb[i] : 0.0;
    }
  };
  const int nk = (kend - kbeg + kDgBK - 1) / kDgBK;
  load(kbeg);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(kbeg + (kt + 1) * kDgBK);
    const double* as = As[cur] + (wr * 32 + (lane & 15)) * LDA_S + (lane >> 4);
    const double* bs = Bs[cur] + (lane >> 4) * LDB_S + ct0 * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < kDgBK / 4; ++ks) {
      const double a0 = as[4 * ks], a1 = as[16 * LDA_S + 4 * ks];
#pragma unroll
      for (int j = 0; j < NT0; ++j)
        if (j < nct) {
          const double b = bs[4 * ks * LDB_S + j * 16];
          acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < NT0; ++j) {
      if (j >= nct) continue;
      const int col = col0 + (ct0 + j) * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + t * 16 + 4 * r + (lane >> 4);
        if (row < M && col < N) C[(size_t)row * ldc + col] = alpha * acc[t][j][r];
      }
    }
}

// C[r][c] = alpha * sum_z ws[z][r][c] in order z = 0 .. nz - 1 (ws slices M x N).
__global__ void k_sum_splits(const double* __restrict__ ws, int nz, int M, int N,
                             double* __restrict__ C, int ldc, double alpha) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t mn = (size_t)M * N;
  if (e >= mn) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += ws[(size_t)z * mn + e];
  C[(e / N) * ldc + e % N] = alpha * s;
}

template <int NT>
hipError_t launch_dgemm_nt(dim3 grid, int M, int N, int K, int chunk, const double* A, int lda,
                           const double* B, int ldb, double* C, int ldc, size_t cz, double alpha,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_dgemm_mfma<NT>, grid, dim3(kDgThreads), 0, s, M, N, K, chunk, A, lda, B,
                     ldb, C, ldc, cz, alpha);
  return hipGetLastError();
}

hipError_t dgemm_mfma(int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                      double* C, int ldc, double alpha, hipStream_t s) {
  const int gx = (N + 127) / 128;                     // column blocks of at most 8 tiles
  const int NT = ((N + gx - 1) / gx + 15) / 16;
  const int BNC = 16 * NT;
  const int gy = (M + kDgBM - 1) / kDgBM;
  int splits = dgemm_splits(M, N, K, g_eig_env.num_cu);
  if (splits > 1 && (g_eig_env.ws == nullptr || (size_t)splits * M * N > g_eig_env.ws_doubles))
    splits = 1;
  int chunk = ((K + splits - 1) / splits + kDgBK - 1) / kDgBK * kDgBK;
  splits = (K + chunk - 1) / chunk;
  double* out = splits > 1 ? g_eig_env.ws : C;
  const int ldo = splits > 1 ? N : ldc;
  const size_t cz = splits > 1 ? (size_t)M * N : 0;
  const double al = splits > 1 ? 1.0 : alpha;
  const dim3 grid(gx, gy, splits);
  hipError_t e = hipErrorInvalidValue;
  switch (NT) {
#define TLDA_DG(n) \
  case n: e = launch_dgemm_nt<n>(grid, M, N, K, chunk, A, lda, B, ldb, out, ldo, cz, al, s); break;
    TLDA_DG(1) TLDA_DG(2) TLDA_DG(3) TLDA_DG(4) TLDA_DG(5) TLDA_DG(6) TLDA_DG(7) TLDA_DG(8)
#undef TLDA_DG
    default: break;
  }
  if (e != hipSuccess || splits == 1) return e;
  const size_t mn = (size_t)M * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s,
                     g_eig_env.ws, splits, M, N, C, ldc, alpha);
  return hipGetLastError();
}

// Out[e] = alpha * sum_z part[z][e] over nz chunks: four lanes per entry,
// lane c adding the c-th quarter of the chunks in chunk order, the quarters
// then combined as (q0 + q1) + (q2 + q3) (a fixed order, so the sum is
// deterministic).  A lane issues the loads of 16 chunks before adding them;
// the last batch loads from chunk indexes clamped into its quarter and adds
// only the chunks that exist.
__global__ void k_sum_partials(const double* __restrict__ part, int nz, size_t mn, int N, int ldc,
                               double alpha, double* __restrict__ C) {
  constexpr int kU = 16;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t e = t >> 2;
  const int c = (int)(t & 3);
  const bool in = e < mn;
  const size_t ec = in ? e : mn - 1;
  const int per = (nz + 3) / 4;
  const int z0 = min(c * per, nz), z1 = min(z0 + per, nz);
  double s = 0.0;
  for (int z = z0; z < z1; z += kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = part[(size_t)min(z + u, z1 - 1) * mn + ec];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (z + u < z1) s += v[u];
  }
  s += __shfl_xor(s, 1, 64);                    // (q0 + q1), (q2 + q3)
  s += __shfl_xor(s, 2, 64);                    // (q0 + q1) + (q2 + q3)
  if (in && c == 0) C[(e / N) * ldc + e % N] = alpha * s;
}

hipError_t gemm(bool transA, int M, int N, int Kd, const double* A, int lda, const double* B,
                int ldb, double* C, int ldc, double alpha, int splits, hipStream_t s) {
  if (transA && g_eig_env.part != nullptr && (size_t)M * N <= g_eig_env.part_mn &&
      g_eig_env.part_chunks > 0) {
    // A^T B over many rows: row chunks of at least 64 write their own
    // partials, then one pass adds them in order (no atomics)
    int nz = (Kd + 63) / 64;
    if (nz > g_eig_env.part_chunks) nz = g_eig_env.part_chunks;
    if (nz < 1) nz = 1;
    const int chunk = ((Kd + nz - 1) / nz + 15) / 16 * 16;
    nz = (Kd + chunk - 1) / chunk;
    const size_t mn = (size_t)M * N;
    dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
    hipLaunchKernelGGL(k_gemm64<true>, grid, dim3(256), 0, s, M, N, Kd, A, lda, B, ldb,
                       g_eig_env.part, N, 1.0, chunk, 0, mn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((4 * mn + 255) / 256)), dim3(256), 0, s,
                       g_eig_env.part, nz, mn, N, ldc, alpha, C);
    return hipGetLastError();
  }
  if (!transA && g_eig_env.route == 0) return dgemm_mfma(M, N, Kd, A, lda, B, ldb, C, ldc, alpha, s);
  if (splits < 1) splits = 1;
  int chunk = (Kd + splits - 1) / splits;
  chunk = (chunk + 15) / 16 * 16;
  splits = (Kd + chunk - 1) / chunk;
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  const int atomic_out = splits > 1 ? 1 : 0;
  if (atomic_out) {
    hipError_t e = launch_zero(C, (size_t)M * ldc * sizeof(double), s);
    if (e != hipSuccess) return e;
  }
  if (transA)
    hipLaunchKernelGGL(k_gemm64<true>, grid, dim3(256), 0, s, M, N, Kd, A, lda, B, ldb, C, ldc,
                       alpha, chunk, atomic_out, (size_t)0);
  else
    hipLaunchKernelGGL(k_gemm64<false>, grid, dim3(256), 0, s, M, N, Kd, A, lda, B, ldb, C, ldc,
                       alpha, chunk, atomic_out, (size_t)0);
  return hipGetLastError();
}

// splitmix64 (Steele, Lea & Flood 2014) as a counter-based generator for the
// refresh's start block: entry (i, c) is uniform in [-1, 1).
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_random_block(double* __restrict__ Q, int V, int p, uint64_t seed) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)V * p) return;
  const uint64_t r = splitmix64(seed * 0x100000001B3ull + idx);
  Q[idx] = (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// Y[i][c] -= scale_m * m[i] * t[c]   (the -M1 M1^T part of M2~ applied to Q)
__global__ void k_rank1_update(double* __restrict__ Y, const double* __restrict__ m,
                               const double* __restrict__ t, int V, int p, double scale_m) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)V * p) return;
  const int i = (int)(idx / p), c = (int)(idx % p);
  Y[idx] -= scale_m * m[i] * t[c];
}

// Right-looking Cholesky of the p x p matrix G + shift * max(diag) * I in
// place (lower triangle); one block.  info[0] != 0 on a non-positive pivot.
__global__ void __launch_bounds__(1024) k_cholesky(double* __restrict__ G, int p, double shift_rel,
                                                   int* __restrict__ info) {
  __shared__ double sh_shift;
  __shared__ int sh_fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < p; ++i) mx = fmax(mx, G[(size_t)i * p + i]);
    sh_shift = shift_rel * mx;
    sh_fail = 0;
  }
  __syncthreads();
  for (int i = tid; i < p; i += nt) G[(size_t)i * p + i] += sh_shift;
  __threadfence_block();
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    if (tid == 0) {
      const double d = G[(size_t)j * p + j];
      if (!(d > 0.0)) {
        sh_fail = 1;
        G[(size_t)j * p + j] = 1.0;
      } else {
        G[(size_t)j * p + j] = sqrt(d);
      }
    }
    __threadfence_block();
    __syncthreads();
    const double djj = G[(size_t)j * p + j];
    for (int i = j + 1 + tid; i < p; i += nt) G[(size_t)i * p + j] /= djj;
    __threadfence_block();
    __syncthreads();
    const int rem = p - j - 1;
    for (int idx = tid; idx < rem * rem; idx += nt) {
      const int i = j + 1 + idx / rem, k = j + 1 + idx % rem;
      if (k <= i) G[(size_t)i * p + k] -= G[(size_t)i * p + j] * G[(size_t)k * p + j];
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0 && sh_fail) atomicOr(info, 1);
}

// The same factorisation with the matrix held in LDS (p <= kLdsP): two
// barriers per column instead of round trips through global memory.
constexpr int kLdsP = 128;
__global__ void __launch_bounds__(1024) k_cholesky_lds(double* __restrict__ G, int p,
                                                       double shift_rel, int* __restrict__ info) {
  __shared__ double A[kLdsP * kLdsP];
  __shared__ double red[1024];
  __shared__ int sh_fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  double mx = 0.0;
  for (int idx = tid; idx < p * p; idx += nt) {
    const double v = G[idx];
    A[idx] = v;
    if (idx / p == idx % p) mx = fmax(mx, v);
  }
  red[tid] = mx;
  if (tid == 0) sh_fail = 0;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double shift = shift_rel * red[0];
  for (int i = tid; i < p; i += nt) A[i * p + i] += shift;
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    const double d = A[j * p + j];
    const double sq = d > 0.0 ? sqrt(d) : 1.0;
    for (int i = j + 1 + tid; i < p; i += nt) A[i * p + j] /= sq;
    __syncthreads();
    if (tid == 0) {
      if (!(d > 0.0)) sh_fail = 1;
      A[j * p + j] = sq;
    }
    // trailing lower triangle (j < k <= i < p), threads as a 32 x 32 grid
    for (int i = j + 1 + (tid >> 5); i < p; i += 32) {
      const double aij = A[i * p + j];
      for (int k = j + 1 + (tid & 31); k <= i; k += 32) A[i * p + k] -= aij * A[k * p + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < p * p; idx += nt) G[idx] = A[idx];
  if (tid == 0 && sh_fail) atomicOr(info, 1);
}

// Binv = (L^-1)^T: wave c computes column c of X = L^-1 by forward
// substitution, x_i = (delta_ic - sum_{c <= k < i} L[i][k] x_k) / L[i][i].
// Lane l keeps x_k for k = c + l + 64 j in registers; each row's sum is
// split over the lanes and added by a butterfly (every lane gets the same
// value), and row i + 1 of L is loaded while row i is reduced (staging L
// in LDS measured no faster).  p <= 512.
constexpr int kInvJ = 8;
__global__ void __launch_bounds__(256) k_tri_inverse_waves(const double* __restrict__ G, int p,
                                                           double* __restrict__ Binv) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= p) return;                          // the whole wave
  double xr[kInvJ], ln[kInvJ];
#pragma unroll
  for (int j = 0; j < kInvJ; ++j) xr[j] = 0.0;
  auto load_row = [&](int i, double (&l)[kInvJ]) {
#pragma unroll
    for (int j = 0; j < kInvJ; ++j) {
      const int k = c + lane + 64 * j;
      l[j] = k < i ? G[(size_t)i * p + k] : 0.0;
    }
  };
  load_row(c, ln);
  double diag = G[(size_t)c * p + c];
  for (int i = c; i < p; ++i) {
    double lc[kInvJ];
#pragma unroll
    for (int j = 0; j < kInvJ; ++j) lc[j] = ln[j];
    const double dg = diag;
    if (i + 1 < p) {
      load_row(i + 1, ln);
      diag = G[(size_t)(i + 1) * p + i + 1];
    }
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < kInvJ; ++j) part += lc[j] * xr[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    const double xi = ((i == c ? 1.0 : 0.0) - part) / dg;
    const int t = i - c;
#pragma unroll
    for (int j = 0; j < kInvJ; ++j)
      if (lane == (t & 63) && j == (t >> 6)) xr[j] = xi;
  }
  for (int k = lane; k < c; k += 64) Binv[(size_t)c * p + k] = 0.0;
#pragma unroll
  for (int j = 0; j < kInvJ; ++j) {
    const int k = c + lane + 64 * j;
    if (k < p) Binv[(size_t)c * p + k] = xr[j];
  }
}

// Cyclic Jacobi with the round-robin parallel ordering: in each round the
// m/2 disjoint pairs (circle method) are rotated at once, so every pair of
// indices is visited once per sweep.  A pair is rotated only while its
// off-diagonal entry is significant relative to its diagonal entries
// (|a_ij| > 1e-15 sqrt|a_ii a_jj|) and to the matrix (|a_ij| > 1e-20 |A|_F);
// a sweep without rotations ends the iteration.  A (p x p, symmetric) is
// diagonalised in place, Z accumulates the rotations, ev gets the diagonal.
// info |= 2 if 60 sweeps leave an off-diagonal mass above 1e-10 |A|_F.
__global__ void __launch_bounds__(1024) k_jacobi(double* __restrict__ A, double* __restrict__ Z,
                                                 double* __restrict__ ev, int p,
                                                 int* __restrict__ info) {
  extern __shared__ double sh[];   // c[m/2], s[m/2], pair indices, reduction scratch
  __shared__ int sh_rot;
  __shared__ double sh_norm;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = (p + 1) & ~1;
  const int half = m / 2;
  double* cs = sh;
  double* sn = sh + half;
  int* pi = reinterpret_cast<int*>(sh + 2 * half);
  int* pj = pi + half;
  double* red = sh + 3 * half;     // 2 * nt doubles
  for (int idx = tid; idx < p * p; idx += nt) Z[idx] = (idx / p == idx % p) ? 1.0 : 0.0;
  // Frobenius norm (invariant under the rotations)
  double tot = 0.0;
  for (int idx = tid; idx < p * p; idx += nt) tot += A[idx] * A[idx];
  red[tid] = tot;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) sh_norm = sqrt(red[0]);
  __threadfence_block();
  __syncthreads();
  const double tiny = 1e-20 * sh_norm;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) sh_rot = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < half; k += nt) {
        int i, j;
        if (k == 0) { i = 0; j = 1 + r; }
        else {
          i = 1 + (r + k) % (m - 1);
          j = 1 + (r - k + (m - 1)) % (m - 1);
        }
        if (i > j) { const int t = i; i = j; j = t; }
        double c = 1.0, s = 0.0;
        if (j < p) {
          const double aij = A[(size_t)i * p + j];
          const double aii = A[(size_t)i * p + i], ajj = A[(size_t)j * p + j];
          if (fabs(aij) > tiny && fabs(aij) > 1e-15 * sqrt(fabs(aii * ajj))) {
            const double tau = (ajj - aii) / (2.0 * aij);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            sh_rot = 1;
          }
        }
        pi[k] = i;
        pj[k] = j;
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // columns i, j of A and Z
      for (int idx = tid; idx < half * p; idx += nt) {
        const int k = idx / p, row = idx % p;
        const int i = pi[k], j = pj[k];
        const double s = sn[k];
        if (j >= p || s == 0.0) continue;
        const double c = cs[k];
        const double ai = A[(size_t)row * p + i], aj = A[(size_t)row * p + j];
        A[(size_t)row * p + i] = c * ai - s * aj;
        A[(size_t)row * p + j] = s * ai + c * aj;
        const double zi = Z[(size_t)row * p + i], zj = Z[(size_t)row * p + j];
        Z[(size_t)row * p + i] = c * zi - s * zj;
        Z[(size_t)row * p + j] = s * zi + c * zj;
      }
      __threadfence_block();
      __syncthreads();
      // rows i, j of A
      for (int idx = tid; idx < half * p; idx += nt) {
        const int k = idx / p, col = idx % p;
        const int i = pi[k], j = pj[k];
        const double s = sn[k];
        if (j >= p || s == 0.0) continue;
        const double c = cs[k];
        const double ai = A[(size_t)i * p + col], aj = A[(size_t)j * p + col];
        A[(size_t)i * p + col] = c * ai - s * aj;
        A[(size_t)j * p + col] = s * ai + c * aj;
      }
      __threadfence_block();
      __syncthreads();
    }
    if (sh_rot == 0) break;
    __syncthreads();
  }
  // final check of the remaining off-diagonal mass
  double off = 0.0;
  for (int idx = tid; idx < p * p; idx += nt)
    if (idx / p != idx % p) off += A[idx] * A[idx];
  red[tid] = off;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && sqrt(red[0]) > 1e-10 * sh_norm) atomicOr(info, 2);
  for (int i = tid; i < p; i += nt) ev[i] = A[(size_t)i * p + i];
}

// The same iteration with the p x p matrix in LDS (p <= kLdsP).  ZL: the
// rotation accumulator Z is in LDS as well (p <= kLdsPZ, the two matrices
// fill the 160 KB), and Z's array doubles as the reduction scratch before Z
// is formed and after it is written out; otherwise Z stays in global memory.
constexpr int kLdsPZ = 100;
template <bool ZL>
__global__ void __launch_bounds__(1024) k_jacobi_lds(double* __restrict__ Ag, double* __restrict__ Zg,
                                                 double* __restrict__ ev, int p,
                                                 int* __restrict__ info) {
  constexpr int PA = ZL ? kLdsPZ : kLdsP;
  __shared__ double A[PA * PA];
  __shared__ double Zl[ZL ? PA * PA : 1];
  __shared__ double sh[3 * (PA / 2) + (ZL ? 0 : 2 * 1024)];   // c, s, pair indices (, scratch)
  __shared__ int sh_rot;
  __shared__ double sh_norm;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = (p + 1) & ~1;
  const int half = m / 2;
  double* cs = sh;
  double* sn = sh + half;
  int* pi = reinterpret_cast<int*>(sh + 2 * half);
  int* pj = pi + half;
  double* red = ZL ? Zl : sh + 3 * half;     // 2 * nt doubles
  double* Z = ZL ? Zl : Zg;
  for (int idx = tid; idx < p * p; idx += nt) {
    A[idx] = Ag[idx];
    if (!ZL) Z[idx] = (idx / p == idx % p) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Frobenius norm (invariant under the rotations)
  double tot = 0.0;
  for (int idx = tid; idx < p * p; idx += nt) tot += A[idx] * A[idx];
  red[tid] = tot;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) sh_norm = sqrt(red[0]);
  __threadfence_block();
  __syncthreads();
  const double tiny = 1e-20 * sh_norm;
  if (ZL) {
    for (int idx = tid; idx < p * p; idx += nt) Z[idx] = (idx / p == idx % p) ? 1.0 : 0.0;
    __syncthreads();
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) sh_rot = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < half; k += nt) {
        int i, j;
        if (k == 0) { i = 0; j = 1 + r; }
        else {
          i = 1 + (r + k) % (m - 1);
          j = 1 + (r - k + (m - 1)) % (m - 1);
        }
        if (i > j) { const int t = i; i = j; j = t; }
        double c = 1.0, s = 0.0;
        if (j < p) {
          const double aij = A[(size_t)i * p + j];
          const double aii = A[(size_t)i * p + i], ajj = A[(size_t)j * p + j];
          if (fabs(aij) > tiny && fabs(aij) > 1e-15 * sqrt(fabs(aii * ajj))) {
            const double tau = (ajj - aii) / (2.0 * aij);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            sh_rot = 1;
          }
        }
        pi[k] = i;
        pj[k] = j;
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // A <- J^T A J in one pass: a thread owns the 2 x 2 block of A at the
      // rows of pair a and the columns of pair b, rotated by b's columns and
      // then by a's rows (the same operations, in the same order, as a column
      // pass followed by a row pass).  Entries at the padding index p do not
      // exist.
      // Lane l of every wave owns column pair b = l (half <= 64), the waves
      // take the row pairs a in turn.
      const int lb = tid & 63, nw = nt >> 6;
      const bool own = lb < half;
      const double sb = own ? sn[lb] : 0.0, cb = own ? cs[lb] : 1.0;
      const int ib = own ? pi[lb] : 0, jb = own ? pj[lb] : p;
      const bool rb = jb < p;
      for (int a = own ? (tid >> 6) : half; a < half; a += nw) {
        const double sa = sn[a];
        if (sa == 0.0 && sb == 0.0) continue;
        const int ia = pi[a], ja = pj[a];
        const bool ra = ja < p;
        const double ca = cs[a];
        double x00 = A[(size_t)ia * p + ib];
        double x01 = rb ? A[(size_t)ia * p + jb] : 0.0;
        double x10 = ra ? A[(size_t)ja * p + ib] : 0.0;
        double x11 = ra && rb ? A[(size_t)ja * p + jb] : 0.0;
        if (sb != 0.0) {
          const double y00 = cb * x00 - sb * x01, y01 = sb * x00 + cb * x01;
          const double y10 = cb * x10 - sb * x11, y11 = sb * x10 + cb * x11;
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        if (sa != 0.0) {
          const double y00 = ca * x00 - sa * x10, y10 = sa * x00 + ca * x10;
          const double y01 = ca * x01 - sa * x11, y11 = sa * x01 + ca * x11;
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        A[(size_t)ia * p + ib] = x00;
        if (rb) A[(size_t)ia * p + jb] = x01;
        if (ra) A[(size_t)ja * p + ib] = x10;
        if (ra && rb) A[(size_t)ja * p + jb] = x11;
      }
      // Z <- Z J: the same lane owns the same pair b in every row, the waves
      // take the rows in turn, and each thread issues kZ rows' loads before
      // its stores
      constexpr int kZ = 8;
      if (rb && sb != 0.0) {
        for (int r0 = tid >> 6; r0 < p; r0 += kZ * nw) {
          double zi[kZ], zj[kZ];
#pragma unroll
          for (int u = 0; u < kZ; ++u) {
            const int row = r0 + u * nw;
            zi[u] = zj[u] = 0.0;
            if (row < p) {
              zi[u] = Z[(size_t)row * p + ib];
              zj[u] = Z[(size_t)row * p + jb];
            }
          }
#pragma unroll
          for (int u = 0; u < kZ; ++u) {
            const int row = r0 + u * nw;
            if (row < p) {
              Z[(size_t)row * p + ib] = cb * zi[u] - sb * zj[u];
              Z[(size_t)row * p + jb] = sb * zi[u] + cb * zj[u];
            }
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    if (sh_rot == 0) break;
    __syncthreads();
  }
  if (ZL) {
    for (int idx = tid; idx < p * p; idx += nt) Zg[idx] = Z[idx];
    __syncthreads();
  }
  // final check of the remaining off-diagonal mass
  double off = 0.0;
  for (int idx = tid; idx < p * p; idx += nt)
    if (idx / p != idx % p) off += A[idx] * A[idx];
  red[tid] = off;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && sqrt(red[0]) > 1e-10 * sh_norm) atomicOr(info, 2);
  for (int i = tid; i < p; i += nt) ev[i] = A[(size_t)i * p + i];
  for (int idx = tid; idx < p * p; idx += nt) Ag[idx] = A[idx];
}

// Sorts the Ritz values in decreasing order (ties: lower index first), keeps
// the top D, and gathers the matching eigenvector columns into Zs [p][D].
__global__ void __launch_bounds__(256) k_select_top(const double* __restrict__ Z,
                                                    const double* __restrict__ ev, int p, int D,
                                                    double* __restrict__ Zs,
                                                    double* __restrict__ eigD) {
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    int rank = 0;
    const double v = ev[c];
    for (int k = 0; k < p; ++k) {
      const double w = ev[k];
      if (w > v || (w == v && k < c)) ++rank;
    }
    if (rank < D) {
      eigD[rank] = v;
      for (int r = 0; r < p; ++r) Zs[(size_t)r * D + rank] = Z[(size_t)r * p + c];
    }
  }
}

// Sign rule: the entry of largest magnitude of every column of U (V x D) is
// made positive (lowest row index on ties).  One block per column.
__global__ void __launch_bounds__(256) k_sign_fix(double* __restrict__ U, int V, int D) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int col = blockIdx.x, tid = threadIdx.x;
  double best = -1.0;
  int besti = V;
  for (int i = tid; i < V; i += blockDim.x) {
    const double a = fabs(U[(size_t)i * D + col]);
    if (a > best) { best = a; besti = i; }
  }
  bv[tid] = best;
  bi[tid] = besti;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      if (bv[tid + w] > bv[tid] || (bv[tid + w] == bv[tid] && bi[tid + w] < bi[tid])) {
        bv[tid] = bv[tid + w];
        bi[tid] = bi[tid + w];
      }
    }
    __syncthreads();
  }
  const bool flip = bi[0] < V && U[(size_t)bi[0] * D + col] < 0.0;
  __syncthreads();
  if (flip)
    for (int i = tid; i < V; i += blockDim.x) U[(size_t)i * D + col] = -U[(size_t)i * D + col];
}

// W = U diag(eig)^(-1/2) in FP64 and its FP32 copy with row stride Dp (zero
// padding beyond D).
__global__ void k_form_w(const double* __restrict__ U, const double* __restrict__ eig, int V, int D,
                         int Dp, double* __restrict__ W, float* __restrict__ W32) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)V * Dp) return;
  const int i = (int)(idx / Dp), d = (int)(idx % Dp);
  if (d < D) {
    const double w = U[(size_t)i * D + d] / sqrt(eig[d]);
    W[(size_t)i * D + d] = w;
    W32[idx] = (float)w;
  } else {
    W32[idx] = 0.0f;
  }
}

// mw32[d] = sum_i W[i][d] m[i] (FP64 sum, one block per column); padding zero.
__global__ void __launch_bounds__(256) k_mw(const double* __restrict__ W, const double* __restrict__ m,
                                            int V, int D, int Dp, float* __restrict__ mw32) {
  __shared__ double red[256];
  const int d = blockIdx.x, tid = threadIdx.x;
  if (d >= D) {
    if (tid == 0) mw32[d] = 0.0f;
    return;
  }
  double s = 0.0;
  for (int i = tid; i < V; i += blockDim.x) s += W[(size_t)i * D + d] * m[i];
  red[tid] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) mw32[d] = (float)red[0];
}

// For an injected W: eig[d] = 1 / |w_d|^2 and U = W diag(eig)^(1/2).
__global__ void __launch_bounds__(256) k_from_injected(const double* __restrict__ W, int V, int D,
                                                       double* __restrict__ U,
                                                       double* __restrict__ eig) {
  __shared__ double red[256];
  const int d = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < V; i += blockDim.x) {
    const double w = W[(size_t)i * D + d];
    s += w * w;
  }
  red[tid] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double nrm2 = red[0];
  if (tid == 0) eig[d] = nrm2 > 0.0 ? 1.0 / nrm2 : 0.0;
  const double sc = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  for (int i = tid; i < V; i += blockDim.x) U[(size_t)i * D + d] = W[(size_t)i * D + d] * sc;
}

inline int blocks_for(size_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_random_block(double* Q, int V, int p, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_random_block, dim3(blocks_for((size_t)V * p, 256)), dim3(256), 0, s, Q, V,
                     p, seed);
  return hipGetLastError();
}

hipError_t launch_vecT_mat(const double* m, const double* Q, double* t, int V, int p,
                           hipStream_t s) {
  // t (1 x p) = m^T Q as a GEMM with op(A) = m^T
  const int splits = (V + 4095) / 4096;
  return gemm(true, 1, p, V, m, 1, Q, p, t, p, 1.0, splits, s);
}

hipError_t launch_m2_apply(const double* S2, const double* m, const double* t, const double* Q,
                           double* Y, int V, int p, double scale_s, double scale_m,
                           hipStream_t s) {
  hipError_t e = gemm(false, V, p, V, S2, V, Q, p, Y, p, scale_s, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank1_update, dim3(blocks_for((size_t)V * p, 256)), dim3(256), 0, s, Y, m,
                     t, V, p, scale_m);
  return hipGetLastError();
}

hipError_t launch_gram(const double* A, const double* B, double* G, int V, int p, hipStream_t s) {
  const int splits = (V + 2047) / 2048;
  return gemm(true, p, p, V, A, p, B, p, G, p, 1.0, splits, s);
}

hipError_t launch_cholesky(double* G, int p, double shift_rel, int* info, hipStream_t s) {
  if (p <= kLdsP)
    hipLaunchKernelGGL(k_cholesky_lds, dim3(1), dim3(1024), 0, s, G, p, shift_rel, info);
  else
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, G, p, shift_rel, info);
  return hipGetLastError();
}

// Y (V x p) <- Y L^-T, written to Out; Binv is p x p scratch.
hipError_t launch_trsm_right_into(const double* Y, const double* G, double* Binv, double* Out, int V,
                                  int p, hipStream_t s) {
  if (p > 64 * kInvJ) return hipErrorInvalidValue;   // a lane keeps kInvJ entries of a column
  hipLaunchKernelGGL(k_tri_inverse_waves, dim3((p + 3) / 4), dim3(256), 0, s, G, p, Binv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return gemm(false, V, p, p, Y, p, Binv, p, Out, p, 1.0, 1, s);
}

hipError_t launch_jacobi(double* A, double* Z, double* ev, int p, int* info, hipStream_t s) {
  if (p <= kLdsPZ) {
    hipLaunchKernelGGL(k_jacobi_lds<true>, dim3(1), dim3(1024), 0, s, A, Z, ev, p, info);
    return hipGetLastError();
  }
  if (p <= kLdsP) {
    hipLaunchKernelGGL(k_jacobi_lds<false>, dim3(1), dim3(1024), 0, s, A, Z, ev, p, info);
    return hipGetLastError();
  }
  const int m = (p + 1) & ~1;
  const int nt = 1024;
  const size_t shmem = sizeof(double) * (3 * (m / 2) + 2 * nt) + sizeof(int) * m;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(nt), shmem, s, A, Z, ev, p, info);
  return hipGetLastError();
}

hipError_t launch_block_product(const double* Q, const double* Z, double* Out, int V, int p,
                                hipStream_t s) {
  return gemm(false, V, p, p, Q, p, Z, p, Out, p, 1.0, 1, s);
}

hipError_t launch_ritz_vectors(const double* Q, const double* Z, const double* ev, int V, int p,
                               int D, double* U, double* eigD, hipStream_t s) {
  // Zs is placed right after eigD's D entries in caller scratch: eigD [D], Zs [p][D]
  double* Zs = eigD + D;
  hipLaunchKernelGGL(k_select_top, dim3(1), dim3(256), 0, s, Z, ev, p, D, Zs, eigD);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = gemm(false, V, D, p, Q, p, Zs, D, U, D, 1.0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sign_fix, dim3(D), dim3(256), 0, s, U, V, D);
  return hipGetLastError();
}

hipError_t launch_form_whitening(const double* U, const double* eig, const double* m, int V, int D,
                                 int Dp, double* W, float* W32, float* mw32, hipStream_t s) {
  hipLaunchKernelGGL(k_form_w, dim3(blocks_for((size_t)V * Dp, 256)), dim3(256), 0, s, U, eig, V,
                     D, Dp, W, W32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mw, dim3(Dp), dim3(256), 0, s, W, m, V, D, Dp, mw32);
  return hipGetLastError();
}

hipError_t launch_from_injected(const double* W, int V, int D, double* U, double* eig,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_from_injected, dim3(D), dim3(256), 0, s, W, V, D, U, eig);
  return hipGetLastError();
}

int dgemm_splits(int M, int N, int K, int num_cu) {
  // blocks resident at once: two 8-wave blocks per CU; the time of a product
  // goes as (rounds of resident blocks) / splits, so pick the split count in
  // 1 .. 8 (chunks of at least 1024) with the fewest rounds per split,
  // the smallest count on ties
  const long long blocks = (long long)((N + 127) / 128) * ((M + kDgBM - 1) / kDgBM);
  const long long slots = 2LL * num_cu;
  if (K < 2048 || blocks <= 0) return 1;
  int best = 1;
  double best_t = (double)((blocks + slots - 1) / slots);
  for (int sp = 2; sp <= 8 && K / sp >= 1024; ++sp) {
    const double t = (double)((blocks * sp + slots - 1) / slots) / sp;
    if (t < best_t - 1e-9) {
      best_t = t;
      best = sp;
    }
  }
  return best;
}

}  // namespace tlda
