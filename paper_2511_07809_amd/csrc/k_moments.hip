// Moment accumulation: document statistics, sum f and the upper triangle of
// sum f f^T over the kept documents of a CSR batch (section "Computing the
// Centered Cumulants"; documents with fewer than three tokens are dropped).
#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kWave = 64;

__device__ inline long long wave_sum_ll(long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline int wave_sum_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Each wave checks one row: bounds of row_ptr, column range and order, and
// that counts are positive integers <= 2^24.  Any failure sets *err.
__global__ void __launch_bounds__(256) k_validate_csr(const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const float* __restrict__ val, int n_rows,
                                                     int nnz, int V, int* __restrict__ err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (row >= n_rows) return;
  const int b = row_ptr[row], e = row_ptr[row + 1];
  int bad = 0;
  if (row == 0 && b != 0) bad = 1;
  if (row == n_rows - 1 && e != nnz) bad = 1;
  if (b < 0 || e < b || e > nnz) {
    bad = 1;
  } else {
    for (int j = b + lane; j < e; j += kWave) {
      const int c = col_idx[j];
      const float v = val[j];
      if (c < 0 || c >= V) bad = 1;
      if (j > b && col_idx[j - 1] >= c) bad = 1;
      if (!(v >= 1.0f) || v > 16777216.0f || v != rintf(v)) bad = 1;
    }
  }
  if (wave_sum_i(bad) != 0 && lane == 0) {
    atomicOr(err, 1);
    atomicMax(err + 1, n_rows - row);   // the first rejected row has the largest n_rows - row
  }
}

// Exact, order-independent accumulation of FP64 terms in [0, 2^63): every
// term t becomes the integer floor(t 2^64) (fixed point with 2^-64
// resolution; the truncation loses less than 2^-64 per term) and is added to
// a 128-bit accumulator {lo, hi} with 64-bit integer atomics: lo takes the
// low word, and when that add wraps (seen from the value the atomic returns)
// the carry goes to hi with the integer part.  Integer addition is
// associative, so the final {hi, lo} is the same bits for any order of the
// terms: the moments, and the W computed from them, are bit-reproducible.
__device__ __forceinline__ void fx_add(unsigned long long* __restrict__ acc, double t) {
  const double ip = floor(t);
  unsigned long long hi = (unsigned long long)ip;
  const unsigned long long lo = (unsigned long long)ldexp(t - ip, 64);
  if (lo != 0ull) {
    const unsigned long long old = atomicAdd(acc, lo);
    if (old + lo < old) ++hi;
  }
  if (hi != 0ull) atomicAdd(acc + 1, hi);
}

__device__ __forceinline__ double fx_value(const unsigned long long* __restrict__ acc) {
  return (double)acc[1] + ldexp((double)acc[0], -64);
}

// Entry (j, k), j <= k, of the packed upper triangle of a V x V matrix: row
// j holds columns j .. V - 1 and starts at j V - j (j - 1) / 2.
__device__ __forceinline__ size_t tri_index(int j, int k, int V) {
  return (size_t)j * V - (size_t)j * (j - 1) / 2 + (size_t)(k - j);
}

// One wave per document, grid-stride over the batch.  Token totals use 64-bit
// integer atomics and the frequency sums and pair sums the exact fixed-point
// accumulation above.  The pair loop enumerates the upper triangle (j <= k)
// of the row's nnz positions; as columns are strictly increasing,
// col_j <= col_k and the pair lands in the packed upper triangle of the
// accumulator.  Kept/dropped document counts are kept per block and added by
// k_add_counts, so no address is hit by every row.
// CLASSIC: the pair sum takes the unbiased piece of the appendix's second
// moment, c_j c_k / (L (L - 1)) off the diagonal and c_j (c_j - 1) / (L (L - 1))
// on it, in place of f_j f_k.
constexpr int kAccMaxBlocks = kWhitenBlockCounts;

template <bool CLASSIC>
__global__ void __launch_bounds__(256) k_accumulate(const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx,
                                                    const float* __restrict__ val, int n_rows,
                                                    int V, int* __restrict__ block_counts,
                                                    unsigned long long* __restrict__ totals,
                                                    unsigned long long* __restrict__ fsum,
                                                    unsigned long long* __restrict__ S2) {
  __shared__ int kept_s[4], drop_s[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  int kept = 0, dropped = 0;
  for (int row = blockIdx.x * 4 + wave; row < n_rows; row += gridDim.x * 4) {
    const int b = row_ptr[row], e = row_ptr[row + 1];
    const int n = e - b;
    long long part = 0;
    for (int j = lane; j < n; j += kWave) part += (long long)val[b + j];
    const long long L = wave_sum_ll(part);
    if (L < 3) {
      ++dropped;
      continue;
    }
    ++kept;
    const double invL = 1.0 / (double)L;
    const double l2 = 1.0 / ((double)L * (double)(L - 1));
    for (int j = lane; j < n; j += kWave) {
      const int c = col_idx[b + j];
      const float v = val[b + j];
      atomicAdd(&totals[c], (unsigned long long)v);
      fx_add(fsum + 2 * (size_t)c, (double)v * invL);
    }
    const long long P = (long long)n * (n + 1) / 2;
    const double tn = 2.0 * n + 1.0;
    for (long long p = lane; p < P; p += kWave) {
      // row j of the packed triangle starts at base(j) = j*n - j*(j-1)/2
      int j = (int)((tn - sqrt(tn * tn - 8.0 * (double)p)) * 0.5);
      if (j < 0) j = 0;
      if (j > n - 1) j = n - 1;
      while (j + 1 < n && (long long)(j + 1) * n - (long long)(j + 1) * j / 2 <= p) ++j;
      while (j > 0 && (long long)j * n - (long long)j * (j - 1) / 2 > p) --j;
      const long long base = (long long)j * n - (long long)j * (j - 1) / 2;
      const int k = j + (int)(p - base);
      const int cj = col_idx[b + j], ck = col_idx[b + k];
      double prod;
      if (CLASSIC) {
        const double vj = (double)val[b + j], vk = (double)val[b + k];
        prod = (j == k ? vj * (vj - 1.0) : vj * vk) * l2;
      } else {
        prod = ((double)val[b + j] * invL) * ((double)val[b + k] * invL);
      }
      fx_add(S2 + 2 * tri_index(cj, ck, V), prod);
    }
  }
  if (lane == 0) {
    kept_s[wave] = kept;
    drop_s[wave] = dropped;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    block_counts[2 * blockIdx.x] = kept_s[0] + kept_s[1] + kept_s[2] + kept_s[3];
    block_counts[2 * blockIdx.x + 1] = drop_s[0] + drop_s[1] + drop_s[2] + drop_s[3];
  }
}

// counts[0] += kept, counts[1] += dropped over the per-block counts (one block).
__global__ void __launch_bounds__(256) k_add_counts(const int* __restrict__ block_counts, int nb,
                                                    unsigned long long* __restrict__ counts) {
  __shared__ long long rk[256], rd[256];
  long long k = 0, d = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    k += block_counts[2 * i];
    d += block_counts[2 * i + 1];
  }
  rk[threadIdx.x] = k;
  rd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rk[threadIdx.x] += rk[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[0] += (unsigned long long)rk[0];
    counts[1] += (unsigned long long)rd[0];
  }
}

// The FP64 symmetric S2 of the refresh's products from the packed upper
// triangle of the fixed-point accumulator: a 32 x 32 tile of the upper
// triangle is converted row-wise, written in place and, through LDS,
// transposed into the lower triangle, so reads and writes are coalesced.
__global__ void __launch_bounds__(256) k_fx_symmetric(const unsigned long long* __restrict__ acc,
                                                      int V, double* __restrict__ S2) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;     // source tile (bi, bj) of the upper triangle
  if (bi > bj) return;
  const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int gi = bi * 32 + r, gj = bj * 32 + tx;
    double v = 0.0;
    if (gi < V && gj < V && gi <= gj) {
      v = fx_value(acc + 2 * tri_index(gi, gj, V));
      S2[(size_t)gi * V + gj] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int gi = bj * 32 + r, gj = bi * 32 + tx;   // destination (gi, gj), gi > gj
    if (gi < V && gj < V && gj < gi) S2[(size_t)gi * V + gj] = tile[tx][r];
  }
}

__global__ void k_mean(const unsigned long long* __restrict__ fsum,
                       const unsigned long long* __restrict__ counts, double* __restrict__ m,
                       int V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) m[i] = fx_value(fsum + 2 * (size_t)i) / (double)counts[0];
}

// Widening of a compact staged batch, four entries per thread.
__global__ void __launch_bounds__(256) k_widen_u16(const uint16_t* __restrict__ col16,
                                                   const uint16_t* __restrict__ val16, size_t nnz,
                                                   int32_t* __restrict__ col,
                                                   float* __restrict__ val) {
  const size_t base = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t j = base + q;
    if (j < nnz) {
      col[j] = (int32_t)col16[j];
      val[j] = (float)val16[j];
    }
  }
}

}  // namespace

hipError_t launch_widen_u16(const uint16_t* col16, const uint16_t* val16, size_t nnz,
                            int32_t* col, float* val, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  const size_t threads = (nnz + 3) / 4;
  hipLaunchKernelGGL(k_widen_u16, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, col16,
                     val16, nnz, col, val);
  return hipGetLastError();
}

hipError_t launch_validate_csr(const tlda_csr_batch& b, int V, int* err, hipStream_t s) {
  const int rows_per_block = 256 / kWave;
  const int grid = (b.n_rows + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL(k_validate_csr, dim3(grid), dim3(256), 0, s, b.row_ptr, b.col_idx, b.val,
                     b.n_rows, b.nnz, V, err);
  return hipGetLastError();
}

hipError_t launch_accumulate(const tlda_csr_batch& b, int V, const Moments& m, int* block_counts,
                             bool classic, hipStream_t s) {
  const int rows_per_block = 256 / kWave;
  int grid = (b.n_rows + rows_per_block - 1) / rows_per_block;
  if (grid > kAccMaxBlocks) grid = kAccMaxBlocks;
  if (classic)
    hipLaunchKernelGGL(k_accumulate<true>, dim3(grid), dim3(256), 0, s, b.row_ptr, b.col_idx,
                       b.val, b.n_rows, V, block_counts, m.totals, m.fsum, m.acc);
  else
    hipLaunchKernelGGL(k_accumulate<false>, dim3(grid), dim3(256), 0, s, b.row_ptr, b.col_idx,
                       b.val, b.n_rows, V, block_counts, m.totals, m.fsum, m.acc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_add_counts, dim3(1), dim3(256), 0, s, block_counts, grid, m.counts);
  return hipGetLastError();
}

hipError_t launch_fx_symmetric(const unsigned long long* acc, int V, double* S2, hipStream_t s) {
  const int nt = (V + 31) / 32;
  hipLaunchKernelGGL(k_fx_symmetric, dim3(nt, nt), dim3(32, 8), 0, s, acc, V, S2);
  return hipGetLastError();
}

hipError_t launch_mean(const unsigned long long* fsum, const unsigned long long* counts, double* m,
                       int V, hipStream_t s) {
  hipLaunchKernelGGL(k_mean, dim3((V + 255) / 256), dim3(256), 0, s, fsum, counts, m, V);
  return hipGetLastError();
}

}  // namespace tlda
