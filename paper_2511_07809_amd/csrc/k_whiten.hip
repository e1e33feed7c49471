// Whitening SpMM (online second-moment section): for each document of a CSR
// batch, x = W^T (f - M1) = (1/L) sum_j c_j W[col_j, :] - W^T M1, computed
// without ever forming the dense centred batch.
//
// Mapping: a group of G lanes owns one document and holds its D-vector as one
// float4 per lane (G = next power of two of Dp/4, so 64/G documents share a
// wave).  For every nonzero the (column, count) pair is read once per group
// and the group reads the W row as one coalesced 16 * G byte access; rows of
// the FP32 W copy are padded to Dp floats (a cache-line multiple once
// D >= 32).  Four nonzeros are issued before their FMAs so that four row
// gathers are in flight per group.  The 1/L scale and the -W^T M1 shift are
// applied in registers at the end of the row, and the row is written once.
#include "tlda_internal.h"

namespace tlda {
namespace {

template <int G>
__global__ void __launch_bounds__(256) k_whiten(const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col_idx,
                                                const float* __restrict__ val, int n_rows,
                                                const float* __restrict__ W32,
                                                const float* __restrict__ mw32, int D, int Dp,
                                                float* __restrict__ X, int* __restrict__ n_kept,
                                                int* __restrict__ sync) {
  constexpr int RPW = 64 / G;
  __shared__ int block_kept;
  if (threadIdx.x == 0) block_kept = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gl = lane % G;
  const int row = (blockIdx.x * 4 + wave) * RPW + lane / G;
  const int c4 = gl * 4;                       // first of this lane's four columns
  const bool active = c4 < Dp;
  int kept = 0;
  if (row < n_rows) {
    const int b = row_ptr[row], e = row_ptr[row + 1];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    float L = 0.f;
    int j = b;
    for (; j + 4 <= e; j += 4) {
      const int i0 = col_idx[j], i1 = col_idx[j + 1], i2 = col_idx[j + 2], i3 = col_idx[j + 3];
      const float v0 = val[j], v1 = val[j + 1], v2 = val[j + 2], v3 = val[j + 3];
      float4 w0 = make_float4(0.f, 0.f, 0.f, 0.f), w1 = w0, w2 = w0, w3 = w0;
      if (active) {
        w0 = *reinterpret_cast<const float4*>(W32 + (size_t)i0 * Dp + c4);
        w1 = *reinterpret_cast<const float4*>(W32 + (size_t)i1 * Dp + c4);
        w2 = *reinterpret_cast<const float4*>(W32 + (size_t)i2 * Dp + c4);
        w3 = *reinterpret_cast<const float4*>(W32 + (size_t)i3 * Dp + c4);
      }
      acc.x = fmaf(v0, w0.x, acc.x); acc.y = fmaf(v0, w0.y, acc.y);
      acc.z = fmaf(v0, w0.z, acc.z); acc.w = fmaf(v0, w0.w, acc.w);
      acc.x = fmaf(v1, w1.x, acc.x); acc.y = fmaf(v1, w1.y, acc.y);
      acc.z = fmaf(v1, w1.z, acc.z); acc.w = fmaf(v1, w1.w, acc.w);
      acc.x = fmaf(v2, w2.x, acc.x); acc.y = fmaf(v2, w2.y, acc.y);
      acc.z = fmaf(v2, w2.z, acc.z); acc.w = fmaf(v2, w2.w, acc.w);
      acc.x = fmaf(v3, w3.x, acc.x); acc.y = fmaf(v3, w3.y, acc.y);
      acc.z = fmaf(v3, w3.z, acc.z); acc.w = fmaf(v3, w3.w, acc.w);
      L += (v0 + v1) + (v2 + v3);
    }
    for (; j < e; ++j) {
      const int i0 = col_idx[j];
      const float v0 = val[j];
      float4 w0 = make_float4(0.f, 0.f, 0.f, 0.f);
      if (active) w0 = *reinterpret_cast<const float4*>(W32 + (size_t)i0 * Dp + c4);
      acc.x = fmaf(v0, w0.x, acc.x); acc.y = fmaf(v0, w0.y, acc.y);
      acc.z = fmaf(v0, w0.z, acc.z); acc.w = fmaf(v0, w0.w, acc.w);
      L += v0;
    }
    float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
    if (L >= 3.f) {
      kept = 1;
      if (active) {
        const float invL = 1.0f / L;
        const float4 mw = *reinterpret_cast<const float4*>(mw32 + c4);
        x.x = fmaf(acc.x, invL, -mw.x);
        x.y = fmaf(acc.y, invL, -mw.y);
        x.z = fmaf(acc.z, invL, -mw.z);
        x.w = fmaf(acc.w, invL, -mw.w);
      }
    }
    float* out = X + (size_t)row * D;
    if (c4 + 0 < D) out[c4 + 0] = x.x;
    if (c4 + 1 < D) out[c4 + 1] = x.y;
    if (c4 + 2 < D) out[c4 + 2] = x.z;
    if (c4 + 3 < D) out[c4 + 3] = x.w;
  }
  if (n_kept == nullptr) return;
  // kept-row count: per-block sum, then one device atomic per block; the last
  // block to finish publishes the total and re-arms the counters (sync[0]:
  // running sum, sync[1]: finished blocks) for the next call on this context
  const unsigned long long mask = __ballot(kept && gl == 0);
  if (lane == 0 && mask != 0ull) atomicAdd(&block_kept, (int)__popcll(mask));
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&sync[0], block_kept);
    __threadfence();
    const int done = atomicAdd(&sync[1], 1);
    if (done == (int)gridDim.x - 1) {
      __threadfence();
      *n_kept = atomicExch(&sync[0], 0);
      atomicExch(&sync[1], 0);
    }
  }
}

__global__ void k_zero(uint32_t* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_zero_bytes(unsigned char* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <int G>
hipError_t launch_g(const tlda_csr_batch& b, const float* W32, const float* mw32, int D, int Dp,
                    float* X, int* n_kept, int* sync, hipStream_t s) {
  const int rows_per_block = 4 * (64 / G);
  const int grid = (b.n_rows + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL(k_whiten<G>, dim3(grid), dim3(256), 0, s, b.row_ptr, b.col_idx, b.val,
                     b.n_rows, W32, mw32, D, Dp, X, n_kept, sync);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((bytes % 4) == 0 && (reinterpret_cast<uintptr_t>(ptr) % 4) == 0) {
    const size_t n = bytes / 4;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       static_cast<uint32_t*>(ptr), n);
  } else {
    hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, s,
                       static_cast<unsigned char*>(ptr), bytes);
  }
  return hipGetLastError();
}

hipError_t launch_whiten(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                         int Dp, float* X, int* n_kept, int* sync, hipStream_t s) {
  if (b.n_rows == 0) return n_kept != nullptr ? launch_zero(n_kept, sizeof(int), s) : hipSuccess;
  const int q = Dp / 4;   // float4 columns per row, Dp is a multiple of 4 and <= 256
  if (q <= 2) return launch_g<2>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
  if (q <= 4) return launch_g<4>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
  if (q <= 8) return launch_g<8>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
  if (q <= 16) return launch_g<16>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
  if (q <= 32) return launch_g<32>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
  return launch_g<64>(b, W32, mw32, D, Dp, X, n_kept, sync, s);
}

}  // namespace tlda
