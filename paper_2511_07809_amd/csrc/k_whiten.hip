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

// Kernel-wide count of kept rows without same-address device atomics (which
// serialise across the XCDs): every block stores its own count, and a
// one-block kernel adds the counts in block order.
constexpr int kWhitenMaxBlocks = kWhitenBlockCounts;

// 16-byte gather of W32 at a 32-bit byte offset (W32 is far below 4 GiB).
__device__ inline float4 ld_b128(const float* __restrict__ base, int byte_off) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(base) + byte_off);
}

// G lanes per document, V4 float4 columns per lane.
template <int G, int V4>
__global__ void __launch_bounds__(256) k_whiten(const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col_idx,
                                                const float* __restrict__ val, int n_rows,
                                                const float* __restrict__ W32, int V,
                                                const float* __restrict__ mw32, int D, int Dp,
                                                int S, float* __restrict__ X,
                                                int* __restrict__ block_counts) {
  constexpr int RPW = 64 / G;
  constexpr int RPB = 4 * RPW;                  // rows per block per sweep
  constexpr int NB = 16 / V4;                   // nonzeros per step of a row
  constexpr int SLOTS = G >= NB ? 1 : NB / G;   // nonzeros each lane fetches per step
  __shared__ int wave_kept[4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gl = lane % G;
  // Column chunk of this block: workgroups go round-robin to the 8 XCDs, so
  // block b runs on XCD b % 8 and chunk b % S keeps every XCD on one slice of
  // W (Dp / S columns), which then stays in that XCD's L2.
  const int chunk = blockIdx.x % S;
  const int c0 = chunk * (Dp / S) + gl * 4 * V4;   // first of this lane's columns
  const bool active = gl * 4 * V4 < Dp / S;
  const int nblk_chunk = gridDim.x / S;
  int kept_total = 0;
  for (int base = (blockIdx.x / S) * RPB; base < n_rows; base += nblk_chunk * RPB) {
    const int row = base + wave * RPW + lane / G;
    const bool valid = row < n_rows;
    int b = 0, e = 0;
    if (valid) {
      b = row_ptr[row];
      e = row_ptr[row + 1];
    }
    float4 acc[V4];
#pragma unroll
    for (int v = 0; v < V4; ++v) acc[v] = make_float4(0.f, 0.f, 0.f, 0.f);
    float Lp = 0.f;
    // Step through the row NB nonzeros at a time: the G lanes of the row fetch
    // the step's (column, count) pairs together (one memory round trip), pass
    // them around with lane shuffles, and issue all of the step's W-row
    // gathers before using any of them.
    for (int jb = b; jb < e; jb += NB) {
      int cidx[SLOTS];
      float cval[SLOTS];
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int j = jb + q * G + gl;
        const bool in = (q * G + gl) < NB && j < e;
        cidx[q] = in ? col_idx[j] : 0;
        cval[q] = in ? val[j] : 0.f;
        Lp += cval[q];
      }
      float4 w[NB][V4];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const int c = G == 1 ? cidx[t] : __shfl(cidx[t / G < SLOTS ? t / G : 0], t % G, G);
        const int off = (c * Dp + c0) * (int)sizeof(float);
#pragma unroll
        for (int v = 0; v < V4; ++v) {
          w[t][v] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (active && jb + t < e) w[t][v] = ld_b128(W32, off + 16 * v);
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const float x = G == 1 ? cval[t] : __shfl(cval[t / G < SLOTS ? t / G : 0], t % G, G);
#pragma unroll
        for (int v = 0; v < V4; ++v) {
          acc[v].x = fmaf(x, w[t][v].x, acc[v].x);
          acc[v].y = fmaf(x, w[t][v].y, acc[v].y);
          acc[v].z = fmaf(x, w[t][v].z, acc[v].z);
          acc[v].w = fmaf(x, w[t][v].w, acc[v].w);
        }
      }
    }
    // document length: sum of the lanes' partial counts within the group
    float L = Lp;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) L += __shfl_xor(L, off, G);
    int kept = 0;
    if (valid) {
      if (L >= 3.f) kept = 1;
      if (active) {
        const float invL = 1.0f / L;
        float* out = X + (size_t)row * D;
#pragma unroll
        for (int v = 0; v < V4; ++v) {
          const int c4 = c0 + 4 * v;
          float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
          if (kept) {
            const float4 mw = *reinterpret_cast<const float4*>(mw32 + c4);
            x.x = fmaf(acc[v].x, invL, -mw.x);
            x.y = fmaf(acc[v].y, invL, -mw.y);
            x.z = fmaf(acc[v].z, invL, -mw.z);
            x.w = fmaf(acc[v].w, invL, -mw.w);
          }
          if (c4 + 0 < D) out[c4 + 0] = x.x;
          if (c4 + 1 < D) out[c4 + 1] = x.y;
          if (c4 + 2 < D) out[c4 + 2] = x.z;
          if (c4 + 3 < D) out[c4 + 3] = x.w;
        }
      }
    }
    kept_total += __popcll(__ballot(kept && gl == 0));
  }
  if (lane == 0) wave_kept[wave] = kept_total;
  __syncthreads();
  if (threadIdx.x == 0)
    block_counts[blockIdx.x] =
        chunk == 0 ? wave_kept[0] + wave_kept[1] + wave_kept[2] + wave_kept[3] : 0;
}

__global__ void __launch_bounds__(256) k_sum_counts(const int* __restrict__ block_counts, int n,
                                                    int* __restrict__ out) {
  __shared__ int red[256];
  int s = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += block_counts[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_zero(uint32_t* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_zero_bytes(unsigned char* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <int G, int V4>
hipError_t launch_g(const tlda_csr_batch& b, const float* W32, int V, const float* mw32, int D,
                    int Dp, int S, float* X, int* n_kept, int* block_counts, hipStream_t s) {
  const int rows_per_block = 4 * (64 / G);
  int per_chunk = (b.n_rows + rows_per_block - 1) / rows_per_block;
  if (per_chunk * S > kWhitenMaxBlocks) per_chunk = kWhitenMaxBlocks / S;
  const int grid = per_chunk * S;
  launch_main(k_whiten<G, V4>, dim3(grid), dim3(256), 0, s, b.row_ptr, b.col_idx, b.val, b.n_rows,
              W32, V, mw32, D, Dp, S, X, block_counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_kept == nullptr) return e;
  hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(256), 0, s, block_counts, grid, n_kept);
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

hipError_t launch_sum_counts(const int* block_counts, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(256), 0, s, block_counts, n, out);
  return hipGetLastError();
}

// Number of column chunks of the whitening: the smallest of 1, 2, 4, 8 that
// makes one chunk of the FP32 W copy (V x Dp/S floats) fit in 3 MiB, the L2
// share an XCD can spare beside the streaming CSR and X traffic, with at least
// four columns per chunk.
int whiten_chunks(int V, int Dp) {
  int S = 1;
  while (S < 8 && (size_t)V * (Dp / S) * sizeof(float) > (3u << 20) && (Dp / (2 * S)) % 4 == 0)
    S *= 2;
  return S;
}

hipError_t launch_whiten(const tlda_csr_batch& b, const float* W32, const float* mw32, int V, int D,
                         int Dp, float* X, int* n_kept, int* block_counts, const Tuning& t,
                         hipStream_t s) {
  if (b.n_rows == 0) return n_kept != nullptr ? launch_zero(n_kept, sizeof(int), s) : hipSuccess;
  // Measured on MI355X at V = 20 000, D = 50: one chunk and one float4 per
  // lane is fastest; the XCD column split and two float4 per lane are kept as
  // tuning options.
  int S = 1;
  if (t.whiten_chunks < 0) S = whiten_chunks(V, Dp);
  if (t.whiten_chunks == 2 || t.whiten_chunks == 4 || t.whiten_chunks == 8)
    if ((Dp / t.whiten_chunks) % 4 == 0) S = t.whiten_chunks;
  const int wc = Dp / S;   // columns per chunk, a multiple of 4
  if (wc % 8 == 0 && t.whiten_v4 == 2) {
    const int g = wc / 8;
    if (g <= 1) return launch_g<1, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
    if (g <= 2) return launch_g<2, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
    if (g <= 4) return launch_g<4, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
    if (g <= 8) return launch_g<8, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
    if (g <= 16) return launch_g<16, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
    return launch_g<32, 2>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  }
  const int g = wc / 4;
  if (g <= 1) return launch_g<1, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  if (g <= 2) return launch_g<2, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  if (g <= 4) return launch_g<4, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  if (g <= 8) return launch_g<8, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  if (g <= 16) return launch_g<16, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  if (g <= 32) return launch_g<32, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
  return launch_g<64, 1>(b, W32, V, mw32, D, Dp, S, X, n_kept, block_counts, s);
}

}  // namespace tlda
