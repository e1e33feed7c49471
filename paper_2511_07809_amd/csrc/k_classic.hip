// CP-gradient data term on the classic alpha0-corrected moments (the
// appendix's cumulants, run through the batched SGD of section "Online
// Learning of the Third Moment").  Per kept document with counts c, length L,
// l2 = 1/(L(L-1)), l3 = l2/(L-2), the piece of M3 contracted with
// (W, phi_k, phi_k) is, with y = W^T c, z_w = Phi^T W_w (row w of Z = W Phi),
// s = sum_w c_w z_w, q = sum_w c_w z_w^2, r = Phi^T (W^T M1):
//   c3 l3 (y s^2 - 2 s g - y q + 2 h) - c2 l2 (2 r (y s - g) + m_w (s^2 - q))
//   + alpha0^2 m_w r^2,        g = sum_w c_w W_w z_w,  h = sum_w c_w W_w z_w^2,
// column k taking the k-th entries of s, q, r, z (c2 = alpha0(alpha0+1)/2,
// c3 = (alpha0+1)(alpha0+2)/2, m_w = W^T M1).  Grouped by what multiplies W
// rows (y_d = sum_w c_w W_w), the batch sum divided by c3 is one reduction
// with a row per nonzero (d, w),
//   sum over nonzeros (d, w):  W_w  (x)  c_w (a_d + b_d * z_w + g_d z_w^2)
//   plus m_w (x) sum_d e_d,
// with a = l3 (s^2 - q) - 2 (c2/c3) l2 r s, b = -2 l3 s + 2 (c2/c3) l2 r,
// g_d = 2 l3 and e = -(c2/c3) l2 (s^2 - q) + (alpha0^2/c3) r^2 (zero for
// dropped documents).
//
// k_classic_z forms Z (FP32, V x Kp) and r once per step.  k_classic_cp runs
// over tiles of 16 documents: phase 1 (a wave per document) gathers the Z rows
// of the document's words for s, q and the coefficients; phase 2 stages the
// tile's nonzero rows (W rows with their scaled Z rows) in LDS, kRows at a
// time and double-buffered, and accumulates the D x K outer products on FP32
// matrix cores.  Each block writes its partial sum and its kept-document
// count; the shared finish kernel adds them in block order, forms the
// gradient with the penalty term and updates Phi.
#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kThreads = 256;
constexpr int kDocs = 16;    // documents per tile
constexpr int kRows = 16;    // reduction rows per staged chunk (two buffers)
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Z[w][k] = sum_d W32[w][d] Phi[d][k] (zero for K <= k < Kp); block 0 also
// writes r[k] = sum_d mw32[d] Phi[d][k] and the copy of Phi that the finish
// kernel reads while it overwrites Phi.  Phi is staged in LDS (D*K <= 16384).
__global__ void __launch_bounds__(kThreads) k_classic_z(const float* __restrict__ W32, int V,
                                                        int D, int Dp,
                                                        const float* __restrict__ Phi, int K,
                                                        int Kp, const float* __restrict__ mw32,
                                                        float* __restrict__ Z,
                                                        float* __restrict__ r,
                                                        float* __restrict__ phi_copy) {
  extern __shared__ float ph[];
  const int tid = threadIdx.x;
  for (int e = tid; e < D * K; e += kThreads) ph[e] = Phi[e];
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < D * K; e += kThreads) phi_copy[e] = ph[e];
    for (int k = tid; k < Kp; k += kThreads) {
      float s = 0.f;
      if (k < K)
        for (int d = 0; d < D; ++d) s = fmaf(mw32[d], ph[d * K + k], s);
      r[k] = s;
    }
  }
  const size_t n = (size_t)V * Kp;
  for (size_t e = (size_t)blockIdx.x * kThreads + tid; e < n; e += (size_t)gridDim.x * kThreads) {
    const int w = (int)(e / Kp), k = (int)(e % Kp);
    float s = 0.f;
    if (k < K) {
      const float* wr = W32 + (size_t)w * Dp;
      for (int d = 0; d < D; ++d) s = fmaf(wr[d], ph[d * K + k], s);
    }
    Z[e] = s;
  }
}

template <int DQ, int KQ>
__global__ void __launch_bounds__(kThreads, 2) k_classic_cp(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const float* __restrict__ W32, int Dp,
    const float* __restrict__ Z, int Kp, const float* __restrict__ mw32,
    const float* __restrict__ r_g, int D, int K, float c2r, float a0r, int nblk,
    float* __restrict__ partial, int* __restrict__ block_counts) {
  constexpr int LDA = DQ + 4, LDB = KQ + 4;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NRT = NDT * NCT;
  constexpr int RT = (NRT + 3) / 4;
  constexpr int NK = (KQ + 63) / 64;                        // phase-1 columns per lane
  constexpr int GA = DQ / 4, GB = KQ / 4;                   // float4 groups per staged row
  constexpr int TPR = kThreads / kRows;                     // threads per staged row
  constexpr int UA = (GA + TPR - 1) / TPR, UB = (GB + TPR - 1) / TPR;
  constexpr int NB = 8;                                     // nonzeros per gather step
  static_assert(kThreads % kRows == 0, "staging maps whole rows to threads");
  __shared__ __attribute__((aligned(16))) float As[2][kRows * LDA];
  __shared__ __attribute__((aligned(16))) float Bs[2][kRows * LDB];
  __shared__ __attribute__((aligned(16))) float Al[kDocs * LDB];
  __shared__ __attribute__((aligned(16))) float Be[kDocs * LDB];
  __shared__ float gam[kDocs];
  __shared__ int rps[kDocs + 1];
  __shared__ float rsh[KQ];
  __shared__ float dsh[4][KQ];
  __shared__ int wave_kept[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int srow = tid / TPR, ssub = tid % TPR;   // staged row and column-group lane

  for (int k = tid; k < KQ; k += kThreads) rsh[k] = k < K ? r_g[k] : 0.f;
  float dl[NK];
#pragma unroll
  for (int u = 0; u < NK; ++u) dl[u] = 0.f;
  floatx4 acc[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  int kept_total = 0;
  int buf = 0;

  const int ntiles = (n_rows + kDocs - 1) / kDocs;
  for (int tile = blockIdx.x; tile < ntiles; tile += nblk) {
    const int t0 = tile * kDocs;
    const int nd = n_rows - t0 < kDocs ? n_rows - t0 : kDocs;
    __syncthreads();   // the previous tile's LDS reads are done
    if (tid <= kDocs) rps[tid] = row_ptr[t0 + (tid < nd ? tid : nd)];
    __syncthreads();
    // ---- phase 1: per-document s, q, L and coefficients (a wave per document) ----
    for (int ld = wave; ld < kDocs; ld += 4) {
      float s[NK], q[NK];
#pragma unroll
      for (int u = 0; u < NK; ++u) s[u] = q[u] = 0.f;
      float L = 0.f;
      if (ld < nd) {
        const int b = rps[ld], e = rps[ld + 1];
        for (int jb = b; jb < e; jb += NB) {
          int mc = 0;
          float mv = 0.f;
          if (lane < NB && jb + lane < e) {
            mc = col_idx[jb + lane];
            mv = val[jb + lane];
          }
          float zv[NB][NK];
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const int c = __shfl(mc, t, 64);   // 0 (a valid row) past the document's end
#pragma unroll
            for (int u = 0; u < NK; ++u) {
              const int k = lane + 64 * u;
              zv[t][u] = k < Kp ? Z[(size_t)c * Kp + k] : 0.f;
            }
          }
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const float v = __shfl(mv, t, 64);   // 0 past the document's end
            L += v;
#pragma unroll
            for (int u = 0; u < NK; ++u) {
              s[u] = fmaf(v, zv[t][u], s[u]);
              q[u] = fmaf(v * zv[t][u], zv[t][u], q[u]);
            }
          }
        }
      }
      const bool keep = ld < nd && L >= 3.f;   // L is the same on every lane
      const float l2 = keep ? 1.0f / (L * (L - 1.0f)) : 0.f;
      const float l3 = keep ? l2 / (L - 2.0f) : 0.f;
#pragma unroll
      for (int u = 0; u < NK; ++u) {
        const int k = lane + 64 * u;
        if (k < KQ) {
          const float rk = rsh[k], sk = s[u], d2 = s[u] * s[u] - q[u];
          Al[ld * LDB + k] = l3 * d2 - 2.0f * c2r * l2 * rk * sk;
          Be[ld * LDB + k] = -2.0f * l3 * sk + 2.0f * c2r * l2 * rk;
          if (keep) dl[u] += -c2r * l2 * d2 + a0r * rk * rk;
        }
      }
      if (lane == 0) gam[ld] = 2.0f * l3;
      kept_total += keep ? 1 : 0;
    }
    __syncthreads();
    // ---- phase 2: one reduction row per nonzero, staged kRows at a time
    // (double-buffered: the gathers of chunk i+1 are in flight during the
    // matrix-core work on chunk i) ----
    const int nb0 = rps[0];
    const int nnz = rps[nd] - nb0;
    float4 wr[UA], zr[UB];
    float pv = 0.f;
    int pdoc = 0;
    auto fetch = [&](int cs) {
      const int gi = cs + srow;
      const bool in = gi < nnz;
      const int j = nb0 + (in ? gi : 0);
      const int col = col_idx[j];
      pv = in ? val[j] : 0.f;            // rows past the tile's end add zero
      int lo = 0, hi = nd;               // rps[lo] <= j < rps[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rps[mid] <= j) lo = mid;
        else hi = mid;
      }
      pdoc = lo;
#pragma unroll
      for (int u = 0; u < UA; ++u) {
        const int g = ssub + TPR * u;
        wr[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < GA && 4 * g < Dp) wr[u] = *reinterpret_cast<const float4*>(W32 + (size_t)col * Dp + 4 * g);
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int g = ssub + TPR * u;
        zr[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < GB && 4 * g < Kp) zr[u] = *reinterpret_cast<const float4*>(Z + (size_t)col * Kp + 4 * g);
      }
    };
    if (nnz > 0) fetch(0);
    for (int cs = 0; cs < nnz; cs += kRows) {
      // B row = c (a_d + b_d * z + g_d z^2); A row = W row
      const float g = gam[pdoc];
#pragma unroll
      for (int u = 0; u < UA; ++u) {
        const int gg = ssub + TPR * u;
        if (gg < GA) *reinterpret_cast<float4*>(&As[buf][srow * LDA + 4 * gg]) = wr[u];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int gg = ssub + TPR * u;
        if (gg < GB) {
          const float4 al = *reinterpret_cast<const float4*>(Al + pdoc * LDB + 4 * gg);
          const float4 be = *reinterpret_cast<const float4*>(Be + pdoc * LDB + 4 * gg);
          const float4 z = zr[u];
          float4 o;
          o.x = pv * fmaf(g * z.x + be.x, z.x, al.x);
          o.y = pv * fmaf(g * z.y + be.y, z.y, al.y);
          o.z = pv * fmaf(g * z.z + be.z, z.z, al.z);
          o.w = pv * fmaf(g * z.w + be.w, z.w, al.w);
          *reinterpret_cast<float4*>(&Bs[buf][srow * LDB + 4 * gg]) = o;
        }
      }
      __syncthreads();
      if (cs + kRows < nnz) fetch(cs + kRows);
      const float* Ab = As[buf];
      const float* Bb = Bs[buf];
#pragma unroll
      for (int rs = 0; rs < kRows / 4; ++rs) {
        const float* xa = Ab + (rs * 4 + l4) * LDA + l16;
        const float* sb = Bb + (rs * 4 + l4) * LDB + l16;
#pragma unroll
        for (int q = 0; q < RT; ++q) {
          const int t = wave + 4 * q;
          if (t < NRT)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[(t / NCT) * 16], sb[(t % NCT) * 16],
                                                          acc[q], 0, 0, 0);
        }
      }
      buf ^= 1;
    }
  }
  // ---- m_w (x) sum e, then the block's partial and kept count ----
#pragma unroll
  for (int u = 0; u < NK; ++u) {
    const int k = lane + 64 * u;
    if (k < KQ) dsh[wave][k] = dl[u];
  }
  if (lane == 0) wave_kept[wave] = kept_total;
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int t = wave + 4 * q;
    if (t < NRT) {
      const int k = (t % NCT) * 16 + l16;
      const float es = dsh[0][k] + dsh[1][k] + dsh[2][k] + dsh[3][k];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = (t / NCT) * 16 + 4 * l4 + r;
        if (d < D && k < K) out[d * K + k] = fmaf(mw32[d], es, acc[q][r]);
      }
    }
  }
  if (tid == 0) block_counts[blockIdx.x] = wave_kept[0] + wave_kept[1] + wave_kept[2] + wave_kept[3];
}

// ---------------------------------------------------------------------------
// BF16 variant (contexts created with TLDA_CLASSIC | TLDA_BF16): the BF16
// whitening copy W16 (with its mean projection mw16) in place of W, Z16 =
// bf16(W16 Phi) in place of Z, and the reduction rows rounded to BF16 for
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the per-document sums s,
// q and the coefficients stay FP32.  Phase 1 gathers 2 bytes per column of a
// Z16 row; phase 2 stages each chunk of 32 rows column-major in LDS (a lane's
// MFMA operand is 8 consecutive rows of one column).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// FP32 -> BF16 bits, round to nearest even (hardware conversion).
__device__ __forceinline__ uint16_t f_to_bf(float f) {
  const __bf16 h = (__bf16)f;
  return __builtin_bit_cast(uint16_t, h);
}

// Z16[w][k] = bf16(sum_d W16[w][d] Phi[d][k]) (zero for K <= k < Kh); block 0
// also writes r[k] = sum_d mw16[d] Phi[d][k] and the copy of Phi.
__global__ void __launch_bounds__(kThreads) k_classic_z16(const uint16_t* __restrict__ W16, int V,
                                                          int D, int Dh,
                                                          const float* __restrict__ Phi, int K,
                                                          int Kh, const float* __restrict__ mw16,
                                                          uint16_t* __restrict__ Z16,
                                                          float* __restrict__ r,
                                                          float* __restrict__ phi_copy) {
  extern __shared__ float ph[];
  const int tid = threadIdx.x;
  for (int e = tid; e < D * K; e += kThreads) ph[e] = Phi[e];
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < D * K; e += kThreads) phi_copy[e] = ph[e];
    for (int k = tid; k < Kh; k += kThreads) {
      float s = 0.f;
      if (k < K)
        for (int d = 0; d < D; ++d) s = fmaf(mw16[d], ph[d * K + k], s);
      r[k] = s;
    }
  }
  const size_t n = (size_t)V * Kh;
  for (size_t e = (size_t)blockIdx.x * kThreads + tid; e < n; e += (size_t)gridDim.x * kThreads) {
    const int w = (int)(e / Kh), k = (int)(e % Kh);
    float s = 0.f;
    if (k < K) {
      const uint16_t* wr = W16 + (size_t)w * Dh;
      for (int d = 0; d < D; ++d) s = fmaf(bf_to_f(wr[d]), ph[d * K + k], s);
    }
    Z16[e] = f_to_bf(s);
  }
}

template <int DQ, int KQ>
__global__ void __launch_bounds__(kThreads, 2) k_classic_cp16(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const uint16_t* __restrict__ W16, int Dh,
    const uint16_t* __restrict__ Z16, int Kh, const float* __restrict__ mw16,
    const float* __restrict__ r_g, int D, int K, float c2r, float a0r, int nblk,
    float* __restrict__ partial, int* __restrict__ block_counts) {
  constexpr int R = 32;                                     // rows per chunk (one MFMA k-step)
  constexpr int LDR = R + 8;                                // column stride of the staged tiles
  constexpr int LDB = KQ + 4;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NRT = NDT * NCT;
  constexpr int RT = (NRT + 3) / 4;
  constexpr int NK = (KQ + 63) / 64;
  constexpr int GA = DQ / 8, GB = KQ / 8;                   // 8-column groups per staged row
  constexpr int TPR = kThreads / R;                         // threads per staged row (8)
  constexpr int UA = (GA + TPR - 1) / TPR, UB = (GB + TPR - 1) / TPR;
  constexpr int NB = 8;
  __shared__ __attribute__((aligned(16))) uint16_t WsT[DQ * LDR];
  __shared__ __attribute__((aligned(16))) uint16_t BsT[KQ * LDR];
  __shared__ __attribute__((aligned(16))) float Al[kDocs * LDB];
  __shared__ __attribute__((aligned(16))) float Be[kDocs * LDB];
  __shared__ float gam[kDocs];
  __shared__ int rps[kDocs + 1];
  __shared__ float rsh[KQ];
  __shared__ float dsh[4][KQ];
  __shared__ int wave_kept[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int srow = tid / TPR, ssub = tid % TPR;
  const unsigned char* W16b = reinterpret_cast<const unsigned char*>(W16);
  const unsigned char* Z16b = reinterpret_cast<const unsigned char*>(Z16);

  for (int k = tid; k < KQ; k += kThreads) rsh[k] = k < K ? r_g[k] : 0.f;
  float dl[NK];
#pragma unroll
  for (int u = 0; u < NK; ++u) dl[u] = 0.f;
  floatx4 acc[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  int kept_total = 0;

  const int ntiles = (n_rows + kDocs - 1) / kDocs;
  for (int tile = blockIdx.x; tile < ntiles; tile += nblk) {
    const int t0 = tile * kDocs;
    const int nd = n_rows - t0 < kDocs ? n_rows - t0 : kDocs;
    __syncthreads();
    if (tid <= kDocs) rps[tid] = row_ptr[t0 + (tid < nd ? tid : nd)];
    __syncthreads();
    // ---- phase 1: s, q, L and the coefficients (a wave per document) ----
    for (int ld = wave; ld < kDocs; ld += 4) {
      float s[NK], q[NK];
#pragma unroll
      for (int u = 0; u < NK; ++u) s[u] = q[u] = 0.f;
      float L = 0.f;
      if (ld < nd) {
        const int b = rps[ld], e = rps[ld + 1];
        for (int jb = b; jb < e; jb += NB) {
          int mc = 0;
          float mv = 0.f;
          if (lane < NB && jb + lane < e) {
            mc = col_idx[jb + lane];
            mv = val[jb + lane];
          }
          float zv[NB][NK];
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const int c = __shfl(mc, t, 64);
#pragma unroll
            for (int u = 0; u < NK; ++u) {
              const int k = lane + 64 * u;
              zv[t][u] = k < Kh ? bf_to_f(Z16[(size_t)c * Kh + k]) : 0.f;
            }
          }
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const float v = __shfl(mv, t, 64);
            L += v;
#pragma unroll
            for (int u = 0; u < NK; ++u) {
              s[u] = fmaf(v, zv[t][u], s[u]);
              q[u] = fmaf(v * zv[t][u], zv[t][u], q[u]);
            }
          }
        }
      }
      const bool keep = ld < nd && L >= 3.f;
      const float l2 = keep ? 1.0f / (L * (L - 1.0f)) : 0.f;
      const float l3 = keep ? l2 / (L - 2.0f) : 0.f;
#pragma unroll
      for (int u = 0; u < NK; ++u) {
        const int k = lane + 64 * u;
        if (k < KQ) {
          const float rk = rsh[k], sk = s[u], d2 = s[u] * s[u] - q[u];
          Al[ld * LDB + k] = l3 * d2 - 2.0f * c2r * l2 * rk * sk;
          Be[ld * LDB + k] = -2.0f * l3 * sk + 2.0f * c2r * l2 * rk;
          if (keep) dl[u] += -c2r * l2 * d2 + a0r * rk * rk;
        }
      }
      if (lane == 0) gam[ld] = 2.0f * l3;
      kept_total += keep ? 1 : 0;
    }
    __syncthreads();
    // ---- phase 2: the tile's nonzero rows in chunks of R, column-major ----
    const int nb0 = rps[0];
    const int nnz = rps[nd] - nb0;
    for (int cs = 0; cs < nnz; cs += R) {
      const int gi = cs + srow;
      const bool in = gi < nnz;
      const int j = nb0 + (in ? gi : 0);
      const int col = col_idx[j];
      const float v = in ? val[j] : 0.f;    // rows past the tile's end add zero
      int lo = 0, hi = nd;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rps[mid] <= j) lo = mid;
        else hi = mid;
      }
      const float g = gam[lo];
#pragma unroll
      for (int u = 0; u < UA; ++u) {
        const int gg = ssub + TPR * u;
        if (gg < GA) {
          u32x4_t w = u32x4_t{0u, 0u, 0u, 0u};
          if (8 * gg < Dh)
            w = *reinterpret_cast<const u32x4_t*>(W16b + ((size_t)col * Dh + 8 * gg) * 2u);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t wi = w[i];
            WsT[(8 * gg + 2 * i) * LDR + srow] = (uint16_t)(wi & 0xffffu);
            WsT[(8 * gg + 2 * i + 1) * LDR + srow] = (uint16_t)(wi >> 16);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int gg = ssub + TPR * u;
        if (gg < GB) {
          u32x4_t z = u32x4_t{0u, 0u, 0u, 0u};
          if (8 * gg < Kh)
            z = *reinterpret_cast<const u32x4_t*>(Z16b + ((size_t)col * Kh + 8 * gg) * 2u);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t zi = z[i];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int kk = 8 * gg + 2 * i + h;
              const float zf = __uint_as_float(h == 0 ? (zi << 16) : (zi & 0xffff0000u));
              const float o = v * fmaf(g * zf + Be[lo * LDB + kk], zf, Al[lo * LDB + kk]);
              BsT[kk * LDR + srow] = f_to_bf(o);
            }
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        const int t = wave + 4 * q;
        if (t < NRT) {
          const u32x4_t a = *reinterpret_cast<const u32x4_t*>(WsT + ((t / NCT) * 16 + l16) * LDR + 8 * l4);
          const u32x4_t b = *reinterpret_cast<const u32x4_t*>(BsT + ((t % NCT) * 16 + l16) * LDR + 8 * l4);
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                          __builtin_bit_cast(bf16x8_t, b), acc[q],
                                                          0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int u = 0; u < NK; ++u) {
    const int k = lane + 64 * u;
    if (k < KQ) dsh[wave][k] = dl[u];
  }
  if (lane == 0) wave_kept[wave] = kept_total;
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int t = wave + 4 * q;
    if (t < NRT) {
      const int k = (t % NCT) * 16 + l16;
      const float es = dsh[0][k] + dsh[1][k] + dsh[2][k] + dsh[3][k];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = (t / NCT) * 16 + 4 * l4 + r;
        if (d < D && k < K) out[d * K + k] = fmaf(mw16[d], es, acc[q][r]);
      }
    }
  }
  if (tid == 0) block_counts[blockIdx.x] = wave_kept[0] + wave_kept[1] + wave_kept[2] + wave_kept[3];
}

template <int DQ, int KQ>
hipError_t launch_classic16_t(const tlda_csr_batch& b, const uint16_t* W16, int Dh,
                              const uint16_t* Z16, int Kh, const float* mw16, const float* r, int D,
                              int K, double alpha0, int nblk, float* partial, int* block_counts,
                              hipStream_t s) {
  if (partial == nullptr) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_classic_cp16<DQ, KQ>,
                                                                 kThreads, 0);
    *block_counts = per_cu;
    return e;
  }
  const double c2 = alpha0 * (alpha0 + 1.0) / 2.0;
  const double c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0;
  launch_main(k_classic_cp16<DQ, KQ>, dim3(nblk), dim3(kThreads), 0, s, b.row_ptr, b.col_idx,
              b.val, b.n_rows, W16, Dh, Z16, Kh, mw16, r, D, K, (float)(c2 / c3),
              (float)(alpha0 * alpha0 / c3), nblk, partial, block_counts);
  return hipGetLastError();
}

template <int DQ, int KQ>
hipError_t launch_classic_t(const tlda_csr_batch& b, const float* W32, int Dp, const float* Z,
                            int Kp, const float* mw32, const float* r, int D, int K, double alpha0,
                            int nblk, float* partial, int* block_counts, hipStream_t s) {
  if (partial == nullptr) {   // occupancy query: resident blocks per CU in *block_counts
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_classic_cp<DQ, KQ>,
                                                                 kThreads, 0);
    *block_counts = per_cu;
    return e;
  }
  const double c2 = alpha0 * (alpha0 + 1.0) / 2.0;
  const double c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0;
  launch_main(k_classic_cp<DQ, KQ>, dim3(nblk), dim3(kThreads), 0, s, b.row_ptr, b.col_idx,
              b.val, b.n_rows, W32, Dp, Z, Kp, mw32, r, D, K, (float)(c2 / c3),
              (float)(alpha0 * alpha0 / c3), nblk, partial, block_counts);
  return hipGetLastError();
}

// Padded size of a D or K dimension: 16, 32, 64 or 128 (0 above 128).
int classic_bucket(int n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  if (n <= 128) return 128;
  return 0;
}

}  // namespace

bool classic_supported(int D, int K) { return classic_bucket(D) > 0 && classic_bucket(K) > 0; }

hipError_t launch_classic_z(const float* W32, int V, int D, int Dp, const float* Phi, int K,
                            int Kp, const float* mw32, float* Z, float* r, float* phi_copy,
                            int num_cu, hipStream_t s) {
  const size_t n = (size_t)V * Kp;
  size_t grid = (n + kThreads - 1) / kThreads;
  if (grid > (size_t)num_cu * 8) grid = (size_t)num_cu * 8;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_classic_z, dim3((unsigned)grid), dim3(kThreads),
                     (unsigned)(sizeof(float) * D * K), s, W32, V, D, Dp, Phi, K, Kp, mw32, Z, r,
                     phi_copy);
  return hipGetLastError();
}

hipError_t launch_classic_z16(const uint16_t* W16, int V, int D, int Dh, const float* Phi, int K,
                              int Kh, const float* mw16, uint16_t* Z16, float* r, float* phi_copy,
                              int num_cu, hipStream_t s) {
  const size_t n = (size_t)V * Kh;
  size_t grid = (n + kThreads - 1) / kThreads;
  if (grid > (size_t)num_cu * 8) grid = (size_t)num_cu * 8;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_classic_z16, dim3((unsigned)grid), dim3(kThreads),
                     (unsigned)(sizeof(float) * D * K), s, W16, V, D, Dh, Phi, K, Kh, mw16, Z16,
                     r, phi_copy);
  return hipGetLastError();
}

hipError_t launch_classic_cp16(const tlda_csr_batch& b, const uint16_t* W16, int Dh,
                               const uint16_t* Z16, int Kh, const float* mw16, const float* r,
                               int D, int K, double alpha0, int nblk, float* partial,
                               int* block_counts, hipStream_t s) {
  const int dq = classic_bucket(D), kq = classic_bucket(K);
#define TLDA_CLASSIC16(DQ_, KQ_)                                                              \
  if (dq == DQ_ && kq == KQ_)                                                                 \
    return launch_classic16_t<DQ_, KQ_>(b, W16, Dh, Z16, Kh, mw16, r, D, K, alpha0, nblk,      \
                                        partial, block_counts, s);
#define TLDA_CLASSIC16_ROW(DQ_) \
  TLDA_CLASSIC16(DQ_, 16) TLDA_CLASSIC16(DQ_, 32) TLDA_CLASSIC16(DQ_, 64) TLDA_CLASSIC16(DQ_, 128)
  TLDA_CLASSIC16_ROW(16) TLDA_CLASSIC16_ROW(32) TLDA_CLASSIC16_ROW(64) TLDA_CLASSIC16_ROW(128)
#undef TLDA_CLASSIC16_ROW
#undef TLDA_CLASSIC16
  return hipErrorInvalidValue;
}

hipError_t launch_classic_cp(const tlda_csr_batch& b, const float* W32, int Dp, const float* Z,
                             int Kp, const float* mw32, const float* r, int D, int K,
                             double alpha0, int nblk, float* partial, int* block_counts,
                             hipStream_t s) {
  const int dq = classic_bucket(D), kq = classic_bucket(K);
#define TLDA_CLASSIC(DQ_, KQ_)                                                                \
  if (dq == DQ_ && kq == KQ_)                                                                 \
    return launch_classic_t<DQ_, KQ_>(b, W32, Dp, Z, Kp, mw32, r, D, K, alpha0, nblk, partial, \
                                      block_counts, s);
#define TLDA_CLASSIC_ROW(DQ_) \
  TLDA_CLASSIC(DQ_, 16) TLDA_CLASSIC(DQ_, 32) TLDA_CLASSIC(DQ_, 64) TLDA_CLASSIC(DQ_, 128)
  TLDA_CLASSIC_ROW(16) TLDA_CLASSIC_ROW(32) TLDA_CLASSIC_ROW(64) TLDA_CLASSIC_ROW(128)
#undef TLDA_CLASSIC_ROW
#undef TLDA_CLASSIC
  return hipErrorInvalidValue;
}

}  // namespace tlda
