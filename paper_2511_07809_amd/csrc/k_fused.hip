// Fused whitening + CP-gradient reduction: the whitened batch of the online
// second-moment section is formed tile by tile in LDS and fed straight into
// the data term of eq. vec_deriv, R1 = X^T (X Phi)^2, so X never travels
// through HBM (it is written out only when the caller asks for it).
//
// Per block (256 threads), for each of its row tiles of T documents:
//   1. whitening: a group of G lanes owns a document (one float4 of columns
//      per lane); 16 nonzeros per step are fetched in one round trip, shared
//      by lane shuffles, and all 16 W-row gathers are issued before use; the
//      row x = (1/L) sum c W[col] - W^T M1 (zero for dropped documents) goes to
//      LDS;
//   2. S = X_t Phi on FP32 matrix cores, squared into LDS;
//   3. R1 += X_t^T S^2 on FP32 matrix cores, accumulated in registers.
// Blocks resident on the same CU overlap one block's gathers with another
// block's matrix work.  Each block writes its R1 partial and its kept-row
// count (and its share of a copy of Phi); the finish kernel adds them in
// block order, forms the gradient and updates Phi.
#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kThreads = 256;
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int DQ, int KQ, int T, int G>
__global__ void __launch_bounds__(kThreads, 3) k_whiten_cp(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const float* __restrict__ W32,
    const float* __restrict__ mw32, int D, int Dp, const float* __restrict__ Phi, int K,
    int nblk, float* __restrict__ partial, int* __restrict__ block_counts,
    float* __restrict__ Xout, float* __restrict__ phi_copy) {
  constexpr int LDX = DQ + 4, LDS = KQ + 4;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = DQ / 4;
  constexpr int NRT = NDT * NCT;
  constexpr int ST = (NCT + 3) / 4;
  constexpr int RT = (NRT + 3) / 4;
  constexpr int RPW = 64 / G;              // documents per wave per whitening pass
  constexpr int RPB = 4 * RPW;             // documents per block per pass
  constexpr int NB = 8;                    // nonzeros per gather step
  constexpr int SLOTS = G >= NB ? 1 : NB / G;
  constexpr int PASSES = (T + RPB - 1) / RPB;
  __shared__ __attribute__((aligned(16))) float Xs[T * LDX];
  __shared__ __attribute__((aligned(16))) float Ss[T * LDS];
  __shared__ int wave_kept[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int gl = lane % G;
  const int c4 = gl * 4;
  const bool active = c4 < Dp;             // lane holds real (or zero-padded) W columns
  const bool in_lds = c4 < DQ;             // its columns exist in the LDS tile

  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];
  for (int e = tid; e < T * LDX; e += kThreads) Xs[e] = 0.f;
  float bf[ST][NKS];
#pragma unroll
  for (int q = 0; q < ST; ++q) {
    const int ct = wave + 4 * q;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int d = 4 * ks + l4, k = 16 * ct + l16;
      bf[q][ks] = (ct < NCT && d < D && k < K) ? Phi[d * K + k] : 0.f;
    }
  }
  floatx4 acc[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  float4 mw = make_float4(0.f, 0.f, 0.f, 0.f);
  if (active) mw = *reinterpret_cast<const float4*>(mw32 + c4);
  int kept_total = 0;

  const int ntiles = (n_rows + T - 1) / T;
  for (int tile = blockIdx.x; tile < ntiles; tile += nblk) {
    __syncthreads();
    // ---- 1. whitening of the tile into LDS ----
#pragma unroll 1
    for (int pass = 0; pass < PASSES; ++pass) {
      const int lr = pass * RPB + wave * RPW + lane / G;   // row within the tile
      const int row = tile * T + lr;
      const bool valid = lr < T && row < n_rows;
      int b = 0, e = 0;
      if (valid) {
        b = row_ptr[row];
        e = row_ptr[row + 1];
      }
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      float Lp = 0.f;
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
        float4 w[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const int c = __shfl(cidx[t / G < SLOTS ? t / G : 0], t % G, G);
          w[t] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (active && jb + t < e) w[t] = *reinterpret_cast<const float4*>(W32 + (size_t)c * Dp + c4);
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const float v = __shfl(cval[t / G < SLOTS ? t / G : 0], t % G, G);
          a.x = fmaf(v, w[t].x, a.x);
          a.y = fmaf(v, w[t].y, a.y);
          a.z = fmaf(v, w[t].z, a.z);
          a.w = fmaf(v, w[t].w, a.w);
        }
      }
      float L = Lp;
#pragma unroll
      for (int off = 1; off < G; off <<= 1) L += __shfl_xor(L, off, G);
      const int kept = (valid && L >= 3.f) ? 1 : 0;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kept && active) {
        const float invL = 1.0f / L;
        x.x = fmaf(a.x, invL, -mw.x);
        x.y = fmaf(a.y, invL, -mw.y);
        x.z = fmaf(a.z, invL, -mw.z);
        x.w = fmaf(a.w, invL, -mw.w);
      }
      if (in_lds && lr < T) *reinterpret_cast<float4*>(Xs + lr * LDX + c4) = x;
      if (Xout != nullptr && valid && active) {
        float* out = Xout + (size_t)row * D;
        if (c4 + 0 < D) out[c4 + 0] = x.x;
        if (c4 + 1 < D) out[c4 + 1] = x.y;
        if (c4 + 2 < D) out[c4 + 2] = x.z;
        if (c4 + 3 < D) out[c4 + 3] = x.w;
      }
      kept_total += __popcll(__ballot(kept && gl == 0));
    }
    __syncthreads();
    // ---- 2. S = X_t Phi, squared into LDS ----
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      const int ct = wave + 4 * q;
      if (ct < NCT) {
#pragma unroll
        for (int rt0 = 0; rt0 < T / 16; rt0 += 4) {
          floatx4 sacc[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) sacc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
          const float* xa = Xs + (rt0 * 16 + l16) * LDX + l4;
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (rt0 + u < T / 16)
                sacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u * 16 * LDX + 4 * ks],
                                                               bf[q][ks], sacc[u], 0, 0, 0);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (rt0 + u < T / 16)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                Ss[((rt0 + u) * 16 + 4 * l4 + r) * LDS + ct * 16 + l16] = sacc[u][r] * sacc[u][r];
        }
      }
    }
    __syncthreads();
    // ---- 3. R1 += X_t^T S^2 ----
#pragma unroll
    for (int rs = 0; rs < T / 4; ++rs) {
      const float* xa = Xs + (rs * 4 + l4) * LDX + l16;
      const float* sb = Ss + (rs * 4 + l4) * LDS + l16;
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        const int t = wave + 4 * q;
        if (t < NRT)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[(t / NCT) * 16], sb[(t % NCT) * 16],
                                                        acc[q], 0, 0, 0);
      }
    }
  }
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int t = wave + 4 * q;
    if (t < NRT) {
      const int k = (t % NCT) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = (t / NCT) * 16 + 4 * l4 + r;
        if (d < D && k < K) out[d * K + k] = acc[q][r];
      }
    }
  }
  if (lane == 0) wave_kept[wave] = kept_total;
  __syncthreads();
  if (tid == 0) block_counts[blockIdx.x] = wave_kept[0] + wave_kept[1] + wave_kept[2] + wave_kept[3];
}

template <int DQ, int KQ, int T, int G>
hipError_t launch_fused_t(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                          int Dp, const float* Phi, int K, int nblk, float* partial,
                          int* block_counts, float* Xout, float* phi_copy, hipStream_t s) {
  if (partial == nullptr) {   // occupancy query: resident blocks per CU in nblk's place
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_whiten_cp<DQ, KQ, T, G>,
                                                                 kThreads, 0);
    *block_counts = per_cu;
    return e;
  }
  launch_main(k_whiten_cp<DQ, KQ, T, G>, dim3(nblk), dim3(kThreads), 0, s, b.row_ptr, b.col_idx,
              b.val, b.n_rows, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout,
              phi_copy);
  return hipGetLastError();
}

template <int DQ, int KQ, int T>
hipError_t launch_fused_g(int G, const tlda_csr_batch& b, const float* W32, const float* mw32,
                          int D, int Dp, const float* Phi, int K, int nblk, float* partial,
                          int* block_counts, float* Xout, float* phi_copy, hipStream_t s) {
  switch (G) {
    case 1: return launch_fused_t<DQ, KQ, T, 1>(b, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout, phi_copy, s);
    case 2: return launch_fused_t<DQ, KQ, T, 2>(b, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout, phi_copy, s);
    case 4: return launch_fused_t<DQ, KQ, T, 4>(b, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout, phi_copy, s);
    case 8: return launch_fused_t<DQ, KQ, T, 8>(b, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout, phi_copy, s);
    default: return launch_fused_t<DQ, KQ, T, 16>(b, W32, mw32, D, Dp, Phi, K, nblk, partial, block_counts, Xout, phi_copy, s);
  }
}

}  // namespace

// Shapes the fused kernel covers: D, K <= 64 (padded to 16, 32 or 64).  Above
// that its registers spill (measured at D = K = 100: 708 us per batch against
// 540 us for the two separate kernels), so larger shapes run the two calls.
bool fused_supported(int D, int K, int Dp) {
  return mfma_bucket(D) > 0 && mfma_bucket(D) <= 64 && mfma_bucket(K) > 0 &&
         mfma_bucket(K) <= 64 && Dp <= 64;
}

int fused_tile_rows(int D, int K) {
  return cp_mfma_tile_rows(D, K);
}

hipError_t launch_whiten_cp(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                            int Dp, const float* Phi, int K, int nblk, float* partial,
                            int* block_counts, float* Xout, float* phi_copy, hipStream_t s) {
  const int dq = mfma_bucket(D), kq = mfma_bucket(K);
  const int T = fused_tile_rows(D, K);
  int G = Dp / 4;   // lanes per document: Dp is 4, 8, 16, 32 or 64 here
  if (G < 1) G = 1;
  if (G > 16) G = 16;
#define TLDA_FUSED(DQ_, KQ_)                                                                   \
  if (dq == DQ_ && kq == KQ_)                                                                  \
    return T == 64 ? launch_fused_g<DQ_, KQ_, 64>(G, b, W32, mw32, D, Dp, Phi, K, nblk, partial, \
                                                  block_counts, Xout, phi_copy, s)             \
                   : launch_fused_g<DQ_, KQ_, 32>(G, b, W32, mw32, D, Dp, Phi, K, nblk, partial, \
                                                  block_counts, Xout, phi_copy, s);
#define TLDA_FUSED_ROW(DQ_) TLDA_FUSED(DQ_, 16) TLDA_FUSED(DQ_, 32) TLDA_FUSED(DQ_, 64)
  TLDA_FUSED_ROW(16) TLDA_FUSED_ROW(32) TLDA_FUSED_ROW(64)
#undef TLDA_FUSED_ROW
#undef TLDA_FUSED
  return hipErrorInvalidValue;
}

}  // namespace tlda
