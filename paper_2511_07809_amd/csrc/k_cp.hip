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
                                                        float* __restrict__ partial,
                                                        float* __restrict__ phi_copy) {
  extern __shared__ float smem[];
  const int Dq = (D + 3) & ~3, Kq = (K + 3) & ~3;
  float* Ps = smem;                 // [Dq][Kq]
  float* Xs = Ps + Dq * Kq;         // [T][Dq]
  float* Ss = Xs + T * Dq;          // [T][Kq]
  const int tid = threadIdx.x;
  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];
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

// ---------------------------------------------------------------------------
// FP32 matrix-core variant of the reduction (D, K <= 128 after padding to
// 16).  Per row tile (T rows of X staged in LDS):
//   S = X_t Phi      with v_mfma_f32_16x16x4_f32; each wave owns S column
//                    tiles ct = wave, wave + 4, ... and keeps the Phi
//                    fragments of those columns in registers for the whole
//                    kernel (Phi is read from memory once per block);
//   S^2 -> LDS;
//   R1 += X_t^T S^2  with the same instruction, each wave owning R1 tiles
//                    t = wave, wave + 4, ... accumulated in registers over
//                    every tile of the block.
// Operand layout of the 16x16x4 instruction: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; it receives D[4*(l/16) + r][l%16], r = 0..3.
// The next row tile is prefetched into registers while the current one is
// multiplied.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));


// The padded shape (DQ x KQ, multiples of 16) and the row tile T are
// compile-time constants, so every loop is fully unrolled, accumulators stay
// in place across the matrix instructions and only the row bound is checked
// at run time.
// Waves per block of the matrix-core reduction: 16 when D is padded past 64,
// or K is and D is at least 32, so that the R1 tiles (and the Phi fragments
// and staged rows) spread over four times the waves and the kernel keeps
// several waves per SIMD instead of one or two; 4 otherwise.
constexpr int cp_waves(int DQ, int KQ) { return (DQ > 64 || (KQ > 64 && DQ >= 32)) ? 16 : 4; }

template <int DQ, int KQ, int T>
__global__ void __launch_bounds__(64 * cp_waves(DQ, KQ)) k_cp_reduce_mfma(const float* __restrict__ X,
                                                             int n_rows,
                                                             const float* __restrict__ Phi,
                                                             int D, int K, int nblk,
                                                             float* __restrict__ partial,
                                                             float* __restrict__ phi_copy) {
  constexpr int NW = cp_waves(DQ, KQ);
  constexpr int kThreads = NW * 64;
  constexpr int LDX = DQ + 4, LDS = KQ + 4;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = DQ / 4;
  constexpr int NRT = NDT * NCT;
  constexpr int ST = (NCT + NW - 1) / NW;        // S column tiles per wave (max)
  constexpr int RT = (NRT + NW - 1) / NW;        // R1 tiles per wave (max)
  // X tile staging: thread t owns column t % CP of rows t / CP + i * RPI,
  // CP = DQ rounded up to a power of two; rows past the batch and padding
  // columns load a clamped, in-bounds address and are zeroed by a select.
  constexpr int CP = DQ <= 16 ? 16 : (DQ <= 32 ? 32 : (DQ <= 64 ? 64 : 128));
  constexpr int RPI = kThreads / CP;
  constexpr int PER = T / RPI;
  static_assert(T % RPI == 0, "tile must split evenly over the block");
  __shared__ float Xs[T * LDX];
  __shared__ float Ss[T * LDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];

  // Phi fragments of this wave's S column tiles: bf[q][ks] = Phi[4 ks + l4][16 ct + l16]
  float bf[ST][NKS];
#pragma unroll
  for (int q = 0; q < ST; ++q) {
    const int ct = wave + NW * q;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int d = 4 * ks + l4, k = 16 * ct + l16;
      bf[q][ks] = (ct < NCT && d < D && k < K) ? Phi[d * K + k] : 0.f;
    }
  }
  floatx4 acc[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int sd = tid % CP, sr = tid / CP;
  const bool dval = sd < D;
  const int dcl = dval ? sd : 0;
  float pre[PER];
  const int ntiles = (n_rows + T - 1) / T;
  auto fetch = [&](int tile) {
    const int r0 = tile * T;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int r = r0 + sr + i * RPI;
      const int rc = r < n_rows ? r : n_rows - 1;
      const float v = X[(size_t)rc * D + dcl];
      pre[i] = (dval && r < n_rows) ? v : 0.f;
    }
  };
  if (blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += nblk) {
    __syncthreads();
    if (sd < DQ)
#pragma unroll
      for (int i = 0; i < PER; ++i) Xs[(sr + i * RPI) * LDX + sd] = pre[i];
    __syncthreads();
    if (tile + nblk < ntiles) fetch(tile + nblk);
    // S = X_t Phi, squared into LDS (four independent 16-row chains at a time)
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      const int ct = wave + NW * q;
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
    // R1 += X_t^T S^2: for every 4-row step, one instruction per owned tile
#pragma unroll
    for (int rs = 0; rs < T / 4; ++rs) {
      const float* xa = Xs + (rs * 4 + l4) * LDX + l16;
      const float* sb = Ss + (rs * 4 + l4) * LDS + l16;
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        const int t = wave + NW * q;
        if (t < NRT)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[(t / NCT) * 16], sb[(t % NCT) * 16],
                                                        acc[q], 0, 0, 0);
      }
    }
  }
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int t = wave + NW * q;
    if (t < NRT) {
      const int k = (t % NCT) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = (t / NCT) * 16 + 4 * l4 + r;
        if (d < D && k < K) out[d * K + k] = acc[q][r];
      }
    }
  }
}

// Gradient and update, after a reduction kernel has written its per-block R1
// partials and a copy Phi0 of the Phi it read.  Block b (1024 threads) owns
// 16 consecutive entries e = d*K + k of the D x K result:
//   1. its 64 lane groups of 16 add the partials of blocks g, g + 64, ...
//      (one lane per entry, FP64, four independent chains, so each lane
//      waits on few dependent loads); the group sums are combined in group
//      order, giving R1 with a fixed summation order;
//   2. with Phi0 in LDS, the 64 lanes of wave w form the penalty of entry w,
//      P[d][k] = sum_j Phi0[d][j] (phi0_j . phi0_k)^2 (FP64), lane l taking
//      j = l, l + 64, ...; the squared dot products come from gsq (K x K,
//      formed once per step by k_gram_sq) when it is given, else each wave
//      forms the ones it needs;
//   3. grad = 3(1+theta) P - 3 c3 / n R1 and Phi = Phi0 - beta grad.
// n is the sum of counts[0 .. ncounts) (per-block kept-row counts, or one
// caller-supplied count) or n_default when counts is NULL; n <= 0 gives a
// zero gradient and leaves Phi unchanged.  Phi is only written, Phi0 only
// read, so no block sees another block's update.
constexpr int kFinEntries = kFinishEntries;
constexpr int kFinThreads = 1024;
constexpr int kFinGroups = kFinThreads / kFinEntries;   // 64
constexpr int kFinPre = 4;        // quads of partials issued before the penalty
constexpr int kFinStage = 4;      // Phi0 entries per thread per staging round
constexpr int kFinPad = 64;       // LDS floats after the copy of Phi0 (staging pad)

template <int FE>
__device__ __forceinline__ void cp_finish_block(
    int blk, const float* __restrict__ partial, int nblk, const int* __restrict__ counts,
    int ncounts, int n_default, const float* __restrict__ Phi0, int D, int K, double alpha0,
    double theta, float beta, float* __restrict__ Phi, float* __restrict__ grad,
    double* __restrict__ R1, int* __restrict__ n_out, float* __restrict__ ph,
    const double* __restrict__ gsq) {
  // FE entries of D x K per block, FG = kFinThreads / FE groups of partials
  constexpr int FG = kFinThreads / FE;
  __shared__ double red[FG][FE + 1];
  __shared__ double pen_s[FE];
  __shared__ int nred[kFinThreads / 64];
  const int tid = threadIdx.x, el = tid % FE, grp = tid / FE;
  const int lane = tid & 63, wave = tid >> 6;
  const int DK = D * K;
  const int e = blk * FE + el;
  // Phi0 into LDS and the kept-row counts, with the loads of a round issued
  // together (clamped indexes, unconditional) so that one memory round trip
  // serves up to kFinStage * kFinThreads entries.  With the squared Gram
  // entries given, the block needs only the rows of Phi0 its entries lie in
  // (two at most where FE <= K: from D K >= 4096 on, where D <= 256 makes
  // K >= 16, and always for the 32 and 64 entries per block; more at a small
  // K, whose Gram entries the BF16 fused step also forms): ph then holds
  // Phi0[base .. base + n_ph), n_ph <= FE + 2 K - 2 <= 574 <= D K.
  int cnt = 0;
  const bool have_counts = counts != nullptr && ncounts > 0;
  int c_first = 0;
  const bool rows_only = gsq != nullptr;
  const int e_first = min(blk * FE, DK - 1);
  const int e_last = min(blk * FE + FE - 1, DK - 1);
  const int base = rows_only ? e_first / K * K : 0;
  const int n_ph = rows_only ? (e_last / K + 1) * K - base : DK;
  if (rows_only) {
    // one straight-line round: n_ph < kFinThreads; a lane past n_ph stores
    // into the pad after the copy (index n_ph + lane < D K + kFinPad)
    const float v = Phi0[base + min(tid, n_ph - 1)];
    if (have_counts) c_first = counts[min(tid, ncounts - 1)];
    ph[tid < n_ph ? tid : n_ph + lane] = v;
  } else if (DK <= kFinStage * kFinThreads) {
    // one round, straight-line; lanes past the end store into the
    // kFinPad-float pad after Phi0's copy, one slot per lane (no two lanes
    // of a wave on one LDS address)
    float v[kFinStage];
#pragma unroll
    for (int u = 0; u < kFinStage; ++u) v[u] = Phi0[min(tid + u * kFinThreads, DK - 1)];
    if (have_counts) c_first = counts[min(tid, ncounts - 1)];
#pragma unroll
    for (int u = 0; u < kFinStage; ++u) {
      const int i = tid + u * kFinThreads;
      ph[i < DK ? i : DK + lane] = v[u];
    }
  } else {
    if (have_counts) c_first = counts[min(tid, ncounts - 1)];
    for (int i = tid; i < DK; i += kFinThreads) ph[i] = Phi0[i];
  }
  if (have_counts) {
    cnt = tid < ncounts ? c_first : 0;
    for (int i = tid + kFinThreads; i < ncounts; i += kFinThreads) cnt += counts[i];
  }
  __syncthreads();
  // The first kFinPre quads of this thread's partials (four partials each,
  // FG apart) are all in flight while the penalty below works from
  // LDS (a barrier would wait for them); the first nq of them are added
  // afterwards in the same order as the loop that takes the rest.  The loads
  // are unconditional, from indexes clamped into the buffer: a load under a
  // lane condition is followed by a wait for it where the branches join.
  constexpr int kQuad = 4 * FG;
  float f[4 * kFinPre] = {};
  int nq = 0;
#pragma unroll
  for (int q = 0; q < kFinPre; ++q)
    nq += (e < DK && grp + q * kQuad + 3 * FG < nblk) ? 1 : 0;
  const int ec = e < DK ? e : DK - 1;
  if (nblk >= kFinPre * kQuad) {
    // every prefetched row exists: rows grp + FG t, one stride apart
    const float* pr = partial + (size_t)grp * DK + ec;
    const size_t stride = (size_t)FG * DK;
#pragma unroll
    for (int t = 0; t < 4 * kFinPre; ++t) f[t] = pr[t * stride];
  } else if (nblk > 3 * FG) {
    // some lanes have a full quad (exactly those counted in nq: a lane's
    // first quad is full once nblk > grp + 3 FG); the others load
    // rows they then drop.  Below that no lane has one and nq is 0.
#pragma unroll
    for (int t = 0; t < 4 * kFinPre; ++t)
      f[t] = partial[(size_t)min(grp + t * FG, nblk - 1) * DK + ec];
  }
  // wave w: penalty of entries w, w + 16, ... of the block
  constexpr int kWaves = kFinThreads / 64;
  constexpr int kEW = FE / kWaves;            // entries per wave
  if (gsq != nullptr) {
    // lane l of wave w adds Phi0[d][j] gsq[k][j] over j = l, l + 64, ...,
    // for each of the wave's entries (d, k).  gsq is symmetric bit for bit
    // (the same products in the same chains), so row k is read: consecutive
    // lanes, consecutive addresses.  The loads of the first two 64-column
    // chunks of all kEW entries are issued together (one round trip at
    // K <= 128, where a loop over entries and columns waited for each load in
    // turn), from clamped indexes.  A lane past K adds 0 x g, g a squared dot
    // product (>= 0, finite for a finite Phi0): +0, which leaves the sum
    // unchanged, so every sum takes its terms in the order j = l, l + 64, ...
    // (only the Phi0 factor is selected: a select on g would let the compiler
    // move its load under a lane condition, with a wait for it there).
    double pen[kEW];
    int drow[kEW], krow[kEW];
#pragma unroll
    for (int i = 0; i < kEW; ++i) {
      const int me = min(blk * FE + wave + kWaves * i, DK - 1);
      drow[i] = me / K;
      krow[i] = me % K;
      pen[i] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {             // K <= 256: four chunks of 64
      if (t >= 2 && 64 * t >= K) break;
      const int j = lane + 64 * t;
      const int jc = min(j, K - 1);
      double g[kEW];
      float p[kEW];
#pragma unroll
      for (int i = 0; i < kEW; ++i) {
        g[i] = gsq[(size_t)krow[i] * K + jc];
        p[i] = ph[drow[i] * K + jc - base];
      }
#pragma unroll
      for (int i = 0; i < kEW; ++i)
        pen[i] = fma(j < K ? (double)p[i] : 0.0, g[i], pen[i]);
    }
#pragma unroll
    for (int i = 0; i < kEW; ++i) {
      double v = pen[i];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0 && blk * FE + wave + kWaves * i < DK) pen_s[wave + kWaves * i] = v;
    }
  } else {
    // each wave forms the squared dot products it needs from Phi0 in LDS
    for (int wi = wave; wi < FE; wi += kWaves) {
      const int me = blk * FE + wi;
      if (me >= DK) break;
      const int d = me / K, k = me % K;
      double pen = 0.0;
      for (int j = lane; j < K; j += 64) {
        // (Phi^T Phi)[j][k] in four independent chains
        double dot0 = 0.0, dot1 = 0.0, dot2 = 0.0, dot3 = 0.0;
        int i = 0;
        for (; i + 3 < D; i += 4) {
          const float a0 = ph[i * K + j], a1 = ph[(i + 1) * K + j];
          const float a2 = ph[(i + 2) * K + j], a3 = ph[(i + 3) * K + j];
          const float b0 = ph[i * K + k], b1 = ph[(i + 1) * K + k];
          const float b2 = ph[(i + 2) * K + k], b3 = ph[(i + 3) * K + k];
          dot0 += (double)a0 * (double)b0;
          dot1 += (double)a1 * (double)b1;
          dot2 += (double)a2 * (double)b2;
          dot3 += (double)a3 * (double)b3;
        }
        for (; i < D; ++i) dot0 += (double)ph[i * K + j] * (double)ph[i * K + k];
        const double dot = (dot0 + dot1) + (dot2 + dot3);
        pen += (double)ph[d * K + j] * (dot * dot);
      }
      for (int off = 32; off > 0; off >>= 1) pen += __shfl_xor(pen, off, 64);
      if (lane == 0) pen_s[wi] = pen;
    }
  }
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll
  for (int q = 0; q < kFinPre; ++q)
    if (q < nq) {
      r0 += (double)f[4 * q];
      r1 += (double)f[4 * q + 1];
      r2 += (double)f[4 * q + 2];
      r3 += (double)f[4 * q + 3];
    }
  int b = grp + nq * kQuad;
  if (e < DK) {
    for (; b + 3 * FG < nblk; b += 4 * FG) {
      r0 += (double)partial[(size_t)b * DK + e];
      r1 += (double)partial[(size_t)(b + FG) * DK + e];
      r2 += (double)partial[(size_t)(b + 2 * FG) * DK + e];
      r3 += (double)partial[(size_t)(b + 3 * FG) * DK + e];
    }
    for (; b < nblk; b += FG) r0 += (double)partial[(size_t)b * DK + e];
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) nred[wave] = cnt;
  red[grp][el] = (r0 + r1) + (r2 + r3);
  // the groups' sums, added pairwise in a fixed tree (bit-reproducible)
  for (int h = FG / 2; h > 0; h >>= 1) {
    __syncthreads();
    if (grp < h) red[grp][el] += red[grp + h][el];
  }
  __syncthreads();
  int n = n_default;
  if (counts != nullptr) {
    n = 0;
    for (int w = 0; w < kFinThreads / 64; ++w) n += nred[w];
  }
  if (tid < FE && e < DK) {
    const double tot = red[0][el];
    R1[e] = tot;
    if (n <= 0) {
      grad[e] = 0.f;
    } else {
      const double c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0;
      const float g = (float)(3.0 * (1.0 + theta) * pen_s[el] - 3.0 * c3 / (double)n * tot);
      grad[e] = g;
      Phi[e] = fmaf(-beta, g, ph[e - base]);
    }
  }
  if (blk == 0 && tid == 0 && n_out != nullptr) *n_out = n;
}

// gsq[j][k] = (phi_j . phi_k)^2 for the K columns of Phi (D x K), in FP64:
// the squared Gram entries of the penalty, with the finish kernel's own
// summation: four chains over d (chain c takes d = 4m + c, chain 0 also the
// tail), added as (c0 + c1) + (c2 + c3).  Four lanes per entry, one per
// chain; each block stages Phi in LDS and forms 256 entries.
__global__ void __launch_bounds__(1024) k_gram_sq(const float* __restrict__ Phi, int D, int K,
                                                  double* __restrict__ gsq) {
  extern __shared__ float ph[];                 // [D][K]
  for (int i = threadIdx.x; i < D * K; i += 1024) ph[i] = Phi[i];
  __syncthreads();
  const int t = blockIdx.x * 1024 + threadIdx.x;
  const int e = t >> 2, c = t & 3;
  const bool in = e < K * K;
  const int j = in ? e / K : 0, k = in ? e % K : 0;
  double acc = 0.0;
  const int M = D / 4;
  for (int m = 0; m < M; ++m) {
    const int i = 4 * m + c;
    acc += (double)ph[i * K + j] * (double)ph[i * K + k];
  }
  if (c == 0)
    for (int i = 4 * M; i < D; ++i) acc += (double)ph[i * K + j] * (double)ph[i * K + k];
  acc += __shfl_xor(acc, 1, 64);                // (c0 + c1), (c2 + c3)
  acc += __shfl_xor(acc, 2, 64);                // (c0 + c1) + (c2 + c3)
  if (in && c == 0) gsq[e] = acc * acc;
}

// Two blocks per CU (64 registers per lane) at 16 and 32 entries per block,
// whose grids can exceed the CU count; one at 64 (D K / 64 <= 256 blocks, one
// round), which leaves room for the penalty's squared-Gram loads of four
// entries per wave in flight together.
template <int FE>
__global__ void __launch_bounds__(kFinThreads, FE == 64 ? 4 : 8) k_cp_finish(
    const float* __restrict__ partial, int nblk, const int* __restrict__ counts, int ncounts,
    int n_default, const float* __restrict__ Phi0, int D, int K, double alpha0, double theta,
    float beta, float* __restrict__ Phi, float* __restrict__ grad, double* __restrict__ R1,
    int* __restrict__ n_out, const double* __restrict__ gsq) {
  extern __shared__ float ph[];                 // [D][K] copy of Phi0
  // Workgroups go to the 8 XCDs in turn; block b takes entry chunk
  // (b % 8) per + b / 8, so each XCD reads one contiguous run of every
  // partial row and no cache line of it is fetched by two XCDs.  The grid is
  // 8 per blocks; those past the last chunk have nothing to do.
  const int per = gridDim.x / 8;
  const int chunk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (chunk * FE >= D * K) return;
  cp_finish_block<FE>(chunk, partial, nblk, counts, ncounts, n_default, Phi0, D, K, alpha0, theta,
                      beta, Phi, grad, R1, n_out, ph, gsq);
}

// The finish of every slice of a multi-slice step in one launch: block b
// serves slice fin_slice[b] as its finish block b - fin0.
__global__ void __launch_bounds__(kFinThreads, 8) k_cp_finish_multi(const SliceStep* __restrict__ sl,
                                                                 const int* __restrict__ fin_slice) {
  extern __shared__ float ph[];
  const SliceStep& d = sl[fin_slice[blockIdx.x]];
  cp_finish_block<kFinEntries>(blockIdx.x - d.fin0, d.partial, d.nblk, d.block_counts, d.nblk, 0,
                               d.phi_copy, d.D, d.K, d.alpha0, d.theta, d.beta, d.Phi, d.grad,
                               d.R1, d.n_kept_out, ph, nullptr);
}

}  // namespace

// LDS bytes of the reduction kernel for a row tile of T rows: Phi and the X
// and S tiles.
size_t cp_lds_bytes(int D, int K, int T) {
  const int Dq = (D + 3) & ~3, Kq = (K + 3) & ~3;
  return sizeof(float) * ((size_t)Dq * Kq + (size_t)T * (Dq + Kq));
}

// Row-tile height for the reduction: the largest of 64, 32, 16, 8, 4 whose
// LDS footprint stays within 64 KiB.
int cp_tile_rows(int D, int K) {
  for (int T = 64; T >= 4; T >>= 1)
    if (cp_lds_bytes(D, K, T) <= 65536) return T;
  return 0;
}

// Padded size of a dimension for the matrix-core reduction: the smallest of
// 16, 32, 64, 112, 128 that holds it (0: too large).
int mfma_bucket(int n) {
  const int q = (n + 15) & ~15;
  if (q <= 16) return 16;
  if (q <= 32) return 32;
  if (q <= 64) return 64;
  if (q <= 112) return 112;
  if (q <= 128) return 128;
  return 0;
}

// Row tile of the matrix-core reduction for padded shape (dq, kq): 64 rows
// unless the X and S tiles would pass 48 KiB of LDS, then 32 (0: shape not
// supported by it).
int cp_mfma_tile_rows(int D, int K) {
  const int dq = mfma_bucket(D), kq = mfma_bucket(K);
  if (dq == 0 || kq == 0) return 0;
  return (size_t)64 * (dq + kq + 8) * sizeof(float) <= 49152 ? 64 : 32;
}

int cp_resident_blocks(int D, int K, int num_cu) {
  const int Tm = cp_mfma_tile_rows(D, K);
  int per_cu = 0;
  hipError_t e = hipSuccess;
  if (Tm > 0) {
    const int dq = mfma_bucket(D), kq = mfma_bucket(K);
#define TLDA_OCC(DQ_, KQ_)                                                                      \
  if (dq == DQ_ && kq == KQ_)                                                                   \
    e = Tm == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                \
                       &per_cu, k_cp_reduce_mfma<DQ_, KQ_, 64>, 64 * cp_waves(DQ_, KQ_), 0)         \
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                \
                       &per_cu, k_cp_reduce_mfma<DQ_, KQ_, 32>, 64 * cp_waves(DQ_, KQ_), 0);
#define TLDA_OCC_ROW(DQ_) \
  TLDA_OCC(DQ_, 16) TLDA_OCC(DQ_, 32) TLDA_OCC(DQ_, 64) TLDA_OCC(DQ_, 112) TLDA_OCC(DQ_, 128)
    TLDA_OCC_ROW(16) TLDA_OCC_ROW(32) TLDA_OCC_ROW(64) TLDA_OCC_ROW(112) TLDA_OCC_ROW(128)
#undef TLDA_OCC_ROW
#undef TLDA_OCC
  } else {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cp_reduce, kThreads,
                                                      cp_lds_bytes(D, K, cp_tile_rows(D, K)));
  }
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu * num_cu;
}

int cp_num_blocks(int n_rows, int D, int K, int max_blocks) {
  if (max_blocks <= 0) max_blocks = 1024;
  const int Tm = cp_mfma_tile_rows(D, K);
  const int T = Tm > 0 ? Tm : cp_tile_rows(D, K);
  const int ntiles = (n_rows + T - 1) / T;
  return ntiles < max_blocks ? (ntiles < 1 ? 1 : ntiles) : max_blocks;
}

hipError_t launch_cp_reduce(const float* X, int n_rows, const float* Phi, int D, int K, int nblk,
                            float* partial, float* phi_copy, hipStream_t s) {
  const int Tm = cp_mfma_tile_rows(D, K);
  if (Tm > 0) {
    const int dq = mfma_bucket(D), kq = mfma_bucket(K);
#define TLDA_MFMA(DQ_, KQ_)                                                                   \
  if (dq == DQ_ && kq == KQ_) {                                                               \
    if (Tm == 64)                                                                             \
      launch_main(k_cp_reduce_mfma<DQ_, KQ_, 64>, dim3(nblk), dim3(64 * cp_waves(DQ_, KQ_)), 0, s, X, \
                  n_rows, Phi, D, K, nblk, partial, phi_copy);                                \
    else                                                                                      \
      launch_main(k_cp_reduce_mfma<DQ_, KQ_, 32>, dim3(nblk), dim3(64 * cp_waves(DQ_, KQ_)), 0, s, X, \
                  n_rows, Phi, D, K, nblk, partial, phi_copy);                                \
  }
#define TLDA_MFMA_ROW(DQ_) \
  TLDA_MFMA(DQ_, 16) TLDA_MFMA(DQ_, 32) TLDA_MFMA(DQ_, 64) TLDA_MFMA(DQ_, 112) TLDA_MFMA(DQ_, 128)
    TLDA_MFMA_ROW(16) TLDA_MFMA_ROW(32) TLDA_MFMA_ROW(64) TLDA_MFMA_ROW(112) TLDA_MFMA_ROW(128)
#undef TLDA_MFMA_ROW
#undef TLDA_MFMA
  } else {
    const int T = cp_tile_rows(D, K);
    launch_main(k_cp_reduce, dim3(nblk), dim3(kThreads), (unsigned)cp_lds_bytes(D, K, T), s, X,
                n_rows, Phi, D, K, T, nblk, partial, phi_copy);
  }
  return hipGetLastError();
}

hipError_t launch_cp_finish_multi(const SliceStep* sl, const int* fin_slice, int n_fin,
                                  int max_dk, hipStream_t s) {
  hipLaunchKernelGGL(k_cp_finish_multi, dim3(n_fin), dim3(kFinThreads),
                     sizeof(float) * (max_dk + kFinPad), s,
                     sl, fin_slice);
  return hipGetLastError();
}

hipError_t launch_gram_sq(const float* Phi, int D, int K, double* gsq, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_sq, dim3((4 * K * K + 1023) / 1024), dim3(1024),
                     sizeof(float) * D * K, s, Phi, D, K, gsq);
  return hipGetLastError();
}

hipError_t launch_cp_finish(const float* partial, int nblk, const int* counts, int ncounts,
                            int n_default, const float* Phi0, int D, int K, double alpha0,
                            double theta, float beta, float* Phi, float* grad, double* R1,
                            int* n_out, const double* gsq, hipStream_t s) {
  const int DK = D * K;
  // 16 entries per block, or 32 from D K = 8192 on (64 when also K >= 64):
  // 64 (32, 16) groups of 16 lanes (32, 64) need DK waves (DK / 2, DK / 4),
  // and the wider blocks keep a large D x K within one round of resident
  // blocks (at D = K = 100 with 256 partials, 64 entries per block take
  // about 1 us less per step than 32).
  const bool wide = DK >= 8192;
  const bool wider = wide && K >= 64;
  const int fe = wider ? 64 : wide ? 32 : kFinEntries;
  const int chunks = (DK + fe - 1) / fe;
  const dim3 grid(8 * ((chunks + 7) / 8));
  if (wider)
    hipLaunchKernelGGL(k_cp_finish<64>, grid, dim3(kFinThreads), sizeof(float) * (DK + kFinPad), s,
                       partial, nblk, counts, ncounts, n_default, Phi0, D, K, alpha0, theta, beta,
                       Phi, grad, R1, n_out, gsq);
  else if (wide)
    hipLaunchKernelGGL(k_cp_finish<32>, grid, dim3(kFinThreads), sizeof(float) * (DK + kFinPad), s,
                       partial, nblk, counts, ncounts, n_default, Phi0, D, K, alpha0, theta, beta,
                       Phi, grad, R1, n_out, gsq);
  else
    hipLaunchKernelGGL(k_cp_finish<kFinEntries>, grid, dim3(kFinThreads),
                       sizeof(float) * (DK + kFinPad), s, partial, nblk, counts, ncounts,
                       n_default, Phi0, D, K, alpha0, theta, beta, Phi, grad, R1, n_out, gsq);
  return hipGetLastError();
}

}  // namespace tlda
