// Fused whitening + CP-gradient reduction: the whitened batch of the online
// second-moment section is formed tile by tile in LDS and fed straight into
// the data term of eq. vec_deriv, R1 = X^T (X Phi)^2, so X never travels
// through HBM (it is written out only when the caller asks for it).
//
// Per block (NW waves), for each of its row tiles of T documents:
//   1. whitening: a group of G lanes owns a document (one float4 of columns
//      per lane); 8 nonzeros per step are fetched in one round trip, shared
//      by lane shuffles, and all 8 W-row gathers are issued before use; the
//      row x = (1/L) sum c W[col] - W^T M1 (zero for dropped documents) goes to
//      LDS;
//   2. S = X_t Phi on FP32 matrix cores, squared into LDS;
//   3. R1 += X_t^T S^2 on FP32 matrix cores, accumulated in registers.
// Blocks resident on the same CU overlap one block's gathers with another
// block's matrix work.  Each block writes its R1 partial and its kept-row
// count (and its share of a copy of Phi); the finish kernel adds them in
// block order, forms the gradient and updates Phi.
//
// Three families of instances: D and K both padded to 64, 112 or 128 take
// the hybrid kernel, one 16-wave block per CU whose waves split into
// whitening and matrix roles; the other shapes with D or K padded to 112 or
// 128 (the other dimension 16 or 32) take 8-wave blocks, 32 lanes per
// document (one float4 of the up to 128 columns each) and 32-row tiles, so
// that two blocks fit on a CU (LDS and 128 registers per lane) and one
// block's gathers overlap the other's matrix work; the rest (D, K <= 64)
// take 4-wave blocks, G = Dp / 4 <= 16 lanes per document and 64- or 32-row
// tiles.
#include "tlda_internal.h"

namespace tlda {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Waves per block of the fused kernel and its resident waves per SIMD.
constexpr int fused_waves(int DQ, int KQ) { return (DQ > 64 || KQ > 64) ? 8 : 4; }
constexpr int fused_min_waves(int DQ, int KQ) { return (DQ > 64 || KQ > 64) ? 4 : 3; }

template <int DQ, int KQ, int T, int G>
__global__ void __launch_bounds__(64 * fused_waves(DQ, KQ), fused_min_waves(DQ, KQ)) k_whiten_cp(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const float* __restrict__ W32,
    const float* __restrict__ mw32, int D, int Dp, const float* __restrict__ Phi, int K,
    int nblk, float* __restrict__ partial, int* __restrict__ block_counts,
    float* __restrict__ Xout, float* __restrict__ phi_copy) {
  constexpr int NW = fused_waves(DQ, KQ);
  constexpr int kThreads = 64 * NW;
  constexpr int LDX = DQ + 4, LDS = KQ + 4;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = DQ / 4;
  constexpr int NRT = NDT * NCT;
  constexpr int ST = (NCT + NW - 1) / NW;  // S column tiles per wave (max)
  // R1 tiles of a wave: wide instances with at least NW / 2 column tiles give
  // wave w column tile w, every row tile (LDS offsets known at compile time;
  // a runtime tile index t / NCT, t % NCT kept an address register per tile
  // live through the gathers and spilled); otherwise tiles w, w + NW, ...
  constexpr bool kColOwner = NW > 4 && 2 * NCT > NW;
  constexpr int RT = kColOwner ? NDT : (NRT + NW - 1) / NW;
  constexpr int RPW = 64 / G;              // documents per wave per whitening pass
  constexpr int RPB = NW * RPW;            // documents per block per pass
  constexpr int NB = NW > 4 ? 4 : 8;       // nonzeros per gather step (wide instances: 4,
                                           // so that their 128 registers hold the rest)
  constexpr int SLOTS = G >= NB ? 1 : NB / G;
  constexpr int PASSES = (T + RPB - 1) / RPB;
  __shared__ __attribute__((aligned(16))) float Xs[T * LDX];
  __shared__ __attribute__((aligned(16))) float Ss[T * LDS];
  __shared__ int wave_kept[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int gl = lane % G;
  const int c4 = gl * 4;
  const bool active = c4 < D;              // lane's float4 holds real W columns (the rest
                                           // of a row past D is zero padding)
  const bool in_lds = c4 < DQ;             // its columns exist in the LDS tile

  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];
  for (int e = tid; e < T * LDX; e += kThreads) Xs[e] = 0.f;
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
          // 32-bit element offset from the kernel's (uniform) base: V Dp < 2^31
          const uint32_t off = (uint32_t)c * (uint32_t)Dp + (uint32_t)c4;
          w[t] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (active && jb + t < e) w[t] = *reinterpret_cast<const float4*>(W32 + off);
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
      const int ct = wave + NW * q;
      if (ct < NCT) {
#pragma unroll
        for (int rt0 = 0; rt0 < T / 16; rt0 += 4) {
          floatx4 sacc[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) sacc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
          const float* xa = Xs + (rt0 * 16 + l16) * LDX + l4;
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (rt0 + u < T / 16)
                sacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u * 16 * LDX + 4 * ks],
                                                               bf[q][ks], sacc[u], 0, 0, 0);
            // wide instances: keep the operand loads of a few k steps in
            // flight, not all of them (their registers would spill)
            if constexpr (NW > 4)
              if (ks % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
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
        if constexpr (kColOwner) {
          if (wave < NCT)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[q * 16], sb[wave * 16], acc[q], 0,
                                                          0, 0);
        } else {
          const int t = wave + NW * q;
          if (t < NRT)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[(t / NCT) * 16], sb[(t % NCT) * 16],
                                                          acc[q], 0, 0, 0);
        }
      }
      if constexpr (NW > 4)
        if (rs % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
  float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int t = kColOwner ? q * NCT + wave : wave + NW * q;
    if ((kColOwner && wave < NCT) || (!kColOwner && t < NRT)) {
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
  if (tid == 0) {
    int n = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) n += wave_kept[w];
    block_counts[blockIdx.x] = n;
  }
}

// ---------------------------------------------------------------------------
// Wide shapes (D or K padded to 112 or 128): 8-wave blocks, 32-row tiles,
// 32 lanes per document (one float4 of the up to 128 columns each), two
// documents per wave and pass, two passes per tile.  The whitening phase is
// latency-bound on chains of dependent memory round trips, so it is
// pipelined across documents: a wave's row pointers are loaded two
// documents ahead and its CSR entries (up to 32, one per lane, in one round
// trip) one document ahead, so a document's own chain is only its W-row
// gather steps (8 nonzeros per step; a document of up to 16 distinct words
// takes two).  The loads for the next tile's first document are in flight
// while the tile's matrix work runs.  Phi lives in LDS (the B operand of
// S = X_t Phi), which leaves the registers to the gathers; each wave owns
// one column tile of S and of R1 (every row tile), so all LDS offsets are
// known at compile time.  Two blocks fit on a CU at 112 x 112 (LDS and 128
// registers per lane), one block's gathers overlapping the other's matrix
// work.
// ---------------------------------------------------------------------------
// LDS of a wide block (Phi, X and S tiles, counts) and its waves per SIMD:
// two blocks per CU while they fit in the 160 KB, else one.
constexpr int wide_lds_bytes(int DQ, int KQ) {
  return (DQ * KQ + 32 * (DQ + 4) + 32 * (KQ + 4)) * 4 + 32;
}
constexpr int wide_min_waves(int DQ, int KQ) { return 2 * wide_lds_bytes(DQ, KQ) <= 163840 ? 4 : 2; }

// NK2: k-steps of S = X_t Phi, DQ / 4 unless the real D ends earlier (the
// columns of X past D are zero): 25 for D <= 100 in the 112 bucket.
template <int DQ, int KQ, int NK2 = DQ / 4>
__global__ void __launch_bounds__(512, wide_min_waves(DQ, KQ)) k_whiten_cp_wide(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const float* __restrict__ W32,
    const float* __restrict__ mw32, int D, int Dp, int Dt, uint32_t tail_base,
    const float* __restrict__ Phi, int K, int nblk, float* __restrict__ partial,
    int* __restrict__ block_counts, float* __restrict__ Xout, float* __restrict__ phi_copy,
    double* __restrict__ gsq) {
  constexpr int NW = 8, kThreads = 512;
  constexpr int T = 32, G = 32, RPW = 2, RPB = NW * RPW, PASSES = T / RPB;
  constexpr int NB = 8;                    // nonzeros per gather step
  constexpr int LDX = DQ + 4, LDS = KQ + 4, LDP = KQ;   // Phi unpadded: 78 KB per block at 112
                                                         // x 112, so two blocks fit on a CU
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = NK2;
  static_assert(NCT <= NW && T % RPB == 0 && NK2 <= DQ / 4, "wide fused shape");
  __shared__ __attribute__((aligned(16))) float Ps[DQ * LDP];
  __shared__ __attribute__((aligned(16))) float Xs[T * LDX];
  __shared__ __attribute__((aligned(16))) float Ss[T * LDS];
  __shared__ int wave_kept[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int gl = lane & (G - 1), half = lane >> 5;
  const int c4 = gl * 4;
  const bool active = c4 < D;              // lane's float4 holds real W columns
  const bool in_lds = c4 < DQ;             // its columns exist in the LDS tile
  const bool owner = wave < NCT;           // wave owns column tile `wave` of S and R1
  // A row's gather reads its whole 128-byte lines from the row itself and
  // the rest (Dt columns) from the compact tail copy, so that a row of
  // D = 100 costs three lines and a sixteenth of a shared one instead of
  // four; lanes past D read the row's first float4 (a line already read).
  const int Dm = Dt > 0 ? D / 32 * 32 : Dp;
  const bool tail_lane = active && c4 >= Dm;
  const uint32_t gmul = tail_lane ? (uint32_t)Dt : (uint32_t)Dp;
  const uint32_t gadd = !active ? 0u : tail_lane ? tail_base + (uint32_t)(c4 - Dm) : (uint32_t)c4;

  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];
  // Phi into LDS, zero padded (first read after the first tile's barrier).
  // Xs needs no clearing: every pass writes all DQ columns of its rows.
  for (int e = tid; e < DQ * LDP; e += kThreads) {
    const int d = e / LDP, k = e % LDP;
    Ps[e] = (d < D && k < K) ? Phi[d * K + k] : 0.f;
  }
  floatx4 acc[NDT];
#pragma unroll
  for (int q = 0; q < NDT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  int kept_total = 0;

  // The documents this lane group whitens, in order: pass g of the block is
  // pass g % PASSES of tile blockIdx.x + (g / PASSES) nblk.
  const int ntiles = (n_rows + T - 1) / T;
  const int my_tiles = blockIdx.x < ntiles ? (ntiles - 1 - blockIdx.x) / nblk + 1 : 0;
  const int n_pass = my_tiles * PASSES;
  auto doc_row = [&](int g) -> int {     // -1: no document
    if (g >= n_pass) return -1;
    const int tile = blockIdx.x + (g / PASSES) * nblk;
    const int row = tile * T + (g % PASSES) * RPB + wave * RPW + half;
    return row < n_rows ? row : -1;
  };
  // row pointers of documents g + 1 and g + 2, CSR entries of document g + 1
  auto load_rp = [&](int g, int& b, int& e) {
    const int r = doc_row(g);
    const int rc = r < 0 ? 0 : r;
    const int b_ = row_ptr[rc], e_ = row_ptr[rc + 1];
    b = r < 0 ? 0 : b_;
    e = r < 0 ? 0 : e_;
  };
  // Unconditional loads from clamped indexes (the launcher passes valid
  // arrays even for a batch without nonzeros): a load under a lane condition
  // sits in a branch whose join waits for every load in flight.
  auto load_csr = [&](int b, int e, int& c, float& v) {
    const int j = b + gl;
    const bool in = j < e;
    const int jc = in ? j : 0;
    const int c_ = col_idx[jc];
    const float v_ = val[jc];
    c = in ? c_ : 0;
    v = in ? v_ : 0.f;
  };
  int b0 = 0, e0 = 0, b1 = 0, e1 = 0;
  load_rp(0, b0, e0);
  load_rp(1, b1, e1);
  int cc = 0;
  float cv = 0.f;
  if (n_pass > 0) load_csr(b0, e0, cc, cv);

#pragma unroll 1
  for (int g = 0; g < n_pass; ++g) {
    const int pass = g % PASSES;
    const int lr = pass * RPB + wave * RPW + half;   // row within the tile
    const int row = doc_row(g);
    const int b = b0, e = e0;
    int c_cur = cc;
    float v_cur = cv;
    // start the next documents' loads: CSR of g + 1, row pointers of g + 2
    load_csr(b1, e1, cc, cv);
    b0 = b1;
    e0 = e1;
    load_rp(g + 2, b1, e1);
    // ---- 1. whitening of this pass's documents into LDS ----
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    float Lp = 0.f;
    for (int base = b; base < e; base += G) {
      if (base != b) load_csr(base, e, c_cur, v_cur);   // documents with more than G words
      Lp += v_cur;
      const int n_here = min(G, e - base);
      for (int t0 = 0; t0 < n_here; t0 += NB) {
        // Branch-free gathers, all NB in flight together: steps past the
        // document's end read a valid row (their count is zeroed below) and
        // lanes past D read column 0 of it (their sums are never used).
        float4 w[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const int c = __shfl(c_cur, (t0 + t) & (G - 1), G);
          // 32-bit element offset from the kernel's (uniform) base:
          // V (Dp + Dt) < 2^31
          const uint32_t off = (uint32_t)c * gmul + gadd;
          w[t] = *reinterpret_cast<const float4*>(W32 + off);
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const float vs = __shfl(v_cur, (t0 + t) & (G - 1), G);
          const float v = t0 + t < n_here ? vs : 0.f;
          a.x = fmaf(v, w[t].x, a.x);
          a.y = fmaf(v, w[t].y, a.y);
          a.z = fmaf(v, w[t].z, a.z);
          a.w = fmaf(v, w[t].w, a.w);
        }
      }
    }
    float L = Lp;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) L += __shfl_xor(L, off, G);
    const int kept = (row >= 0 && L >= 3.f) ? 1 : 0;
    float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kept && active) {
      const float4 mw = *reinterpret_cast<const float4*>(mw32 + c4);
      const float invL = 1.0f / L;
      x.x = fmaf(a.x, invL, -mw.x);
      x.y = fmaf(a.y, invL, -mw.y);
      x.z = fmaf(a.z, invL, -mw.z);
      x.w = fmaf(a.w, invL, -mw.w);
    }
    if (in_lds) *reinterpret_cast<float4*>(Xs + lr * LDX + c4) = x;
    if (Xout != nullptr && row >= 0 && active) {
      float* out = Xout + (size_t)row * D;
      if (c4 + 0 < D) out[c4 + 0] = x.x;
      if (c4 + 1 < D) out[c4 + 1] = x.y;
      if (c4 + 2 < D) out[c4 + 2] = x.z;
      if (c4 + 3 < D) out[c4 + 3] = x.w;
    }
    kept_total += __popcll(__ballot(kept && gl == 0));
    if (pass != PASSES - 1) continue;
    __syncthreads();
    // ---- 2. S = X_t Phi (column tile `wave`), squared into LDS ----
    if (owner) {
      floatx4 sacc[T / 16];
#pragma unroll
      for (int u = 0; u < T / 16; ++u) sacc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
      const float* xa = Xs + l16 * LDX + l4;
      const float* pb = Ps + l4 * LDP + wave * 16 + l16;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const float bv = pb[4 * ks * LDP];
#pragma unroll
        for (int u = 0; u < T / 16; ++u)
          sacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u * 16 * LDX + 4 * ks], bv, sacc[u],
                                                         0, 0, 0);
        if (ks % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int u = 0; u < T / 16; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Ss[(u * 16 + 4 * l4 + r) * LDS + wave * 16 + l16] = sacc[u][r] * sacc[u][r];
    }
    __syncthreads();
    // ---- 3. R1 += X_t^T S^2 (column tile `wave`, every row tile) ----
    if (owner) {
#pragma unroll
      for (int rs = 0; rs < T / 4; ++rs) {
        const float* xa = Xs + (rs * 4 + l4) * LDX + l16;
        const float sv = Ss[(rs * 4 + l4) * LDS + wave * 16 + l16];
#pragma unroll
        for (int q = 0; q < NDT; ++q)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[q * 16], sv, acc[q], 0, 0, 0);
        if (rs % 2 == 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
  }
  // The squared Gram entries (phi_j . phi_k)^2 of the finish, FP64, from the
  // copy of Phi in LDS: the blocks share the K x K entries, four lanes per
  // entry, each summing one chain of d (d = 4m + c, chain 0 also the tail),
  // combined as (c0 + c1) + (c2 + c3) -- the summation of k_gram_sq, which
  // the step then does not launch.  An entry's four lanes are adjacent and
  // 4 K^2 is a multiple of four, so they enter and leave the loop together.
  // (The barrier makes Ps visible also in a block that had no tile.)
  __syncthreads();
  if (gsq != nullptr) {
    for (int e4 = blockIdx.x * kThreads + tid; e4 < 4 * K * K; e4 += nblk * kThreads) {
      const int e = e4 >> 2, c = e4 & 3;
      const int j = e / K, k = e % K;
      double accg = 0.0;
      const int M = D / 4;
      for (int m = 0; m < M; ++m) {
        const int i = 4 * m + c;
        accg += (double)Ps[i * LDP + j] * (double)Ps[i * LDP + k];
      }
      if (c == 0)
        for (int i = 4 * M; i < D; ++i) accg += (double)Ps[i * LDP + j] * (double)Ps[i * LDP + k];
      accg += __shfl_xor(accg, 1, 64);
      accg += __shfl_xor(accg, 2, 64);
      if (c == 0) gsq[e] = accg * accg;
    }
  }
  float* out = partial + (size_t)blockIdx.x * D * K;
  if (owner) {
    const int k = wave * 16 + l16;
#pragma unroll
    for (int q = 0; q < NDT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = q * 16 + 4 * l4 + r;
        if (d < D && k < K) out[d * K + k] = acc[q][r];
      }
  }
  if (lane == 0) wave_kept[wave] = kept_total;
  __syncthreads();
  if (tid == 0) {
    int n = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) n += wave_kept[w];
    block_counts[blockIdx.x] = n;
  }
}

// Sum over each aligned group of G lanes (16 or 32), the result in all of
// them: DPP inside the 16-lane row (pairs, quads, mirrored halves of 8 and of
// 16), then for G = 32 the two rows of the group through a swizzle.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF,
                                                            0xF, false));
}
template <int G>
__device__ __forceinline__ float doc_sum(float s) {
  static_assert(G == 16 || G == 32, "documents of 16 or 32 lanes");
  s += dpp_mov<0xB1>(s);    // quad_perm [1, 0, 3, 2]
  s += dpp_mov<0x4E>(s);    // quad_perm [2, 3, 0, 1]
  s += dpp_mov<0x141>(s);   // row_half_mirror
  s += dpp_mov<0x140>(s);   // row_mirror
  if constexpr (G == 32)    // lane ^ 16 (swizzle bit mode: and 0x1f, or 0, xor 0x10)
    s += __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, s), 0x401F));
  return s;
}

// ---------------------------------------------------------------------------
// Every shape with D and K both padded to 64, 112 or 128 (the tweet-shaped
// K = D = 50 at 64 x 64, the streaming-scale K = D = 100 at 112 x 112): one
// 16-wave block per CU with the waves split by role.  G = 16 lanes per
// document when D pads to 64, else 32.  Waves 0-11 (three per SIMD) whiten
// 48-row tiles, 64 / G documents per wave at a time, into one of two X
// buffers; waves 12-15 (one per SIMD) run S = X_t Phi and R1 += X_t^T S^2
// on the other buffer, each owning column tiles c and c + 4 of S and of R1
// (one tile each when K pads to 64, two each at 128).  One barrier per tile
// hands a buffer over.  Each block takes a contiguous run of the batch's
// passes (RPB documents each), not of whole tiles.  In the 8-wave kernel a CU alternates between gathers
// and matrix work and the two phases add up; here the matrix waves' work
// runs beside the next tile's gathers.  What is left of the matrix phases' cost
// is their issue slots on the whitening waves' SIMDs, so the whitening is
// written for few instructions per nonzero:
//  * the W-row gathers are buffer loads from a 32-bit byte offset, one
//    24-bit multiply-add per nonzero (no 64-bit address arithmetic);
//  * a document's CSR entries (32 at a time, 32 / G per lane, loaded one
//    document ahead: a second chunk, a dependent round trip, is needed only
//    past 32 nonzeros) go to the wave's own LDS rows once, and every lane
//    reads eight of them per step with four 16-byte LDS reads at fixed
//    offsets (instead of two lane shuffles per nonzero);
//  * the word count L is summed across the document's lanes with DPP and one
//    swizzle as soon as its entries arrive, before its gathers.
// Entries past a document's end are (column 0, count 0): they gather row 0
// and add nothing.  S^2 never goes through LDS: the R1 product takes its
// rows in the order the S accumulators hold them.  The per-row arithmetic
// (the nonzeros of a row in CSR order, one FMA each) is the 8-wave kernel's;
// L, a sum of the row's counts, is added in another order, which changes
// nothing for integer counts.  Registers: 84 to 111 per lane, no spills
// (101 at 112 x 112, 88 at 64 x 64, 108 to 111 at 128 x 128); LDS 54 KB at 64 x 64,
// 99 KB at 112 x 112, 121 KB at 128 x 128.  The buffer descriptor needs the
// W32 copy below 4 GiB and V below 2^24 (a 24-bit multiply); the launchers
// check both.
// ---------------------------------------------------------------------------
template <int DQ, int KQ, int NK2, int G>
__global__ void __launch_bounds__(1024, 1) k_whiten_cp_hyb(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const float* __restrict__ W32,
    const float* __restrict__ mw32, int D, int Dp, int Dt, uint32_t tail_base,
    const float* __restrict__ Phi, int K, int nblk, float* __restrict__ partial,
    int* __restrict__ block_counts, float* __restrict__ Xout, float* __restrict__ phi_copy,
    double* __restrict__ gsq) {
  constexpr int NP = 12, NC = 4, kThreads = 1024;   // whitening and matrix waves
  constexpr int T = 48, RPW = 64 / G, RPB = NP * RPW, PASSES = T / RPB;
  constexpr int NB = 8;                              // nonzeros per gather step
  constexpr int EPL = 32 / G, CH = G * EPL;          // CSR entries per lane, per chunk
  constexpr int LDX = DQ + 4, LDP = KQ;
  constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = NK2;
  constexpr int CT = (NCT + NC - 1) / NC;        // column tiles per consumer
  static_assert(T % RPB == 0 && T % 16 == 0 && NKS <= DQ / 4, "hybrid fused shape");
  __shared__ __attribute__((aligned(16))) float Ps[DQ * LDP];
  __shared__ __attribute__((aligned(16))) float Xs[2][T * LDX];
  __shared__ int wave_kept[NP];
  __shared__ __attribute__((aligned(16))) int2 ent[NP][64 / G][CH];   // (column, count) per entry
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;

  for (int e = blockIdx.x * kThreads + tid; e < D * K; e += nblk * kThreads) phi_copy[e] = Phi[e];
  for (int e = tid; e < DQ * LDP; e += kThreads) {
    const int d = e / LDP, k = e % LDP;
    Ps[e] = (d < D && k < K) ? Phi[d * K + k] : 0.f;
  }
  // Work split: the batch in passes of RPB documents, each block a contiguous
  // run of them.  At 262 144 documents on 256 blocks (112 x 112) that is 42
  // or 43 passes per block, where whole 48-row tiles (two passes) dealt out
  // one per block in turn gave 21 or 22.  With an odd count the block's last
  // tile holds one pass of documents and one of empty rows.
  const int n_pass_all = (n_rows + RPB - 1) / RPB;
  const int pass0 = (int)((int64_t)blockIdx.x * n_pass_all / nblk);
  const int my_pass = (int)((int64_t)(blockIdx.x + 1) * n_pass_all / nblk) - pass0;
  const int my_tiles = (my_pass + PASSES - 1) / PASSES;
  __syncthreads();

  if (wave < NP) {
    const int gl = lane & (G - 1), grp = lane / G;   // lane in its document, document in the wave
    const int c4 = gl * 4;
    const bool active = c4 < D;
    const bool in_lds = c4 < DQ;
    const int Dm = Dt > 0 ? D / 32 * 32 : Dp;
    const bool tail_lane = active && c4 >= Dm;
    const uint32_t gmul = tail_lane ? (uint32_t)Dt : (uint32_t)Dp;
    const uint32_t gadd = !active ? 0u : tail_lane ? tail_base + (uint32_t)(c4 - Dm) : (uint32_t)c4;
    const uint32_t gmul4 = gmul * 4u, gadd4 = gadd * 4u;
    const uint32_t w_bytes = (tail_base + tail_base / (uint32_t)Dp * (uint32_t)Dt) * 4u;
    const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(W32), (short)0, (int)w_bytes, 0x00020000);
    auto doc_row = [&](int g) -> int {
      if (g >= my_pass) return -1;
      const int row = (pass0 + g) * RPB + wave * RPW + grp;
      return row < n_rows ? row : -1;
    };
    auto load_rp = [&](int g, int& b, int& e) {
      const int r = doc_row(g);
      const int rc = r < 0 ? 0 : r;
      const int b_ = row_ptr[rc], e_ = row_ptr[rc + 1];
      b = r < 0 ? 0 : b_;
      e = r < 0 ? 0 : e_;
    };
    auto load_csr = [&](int b, int e, int (&c)[EPL], float (&v)[EPL]) {
#pragma unroll
      for (int q = 0; q < EPL; ++q) {
        const int j = b + gl + q * G;
        const bool in = j < e;
        const int jc = in ? j : 0;
        const int c_ = col_idx[jc];
        const float v_ = val[jc];
        c[q] = in ? c_ : 0;
        v[q] = in ? v_ : 0.f;
      }
    };
    auto lane_sum = [](const float (&v)[EPL]) {
      float x = v[0];
#pragma unroll
      for (int q = 1; q < EPL; ++q) x += v[q];
      return x;
    };
    int b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    load_rp(0, b0, e0);
    load_rp(1, b1, e1);
    int cc[EPL] = {};
    float cv[EPL] = {};
    if (my_pass > 0) load_csr(b0, e0, cc, cv);
    int kept_total = 0;
    int g = 0;
    // step s: tile s into buffer s & 1 (the matrix waves meanwhile read
    // tile s - 1 from the other); one step more than tiles, so that the
    // barriers pair up with the matrix waves' loop
#pragma unroll 1
    for (int s = 0; s <= my_tiles; ++s) {
      if (s < my_tiles) {
        float* X = Xs[s & 1];
#pragma unroll 1
        for (int pass = 0; pass < PASSES; ++pass, ++g) {
          const int lr = pass * RPB + wave * RPW + grp;
          const int row = doc_row(g);
          const int b = b0, e = e0;
          int c_cur[EPL];
          float v_cur[EPL];
#pragma unroll
          for (int q = 0; q < EPL; ++q) {
            c_cur[q] = cc[q];
            v_cur[q] = cv[q];
          }
          load_csr(b1, e1, cc, cv);
          b0 = b1;
          e0 = e1;
          load_rp(g + 2, b1, e1);
          float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
          float L = doc_sum<G>(lane_sum(v_cur));   // the first chunk's counts, before its gathers
          int2* my_ent = ent[wave][grp];
          for (int base = b; base < e; base += CH) {
            if (base != b) {
              load_csr(base, e, c_cur, v_cur);
              L += doc_sum<G>(lane_sum(v_cur));
            }
            // this chunk's entries into the wave's LDS rows (the previous
            // chunk's reads were issued earlier by this same wave, and one
            // wave's LDS operations complete in order)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
            for (int q = 0; q < EPL; ++q) my_ent[gl + q * G] = make_int2(c_cur[q], __float_as_int(v_cur[q]));
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int n_here = min(CH, e - base);
            for (int t0 = 0; t0 < n_here; t0 += NB) {
              float4 w[NB];
              int2 en[NB];
#pragma unroll
              for (int t = 0; t < NB; ++t) en[t] = my_ent[t0 + t];
#pragma unroll
              for (int t = 0; t < NB; ++t) {
                const int c = en[t].x;
                const uint32_t off = __umul24((uint32_t)c, gmul4) + gadd4;
                const auto r = __builtin_amdgcn_raw_buffer_load_b128(wrs, off, 0, 0);
                w[t] = make_float4(__uint_as_float(r[0]), __uint_as_float(r[1]),
                                   __uint_as_float(r[2]), __uint_as_float(r[3]));
              }
#pragma unroll
              for (int t = 0; t < NB; ++t) {
                const float v = __int_as_float(en[t].y);
                a.x = fmaf(v, w[t].x, a.x);
                a.y = fmaf(v, w[t].y, a.y);
                a.z = fmaf(v, w[t].z, a.z);
                a.w = fmaf(v, w[t].w, a.w);
              }
            }
          }
          const int kept = (row >= 0 && L >= 3.f) ? 1 : 0;
          float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
          if (kept && active) {
            const float4 mw = *reinterpret_cast<const float4*>(mw32 + c4);
            const float invL = 1.0f / L;
            x.x = fmaf(a.x, invL, -mw.x);
            x.y = fmaf(a.y, invL, -mw.y);
            x.z = fmaf(a.z, invL, -mw.z);
            x.w = fmaf(a.w, invL, -mw.w);
          }
          if (in_lds) *reinterpret_cast<float4*>(X + lr * LDX + c4) = x;
          if (Xout != nullptr && row >= 0 && active) {
            float* out = Xout + (size_t)row * D;
            if (c4 + 0 < D) out[c4 + 0] = x.x;
            if (c4 + 1 < D) out[c4 + 1] = x.y;
            if (c4 + 2 < D) out[c4 + 2] = x.z;
            if (c4 + 3 < D) out[c4 + 3] = x.w;
          }
          kept_total += __popcll(__ballot(kept && gl == 0));
        }
      }
      __syncthreads();
    }
    if (lane == 0) wave_kept[wave] = kept_total;
  } else {
    // matrix wave cw: column tiles cw and cw + NC of S and R1 (K = 112 has
    // seven: waves 12-14 take two, wave 15 one)
    const int cw = wave - NP;
    floatx4 acc[CT][NDT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int q = 0; q < NDT; ++q) acc[c][q] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int s = 0; s <= my_tiles; ++s) {
      if (s >= 1) {   // tile s - 1, whitened in the previous step
        const float* X = Xs[(s - 1) & 1];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int ct = cw + NC * c;
          if (ct < NCT) {
            floatx4 sacc[T / 16];
#pragma unroll
            for (int u = 0; u < T / 16; ++u) sacc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
            const float* xa = X + l16 * LDX + l4;
            const float* pb = Ps + l4 * LDP + ct * 16 + l16;
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
              const float bv = pb[4 * ks * LDP];
#pragma unroll
              for (int u = 0; u < T / 16; ++u)
                sacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u * 16 * LDX + 4 * ks], bv,
                                                               sacc[u], 0, 0, 0);
            }
            // R1 += X_t^T S^2 with S^2 straight from the accumulators: k-step
            // (u, r) sums rows u 16 + 4 k + r (k = l4), the rows this lane
            // already holds, so S never goes through LDS
#pragma unroll
            for (int u = 0; u < T / 16; ++u)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float sv = sacc[u][r] * sacc[u][r];
                const float* xr = X + (u * 16 + 4 * l4 + r) * LDX + l16;
#pragma unroll
                for (int q = 0; q < NDT; ++q)
                  acc[c][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[q * 16], sv, acc[c][q], 0, 0, 0);
                if (r % 2 == 1) __builtin_amdgcn_sched_barrier(0);
              }
          }
        }
      }
      __syncthreads();
    }
    float* out = partial + (size_t)blockIdx.x * D * K;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int ct = cw + NC * c;
      if (ct < NCT) {
        const int k = ct * 16 + l16;
#pragma unroll
        for (int q = 0; q < NDT; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int d = q * 16 + 4 * l4 + r;
            if (d < D && k < K) out[d * K + k] = acc[c][q][r];
          }
      }
    }
  }
  // the squared Gram entries of the finish, as in the wide kernel, dealt
  // first to the blocks with the shorter run of passes (they finish a pass
  // earlier): block b has run floor((b+1) P / n) - floor(b P / n) of the P
  // passes, floor(P / n) + 1 for the floor(b P / n) - b floor(P / n) longer
  // runs before it
  __syncthreads();
  if (gsq != nullptr) {
    const int q = n_pass_all / nblk;
    const int n_short = nblk - (n_pass_all - q * nblk);
    const int long_before = pass0 - (int)blockIdx.x * q;
    const int slot = my_pass == q ? (int)blockIdx.x - long_before : n_short + long_before;
    for (int e4 = slot * kThreads + tid; e4 < 4 * K * K; e4 += nblk * kThreads) {
      const int e = e4 >> 2, c = e4 & 3;
      const int j = e / K, k = e % K;
      double accg = 0.0;
      const int M = D / 4;
      for (int m = 0; m < M; ++m) {
        const int i = 4 * m + c;
        accg += (double)Ps[i * LDP + j] * (double)Ps[i * LDP + k];
      }
      if (c == 0)
        for (int i = 4 * M; i < D; ++i) accg += (double)Ps[i * LDP + j] * (double)Ps[i * LDP + k];
      accg += __shfl_xor(accg, 1, 64);
      accg += __shfl_xor(accg, 2, 64);
      if (c == 0) gsq[e] = accg * accg;
    }
  }
  if (tid == 0) {
    int n = 0;
#pragma unroll
    for (int w = 0; w < NP; ++w) n += wave_kept[w];
    block_counts[blockIdx.x] = n;
  }
}

// W32 (tail_base / Dp = V rows) below 4 GiB and V below 2^24.
inline bool hyb_addressable(int Dp, int Dt, uint32_t tail_base) {
  const uint64_t V = (uint64_t)tail_base / (uint64_t)Dp;
  const uint64_t bytes = 4 * V * (uint64_t)(Dp + Dt);
  return V < (1u << 24) && bytes < (1ull << 32);
}

template <int DQ, int KQ, int NK2, int G>
hipError_t launch_hyb(const tlda_csr_batch& b, const float* W32, const float* mw32, int D, int Dp,
                      int Dt, uint32_t tail_base, const float* Phi, int K, int nblk,
                      float* partial, int* block_counts, float* Xout, float* phi_copy,
                      double* gsq, hipStream_t s) {
  if (partial == nullptr) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, k_whiten_cp_hyb<DQ, KQ, NK2, G>, 1024, 0);
    *block_counts = per_cu;
    return e;
  }
  // as in launch_wide: clamped loads read the row pointers when there are no nonzeros
  const int32_t* ci = b.nnz > 0 ? b.col_idx : b.row_ptr;
  const float* va = b.nnz > 0 ? b.val : reinterpret_cast<const float*>(b.row_ptr);
  launch_main(k_whiten_cp_hyb<DQ, KQ, NK2, G>, dim3(nblk), dim3(1024), 0, s, b.row_ptr, ci, va,
              b.n_rows, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial, block_counts,
              Xout, phi_copy, gsq);
  return hipGetLastError();
}

template <int DQ, int KQ, int NK2 = DQ / 4>
hipError_t launch_wide(const tlda_csr_batch& b, const float* W32, const float* mw32, int D, int Dp,
                       int Dt, uint32_t tail_base, const float* Phi, int K, int nblk,
                       float* partial, int* block_counts, float* Xout, float* phi_copy,
                       double* gsq, hipStream_t s) {
  if constexpr (DQ >= 64 && KQ >= 64) {
    // the hybrid kernel, whose gathers address W32 (V rows of Dp floats from
    // element 0, then V rows of Dt from tail_base = V Dp) with 32-bit byte
    // offsets from 24-bit row numbers; past that, the 8-wave kernel
    constexpr int G = DQ == 64 ? 16 : 32;
    if (hyb_addressable(Dp, Dt, tail_base)) {
      if (D <= (DQ == 64 ? 52 : DQ == 112 ? 100 : 116))
        return launch_hyb<DQ, KQ, (DQ == 64 ? 13 : DQ == 112 ? 25 : 29), G>(
            b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial, block_counts, Xout,
            phi_copy, gsq, s);
      return launch_hyb<DQ, KQ, DQ / 4, G>(b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk,
                                           partial, block_counts, Xout, phi_copy, gsq, s);
    }
  }
  if constexpr (DQ == 112 && NK2 == DQ / 4) {
    if (D <= 100)
      return launch_wide<DQ, KQ, 25>(b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial,
                                     block_counts, Xout, phi_copy, gsq, s);
  }
  if (partial == nullptr) {   // occupancy query: resident blocks per CU in nblk's place
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, k_whiten_cp_wide<DQ, KQ, NK2>, 512, 0);
    *block_counts = per_cu;
    return e;
  }
  // without nonzeros the CSR arrays may be absent: the kernel's clamped loads
  // then read the row pointers instead (the values are discarded)
  const int32_t* ci = b.nnz > 0 ? b.col_idx : b.row_ptr;
  const float* va = b.nnz > 0 ? b.val : reinterpret_cast<const float*>(b.row_ptr);
  launch_main(k_whiten_cp_wide<DQ, KQ, NK2>, dim3(nblk), dim3(512), 0, s, b.row_ptr, ci, va,
              b.n_rows, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial, block_counts,
              Xout, phi_copy, gsq);
  return hipGetLastError();
}

template <int DQ, int KQ, int T, int G>
hipError_t launch_fused_t(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                          int Dp, const float* Phi, int K, int nblk, float* partial,
                          int* block_counts, float* Xout, float* phi_copy, hipStream_t s) {
  if (partial == nullptr) {   // occupancy query: resident blocks per CU in nblk's place
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, k_whiten_cp<DQ, KQ, T, G>, 64 * fused_waves(DQ, KQ), 0);
    *block_counts = per_cu;
    return e;
  }
  launch_main(k_whiten_cp<DQ, KQ, T, G>, dim3(nblk), dim3(64 * fused_waves(DQ, KQ)), 0, s,
              b.row_ptr, b.col_idx,
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

// Shapes the fused kernel covers: D, K <= 128 (each padded to 16, 32, 64,
// 112 or 128); the wide kernels keep Phi, X and S in LDS, at most 97 KB per
// block for the 8-wave kernel and 121 KB for the hybrid (128 x 128).
bool fused_supported(int D, int K, int Dp) {
  return mfma_bucket(D) > 0 && mfma_bucket(K) > 0 && Dp <= 128;
}

namespace {
// the wide kernels (k_whiten_cp_wide, k_whiten_cp_hyb): D or K past 64
bool fused_wide(int D, int K) { return mfma_bucket(D) > 64 || mfma_bucket(K) > 64; }
}  // namespace

int fused_tile_rows(int D, int K) {
  if (mfma_bucket(D) >= 64 && mfma_bucket(K) >= 64) return 48;   // the hybrid kernel
  return fused_wide(D, K) ? 32 : cp_mfma_tile_rows(D, K);        // 8-wave : 4-wave
}

int w32_tail_cols(int D, int K) {
  if (!fused_wide(D, K) || D < 32) return 0;   // only the wide kernels read it
  const int rem = D % 32;
  return rem >= 1 && rem <= 8 ? (rem + 3) / 4 * 4 : 0;
}

namespace {
__global__ void k_w32_tail(float* __restrict__ W32, int V, int Dm, int Dp, int Dt,
                           uint32_t tail_base) {
  const size_t n = (size_t)V * Dt;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t w = e / Dt, j = e % Dt;
    W32[tail_base + e] = W32[w * Dp + Dm + j];
  }
}
}  // namespace

hipError_t launch_w32_tail(float* W32, int V, int D, int Dp, int Dt, uint32_t tail_base,
                           hipStream_t s) {
  if (Dt <= 0) return hipSuccess;
  const size_t n = (size_t)V * Dt;
  const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_w32_tail, dim3(grid), dim3(256), 0, s, W32, V, D / 32 * 32, Dp, Dt,
                     tail_base);
  return hipGetLastError();
}

bool fused_forms_gram(int D, int K) {
  return fused_wide(D, K) || (mfma_bucket(D) >= 64 && mfma_bucket(K) >= 64);
}

hipError_t launch_whiten_cp(const tlda_csr_batch& b, const float* W32, const float* mw32, int D,
                            int Dp, int Dt, uint32_t tail_base, const float* Phi, int K,
                            int nblk, float* partial, int* block_counts, float* Xout,
                            float* phi_copy, double* gsq, hipStream_t s) {
  const int dq = mfma_bucket(D), kq = mfma_bucket(K);
  // D and K in 33..64: the hybrid kernel, 16 lanes per document (13 k-steps
  // of S = X_t Phi up to D = 52); wider hybrid shapes go through launch_wide
  if (dq == 64 && kq == 64 && hyb_addressable(Dp, Dt, tail_base)) {
    if (D <= 52)
      return launch_hyb<64, 64, 13, 16>(b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial,
                                        block_counts, Xout, phi_copy, gsq, s);
    return launch_hyb<64, 64, 16, 16>(b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial,
                                      block_counts, Xout, phi_copy, gsq, s);
  }
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
  // wide shapes: 32 lanes per document (one float4 of up to 128 columns each)
#define TLDA_WIDE(DQ_, KQ_)                                                                    \
  if (dq == DQ_ && kq == KQ_)                                                                  \
    return launch_wide<DQ_, KQ_>(b, W32, mw32, D, Dp, Dt, tail_base, Phi, K, nblk, partial,   \
                                 block_counts, Xout, phi_copy, gsq, s);
#define TLDA_WIDE_ROW(DQ_) \
  TLDA_WIDE(DQ_, 16) TLDA_WIDE(DQ_, 32) TLDA_WIDE(DQ_, 64) TLDA_WIDE(DQ_, 112) TLDA_WIDE(DQ_, 128)
  TLDA_WIDE(16, 112) TLDA_WIDE(16, 128) TLDA_WIDE(32, 112) TLDA_WIDE(32, 128)
  TLDA_WIDE(64, 112) TLDA_WIDE(64, 128) TLDA_WIDE_ROW(112) TLDA_WIDE_ROW(128)
#undef TLDA_WIDE_ROW
#undef TLDA_WIDE
  return hipErrorInvalidValue;
}

}  // namespace tlda
