// BF16 precision path of the whitening SpMM and the CP-gradient reduction
// (the data term R1 = X^T (X Phi)^2 of eq. vec_deriv).
//
// What is rounded to BF16 (round to nearest even), and nothing else:
//   * the whitening copy: W16 = bf16(fp32(W)); its mean projection
//     mw16 = W16^T M1 is formed in FP64 from the rounded values, so the
//     whitened rows are exactly (F - 1 M1^T) W16 up to FP32 accumulation: a
//     whitening by a slightly perturbed W, centred in FP32 before any
//     rounding of X (no mean-correction terms are needed afterwards);
//   * the MFMA operands: X, Phi and the squared scores S^2 = (X Phi)^2.
// Accumulation is FP32 on the matrix cores; the penalty term, the 3 c3 / n
// scaling and the update stay in the FP64/FP32 finish kernel shared with the
// FP32 path.
//
// One kernel template, three modes:
//   kFused      CSR batch -> whitened tile in LDS -> S^2 -> R1 partials
//   kFromX      FP32 X rows from HBM -> same contractions (tlda_cp_step)
//   kWhitenOnly CSR batch -> FP32 X rows in HBM (tlda_whiten_batch)
//
// Per tile of 64 documents (256 threads = 4 waves):
//   1. G lanes own a document, 8 columns (16 bytes of W16) per lane; 8
//      nonzeros per step are fetched cooperatively one step ahead, broadcast
//      by shuffles, and all their W16-row gathers are issued before use.
//      Counts that are exact in BF16 (integers up to 256, every count of a
//      short document in practice) accumulate with v_dot2_f32_bf16 (one
//      instruction per column, the BF16 x BF16 product being exact in FP32),
//      any other step with plain FMAs.  The centred row goes to LDS twice in
//      BF16: row-major (operand of X Phi) and column-major (operand of
//      X^T S^2).
//   2. S = X Phi with v_mfma_f32_16x16x32_bf16 (Phi fragments in registers),
//      S^2 rounded to BF16 into LDS column-major.
//   3. R1 += X^T S^2 with the same instruction, accumulators in registers.
// A K-permutation applied equally to both operands of an MFMA leaves the
// product unchanged, so only the row/column lane mapping (shared with the
// FP32 16x16x4 instruction) is relied on.
#include "tlda_internal.h"

namespace tlda {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;       // documents per tile
constexpr int kNB = 8;          // nonzeros per gather step

enum { kFused = 0, kFromX = 1, kWhitenOnly = 2 };

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even on the upper 16 bits; NaN stays NaN.
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
// Two FP32 values to packed BF16 (a in the low half), round to nearest even
// (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
  const b16x2 h = __builtin_convertvector((f32x2{a, b}), b16x2);
  return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ floatx4 mfma_bf16(u32x4 a, u32x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__global__ void k_form_w16(const double* __restrict__ W, int V, int D, int Dh,
                           uint16_t* __restrict__ W16) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)V * Dh) return;
  const int i = (int)(idx / Dh), d = (int)(idx % Dh);
  W16[idx] = d < D ? (uint16_t)bf16_rne((float)W[(size_t)i * D + d]) : (uint16_t)0;
}

// mw16[d] = sum_i W16[i][d] m[i] in FP64 (one block per column); padding zero.
__global__ void __launch_bounds__(256) k_mw16(const uint16_t* __restrict__ W16,
                                              const double* __restrict__ m, int V, int D, int Dh,
                                              float* __restrict__ mw16) {
  __shared__ double red[256];
  const int d = blockIdx.x, tid = threadIdx.x;
  if (d >= D) {
    if (tid == 0) mw16[d] = 0.0f;
    return;
  }
  double s = 0.0;
  for (int i = tid; i < V; i += blockDim.x) s += (double)bf16_lo(W16[(size_t)i * Dh + d]) * m[i];
  red[tid] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) mw16[d] = (float)red[0];
}

// Sum over each group of G lanes (G <= 16, aligned), the result in all of
// them: a DPP butterfly inside the 16-lane row (pairs, quads, mirrored halves
// of 8, mirrored halves of 16), the same pairings as lane xors 1, 2, 4, 8.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF,
                                                            0xF, false));
}
template <int G>
__device__ __forceinline__ float group_sum(float s) {
  static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "group of 1 to 16 lanes");
  if constexpr (G >= 2) s += dpp_mov<0xB1>(s);    // quad_perm [1, 0, 3, 2]
  if constexpr (G >= 4) s += dpp_mov<0x4E>(s);    // quad_perm [2, 3, 0, 1]
  if constexpr (G >= 8) s += dpp_mov<0x141>(s);   // row_half_mirror
  if constexpr (G >= 16) s += dpp_mov<0x140>(s);  // row_mirror
  return s;
}

// Waves per block: 16 when both D and K are padded past 64 and 8 when one is,
// so that the R1 accumulators (DQ x KQ per block) spread over more waves and
// each keeps few enough registers for 4 waves per SIMD (with 4-wave blocks
// these shapes ran at 2 or 3); 4 otherwise.
constexpr int bf16_waves(int DQ, int KQ) {
  return (DQ > 64 && KQ > 64) ? 16 : (DQ > 64 || KQ > 64) ? 8 : 4;
}

template <int DQ, int KQ, int NW = 4, int TR = kTile>
struct Bf16Shape {
  static constexpr int LDA = DQ + 8;        // row-major X tile stride (bf16)
  static constexpr int LDT = TR + 8;        // column-major tiles stride (bf16)
  static constexpr int NCT = KQ / 16, NDT = DQ / 16, NKS = DQ / 32;
  static constexpr int ST = (NCT + NW - 1) / NW;       // column tiles of S per wave
  static constexpr int WD = NDT >= 4 ? 4 : NDT;
  static constexpr int WK = NW / WD;
  static constexpr int TDW = NDT / WD;                 // R1 row tiles per wave
  static constexpr int TKW = (NCT + WK - 1) / WK;      // R1 column tiles per wave
};

// The work of one block: block `blk` of `nblk` blocks that share one batch,
// in row tiles of TR documents (64 for the single-batch kernels; the
// multi-slice kernels also take 32).  LDS comes from the caller (Xs: TR x LDA,
// XsT: DQ x LDT, twice that with kDbl, SsT: KQ x LDT BF16 values, wave_kept:
// NW ints, ent: 64 NW entries), so one kernel can serve several shapes.
template <int DQ, int KQ, int G, int MODE, int NW, int TR = kTile, bool kDbl = false>
__device__ __forceinline__ void cp_bf16_block(
    int blk, int nblk, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const uint16_t* __restrict__ W16,
    const float* __restrict__ mw16, int Dh, const float* __restrict__ Xin, int D,
    const float* __restrict__ Phi, int K, float* __restrict__ partial,
    int* __restrict__ block_counts, float* __restrict__ Xout, float* __restrict__ phi_copy,
    uint16_t* __restrict__ Xs, uint16_t* __restrict__ XsT, uint16_t* __restrict__ SsT,
    int* __restrict__ wave_kept, int2* __restrict__ ent) {
  typedef Bf16Shape<DQ, KQ, NW, TR> Sh;
  static_assert(TR % 32 == 0, "tile rows: a multiple of the 32-row MFMA step");
  constexpr bool kCp = MODE != kWhitenOnly;
  constexpr int kThreads = NW * 64;
  constexpr int RPW = 64 / G;
  constexpr int RPB = NW * RPW;
  constexpr int PASSES = (TR + RPB - 1) / RPB;
  constexpr int SLOTS = G >= kNB ? 1 : kNB / G;
  // G >= kNB: a step's entries sit in lanes 0 .. kNB - 1 of the group, which
  // write them to the group's LDS row (G entries, one per lane); every lane
  // then reads all kNB with 16-byte reads at fixed offsets
  constexpr bool kStage = G >= kNB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int gl = lane % G;
  const int c8 = gl * 8;               // first column of this lane (c8 < Dh <= DQ)
  const bool pair_lo = ((lane / G) & 1) == 0;
  const unsigned char* W16b = reinterpret_cast<const unsigned char*>(W16);
  int2* my_ent = ent + (kStage ? (lane / G) * G + wave * 64 : 0);   // this group's LDS row
  const uint32_t row_bytes = (uint32_t)Dh * 2u, col_bytes = (uint32_t)c8 * 2u;

  if (kCp) {
    for (int e = blk * kThreads + tid; e < D * K; e += nblk * kThreads)
      phi_copy[e] = Phi[e];
    for (int e = tid; e < TR * Sh::LDA; e += kThreads) Xs[e] = 0;
    for (int e = tid; e < (kDbl ? 2 : 1) * DQ * Sh::LDT; e += kThreads) XsT[e] = 0;
  }
  // Phi fragments: bphi[q][ks] holds Phi[32 ks + 8 l4 + i][16 ct + l16], i = 0..7
  u32x4 bphi[Sh::ST][Sh::NKS];
#pragma unroll
  for (int q = 0; q < Sh::ST; ++q) {
    const int ct = wave + NW * q;
    const int k = 16 * ct + l16;
#pragma unroll
    for (int ks = 0; ks < Sh::NKS; ++ks) {
      float f[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int d = 32 * ks + 8 * l4 + i;
        f[i] = (kCp && ct < Sh::NCT && d < D && k < K) ? Phi[d * K + k] : 0.f;
      }
      bphi[q][ks] = u32x4{pack_bf16(f[0], f[1]), pack_bf16(f[2], f[3]), pack_bf16(f[4], f[5]),
                          pack_bf16(f[6], f[7])};
    }
  }
  floatx4 acc[Sh::TDW][Sh::TKW];
#pragma unroll
  for (int a = 0; a < Sh::TDW; ++a)
#pragma unroll
    for (int b = 0; b < Sh::TKW; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  float mw[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) mw[i] = MODE == kFromX ? 0.f : mw16[c8 + i];
  int kept_total = 0;

  const int ntiles = (n_rows + TR - 1) / TR;
  // kDbl: two column-major tiles in turn, so a tile's rows can be written
  // while other waves still read the previous tile's in the R1 phase (the
  // row-major tile and S^2 are free by then: every wave has passed the
  // barrier after the S phase, and the next S phase follows the barrier
  // after the whitening); one barrier per tile fewer
  if (kDbl) __syncthreads();
  uint16_t* const XsT0 = XsT;
  int parity = 0;
  for (int tile = blk; tile < ntiles; tile += nblk, parity ^= 1) {
    if (kCp && !kDbl) __syncthreads();
    if (kDbl) XsT = XsT0 + parity * DQ * Sh::LDT;
    // ---- 1. rows of the tile ----
#pragma unroll 1
    for (int pass = 0; pass < PASSES; ++pass) {
      const int lr = pass * RPB + wave * RPW + lane / G;
      const int row = tile * TR + lr;
      const bool valid = lr < TR && row < n_rows;
      float x[8];
      int kept = 0;
      if (MODE == kFromX) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          x[i] = (valid && c8 + i < D) ? Xin[(size_t)row * D + c8 + i] : 0.f;
      } else {
        int b = 0, e = 0;
        if (valid) {
          b = row_ptr[row];
          e = row_ptr[row + 1];
        }
        float a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = 0.f;
        float Lp = 0.f;
        // nonzeros jb .. jb + 7 of the row, fetched cooperatively (lane gl
        // of the group loads entries gl, gl + G, ...); indices are clamped
        // to the row, and entries past it become (column 0, count 0)
        int cn[SLOTS];
        float vn[SLOTS];
        auto fetch = [&](int jb) {
#pragma unroll
          for (int q = 0; q < SLOTS; ++q) {
            const int j = jb + q * G + gl;
            const bool in = (q * G + gl) < kNB && j < e;
            const int jc = j < e ? j : e - 1;
            const int cc = col_idx[jc];
            const float vv = val[jc];
            cn[q] = in ? cc : 0;
            vn[q] = in ? vv : 0.f;
          }
        };
        if (b < e) fetch(b);
        for (int jb = b; jb < e; jb += kNB) {
          int cidx[SLOTS];
          float cval[SLOTS];
          bool inexact = false;
#pragma unroll
          for (int q = 0; q < SLOTS; ++q) {
            cidx[q] = cn[q];
            cval[q] = vn[q];
            Lp += cval[q];
            inexact |= (__float_as_uint(cval[q]) & 0xffffu) != 0u;
          }
          if (jb + kNB < e) fetch(jb + kNB);      // next step's entries, in flight meanwhile
          uint32_t cs[kNB];
          float v[kNB];
          if constexpr (kStage) {
            // the previous step's reads of the row were issued earlier by this
            // wave, and one wave's LDS operations complete in order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            my_ent[gl] = make_int2(cidx[0], __float_as_int(cval[0]));
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            int2 en[kNB];
#pragma unroll
            for (int t = 0; t < kNB; ++t) en[t] = my_ent[t];
#pragma unroll
            for (int t = 0; t < kNB; ++t) {
              cs[t] = (uint32_t)en[t].x;
              v[t] = __int_as_float(en[t].y);
            }
          } else {
#pragma unroll
            for (int t = 0; t < kNB; ++t) {
              cs[t] = (uint32_t)__shfl(cidx[t / G < SLOTS ? t / G : 0], t % G, G);
              v[t] = __shfl(cval[t / G < SLOTS ? t / G : 0], t % G, G);
            }
          }
          // all gathers first: 16 bytes of row c of W16 per lane, 32-bit byte
          // offsets from a 24-bit multiply (V < 2^24, V Dh 2 < 2^32)
          u32x4 w[kNB];
#pragma unroll
          for (int t = 0; t < kNB; ++t)
            w[t] = *reinterpret_cast<const u32x4*>(W16b + (__umul24(cs[t], row_bytes) + col_bytes));
          if (!__any(inexact)) {
            // every count of the step is exact in BF16 (integers <= 256): one
            // dot-2 per column, w.lo * v + w.hi * 0 + a (products exact in FP32)
#pragma unroll
            for (int t = 0; t < kNB; ++t) {
              // an exact count has zero low 16 bits: its FP32 pattern is
              // (0, v) as a BF16 pair, and shifted right it is (v, 0)
              const uint32_t vb = __float_as_uint(v[t]);
              const uint32_t vb_lo = vb >> 16;
              const bf16x2 vlo = __builtin_bit_cast(bf16x2, vb_lo);
              const bf16x2 vhi = __builtin_bit_cast(bf16x2, vb);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                // (bit-cast a named scalar: this compiler folds a bit-cast of a
                // vector subscript to element 0)
                const uint32_t wi = w[t][i];
                const bf16x2 wp = __builtin_bit_cast(bf16x2, wi);
                a[2 * i] = __builtin_amdgcn_fdot2_f32_bf16(wp, vlo, a[2 * i], false);
                a[2 * i + 1] = __builtin_amdgcn_fdot2_f32_bf16(wp, vhi, a[2 * i + 1], false);
              }
            }
          } else {
#pragma unroll
            for (int t = 0; t < kNB; ++t)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                a[2 * i] = fmaf(v[t], bf16_lo(w[t][i]), a[2 * i]);
                a[2 * i + 1] = fmaf(v[t], bf16_hi(w[t][i]), a[2 * i + 1]);
              }
          }
        }
        const float L = group_sum<G>(Lp);
        kept = (valid && L >= 3.f) ? 1 : 0;
        const float invL = kept ? 1.0f / L : 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = kept ? fmaf(a[i], invL, -mw[i]) : 0.f;
        if (Xout != nullptr && valid) {
          float* out = Xout + (size_t)row * D;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (c8 + i < D) out[c8 + i] = x[i];
        }
        kept_total += __popcll(__ballot(kept && gl == 0));
      }
      if (kCp) {
        const u32x4 hp = u32x4{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]),
                               pack_bf16(x[4], x[5]), pack_bf16(x[6], x[7])};
        if (lr < TR) *reinterpret_cast<u32x4*>(Xs + lr * Sh::LDA + c8) = hp;
        // column-major copy: the even document of each pair writes both
        // documents' values of a column as one 32-bit word
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t mine = hp[i];
          const uint32_t other = __shfl_down(mine, G, 64);
          if (pair_lo && lr < TR) {
            *reinterpret_cast<uint32_t*>(XsT + (c8 + 2 * i) * Sh::LDT + lr) =
                (mine & 0xffffu) | (other << 16);
            *reinterpret_cast<uint32_t*>(XsT + (c8 + 2 * i + 1) * Sh::LDT + lr) =
                (mine >> 16) | (other & 0xffff0000u);
          }
        }
      }
    }
    if (!kCp) continue;
    __syncthreads();
    // ---- 2. S = X Phi; S^2 to LDS, column-major ----
#pragma unroll
    for (int q = 0; q < Sh::ST; ++q) {
      const int ct = wave + NW * q;
      if (ct < Sh::NCT) {
#pragma unroll
        for (int rt = 0; rt < TR / 16; ++rt) {
          floatx4 s = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < Sh::NKS; ++ks) {
            const u32x4 av =
                *reinterpret_cast<const u32x4*>(Xs + (16 * rt + l16) * Sh::LDA + 32 * ks + 8 * l4);
            s = mfma_bf16(av, bphi[q][ks], s);
          }
          *reinterpret_cast<u32x2*>(SsT + (16 * ct + l16) * Sh::LDT + 16 * rt + 4 * l4) =
              u32x2{pack_bf16(s[0] * s[0], s[1] * s[1]), pack_bf16(s[2] * s[2], s[3] * s[3])};
        }
      }
    }
    __syncthreads();
    // ---- 3. R1 += X^T S^2 ----
    const int wd = wave % Sh::WD, wk = wave / Sh::WD;
#pragma unroll
    for (int kk = 0; kk < TR / 32; ++kk) {
      u32x4 av[Sh::TDW];
#pragma unroll
      for (int a = 0; a < Sh::TDW; ++a)
        av[a] = *reinterpret_cast<const u32x4*>(XsT + (16 * (wd + Sh::WD * a) + l16) * Sh::LDT +
                                                32 * kk + 8 * l4);
#pragma unroll
      for (int b = 0; b < Sh::TKW; ++b) {
        const int ct = wk + Sh::WK * b;
        if (ct < Sh::NCT) {
          const u32x4 bv =
              *reinterpret_cast<const u32x4*>(SsT + (16 * ct + l16) * Sh::LDT + 32 * kk + 8 * l4);
#pragma unroll
          for (int a = 0; a < Sh::TDW; ++a) acc[a][b] = mfma_bf16(av[a], bv, acc[a][b]);
        }
      }
    }
  }
  if (kCp) {
    const int wd = wave % Sh::WD, wk = wave / Sh::WD;
    float* out = partial + (size_t)blk * D * K;
#pragma unroll
    for (int a = 0; a < Sh::TDW; ++a)
#pragma unroll
      for (int b = 0; b < Sh::TKW; ++b) {
        const int ct = wk + Sh::WK * b;
        const int k = 16 * ct + l16;
        if (ct < Sh::NCT && k < K) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int d = 16 * (wd + Sh::WD * a) + 4 * l4 + r;
            if (d < D) out[d * K + k] = acc[a][b][r];
          }
        }
      }
  }
  if (MODE != kFromX) {
    if (lane == 0) wave_kept[wave] = kept_total;
    __syncthreads();
    if (tid == 0) {
      int n = 0;
      for (int w = 0; w < NW; ++w) n += wave_kept[w];
      block_counts[blk] = n;
    }
  }
}


template <int DQ, int KQ, int G, int MODE>
__global__ void __launch_bounds__(64 * (MODE == kWhitenOnly ? 4 : bf16_waves(DQ, KQ)),
                                  (DQ <= 64 && KQ <= 64) ? 3 : 4)
    k_cp_bf16(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int n_rows, const uint16_t* __restrict__ W16,
    const float* __restrict__ mw16, int Dh, const float* __restrict__ Xin, int D,
    const float* __restrict__ Phi, int K, int nblk, float* __restrict__ partial,
    int* __restrict__ block_counts, float* __restrict__ Xout, float* __restrict__ phi_copy,
    double* __restrict__ gsq) {
  constexpr int NW = MODE == kWhitenOnly ? 4 : bf16_waves(DQ, KQ);
  constexpr bool kCp = MODE != kWhitenOnly;
  // 16-wave blocks (D and K past 64) take 128-document tiles: half the
  // barriers and matrix phases per document of 64-document tiles (118 against
  // 125 us per streaming-scale batch), and two column-major tiles in turn
  // (one barrier per tile fewer: 116.7 against 119.1 us); 144 KiB of LDS at
  // 128 x 128
  constexpr int TRB = (kCp && NW == 16) ? 128 : kTile;
  constexpr bool kDbl = kCp && NW == 16;
  typedef Bf16Shape<DQ, KQ, NW, TRB> Sh;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[kCp ? TRB * Sh::LDA : 8];
  __shared__ __attribute__((aligned(16))) uint16_t XsT[kCp ? (kDbl ? 2 : 1) * DQ * Sh::LDT : 8];
  __shared__ __attribute__((aligned(16))) uint16_t SsT[kCp ? KQ * Sh::LDT : 8];
  __shared__ int wave_kept[NW];
  __shared__ __attribute__((aligned(16))) int2 ent[G >= kNB ? 64 * NW : 2];
  cp_bf16_block<DQ, KQ, G, MODE, NW, TRB, kDbl>(blockIdx.x, nblk, row_ptr, col_idx, val, n_rows, W16, mw16, Dh,
                                 Xin, D, Phi, K, partial, block_counts, Xout, phi_copy, Xs, XsT,
                                 SsT, wave_kept, ent);
  // The fused step also forms the finish's squared Gram entries of Phi (still
  // Phi0 here: the finish writes Phi after this kernel), with k_gram_sq's
  // summation (four lanes per entry, chain c over d = 4m + c, chain 0 also
  // the tail, added as (c0 + c1) + (c2 + c3)), so no launch of its own.
  // 4 K^2 is a multiple of 4, so the four lanes of an entry leave the loop
  // together.  The 16-wave blocks read Phi from an LDS copy in the space of
  // the column-major tiles (free since the block's last barrier; 17 408
  // floats >= D K), the others from global memory.
  constexpr int kThr = 64 * NW;
  if (MODE == kFused && gsq != nullptr && blockIdx.x * kThr < 4 * K * K) {
    const float* P = Phi;
    if constexpr (kDbl) {
      static_assert(!kDbl || 2 * DQ * Sh::LDT / 2 >= TLDA_MAX_DK, "Phi fits the tiles' space");
      float* Pf = reinterpret_cast<float*>(XsT);
      for (int i = threadIdx.x; i < D * K; i += kThr) Pf[i] = Phi[i];
      __syncthreads();
      P = Pf;
    }
    for (int e4 = blockIdx.x * kThr + threadIdx.x; e4 < 4 * K * K; e4 += nblk * kThr) {
      const int e = e4 >> 2, c = e4 & 3;
      const int j = e / K, k = e % K;
      double accg = 0.0;
      const int M = D / 4;
      for (int m = 0; m < M; ++m) {
        const int i = 4 * m + c;
        accg += (double)P[i * K + j] * (double)P[i * K + k];
      }
      if (c == 0)
        for (int i = 4 * M; i < D; ++i) accg += (double)P[i * K + j] * (double)P[i * K + k];
      accg += __shfl_xor(accg, 1, 64);
      accg += __shfl_xor(accg, 2, 64);
      if (c == 0) gsq[e] = accg * accg;
    }
  }
}

// Several batches (the slices of a batched run, each with its own
// whitening, D, K and Phi) in one launch: block b serves slice blk_slice[b],
// as block b - blk0 of that slice's nblk blocks.  One LDS allocation of the
// largest shape (D, K <= 64) serves every slice.  Tile shape: TR documents
// per row tile, NW waves per block (the plan's autotuner picks among the
// instances below).
template <int TR, int NW>
__global__ void __launch_bounds__(64 * NW, NW == 4 ? 3 : 4) k_cp_bf16_multi(
    const SliceStep* __restrict__ sl, const int* __restrict__ blk_slice) {
  constexpr int LDA = 64 + 8, LDT = TR + 8;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[TR * LDA];
  __shared__ __attribute__((aligned(16))) uint16_t XsT[64 * LDT];
  __shared__ __attribute__((aligned(16))) uint16_t SsT[64 * LDT];
  __shared__ int wave_kept[NW];
  __shared__ __attribute__((aligned(16))) int2 ent[64 * NW];
  const SliceStep& d = sl[blk_slice[blockIdx.x]];
  const int blk = blockIdx.x - d.blk0;
#define TLDA_MULTI(DQ_, KQ_, G_)                                                               \
  case multi_shape_id(DQ_, KQ_, G_):                                                           \
    cp_bf16_block<DQ_, KQ_, G_, kFused, NW, TR>(blk, d.nblk, d.row_ptr, d.col_idx, d.val,       \
                                               d.n_rows, d.W16, d.mw16, d.Dh, nullptr, d.D,    \
                                               d.Phi, d.K, d.partial, d.block_counts, nullptr, \
                                               d.phi_copy, Xs, XsT, SsT, wave_kept, ent);       \
    break;
  switch (d.shape) {
    TLDA_MULTI(32, 16, 1) TLDA_MULTI(32, 16, 2) TLDA_MULTI(32, 16, 4)
    TLDA_MULTI(32, 32, 1) TLDA_MULTI(32, 32, 2) TLDA_MULTI(32, 32, 4)
    TLDA_MULTI(32, 64, 1) TLDA_MULTI(32, 64, 2) TLDA_MULTI(32, 64, 4)
    TLDA_MULTI(64, 16, 8) TLDA_MULTI(64, 32, 8) TLDA_MULTI(64, 64, 8)
    default: break;
  }
#undef TLDA_MULTI
}

struct Bf16Args {
  const tlda_csr_batch* b;
  int n_rows;
  const uint16_t* W16;
  const float* mw16;
  int Dh;
  const float* Xin;
  int D;
  const float* Phi;
  int K;
  int nblk;
  float* partial;
  int* block_counts;
  float* Xout;
  float* phi_copy;
  double* gsq;
};

template <int DQ, int KQ, int G, int MODE>
hipError_t launch_t(const Bf16Args& a, int* per_cu, hipStream_t s) {
  constexpr int kBlock = 64 * (MODE == kWhitenOnly ? 4 : bf16_waves(DQ, KQ));
  if (per_cu != nullptr)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_cp_bf16<DQ, KQ, G, MODE>,
                                                        kBlock, 0);
  const int32_t* rp = a.b ? a.b->row_ptr : nullptr;
  const int32_t* ci = a.b ? a.b->col_idx : nullptr;
  const float* va = a.b ? a.b->val : nullptr;
  launch_main(k_cp_bf16<DQ, KQ, G, MODE>, dim3(a.nblk), dim3(kBlock), 0, s, rp, ci, va,
              a.n_rows, a.W16, a.mw16, a.Dh, a.Xin, a.D, a.Phi, a.K, a.nblk, a.partial,
              a.block_counts, a.Xout, a.phi_copy, a.gsq);
  return hipGetLastError();
}

// Lanes per document G = Dh / 8: 1, 2 or 4 below 33 columns (DQ = 32), then
// 8 (DQ = 64) and 16 (DQ = 128).
template <int DQ, int KQ, int MODE>
hipError_t launch_g(int G, const Bf16Args& a, int* per_cu, hipStream_t s) {
  if constexpr (DQ == 32) {
    switch (G) {
      case 1: return launch_t<DQ, KQ, 1, MODE>(a, per_cu, s);
      case 2: return launch_t<DQ, KQ, 2, MODE>(a, per_cu, s);
      case 4: return launch_t<DQ, KQ, 4, MODE>(a, per_cu, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    if (G != DQ / 8) return hipErrorInvalidValue;
    return launch_t<DQ, KQ, DQ / 8, MODE>(a, per_cu, s);
  }
}

int dq_bucket(int D) { return D <= 32 ? 32 : D <= 64 ? 64 : 128; }
int kq_bucket(int K) { return K <= 16 ? 16 : K <= 32 ? 32 : K <= 64 ? 64 : 128; }

int bf16_cols_(int D) {
  int c = 8;
  while (c < D) c <<= 1;
  return c;
}

hipError_t dispatch(int mode, const Bf16Args& a, int* per_cu, hipStream_t s) {
  const int dq = dq_bucket(a.D), kq = kq_bucket(a.K);
  const int G = a.Dh / 8;
  if (mode == kWhitenOnly) {
    // the contraction shapes do not matter without the CP phases
    switch (G) {
      case 1: return launch_t<32, 16, 1, kWhitenOnly>(a, per_cu, s);
      case 2: return launch_t<32, 16, 2, kWhitenOnly>(a, per_cu, s);
      case 4: return launch_t<32, 16, 4, kWhitenOnly>(a, per_cu, s);
      case 8: return launch_t<32, 16, 8, kWhitenOnly>(a, per_cu, s);
      default: return launch_t<32, 16, 16, kWhitenOnly>(a, per_cu, s);
    }
  }
#define TLDA_BF16_SHAPE(DQ_, KQ_)                                                        \
  if (dq == DQ_ && kq == KQ_)                                                      \
    return mode == kFused ? launch_g<DQ_, KQ_, kFused>(G, a, per_cu, s)            \
                          : launch_g<DQ_, KQ_, kFromX>(G, a, per_cu, s);
#define TLDA_BF16_ROW(DQ_) TLDA_BF16_SHAPE(DQ_, 16) TLDA_BF16_SHAPE(DQ_, 32) TLDA_BF16_SHAPE(DQ_, 64) TLDA_BF16_SHAPE(DQ_, 128)
  TLDA_BF16_ROW(32) TLDA_BF16_ROW(64) TLDA_BF16_ROW(128)
#undef TLDA_BF16_ROW
#undef TLDA_BF16_SHAPE
  return hipErrorInvalidValue;
}

}  // namespace

int bf16_cols(int D) { return bf16_cols_(D); }

int multi_shape(int D, int K) {
  if (D < 1 || D > 64 || K < 1 || K > 64) return -1;
  const int dq = D <= 32 ? 32 : 64, kq = K <= 16 ? 16 : K <= 32 ? 32 : 64;
  return multi_shape_id(dq, kq, bf16_cols_(D) / 8);
}

// Tile shapes of the multi-slice kernel: (rows per tile, waves per block).
constexpr int kMultiShapes[kMultiTiles][2] = {{64, 4}, {32, 4}, {64, 8}};

int multi_tile_rows(int v) { return kMultiShapes[v][0]; }
int multi_tile_waves(int v) { return kMultiShapes[v][1]; }

int cp_bf16_multi_per_cu(int v) {
  int per_cu = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (v) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cp_bf16_multi<64, 4>, 256, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cp_bf16_multi<32, 4>, 256, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cp_bf16_multi<64, 8>, 512, 0); break;
    default: break;
  }
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu;
}

hipError_t launch_cp_bf16_multi(const SliceStep* sl, const int* blk_slice, int n_blocks, int v,
                                hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  switch (v) {
    case 0: hipLaunchKernelGGL((k_cp_bf16_multi<64, 4>), dim3(n_blocks), dim3(256), 0, s, sl, blk_slice); break;
    case 1: hipLaunchKernelGGL((k_cp_bf16_multi<32, 4>), dim3(n_blocks), dim3(256), 0, s, sl, blk_slice); break;
    case 2: hipLaunchKernelGGL((k_cp_bf16_multi<64, 8>), dim3(n_blocks), dim3(512), 0, s, sl, blk_slice); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool bf16_supported(int D, int K) { return D >= 1 && D <= 128 && K >= 1 && K <= 128; }

hipError_t launch_form_w16(const double* W, const double* m, int V, int D, int Dh, uint16_t* W16,
                           float* mw16, hipStream_t s) {
  const size_t n = (size_t)V * Dh;
  hipLaunchKernelGGL(k_form_w16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, V, D, Dh,
                     W16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mw16, dim3(Dh), dim3(256), 0, s, W16, m, V, D, Dh, mw16);
  return hipGetLastError();
}

int bf16_resident_blocks(int mode, int D, int K, int Dh, int num_cu) {
  Bf16Args a{};
  a.D = D;
  a.K = K;
  a.Dh = Dh;
  int per_cu = 0;
  if (dispatch(mode, a, &per_cu, nullptr) != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu * num_cu;
}

hipError_t launch_whiten_cp_bf16(const tlda_csr_batch& b, const uint16_t* W16, const float* mw16,
                                 int Dh, int D, const float* Phi, int K, int nblk, float* partial,
                                 int* block_counts, float* Xout, float* phi_copy, double* gsq,
                                 hipStream_t s) {
  Bf16Args a{&b,   b.n_rows, W16,          mw16, Dh,       nullptr, D, Phi, K,
             nblk, partial,  block_counts, Xout, phi_copy, gsq};
  return dispatch(kFused, a, nullptr, s);
}

hipError_t launch_cp_reduce_bf16(const float* X, int n_rows, const float* Phi, int D, int K,
                                 int nblk, float* partial, float* phi_copy, hipStream_t s) {
  Bf16Args a{nullptr, n_rows,  nullptr, nullptr, bf16_cols(D), X,       D,
             Phi,     K,       nblk,    partial, nullptr,      nullptr, phi_copy, nullptr};
  return dispatch(kFromX, a, nullptr, s);
}

hipError_t launch_whiten_bf16(const tlda_csr_batch& b, const uint16_t* W16, const float* mw16,
                              int Dh, int D, int nblk, float* X, int* block_counts,
                              hipStream_t s) {
  Bf16Args a{&b,   b.n_rows, W16,          mw16, Dh,     nullptr, D, nullptr, 1,
             nblk, nullptr,  block_counts, X,    nullptr, nullptr};
  return dispatch(kWhitenOnly, a, nullptr, s);
}

}  // namespace tlda
