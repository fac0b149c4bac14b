// Pair kernels: the O(P^2) Gaussian blob-kernel sums of the particle scheme.
//
// One pass computes, for every row particle I and a column weight vector wh,
//   O_I[n] = sum_J e_IJ V_J[n],   V_J = (wh_J x_J, wh_J),
//   e_IJ   = exp2(min(t_IJ, 0)),  t_IJ = -kappa |x_I - x_J|^2,  kappa = log2(e) / 2h^2,
// over all J including J = I (eq. model_DeteParAppr and the two kernel sums of
// eq. model_DymRepPar).  The squared distance is expanded through augmented
// vectors so that t_IJ is one dot product:
//   Q_I = (x_I, -kappa |x_I|^2, 1),  K_J = (2 kappa x_J, 1, -kappa |x_J|^2),
//   t_IJ = Q_I . K_J.
// The min(., 0) is the clamp of the expanded |x_I - x_J|^2 at zero.
//
// Two implementations share the operand arrays the prep kernel writes:
//  * MFMA: each wavefront owns RB blocks of 16 rows; per 16-column chunk,
//    ceil((D+2)/4) v_mfma_f32_16x16x4_f32 form t for a 16x16 pair tile, the
//    VALU takes exp2, and four more MFMAs accumulate e V.  The accumulator
//    layout of the first product is already the A-operand layout of the second
//    once the chunk's columns are visited in the order 4k + i, which is how the
//    prep kernel stores V.  Operands are pre-swizzled so every lane reads
//    consecutive dwords.
//  * VALU: one thread per row pair, column tiles of 256 staged in LDS, FP32
//    FMAs, v_exp_f32.
//  * MFMA, FP16-split product: t as above on FP32 MFMA, then the e V product
//    on v_mfma_f32_16x16x32_f16 with both factors split into two halves,
//    e = e_hi + e_lo and V = V_hi + V_lo, and e V taken as
//    e_hi V_hi + e_hi V_lo + e_lo V_hi (the dropped e_lo V_lo is 2^-22 of it).
//    Half products are exact in the FP32 accumulator, so the product keeps
//    about 22 bits against 24 for FP32, at three MFMAs per 32 columns instead
//    of eight.  FP16 has a narrow exponent range, so e is computed as
//    2^(t + 15) (the shift enters through the accumulator of the t product)
//    and the column weights in V are divided by their maximum; with e spanning
//    2^15 down to the FP16 subnormals, pairs as weak as 1e-12 of the strongest
//    still count.  The shift and the weight maximum are taken out in FP64 at
//    the end.
//  * MFMA, FP16-split products throughout: as the previous one, and t too on
//    v_mfma_f32_16x16x32_f16 from split halves of sqrt(2 kappa) x, with the
//    squared norms kept in FP32 (layout at pair_rows_f16).
// Column ranges are split over blockIdx.y; every split writes its own partial
// sums, reduced later in a fixed order (deterministic, no float atomics).
//
// Accuracy: the drift needs x_I S_I - M_I, a difference of two sums whose
// magnitudes can exceed it by an order of magnitude (narrow kernels, isolated
// particles).  Plain FP32 accumulation over thousands of columns would leave
// errors of ~1e-6 relative to the sums, amplified by that ratio.  So the FP32
// accumulators are flushed into FP64 running sums every kFlush chunks (16
// columns each), and the kernel itself forms, in FP64,
//   A_I[n] = x_I[n] O_I[D] - O_I[n]  (n < D),   O_I[D] = sum_J e_IJ wh_J,
// i.e. it writes sum_J e_IJ wh_J (x_I - x_J) and the weighted kernel sum.
// With exclude_self the J = I term is left out of both sums: it adds nothing to
// the difference sum, but for an isolated particle it dominates the kernel sum
// and would swamp its neighbours' contributions in FP32.  The caller adds the
// self weight back in FP64.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "vds_internal.h"

namespace vds {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kFlush = 8;  // chunks per FP32 accumulation group

// One wavefront: row blocks rb0 .. rb0 + RB - 1 against column chunks [c0, c1),
// results into out[row][16].  No barriers: waves are independent.
template <int KK, int RB>
__device__ void pair_rows(const float *__restrict__ QB, int nrow_blocks, const float *__restrict__ KA,
                          const float4 *__restrict__ VB, int c0, int c1, const float *__restrict__ xc, int D,
                          int exclude_self, float *__restrict__ out, int rb0) {
  if (rb0 >= nrow_blocks) return;
  const int lane = threadIdx.x & 63;
  // position of the self pair inside a diagonal 16x16 tile, per element i
  const int diag_i = (lane & 15) - 4 * (lane >> 4);  // in 0..3 when this lane holds one

  float qv[RB][KK];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
      qv[r][kk] = (rb0 + r < nrow_blocks) ? QB[((int64_t)(rb0 + r) * KK + kk) * 64 + lane] : 0.f;

  double tot[RB][4];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[r][i] = 0.0;

  float ka[KK];
  float4 vb;
  if (c0 < c1) {
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) ka[kk] = KA[((int64_t)c0 * KK + kk) * 64 + lane];
    vb = VB[(int64_t)c0 * 64 + lane];
  }
  for (int c = c0; c < c1;) {
    const int cg_end = min(c1, c + kFlush);
    floatx4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (; c < cg_end; ++c) {
      // prefetch the next chunk's operands while this one computes
      float kn[KK];
      float4 vn;
      const int cn = (c + 1 < c1) ? c + 1 : c;
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) kn[kk] = KA[((int64_t)cn * KK + kk) * 64 + lane];
      vn = VB[(int64_t)cn * 64 + lane];

#pragma unroll
      for (int r = 0; r < RB; ++r) {
        floatx4 t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) t = __builtin_amdgcn_mfma_f32_16x16x4f32(ka[kk], qv[r][kk], t, 0, 0, 0);
        // e = 2^t clamped to [0, 1] by the instruction's output clamp: the same as
        // clamping the expanded squared distance at zero
        float e0 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[0]), 0.f, 1.f);
        float e1 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[1]), 0.f, 1.f);
        float e2 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[2]), 0.f, 1.f);
        float e3 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[3]), 0.f, 1.f);
        if (exclude_self && c == rb0 + r) {  // scalar branch: the diagonal tile
          e0 = diag_i == 0 ? 0.f : e0;
          e1 = diag_i == 1 ? 0.f : e1;
          e2 = diag_i == 2 ? 0.f : e2;
          e3 = diag_i == 3 ? 0.f : e3;
        }
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(e0, vb.x, acc[r], 0, 0, 0);
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(e1, vb.y, acc[r], 0, 0, 0);
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(e2, vb.z, acc[r], 0, 0, 0);
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(e3, vb.w, acc[r], 0, 0, 0);
      }
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) ka[kk] = kn[kk];
      vb = vn;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) tot[r][i] += (double)acc[r][i];
  }

  // lane holds O[row 4 (lane / 16) + i][column lane % 16] of each row block;
  // the weighted kernel sum O[.][D] sits in lane (lane & 48) + D
  const int n = lane & 15;
  const int src = (lane & 48) + D;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (rb0 + r >= nrow_blocks) break;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double s = __shfl(tot[r][i], src);
      const int64_t row = (int64_t)(rb0 + r) * 16 + 4 * (lane >> 4) + i;
      double v = 0.0;
      if (n < D) v = (double)xc[row * D + n] * s - tot[r][i];
      else if (n == D) v = s;
      out[row * 16 + n] = (float)v;
    }
  }
}

template <int KK, int RB>
__global__ __launch_bounds__(256) void k_pair_mfma(const float *__restrict__ QB, int nrow_blocks,
                                                   const float *__restrict__ KA, const float4 *__restrict__ VB,
                                                   int ncol_chunks, int chunks_per_split,
                                                   const float *__restrict__ xc, int D, int exclude_self,
                                                   float *__restrict__ partial, int64_t part_stride_rows,
                                                   const int *__restrict__ done) {
  if (done != nullptr && *done) return;
  // wave index as a scalar so that row-block tests compile to scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rb0 = ((int)blockIdx.x * 4 + wave) * RB;
  const int c0 = (int)blockIdx.y * chunks_per_split;
  const int c1 = min(ncol_chunks, c0 + chunks_per_split);
  pair_rows<KK, RB>(QB, nrow_blocks, KA, VB, c0, c1, xc, D, exclude_self,
                    partial + (int64_t)blockIdx.y * part_stride_rows * 16, rb0);
}

// ---- FP32, 32x32 distance tiles and 4x4 sum blocks --------------------------
//
// On gfx950 the FP32 matrix instructions and the exponentials do not overlap
// (the VALU work of one wave and the MFMAs of another share the SIMD's issue),
// so a pass costs its MFMA cycles plus its exponential cycles and the MFMA
// work per pair-eval is what to cut.  This form issues, per 1024 pairs (a
// 32-row by 32-column tile):
//  * distances: ceil((D+2)/2) v_mfma_f32_32x32x2f32 over the augmented
//    vectors K_J = (2 kappa x_J, -kappa |x_J|^2, 1) and Q_I = (x_I, 1,
//    -kappa |x_I|^2) (D = 9: 6 instead of 12 16x16x4 steps; the row norm in a
//    K slot costs one 32x32x2 step, what setting every accumulator to it would
//    cost in moves, and no registers);
//  * kernel-weighted sums: 16 * ceil((D+1)/4) v_mfma_f32_4x4x1f32, whose 4x4
//    blocks need only ceil((D+1)/4) groups of four outputs (D = 9: 12 output
//    slots instead of the 16 of a 16x16 tile).
// Lane l of the distance product holds t[J][I] for I = l % 32 and the sixteen
// columns J = 8 (v / 4) + 4 (l / 32) + v % 4 of its registers v.  Taken as the
// A operand of a 4x4x1 product, register v gives block b = l / 4 the rows
// I = 4 (b % 8) + i and the single column J(b, v), which is the layout the
// sums need: block b accumulates O[I][4 g + j] over the columns of lane half
// b / 8, and the two halves are added at every FP64 flush (a permlane32 swap
// that leaves lane half h with rows i = h and i = 2 + h).
// The four waves of a workgroup take the same column chunks, which are staged
// once per workgroup in LDS, double buffered with one barrier per chunk.
// Accumulation: FP32 within groups of kFlush32 chunks (each lane half sums 128
// columns), then FP64, and the difference sums are formed in FP64 as for the
// other forms.

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kFlush32 = 8;  // 32-column chunks per FP32 accumulation group (128 columns per lane half)
constexpr int kStage32 = 2;  // 32-column chunks staged in LDS per barrier (divides kFlush32)

// v_permlane32_swap: exchanges lanes 32..63 of `a` with lanes 0..31 of `b`.
// Inline asm because __builtin_amdgcn_permlane32_swap is mistranslated by this
// compiler when its operands come from MFMA results (both results become the
// first operand).  The compiler does not account for the wait an MFMA result
// needs before a VALU instruction may read it when the reader is inline asm,
// so the asm waits 8 cycles itself (a 4x4x1 result needs fewer).
__device__ inline void permlane32_swap(float &a, float &b) {
  asm volatile("s_nop 7\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}

template <int D>
struct Mfma32Shape {
  static constexpr int KP = mfma32_kslots(D);  // K slots: D coordinates and the two norm terms, even
  static constexpr int NK = KP / 2;             // 32x32x2 steps of the distance product
  static constexpr int NG = (D + 4) / 4;        // four-wide output groups covering the D + 1 sums
  static constexpr int KF4 = KP * 8;            // float4s of a chunk's K operand (KP x 32 floats)
  static constexpr int VS = 5;                  // LDS float4 stride of one column's V (16 floats + 4 padding)
  static constexpr int LF4 = KF4 + 32 * VS;     // LDS float4s of one chunk buffer
  static constexpr int GF4 = KF4 + 128;         // float4s of one chunk in global memory
};

// Largest row-norm term kappa |x_I|^2 that a row block may fold out of the
// exponent (see mfma32_segment): e' <= 2^100, and a group of 128 products
// e' V stays far below the FP32 range.
constexpr float kFoldMax = 100.f;

// LDS of one workgroup of the FP32 32x32 form: staged chunks (double buffered)
// and the FP64 running sums of its four waves (one slot per lane and value;
// only its own lane touches a slot, so plain read-add-write keeps the
// summation order; held in LDS, they leave the registers to the arithmetic).
template <int D, int RB>
struct Mfma32Lds {
  float4 sb[2][kStage32 * Mfma32Shape<D>::LF4];
  double stot[4][RB][Mfma32Shape<D>::NG][2][64];
};

// Waves per SIMD the FP32 32x32 kernels are compiled for: four (128 VGPRs)
// where the workgroup's LDS lets four workgroups share a compute unit.
template <int D, int RB>
constexpr int mfma32_waves() {
  return sizeof(Mfma32Lds<D, RB>) <= 40960 ? 4 : 3;
}

// One segment of the FP32 32x32 form: the workgroup's four waves take row
// group rg (wave w: 32-row blocks (4 rg + w) RB ..), the columns of chunks
// [c0, c1), and write partial sums for their rows to out[row][W] (W >= D + 1).
// Every thread of the workgroup calls it with the same arguments (it holds
// barriers).  With run_len > 0 the segment is part of a run of run_len chunk
// units of which done0 came before it, and every stage sets the waves' issue
// priority by the share of the run still to do (see k_pair_mfma32).
template <int D, int RB, int W>
__device__ __forceinline__ void mfma32_segment(const float *__restrict__ xr, int nrb32, const float4 *__restrict__ KC,
                               const float4 *__restrict__ VC, int rg, int c0, int c1, int exclude_self, float kappa,
                               float *__restrict__ out, Mfma32Lds<D, RB> &lds, int64_t done0 = 0,
                               int64_t run_len = 0) {
  using S = Mfma32Shape<D>;
  // odd D: the last distance step holds only the row-norm slot and padding
  constexpr bool kFold = (D % 2) == 1;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int h = lane >> 5;   // lane half
  const int li = lane & 31;  // row of the 32x32 tile (distance product) / column slot of the K operand
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  auto &sb = lds.sb;
  double(*tot)[S::NG][2][64] = lds.stot[wave];
  constexpr int NST = (S::GF4 + 255) / 256;
  auto stage_dst = [&](int u) { return u < S::KF4 ? u : S::KF4 + ((u - S::KF4) >> 2) * S::VS + ((u - S::KF4) & 3); };
  auto chunk_src = [&](int c, int u) -> float4 {
    return u < S::KF4 ? KC[(int64_t)c * S::KF4 + u] : VC[(int64_t)c * 128 + (u - S::KF4)];
  };
  const int rb0 = (rg * 4 + wave) * RB;  // first 32-row block of this wave

  // row operands: slot 2 kk + h of row I is x_I[k] (k < D), 1 (k == D), the
  // row norm term -kappa |x_I|^2 (k == D + 1), 0 beyond.  With kFold, a wave
  // whose row-norm terms all lie within kFoldMax leaves out the last step (the
  // row-norm slot): its exponents are t + kappa |x_I|^2, and the factor
  // 2^(-kappa |x_I|^2) of each row is applied to its sums in FP64 at the end
  float qv[RB][S::NK];
  bool in_range = true;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rb = rb0 + r < nrb32 ? rb0 + r : 0;  // waves past the rows compute on row block 0, unwritten
    const float *x = xr + ((int64_t)rb * 32 + li) * D;
    float nrm = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) nrm = __builtin_fmaf(x[a], x[a], nrm);
    const float rn = -kappa * nrm;
#pragma unroll
    for (int kk = 0; kk < S::NK; ++kk) {
      const int k = 2 * kk + h;
      qv[r][kk] = k < D ? x[k < D ? k : 0] : (k == D ? 1.f : (k == D + 1 ? rn : 0.f));
    }
    in_range = in_range && rn >= -kFoldMax;
  }
  const int fold = kFold ? __builtin_amdgcn_readfirstlane(__all(in_range ? 1 : 0) ? 1 : 0) : 0;

  // thread t stages float4s t, t + 256, ... of a chunk: the K operand first,
  // then V into rows of VS float4s; a stage is kStage32 consecutive chunks,
  // one barrier each
#pragma unroll
  for (int cc = 0; cc < kStage32; ++cc) {
    if (c0 + cc < c1) {
#pragma unroll
      for (int i = 0; i < NST; ++i) {
        const int v = t + 256 * i;
        if (v < S::GF4) sb[0][cc * S::LF4 + stage_dst(v)] = chunk_src(c0 + cc, v);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int g = 0; g < S::NG; ++g) tot[r][g][0][lane] = tot[r][g][1][lane] = 0.0;
  __syncthreads();

  floatx4 acc[RB][S::NG];
  // one chunk of 32 columns from its LDS buffer; NKS distance steps
  auto chunk = [&](int c, const float4 *cb, auto nks) {
    constexpr int NKS = decltype(nks)::value;
    // per-lane bases; every read below is at a constant offset from them
    const float *sK = reinterpret_cast<const float *>(cb) + h * 32 + li;
    const float4 *sV = cb + S::KF4 + 4 * h * S::VS + (lane & 3);
    float ka[S::NK];
#pragma unroll
    for (int kk = 0; kk < S::NK; ++kk) ka[kk] = sK[kk * 64];
    floatx16 e[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int v = 0; v < 16; ++v) e[r][v] = 0.f;
#pragma unroll
      for (int kk = 0; kk < NKS; ++kk)
        e[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(ka[kk], qv[r][kk], e[r], 0, 0, 0);
      // no clamp: the expanded squared distance exceeds zero only by its rounding
#pragma unroll
      for (int v = 0; v < 16; ++v) e[r][v] = __builtin_amdgcn_exp2f(e[r][v]);
      if (exclude_self && c == rb0 + r) {  // scalar branch: the diagonal tile
        // an empty volatile asm keeps this a branch: if-converted into selects
        // it would cost sixteen VALU instructions on every tile
        asm volatile("" ::: "memory");
#pragma unroll
        for (int v = 0; v < 16; ++v) e[r][v] = (8 * (v >> 2) + 4 * h + (v & 3)) == li ? 0.f : e[r][v];
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float4 vv = sV[(8 * (v >> 2) + (v & 3)) * S::VS];
      const float vg[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int g = 0; g < S::NG; ++g)
          acc[r][g] = __builtin_amdgcn_mfma_f32_4x4x1f32(e[r][v], vg[g], acc[r][g], 0, 0, 0);
    }
  };

  // the chunk loop, in two copies (all steps, or the folded wave's NK - 1);
  // both pass the same barriers
  auto chunks = [&](auto nks) {
  for (int c = c0; c < c1;) {
    // groups start kFlush32 (a multiple of kStage32) chunks apart, so a stage
    // never crosses a group boundary
    const int gend = min(c1, c + kFlush32);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int g = 0; g < S::NG; ++g) acc[r][g] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (; c < gend; c += kStage32) {
      if (run_len > 0) {  // scalar: priority 3 while more than half the run is left, then 2, 1, 0 below 20 %, 5 %
        const int64_t rem = run_len - (done0 + (c - c0));
        if (20 * rem > 10 * run_len) __builtin_amdgcn_s_setprio(3);
        else if (20 * rem > 4 * run_len) __builtin_amdgcn_s_setprio(2);
        else if (20 * rem > run_len) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
      }
      const int buf = ((c - c0) / kStage32) & 1;
      const int cn = c + kStage32;  // first chunk of the next stage
      float4 pre[kStage32][NST];    // the next stage, stored after this one's arithmetic
#pragma unroll
      for (int cc = 0; cc < kStage32; ++cc)
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          const int v = t + 256 * i;
          pre[cc][i] = (cn + cc < c1 && v < S::GF4) ? chunk_src(cn + cc, v) : float4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
      for (int cc = 0; cc < kStage32; ++cc)
        if (c + cc < gend) chunk(c + cc, sb[buf] + cc * S::LF4, nks);
      if (cn < c1) {
#pragma unroll
        for (int cc = 0; cc < kStage32; ++cc)
#pragma unroll
          for (int i = 0; i < NST; ++i) {
            const int v = t + 256 * i;
            if (cn + cc < c1 && v < S::GF4) sb[buf ^ 1][cc * S::LF4 + stage_dst(v)] = pre[cc][i];
          }
      }
      // every stage ends at a barrier, the segment's last one too: the next
      // segment may overwrite either buffer
      __syncthreads();
    }
    // the two lane halves hold the same outputs over different columns: after a
    // swap of rows (0, 1) and one of rows (2, 3), each sum of the pair leaves
    // half h with the full row h and the full row 2 + h
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int g = 0; g < S::NG; ++g) {
        float a0 = acc[r][g][0], a1 = acc[r][g][1], a2 = acc[r][g][2], a3 = acc[r][g][3];
        permlane32_swap(a0, a1);
        permlane32_swap(a2, a3);
        tot[r][g][0][lane] += (double)(a0 + a1);
        tot[r][g][1][lane] += (double)(a2 + a3);
      }
  }
  };
  if (fold)  // scalar branch
    chunks(std::integral_constant<int, S::NK - 1>{});
  else
    chunks(std::integral_constant<int, S::NK>{});

  // lane l holds rows 4 ((l % 32) / 4) + h + 2 s (s = 0, 1) and outputs n = 4 g + l % 4;
  // the weighted kernel sum O[.][D] sits in the lane of the same quad with l % 4 = D % 4
  const int src = (lane & ~3) | (D & 3);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (rb0 + r >= nrb32) break;
#pragma unroll
    for (int sidx = 0; sidx < 2; ++sidx) {
      const int64_t row = (int64_t)(rb0 + r) * 32 + 4 * (li >> 2) + h + 2 * sidx;
      double f = 1.0;  // the factor a folded wave's sums still carry
      if (fold) {
        float nrm = 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) nrm = __builtin_fmaf(xr[row * D + a], xr[row * D + a], nrm);
        f = exp2((double)(-kappa * nrm));
      }
      const double sv = f * tot[r][D / 4][sidx][src];
#pragma unroll
      for (int g = 0; g < S::NG; ++g) {
        const int n = 4 * g + (lane & 3);
        if (n < D) out[row * W + n] = (float)((double)xr[row * D + n] * sv - f * tot[r][g][sidx][lane]);
        else if (n == D) out[row * W + n] = (float)sv;
      }
    }
  }
}

template <int D, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mfma32_waves<D, RB>()))) void k_pair_mfma32(
    const float *__restrict__ xr, int nrb32, const float4 *__restrict__ KC, const float4 *__restrict__ VC,
    SplitMap map, int exclude_self, float kappa, float *__restrict__ partial, int64_t part_stride_rows,
    const int *__restrict__ done) {
  __shared__ Mfma32Lds<D, RB> lds;
  if (done != nullptr && *done) return;  // the whole grid returns: no barrier is left waiting
  // workgroups go to the 8 XCDs round robin by linear id, and each XCD has its
  // own L2: with a multiple of 8 runs, XCD x takes the consecutive runs
  // x G / 8 .. (x + 1) G / 8 - 1, i.e. a band of row groups against all columns
  const int G = (int)gridDim.x;
  const int L = G % 8 == 0 ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int64_t nch = map.nch;
  const int64_t u_beg = map.run_start(L), u_end = map.run_start(L + 1);
  // Four workgroups share a compute unit, and its SIMDs issue for the oldest
  // ready wave first: left alone, the first workgroup placed runs ahead and
  // the four finish one after another (at about 60, 75, 90 and 100 % of the
  // pass), the last with one wave per SIMD to hide latency.  Each workgroup
  // therefore lowers its waves' priority as its run progresses
  // (mfma32_segment), so that the laggards are issued first and the four
  // finish together.
  // one segment per row group this run covers: chunks [c0, c1) of row group rg
  for (int64_t u = u_beg; u < u_end;) {
    const int64_t rg = u / nch;
    const int c0 = (int)(u - rg * nch);
    const int c1 = (int)min(nch, u_end - rg * nch);
    const int slot = (int)(L - map.run_of(rg * nch));
    u = rg * nch + c1;
    // slots in the compact layout: D + 1 floats per row
    mfma32_segment<D, RB, D + 1>(xr, nrb32, KC, VC, (int)rg, c0, c1, exclude_self, kappa,
                                 partial + (int64_t)slot * part_stride_rows * (D + 1), lds,
                                 rg * nch + c0 - u_beg, u_end - u_beg);
  }
}

// Batched form: a persistent grid walks the (ensemble, row group) items; each
// item takes all columns of its ensemble (one slot of partial sums).
template <int D, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mfma32_waves<D, RB>()))) void k_batch_pair32(
    const int2 *__restrict__ items, int nitems, const EnsDesc *__restrict__ ens, const float *__restrict__ xc,
    const float *__restrict__ KC, const float *__restrict__ VC, int KK, float *__restrict__ partial) {
  __shared__ Mfma32Lds<D, RB> lds;
  // this workgroup's chunks over all its items, for the issue priority by
  // progress (see k_pair_mfma32)
  int64_t total = 0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) total += (ens[items[it].x].p.P + 31) / 32;
  int64_t done = 0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const int64_t off = ens[item.x].pad_off;
    const int64_t P = ens[item.x].p.P;
    const int nrb32 = (int)(ens[item.x].p.Ppad / 32);
    const float kappa = ens[item.x].p.kappa;
    const int nc = (int)((P + 31) / 32);
    mfma32_segment<D, RB, 16>(xc + off * D, nrb32, reinterpret_cast<const float4 *>(KC + off * KK * 4),
                          reinterpret_cast<const float4 *>(VC + off * 16), item.y, 0, nc, 1, kappa,
                          partial + off * 16, lds, done, total);
    done += nc;
  }
}

// ---- FP16-split variant ----------------------------------------------------

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

constexpr float kF16Shift = 15.f;  // e = 2^(t + 15) <= 2^15 < FP16 max, t <= 0 up to rounding
constexpr int kFlushPairs = 4;     // chunk pairs (32 columns each) per FP32 group

// (a, b) -> hi = (a, b) rounded toward zero to FP16, lo = the remainders
// a - hi, b - hi (exact in FP32) rounded to nearest FP16.  `one` is 1.0 passed
// in at run time, so that the compiler keeps fma(-hi, one, a) and selects the
// mixed-precision FMA that reads the packed FP16 halves directly.
__device__ inline void split_pair(float a, float b, float one, half2v &hi, half2v &lo) {
  hi = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(a, b));
  const float ra = __builtin_fmaf(-(float)hi.x, one, a);
  const float rb = __builtin_fmaf(-(float)hi.y, one, b);
  lo = half2v{(_Float16)ra, (_Float16)rb};
}

__device__ inline half8 as_half8(uint4 u) {
  half8 h;
  __builtin_memcpy(&h, &u, sizeof(h));
  return h;
}

// One wavefront: row blocks rb0 .. rb0 + RB - 1 against column chunk pairs
// [p0, p1).  VH[cp * 64 + lane] holds, for lane = n + 16 g, the FP16 highs of
// V_J[n] for the eight columns J = 32 cp + 16 s + 4 g + i (slot 4 s + i) and
// VH[lo_off + cp * 64 + lane] the lows.  out_scale multiplies every sum.
//
// t comes from FP32 MFMAs over the QB/KA operands (KQ = 0, KK slices), or
// (KQ > 0) from KQ FP16 MFMAs of 32 products each over the QH/KH operands:
// with c = sqrt(2 kappa) and y = c x split into FP16 halves, slot 3k + (0, 1, 2)
// holds (y_I,hi y_J,hi, y_I,hi y_J,lo, y_I,lo y_J,hi) for component k, and
// slots 3D, 3D + 1 hold 16 times the two halves of -kappa |x_J|^2 / 16.  The
// row norm -kappa |x_I|^2 (RN) enters exactly, in FP32, through the
// accumulator's initial value.
template <int KK, int KQ, int RB>
__device__ __forceinline__ void pair_rows_f16(const float *__restrict__ QB, const uint4 *__restrict__ QH,
                              const float *__restrict__ RN, int nrow_blocks, const float *__restrict__ KA,
                              const uint4 *__restrict__ KH, const uint4 *__restrict__ VH, int64_t lo_off, int p0,
                              int p1, const float *__restrict__ xc, int D, int exclude_self, double out_scale,
                              float one, float *__restrict__ out, int rb0) {
  constexpr bool kQ16 = KQ > 0;
  constexpr int NK = kQ16 ? 1 : KK;  // FP32 operand slices (unused with FP16 distances)
  constexpr int NQ = kQ16 ? KQ : 1;  // FP16 operand slices (unused with FP32 distances)
  if (rb0 >= nrow_blocks) return;
  const int lane = threadIdx.x & 63;
  const int diag_i = (lane & 15) - 4 * (lane >> 4);

  float qv[RB][NK];
  half8 qh[RB][NQ];
  float rinit[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const bool ok = rb0 + r < nrow_blocks;
    if constexpr (kQ16) {
#pragma unroll
      for (int m = 0; m < KQ; ++m)
        qh[r][m] = as_half8(ok ? QH[((int64_t)(rb0 + r) * KQ + m) * 64 + lane] : uint4{0, 0, 0, 0});
      rinit[r] = (ok ? RN[(int64_t)(rb0 + r) * 16 + (lane & 15)] : 0.f) + kF16Shift;
    } else {
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) qv[r][kk] = ok ? QB[((int64_t)(rb0 + r) * KK + kk) * 64 + lane] : 0.f;
      rinit[r] = kF16Shift;
    }
  }

  double tot[RB][4];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[r][i] = 0.0;

  // Operands of one chunk pair (32 columns): distance operands of its two
  // 16-column slices and the V highs and lows.  Two of them alternate so that
  // the loads of the next chunk pair overlap this one's arithmetic without
  // register copies; addresses are a wave-uniform base plus the lane offset.
  struct ColOps {
    float fa[2][NK];
    uint4 ha[2][NQ];
    uint4 h, l;
  };
  auto load_cols = [&](int cp, ColOps &o) {
    if constexpr (kQ16) {
      const uint4 *kb = KH + (int64_t)(2 * cp) * KQ * 64;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int m = 0; m < KQ; ++m) o.ha[s][m] = kb[(s * KQ + m) * 64 + lane];
    } else {
      const float *kb = KA + (int64_t)(2 * cp) * KK * 64;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) o.fa[s][kk] = kb[(s * KK + kk) * 64 + lane];
    }
    const uint4 *vb = VH + (int64_t)cp * 64;
    o.h = vb[lane];
    o.l = vb[lo_off + lane];
  };
  floatx4 acc[RB];
  auto compute = [&](int cp, const ColOps &o) {
    const half8 h8 = as_half8(o.h), l8 = as_half8(o.l);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      float e[8];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        floatx4 t = {rinit[r], rinit[r], rinit[r], rinit[r]};
        if constexpr (kQ16) {
#pragma unroll
          for (int m = 0; m < KQ; ++m)
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_half8(o.ha[s][m]), qh[r][m], t, 0, 0, 0);
        } else {
#pragma unroll
          for (int kk = 0; kk < KK; ++kk) t = __builtin_amdgcn_mfma_f32_16x16x4f32(o.fa[s][kk], qv[r][kk], t, 0, 0, 0);
        }
        // no clamp: e exceeds 2^15 only by the rounding of t, and the RTZ
        // conversion of the split saturates at the FP16 maximum
#pragma unroll
        for (int i = 0; i < 4; ++i) e[4 * s + i] = __builtin_amdgcn_exp2f(t[i]);
      }
      if (exclude_self && (2 * cp == rb0 + r || 2 * cp + 1 == rb0 + r)) {  // scalar branch: diagonal tile
        // an empty volatile asm keeps this a branch: if-converted into
        // selects it would cost four VALU instructions on every tile
        asm volatile("" ::: "memory");
        const int sd = 2 * cp == rb0 + r ? 0 : 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) e[sd + i] = diag_i == i ? 0.f : e[sd + i];
      }
      half8 eh, el;
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        half2v h, l;
        split_pair(e[j], e[j + 1], one, h, l);
        eh[j] = h.x;
        eh[j + 1] = h.y;
        el[j] = l.x;
        el[j + 1] = l.y;
      }
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh, h8, acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh, l8, acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_f16(el, h8, acc[r], 0, 0, 0);
    }
  };
  ColOps b0, b1;
  if (p0 < p1) load_cols(p0, b0);
  // groups of kFlushPairs (even) chunk pairs, so every group but the last
  // starts with its operands in b0; loads past the end re-read the last
  // chunk pair
  for (int cp = p0; cp < p1;) {
    const int g_end = min(p1, cp + kFlushPairs);
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (; cp < g_end; cp += 2) {
      load_cols(min(cp + 1, p1 - 1), b1);
      compute(cp, b0);
      if (cp + 1 < g_end) {
        load_cols(min(cp + 2, p1 - 1), b0);
        compute(cp + 1, b1);
      }
    }
    cp = g_end;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) tot[r][i] += (double)acc[r][i];
  }

  const int n = lane & 15;
  const int src = (lane & 48) + D;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (rb0 + r >= nrow_blocks) break;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double s = __shfl(tot[r][i], src);
      const int64_t row = (int64_t)(rb0 + r) * 16 + 4 * (lane >> 4) + i;
      double v = 0.0;
      if (n < D) v = ((double)xc[row * D + n] * s - tot[r][i]) * out_scale;
      else if (n == D) v = s * out_scale;
      out[row * 16 + n] = (float)v;
    }
  }
}

// Operands of the FP16-split pair pass.
struct PairF16Ops {
  const float *QB, *KA;   // FP32 distance operands (FP32 distances)
  const uint4 *QH, *KH;   // FP16 distance operands (FP16 distances)
  const float *RN;        // row norms -kappa |x_I|^2 (FP16 distances)
  const uint4 *VH;        // V highs, then lows at lo_off
  int64_t lo_off;
};

template <int KK, int KQ, int RB>
__global__ __launch_bounds__(256, 4) void k_pair_mfma16(PairF16Ops ops, int nrow_blocks, int ncol_pairs,
                                                     int pairs_per_split, const float *__restrict__ xc, int D,
                                                     int exclude_self, const float *__restrict__ wscale, float one,
                                                     float *__restrict__ partial, int64_t part_stride_rows,
                                                     const int *__restrict__ done) {
  if (done != nullptr && *done) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rb0 = ((int)blockIdx.x * 4 + wave) * RB;
  const int p0 = (int)blockIdx.y * pairs_per_split;
  const int p1 = min(ncol_pairs, p0 + pairs_per_split);
  const double scale = (wscale != nullptr ? (double)*wscale : 1.0) * 0x1p-15;
  pair_rows_f16<KK, KQ, RB>(ops.QB, ops.QH, ops.RN, nrow_blocks, ops.KA, ops.KH, ops.VH, ops.lo_off, p0, p1, xc, D,
                            exclude_self, scale, one, partial + (int64_t)blockIdx.y * part_stride_rows * 16, rb0);
}

// Batched ensembles: a persistent grid walks a static list of (ensemble, row
// tile) items, sorted by decreasing cost, each over all of its ensemble's
// columns (one split).  Operands of ensemble e start at padded particle
// ens[e].pad_off of the concatenated arrays.
template <int KK, int RB>
__global__ __launch_bounds__(256) void k_batch_pair(const int2 *__restrict__ items, int nitems,
                                                    const EnsDesc *__restrict__ ens, const float *__restrict__ QB,
                                                    const float *__restrict__ KA, const float4 *__restrict__ VB,
                                                    const float *__restrict__ xc, int D, float *__restrict__ partial) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const int64_t off = ens[item.x].pad_off;
    const int64_t P = ens[item.x].p.P;
    const int nrb = (int)(ens[item.x].p.Ppad / 16);
    const int ncc = (int)((P + 15) / 16);
    const int rb0 = (item.y * 4 + wave) * RB;
    pair_rows<KK, RB>(QB + off * KK * 4, nrb, KA + off * KK * 4, VB + off * 4, 0, ncc, xc + off * D, D, 1,
                      partial + off * 16, rb0);
  }
}

// VALU variant.  D is the configuration dimension; the augmented length is D + 2.
// FP32 accumulation over 64 columns, then FP64 running sums (see above).
template <int D>
__global__ __launch_bounds__(256) void k_pair_valu(const float *__restrict__ QB, int64_t nrows,
                                                   const float *__restrict__ KA, const float *__restrict__ VB,
                                                   int64_t ncol_chunks, int64_t chunks_per_split, int exclude_self,
                                                   float *__restrict__ partial, int64_t part_stride_rows,
                                                   const int *__restrict__ done) {
  constexpr int KA_LEN = D + 2;
  constexpr int KK = (D + 2 + 3) / 4;
  constexpr int NV = D + 1;
  constexpr int RT = 2;
  __shared__ float sK[KA_LEN][256];
  __shared__ float sV[NV][256];
  if (done != nullptr && *done) return;

  const int tid = threadIdx.x;
  int64_t rows[RT];
  float q[RT][KA_LEN];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    rows[r] = (int64_t)blockIdx.x * (256 * RT) + r * 256 + tid;
    const int64_t I = rows[r] < nrows ? rows[r] : 0;
#pragma unroll
    for (int k = 0; k < KA_LEN; ++k)
      q[r][k] = QB[((I >> 4) * KK + (k >> 2)) * 64 + (I & 15) + 16 * (k & 3)];
  }
  double tot[RT][NV];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int n = 0; n < NV; ++n) tot[r][n] = 0.0;

  const int64_t c0 = (int64_t)blockIdx.y * chunks_per_split;
  const int64_t c1 = min(ncol_chunks, c0 + chunks_per_split);
  for (int64_t tile = c0; tile < c1; tile += 16) {
    const int64_t c = tile + (tid >> 4);
    const int jj = tid & 15;
    if (c < c1) {
#pragma unroll
      for (int k = 0; k < KA_LEN; ++k) sK[k][tid] = KA[(c * KK + (k >> 2)) * 64 + jj + 16 * (k & 3)];
#pragma unroll
      for (int n = 0; n < NV; ++n) sV[n][tid] = VB[(c * 64 + (jj >> 2) * 16 + n) * 4 + (jj & 3)];
    } else {
#pragma unroll
      for (int k = 0; k < KA_LEN; ++k) sK[k][tid] = 0.f;
#pragma unroll
      for (int n = 0; n < NV; ++n) sV[n][tid] = 0.f;
    }
    __syncthreads();
    for (int j0 = 0; j0 < 256; j0 += 64) {
      float acc[RT][NV];
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int n = 0; n < NV; ++n) acc[r][n] = 0.f;
      for (int j = j0; j < j0 + 64; ++j) {
        const int64_t col = tile * 16 + j;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          float t = 0.f;
#pragma unroll
          for (int k = 0; k < KA_LEN; ++k) t = fmaf(q[r][k], sK[k][j], t);
          float e = __builtin_amdgcn_exp2f(fminf(t, 0.f));
          if (exclude_self && col == rows[r]) e = 0.f;
#pragma unroll
          for (int n = 0; n < NV; ++n) acc[r][n] = fmaf(e, sV[n][j], acc[r][n]);
        }
      }
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int n = 0; n < NV; ++n) tot[r][n] += (double)acc[r][n];
    }
    __syncthreads();
  }
  float *out = partial + (int64_t)blockIdx.y * part_stride_rows * 16;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    if (rows[r] >= nrows) continue;
    const double s = tot[r][D];
#pragma unroll
    for (int n = 0; n < D; ++n) out[rows[r] * 16 + n] = (float)((double)q[r][n] * s - tot[r][n]);
    out[rows[r] * 16 + D] = (float)s;
  }
}

// Batched FP16-split variant over the same work list.  Pass A's V holds the
// weights 1/P_e over their maximum 1/P_e, so its sums are scaled by 1/P_e.
template <int KK, int KQ, int RB>
__global__ __launch_bounds__(256) void k_batch_pair16(const int2 *__restrict__ items, int nitems,
                                                      const EnsDesc *__restrict__ ens, PairF16Ops ops, int pass_a,
                                                      const float *__restrict__ xc, int D, float one,
                                                      float *__restrict__ partial) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const EnsDesc &d = ens[item.x];
    const int64_t off = d.pad_off;
    const int nrb = (int)(d.p.Ppad / 16);
    const int ncp = (int)((d.p.P + 31) / 32);
    const int rb0 = (item.y * 4 + wave) * RB;
    const double scale = (pass_a ? (double)d.p.uniform_w : 1.0) * 0x1p-15;
    const int64_t qoff = (off / 16) * KQ * 64;  // uint4 units of the distance operands
    pair_rows_f16<KK, KQ, RB>(ops.QB + off * KK * 4, ops.QH + qoff, ops.RN + off, nrb, ops.KA + off * KK * 4,
                              ops.KH + qoff, ops.VH + off * 4, d.p.Ppad * 2, 0, ncp, xc + off * D, D, 1, scale,
                              one, partial + off * 16, rb0);
  }
}

template <int KK, int KQ>
static void launch_batch16_k(int rb, int grid, const int2 *items, int nitems, const EnsDesc *ens,
                             const PairF16Ops &ops, int pass_a, const float *xc, int D, float *partial,
                             hipStream_t s) {
  switch (rb) {
    case 1: k_batch_pair16<KK, KQ, 1><<<grid, 256, 0, s>>>(items, nitems, ens, ops, pass_a, xc, D, 1.f, partial); break;
    case 2: k_batch_pair16<KK, KQ, 2><<<grid, 256, 0, s>>>(items, nitems, ens, ops, pass_a, xc, D, 1.f, partial); break;
    default: k_batch_pair16<KK, KQ, 4><<<grid, 256, 0, s>>>(items, nitems, ens, ops, pass_a, xc, D, 1.f, partial); break;
  }
}

template <int KK>
static void launch_batch_kk(int rb, int grid, const int2 *items, int nitems, const EnsDesc *ens, const float *QB,
                            const float *KA, const float *VB, const float *xc, int D, float *partial, hipStream_t s) {
  const float4 *vb = reinterpret_cast<const float4 *>(VB);
  switch (rb) {
    case 1: k_batch_pair<KK, 1><<<grid, 256, 0, s>>>(items, nitems, ens, QB, KA, vb, xc, D, partial); break;
    case 2: k_batch_pair<KK, 2><<<grid, 256, 0, s>>>(items, nitems, ens, QB, KA, vb, xc, D, partial); break;
    default: k_batch_pair<KK, 4><<<grid, 256, 0, s>>>(items, nitems, ens, QB, KA, vb, xc, D, partial); break;
  }
}

template <int D>
static void launch_batch32_d(int rb, int grid, const int2 *items, int nitems, const EnsDesc *ens, const float *xc,
                             const float *KC, const float *VC, int KK, float *partial, hipStream_t s) {
  if (rb == 1)
    k_batch_pair32<D, 1><<<grid, 256, 0, s>>>(items, nitems, ens, xc, KC, VC, KK, partial);
  else
    k_batch_pair32<D, 2><<<grid, 256, 0, s>>>(items, nitems, ens, xc, KC, VC, KK, partial);
}

void launch_batch_pair(int impl, int rb, int grid, int KK, int D, const int2 *items, int nitems, const EnsDesc *ens,
                       const float *QB, const float *KA, const float *VB, const F16Operands &f16, bool pass_a,
                       const float *xc, float *partial, hipStream_t s) {
  if (impl == VDS_PAIR_MFMA32) {
    switch (D) {
      case 3: launch_batch32_d<3>(rb, grid, items, nitems, ens, xc, KA, VB, KK, partial, s); break;
      case 6: launch_batch32_d<6>(rb, grid, items, nitems, ens, xc, KA, VB, KK, partial, s); break;
      case 9: launch_batch32_d<9>(rb, grid, items, nitems, ens, xc, KA, VB, KK, partial, s); break;
      case 12: launch_batch32_d<12>(rb, grid, items, nitems, ens, xc, KA, VB, KK, partial, s); break;
      default: launch_batch32_d<15>(rb, grid, items, nitems, ens, xc, KA, VB, KK, partial, s); break;
    }
    return;
  }
  if (impl == VDS_PAIR_MFMA_F16X2 || impl == VDS_PAIR_MFMA_F16X2_ALL) {
    const PairF16Ops ops{QB, KA, reinterpret_cast<const uint4 *>(f16.QH), reinterpret_cast<const uint4 *>(f16.KH),
                         f16.RN, reinterpret_cast<const uint4 *>(VB), 0};
    const int pa = pass_a ? 1 : 0;
    if (impl == VDS_PAIR_MFMA_F16X2_ALL) {
      if (f16_slices(D) == 1) launch_batch16_k<0, 1>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s);
      else launch_batch16_k<0, 2>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s);
    } else {
      switch (KK) {
        case 2: launch_batch16_k<2, 0>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s); break;
        case 3: launch_batch16_k<3, 0>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s); break;
        case 4: launch_batch16_k<4, 0>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s); break;
        default: launch_batch16_k<5, 0>(rb, grid, items, nitems, ens, ops, pa, xc, D, partial, s); break;
      }
    }
    return;
  }
  switch (KK) {
    case 2: launch_batch_kk<2>(rb, grid, items, nitems, ens, QB, KA, VB, xc, D, partial, s); break;
    case 3: launch_batch_kk<3>(rb, grid, items, nitems, ens, QB, KA, VB, xc, D, partial, s); break;
    case 4: launch_batch_kk<4>(rb, grid, items, nitems, ens, QB, KA, VB, xc, D, partial, s); break;
    default: launch_batch_kk<5>(rb, grid, items, nitems, ens, QB, KA, VB, xc, D, partial, s); break;
  }
}

bool pair_shape_ok(const vds_tuning &t, int D) {
  if (D < 3 || D > kMaxD || D % 3 != 0) return false;
  if (t.col_splits < 1 || t.col_splits > kMaxSplits) return false;
  if (t.impl == VDS_PAIR_MFMA || t.impl == VDS_PAIR_MFMA_F16X2 || t.impl == VDS_PAIR_MFMA_F16X2_ALL)
    return t.rows_per_wave == 1 || t.rows_per_wave == 2 || t.rows_per_wave == 4;
  if (t.impl == VDS_PAIR_MFMA32) return t.rows_per_wave == 1 || t.rows_per_wave == 2;
  return t.impl == VDS_PAIR_VALU;
}

template <int KK>
static void launch_mfma_kk(int rb, dim3 grid, const float *QB, int nrb, const float *KA, const float *VB,
                           int ncc, int cps, const float *xc, int D, int ex, float *partial, int64_t stride,
                           const int *done, hipStream_t s) {
  const float4 *vb = reinterpret_cast<const float4 *>(VB);
  switch (rb) {
    case 1: k_pair_mfma<KK, 1><<<grid, 256, 0, s>>>(QB, nrb, KA, vb, ncc, cps, xc, D, ex, partial, stride, done); break;
    case 2: k_pair_mfma<KK, 2><<<grid, 256, 0, s>>>(QB, nrb, KA, vb, ncc, cps, xc, D, ex, partial, stride, done); break;
    default: k_pair_mfma<KK, 4><<<grid, 256, 0, s>>>(QB, nrb, KA, vb, ncc, cps, xc, D, ex, partial, stride, done); break;
  }
}

template <int KK, int KQ>
static void launch_mfma16_k(int rb, dim3 grid, const PairF16Ops &ops, int nrb, int ncp, int pps, const float *xc,
                            int D, int ex, const float *wscale, float *partial, int64_t stride, const int *done,
                            hipStream_t s) {
  switch (rb) {
    case 1: k_pair_mfma16<KK, KQ, 1><<<grid, 256, 0, s>>>(ops, nrb, ncp, pps, xc, D, ex, wscale, 1.f, partial, stride, done); break;
    case 2: k_pair_mfma16<KK, KQ, 2><<<grid, 256, 0, s>>>(ops, nrb, ncp, pps, xc, D, ex, wscale, 1.f, partial, stride, done); break;
    default: k_pair_mfma16<KK, KQ, 4><<<grid, 256, 0, s>>>(ops, nrb, ncp, pps, xc, D, ex, wscale, 1.f, partial, stride, done); break;
  }
}

template <int D>
static void launch_mfma32_d(int rb, const float *xr, int nrb32, const float *KC, const float *VC, const SplitMap &map,
                            int ex, float kappa, float *partial, int64_t stride, const int *done, hipStream_t s) {
  const float4 *kc = reinterpret_cast<const float4 *>(KC), *vc = reinterpret_cast<const float4 *>(VC);
  const dim3 grid((unsigned)map.G);
  if (rb == 1)
    k_pair_mfma32<D, 1><<<grid, 256, 0, s>>>(xr, nrb32, kc, vc, map, ex, kappa, partial, stride, done);
  else
    k_pair_mfma32<D, 2><<<grid, 256, 0, s>>>(xr, nrb32, kc, vc, map, ex, kappa, partial, stride, done);
}

// Compute units of the current device (256 on MI355X), looked up once per
// device (host threads may race to fill a slot; they store the same value).
int device_cu_count() {
  constexpr int kDevs = 64;
  static std::atomic<int> cache[kDevs];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

SplitMap pair_split_map(const vds_tuning &t, int D, int64_t nrow_blocks, int64_t ncol_chunks) {
  SplitMap m;
  if (t.impl != VDS_PAIR_MFMA32) {
    m.splits = t.col_splits;
    return m;
  }
  m.width = D + 1;  // the compact layout
  // rows in blocks of 32, four waves of RB blocks per row group; columns in chunks of 32
  const int rb = t.rows_per_wave;
  const int64_t nrb32 = nrow_blocks / 2;
  m.rows_per_group = 4 * rb * 32;
  m.n_rg = (nrb32 + 4 * rb - 1) / (4 * rb);
  m.nch = (ncol_chunks + 1) / 2;
  m.splits = kMaxSplits;
  // col_splits workgroups per compute unit; runs of at least qmin units, so
  // that at most kMaxSplits runs meet in one row group
  const int64_t U = m.units();
  const int64_t qmin = (m.nch + kMaxSplits - 2) / (kMaxSplits - 1);
  int64_t G = std::min<int64_t>((int64_t)t.col_splits * device_cu_count(), U / qmin);
  if (G >= 8) G -= G % 8;
  m.G = (int)std::max<int64_t>(G, 1);
  return m;
}

void launch_pair_pass(const vds_tuning &t, int KK, int D, const float *QB, int64_t nrow_blocks, const float *KA,
                      const float *VB, int64_t ncol_chunks, int64_t ncol_pad, const float *xc, bool exclude_self,
                      const float *wscale, const F16Operands &f16, float *partial, int64_t part_stride_rows,
                      const int *done, hipStream_t s, float kappa) {
  const int ex = exclude_self ? 1 : 0;
  const int splits = t.col_splits;
  const int64_t cps = (ncol_chunks + splits - 1) / splits;
  if (t.impl == VDS_PAIR_MFMA32) {
    // rows in blocks of 32 (nrow_blocks counts 16-row blocks of a multiple of 256 rows, so
    // every row group of 4 waves x RB blocks is whole); columns in chunks of 32, the last
    // inside the padding (ncol_pad is a multiple of 256 columns), whose weights are zero
    const SplitMap map = pair_split_map(t, D, nrow_blocks, ncol_chunks);
    const int rb = t.rows_per_wave;
    const int nrb32 = (int)(nrow_blocks / 2);
    switch (D) {
      case 3: launch_mfma32_d<3>(rb, QB, nrb32, KA, VB, map, ex, kappa, partial, part_stride_rows, done, s); break;
      case 6: launch_mfma32_d<6>(rb, QB, nrb32, KA, VB, map, ex, kappa, partial, part_stride_rows, done, s); break;
      case 9: launch_mfma32_d<9>(rb, QB, nrb32, KA, VB, map, ex, kappa, partial, part_stride_rows, done, s); break;
      case 12: launch_mfma32_d<12>(rb, QB, nrb32, KA, VB, map, ex, kappa, partial, part_stride_rows, done, s); break;
      default: launch_mfma32_d<15>(rb, QB, nrb32, KA, VB, map, ex, kappa, partial, part_stride_rows, done, s); break;
    }
    return;
  }
  if (t.impl == VDS_PAIR_MFMA_F16X2 || t.impl == VDS_PAIR_MFMA_F16X2_ALL) {
    // chunk pairs; the second chunk of the last pair lies inside the padding
    // (ncol_pad is a multiple of 32 columns), whose V is zero
    const int64_t ncp = (ncol_chunks + 1) / 2;
    const int64_t pps = (ncp + splits - 1) / splits;
    PairF16Ops ops{QB, KA, reinterpret_cast<const uint4 *>(f16.QH), reinterpret_cast<const uint4 *>(f16.KH), f16.RN,
                   reinterpret_cast<const uint4 *>(VB), ncol_pad / 32 * 64};  // lows follow the highs
    const int rb = t.rows_per_wave;
    dim3 grid((unsigned)((nrow_blocks + 4 * rb - 1) / (4 * rb)), (unsigned)splits);
    const int nrb = (int)nrow_blocks, np = (int)ncp, pp = (int)pps;
    if (t.impl == VDS_PAIR_MFMA_F16X2_ALL) {
      if (f16_slices(D) == 1)
        launch_mfma16_k<0, 1>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s);
      else
        launch_mfma16_k<0, 2>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s);
    } else {
      switch (KK) {
        case 2: launch_mfma16_k<2, 0>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s); break;
        case 3: launch_mfma16_k<3, 0>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s); break;
        case 4: launch_mfma16_k<4, 0>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s); break;
        default: launch_mfma16_k<5, 0>(rb, grid, ops, nrb, np, pp, xc, D, ex, wscale, partial, part_stride_rows, done, s); break;
      }
    }
  } else if (t.impl == VDS_PAIR_MFMA) {
    const int rb = t.rows_per_wave;
    dim3 grid((unsigned)((nrow_blocks + 4 * rb - 1) / (4 * rb)), (unsigned)splits);
    switch (KK) {
      case 2: launch_mfma_kk<2>(rb, grid, QB, (int)nrow_blocks, KA, VB, (int)ncol_chunks, (int)cps, xc, D, ex, partial, part_stride_rows, done, s); break;
      case 3: launch_mfma_kk<3>(rb, grid, QB, (int)nrow_blocks, KA, VB, (int)ncol_chunks, (int)cps, xc, D, ex, partial, part_stride_rows, done, s); break;
      case 4: launch_mfma_kk<4>(rb, grid, QB, (int)nrow_blocks, KA, VB, (int)ncol_chunks, (int)cps, xc, D, ex, partial, part_stride_rows, done, s); break;
      default: launch_mfma_kk<5>(rb, grid, QB, (int)nrow_blocks, KA, VB, (int)ncol_chunks, (int)cps, xc, D, ex, partial, part_stride_rows, done, s); break;
    }
  } else {
    const int64_t nrows = nrow_blocks * 16;
    dim3 grid((unsigned)((nrows + 511) / 512), (unsigned)splits);
    switch (D) {
      case 3: k_pair_valu<3><<<grid, 256, 0, s>>>(QB, nrows, KA, VB, ncol_chunks, cps, ex, partial, part_stride_rows, done); break;
      case 6: k_pair_valu<6><<<grid, 256, 0, s>>>(QB, nrows, KA, VB, ncol_chunks, cps, ex, partial, part_stride_rows, done); break;
      case 9: k_pair_valu<9><<<grid, 256, 0, s>>>(QB, nrows, KA, VB, ncol_chunks, cps, ex, partial, part_stride_rows, done); break;
      case 12: k_pair_valu<12><<<grid, 256, 0, s>>>(QB, nrows, KA, VB, ncol_chunks, cps, ex, partial, part_stride_rows, done); break;
      default: k_pair_valu<15><<<grid, 256, 0, s>>>(QB, nrows, KA, VB, ncol_chunks, cps, ex, partial, part_stride_rows, done); break;
    }
  }
}

}  // namespace vds
