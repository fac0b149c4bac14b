// Galerkin reduced model of the particle scheme (C ABI of include/vds_pod.h).
//
// Per freeze: reconstruct q~ = U p, run the two kernel passes at q~ for
// S = Z w and T = Z (w/S), form Y = Z [w U_a | (w/S) U_a]_a with the kernel
// matrix generated tile by tile on MFMA (never stored), then contract with the
// mode blocks into X^B1 and X^B2.  Between freezes a single workgroup takes the
// explicit Euler steps of the reduced equation.  Midpoint freezes add a second
// freeze per window, at the state half a window on.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include <rocblas/rocblas.h>

#include "vds_ctx.h"
#include "vds_linalg.h"
#include "vds_pod.h"

using namespace vds;

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr int kMaxR = 1024;
constexpr int kNBG = 8;       // 16-column output blocks per workgroup of the kernel-GEMM
constexpr int kKgFlush = 8;   // chunks per FP32 accumulation group
constexpr int kK32Waves = 8;  // waves (32-row blocks) per workgroup of the FP32 32x32 kernel-GEMM
constexpr int kK32MaxNB = 4;  // its column blocks of 32 per workgroup: 1 to 4 (B holds 4 slots per lane and row)
// floats of one (row group, column group) output tile with nb column blocks
constexpr int kgemm32_tile(int nb) { return kK32Waves * 32 * 32 * nb; }

// (row group, column group) items of the FP32 kernel-GEMM with nb column blocks
int64_t kgemm32_items(int64_t Ppad, int ncols, int nb) {
  return (Ppad / 32 + kK32Waves - 1) / kK32Waves * ((ncols + 32 * nb - 1) / (32 * nb));
}

// Runs (workgroups) of the FP32 kernel-GEMM's balanced grid for Ppad rows and
// ncols output columns: two per compute unit (one round), at most one per
// (row group, column group) item, so that no item spans more than two runs;
// a multiple of 8 from 8 on (consecutive runs share an XCD).
int kgemm32_runs(int64_t Ppad, int ncols, int nb) {
  int64_t G = std::min<int64_t>(2 * (int64_t)device_cu_count(), kgemm32_items(Ppad, ncols, nb));
  if (G >= 8) G -= G % 8;
  return (int)std::max<int64_t>(G, 1);
}

// Column blocks per workgroup: the count whose issue cycles per run are fewest.
// Per chunk of an item, the distance product and the exponentials cost
// 64 NK + 128 cycles and each column block 16 x 64; columns past ncols in the
// last group are computed too.  Wide groups amortise the distances (at
// P = 20000, R = 180: four blocks); where the items are fewer than the runs a
// full round would hold (small P), narrow groups give more, shorter runs.
int kgemm32_nb(int64_t Ppad, int ncols, int D) {
  const double ko = 64.0 * (mfma32_kslots(D) / 2) + 128.0;
  int best = kK32MaxNB;
  double best_cost = 0.0;
  for (int nb = kK32MaxNB; nb >= 1; --nb) {
    const double items = (double)kgemm32_items(Ppad, ncols, nb);
    const double cost = items * (ko + 1024.0 * nb) / kgemm32_runs(Ppad, ncols, nb);
    if (nb == kK32MaxNB || cost < best_cost) {
      best = nb;
      best_cost = cost;
    }
  }
  return best;
}

struct RomLayout {
  size_t Ude, Mbig, XH, I1, XB1, XB2, XB, Bsw, Y, qt, T, invS, part, red, psave, pprev, total;
  int NB16;
  int64_t ldy;
  int kg_nb;    // column blocks per workgroup of the FP32 kernel-GEMM
  int kg_runs;  // runs of its balanced grid (its continuation slots are sized for them)
};

RomLayout rom_layout(const vds_problem &p, int R) {
  RomLayout L{};
  const int64_t P = p.P, Ppad = round_up(P, kRowAlign);
  const int ncols = 2 * 3 * R;
  L.NB16 = (ncols + 15) / 16;
  L.ldy = (int64_t)L.NB16 * 16;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  L.Ude = take(sizeof(float) * 3 * (size_t)R * P);
  L.Mbig = take(sizeof(float) * 9 * (size_t)R * R);
  L.XH = take(sizeof(float) * R * R);
  L.I1 = take(sizeof(float) * R * R);
  L.XB1 = take(sizeof(float) * R * R);
  L.XB2 = take(sizeof(float) * R * R);
  L.XB = take(sizeof(float) * R * R);
  // B of the kernel-GEMM: the 16-column swizzled layout, or that of the 32x32 form
  L.kg_nb = kgemm32_nb(Ppad, ncols, 3 * p.nb);
  const int64_t ncg32 = (ncols + 32 * L.kg_nb - 1) / (32 * L.kg_nb);
  L.Bsw = take(sizeof(float) * (size_t)Ppad * std::max<int64_t>(L.ldy, ncg32 * 128));
  L.Y = take(sizeof(float) * (size_t)Ppad * L.ldy);
  L.qt = take(sizeof(float) * (size_t)p.nb * P * 3);
  L.T = take(sizeof(float) * Ppad);
  L.invS = take(sizeof(float) * Ppad);
  const int64_t m = 3 * P;
  // (the GEMMs' split partials, or the kernel-GEMM's continuation tiles: one per run)
  L.kg_runs = kgemm32_runs(Ppad, ncols, L.kg_nb);
  const size_t part = std::max({sizeof(float) * (size_t)gemm_splits(3 * R, 3 * R, P) * 9 * R * R,
                                sizeof(float) * (size_t)gemm_splits(R, R, P) * R * R,
                                sizeof(float) * (size_t)m * p.nb,
                                sizeof(float) * (size_t)L.kg_runs * kgemm32_tile(L.kg_nb)});
  L.part = take(part);
  L.red = take(sizeof(double) * 16);
  L.psave = take(sizeof(float) * (size_t)p.nb * R);
  L.pprev = take(sizeof(float) * (size_t)p.nb * R);
  L.total = off;
  return L;
}

// Ude[a][s][I] = U[s m + 3 I + a]: the mode blocks U_a, K-contiguous over I.
__global__ void k_deinterleave(const float *__restrict__ U, int64_t P, int R, float *__restrict__ Ude) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 3 * (int64_t)R * P) return;
  const int64_t I = t % P;
  const int64_t rest = t / P;
  const int s = (int)(rest % R), a = (int)(rest / R);
  Ude[t] = U[(int64_t)s * 3 * P + 3 * I + a];
}

// X^H = sum_ab G_ab M_ab and I1 = sum_a M_aa from Mbig[(a R + s)][(b R + t)].
__global__ void k_hydro(const float *__restrict__ Mbig, int R, EvalParams p, float *__restrict__ XH,
                        float *__restrict__ I1) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)R * R) return;
  const int s = (int)(t / R), u = (int)(t % R);
  const int64_t ld = 3 * (int64_t)R;
  float h = 0.f, id = 0.f;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const float m = Mbig[(a * (int64_t)R + s) * ld + b * R + u];
      h += p.G[3 * a + b] * m;
      if (a == b) id += m;
    }
  XH[t] = h;
  I1[t] = id;
}

// T_I = w_I / S_I + sum_{K != I} (w_K / S_K) e_IK from the pass-B partials, and 1/S.
__global__ void k_rom_scalars(const float *__restrict__ part, SplitMap splits, int64_t Ppad, int64_t P, int D,
                              const float *__restrict__ S, const float *__restrict__ wv, float *__restrict__ T,
                              float *__restrict__ invS) {
  const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (I >= Ppad) return;
  if (I >= P) {
    T[I] = 0.f;
    invS[I] = 0.f;
    return;
  }
  const double o = ordered_sum<double>(part + I * splits.width + D, splits.count(I), Ppad * splits.width);
  const double Si = (double)S[I];
  T[I] = (float)(o + (double)wv[I] / Si);
  invS[I] = (float)(1.0 / Si);
}

// Kernel-GEMM right operand B[J][col], col = h dR + a R + t:
// (h = 0: w_J, h = 1: w_J / S_J) * U_a[t][J], in the swizzled MFMA layout
// Bsw[((c NB16 + nbk) 64 + lane) 4 + i] = B[16 c + 4 (lane / 16) + i][16 nbk + lane % 16].
__global__ void k_rom_bsw(const float *__restrict__ Ude, const float *__restrict__ wv, const float *__restrict__ invS,
                          int64_t P, int64_t Ppad, int R, int NB16, float *__restrict__ Bsw) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ldy = (int64_t)NB16 * 16;
  if (t >= Ppad * ldy) return;
  const int64_t J = t / ldy;
  const int col = (int)(t % ldy);
  const int dR = 3 * R;
  float v = 0.f;
  if (J < P && col < 2 * dR) {
    const int h = col / dR, rem = col % dR, a = rem / R, tt = rem % R;
    const float wgt = h == 0 ? wv[J] : wv[J] * invS[J];
    v = wgt * Ude[((int64_t)a * R + tt) * P + J];
  }
  const int64_t c = J >> 4;
  const int jj = (int)(J & 15);
  const int lane = 16 * (jj >> 2) + (col & 15);
  const int nbk = col >> 4;
  Bsw[((c * NB16 + nbk) * 64 + lane) * 4 + (jj & 3)] = v;
}

// Y[I][col] = sum_J Z_IJ B[J][col], Z_IJ = exp(-|x_I - x_J|^2 / 2h^2) (Z_II = 1),
// from the Q/K operands of the pair kernels.  One 16-row block per wavefront,
// kNBG 16-column output blocks per workgroup; FP32 accumulation flushed to FP64.
template <int KK>
__global__ __launch_bounds__(256) void k_kernel_gemm(const float *__restrict__ QB, const float *__restrict__ KA,
                                                     int nrow_blocks, int ncol_chunks,
                                                     const float4 *__restrict__ Bsw, int NB16,
                                                     float *__restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rb = (int)blockIdx.x * 4 + wave;
  if (rb >= nrow_blocks) return;
  const int nb0 = (int)blockIdx.y * kNBG;
  const int nbn = min(kNBG, NB16 - nb0);
  const int diag_i = (lane & 15) - 4 * (lane >> 4);
  float qv[KK];
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) qv[kk] = QB[((int64_t)rb * KK + kk) * 64 + lane];
  double tot[kNBG][4];
#pragma unroll
  for (int g = 0; g < kNBG; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[g][i] = 0.0;

  for (int c = 0; c < ncol_chunks;) {
    const int cg_end = min(ncol_chunks, c + kKgFlush);
    floatx4 acc[kNBG];
#pragma unroll
    for (int g = 0; g < kNBG; ++g) acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (; c < cg_end; ++c) {
      floatx4 t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < KK; ++kk)
        t = __builtin_amdgcn_mfma_f32_16x16x4f32(KA[((int64_t)c * KK + kk) * 64 + lane], qv[kk], t, 0, 0, 0);
      float e0 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[0]), 0.f, 1.f);
      float e1 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[1]), 0.f, 1.f);
      float e2 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[2]), 0.f, 1.f);
      float e3 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(t[3]), 0.f, 1.f);
      if (c == rb) {  // the self pair has Z_II = K_h(0) = 1 exactly
        e0 = diag_i == 0 ? 1.f : e0;
        e1 = diag_i == 1 ? 1.f : e1;
        e2 = diag_i == 2 ? 1.f : e2;
        e3 = diag_i == 3 ? 1.f : e3;
      }
      const float4 *bp = Bsw + ((int64_t)c * NB16 + nb0) * 64 + lane;
#pragma unroll
      for (int g = 0; g < kNBG; ++g) {
        if (g < nbn) {
          const float4 b = bp[(int64_t)g * 64];
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(e0, b.x, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(e1, b.y, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(e2, b.z, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(e3, b.w, acc[g], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kNBG; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) tot[g][i] += (double)acc[g][i];
  }
#pragma unroll
  for (int g = 0; g < kNBG; ++g) {
    if (g >= nbn) break;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = (int64_t)rb * 16 + 4 * (lane >> 4) + i;
      Y[row * ldy + (int64_t)(nb0 + g) * 16 + (lane & 15)] = (float)tot[g][i];
    }
  }
}

// ---- FP32 kernel-GEMM on 32x32 tiles (the operands of VDS_PAIR_MFMA32) -----
//
// Y[I][col] = sum_J Z_IJ B[J][col] with a workgroup of kK32Waves waves owning
// kK32Waves 32-row blocks (256 rows) and NB column blocks of 32 (32 NB
// columns; NB from 1 to 4 by the problem's size).  Per chunk of 32 columns of
// Z it stages the chunk's B block and the K operand of its distance product
// (the pair kernel's per-chunk KC layout) in LDS once, double buffered with one
// barrier.  Each wave forms its
// 32x32 piece of Z on v_mfma_f32_32x32x2_f32 from the centred row coordinates
// (Z_II = 1 set exactly) and multiplies it by the staged B block on the same
// instruction: the distance product leaves lane l with row I = l % 32 and, in
// register v, column J = 8 (v / 4) + 4 (l / 32) + v % 4, which is the A-operand
// layout of step v of the product over J.  B of step v for column block nb
// sits in lane l at row J(v, l / 32), column 32 nb + l % 32.  FP32
// accumulation over all columns of Z (as the FP16-split form: ~1e-6 of the
// sums).
// B of the FP32 32x32 kernel-GEMM, one block of 32 rows J x 32 NB columns per
// (chunk c, column group cg): element (jj, col = 32 NB cg + 32 nb + l) at
// [((c NCG + cg) 32 + jj) 128 + 4 l + nb], one float4 per lane and row
// (slots nb >= NB are zero).
__global__ void k_rom_b32(const float *__restrict__ Ude, const float *__restrict__ wv, const float *__restrict__ invS,
                          int64_t P, int64_t Ppad, int R, int NCG, int NB, float *__restrict__ Bk) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= Ppad * NCG * 128) return;
  const int e = (int)(t & 127);
  const int64_t blk = t >> 7;  // (c NCG + cg) 32 + jj
  const int jj = (int)(blk & 31);
  const int64_t cb = blk >> 5;
  const int cg = (int)(cb % NCG);
  const int64_t J = (cb / NCG) * 32 + jj;
  const int l = e >> 2, nb = e & 3;
  const int col = cg * 32 * NB + 32 * nb + l;
  const int dR = 3 * R;
  float v = 0.f;
  if (nb < NB && J < P && col < 2 * dR) {
    const int h = col / dR, rem = col % dR, a = rem / R, tt = rem % R;
    const float wgt = h == 0 ? wv[J] : wv[J] * invS[J];
    v = wgt * Ude[((int64_t)a * R + tt) * P + J];
  }
  Bk[t] = v;
}

// Balanced grid: the (column group, row group) items, column-group major,
// times their nch chunks, cut into G equal runs (one workgroup each; at most
// one run per item, so an item meets at most two runs).  A run's segment that
// starts an item writes the item's output tile to Y; a run whose first segment
// continues an item begun by the previous run writes that part to its slot,
// slots[L] (kgemm32_tile(NB) floats: 256 rows x 32 NB columns), which
// k_kgemm32_fixup then adds to Y.  Consecutive runs share an XCD (and its L2's
// B blocks).
template <int D, int NB>
__global__ __launch_bounds__(kK32Waves * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_kernel_gemm32(
    const float *__restrict__ xr, int nrb32, const float4 *__restrict__ KC, int nch, const float4 *__restrict__ Bk,
    int NCG, int ncols, float kappa, float *__restrict__ Y, int64_t ldy, float *__restrict__ slots) {
  constexpr int KP = mfma32_kslots(D), NK = KP / 2;
  constexpr int KF4 = KP * 8;             // float4s of a chunk's K operand
  constexpr int BF4 = 32 * 128 / 4;       // float4s of a chunk's B block
  constexpr int SF4 = KF4 + BF4;          // float4s staged per chunk
  constexpr int NST = (SF4 + kK32Waves * 64 - 1) / (kK32Waves * 64);
  __shared__ float4 sb[2][SF4];
  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, li = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int n_rg = (nrb32 + kK32Waves - 1) / kK32Waves;
  const int64_t U = (int64_t)NCG * n_rg * nch;
  const int G = (int)gridDim.x;
  const int L = G % 8 == 0 ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int64_t u_beg = (int64_t)L * U / G, u_end = (int64_t)(L + 1) * U / G;
  // the segments that start an item first (every run's first segment then
  // starts at chunk 0, so the runs of a column group read its B blocks nearly
  // in step through their XCD's L2), a continued item's part last
  const int64_t i_first = u_beg / nch;
  const bool continued = u_beg > i_first * nch;
  const int64_t i_lo = continued ? i_first + 1 : i_first;
  const int64_t n_seg = (u_end - 1) / nch - i_lo + 1 + (continued ? 1 : 0);
  const int64_t run_len = u_end - u_beg;
  int64_t seg_done = 0;  // units of the run in the segments before this one
  for (int64_t sgi = 0; sgi < n_seg; ++sgi) {
    const int64_t item = continued && sgi == n_seg - 1 ? i_first : i_lo + sgi;
    const int c0 = (int)(max(u_beg, item * nch) - item * nch);
    const int c1 = (int)(min(u_end, (item + 1) * nch) - item * nch);
    const int cg = (int)(item / n_rg);
    const int rb = (int)(item % n_rg) * kK32Waves + wave;  // this wave's 32-row block
    // row operands: slot 2 kk + h of row I is x_I[k] (k < D), 1 (k == D), the
    // row norm term (k == D + 1), 0 beyond
    float qv[NK];
    {
      const int rr = rb < nrb32 ? rb : 0;  // waves past the rows compute on block 0, unwritten
      const float *x = xr + ((int64_t)rr * 32 + li) * D;
      float nrm = 0.f;
#pragma unroll
      for (int a = 0; a < D; ++a) nrm = __builtin_fmaf(x[a], x[a], nrm);
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const int k = 2 * kk + h;
        qv[kk] = k < D ? x[k < D ? k : 0] : (k == D ? 1.f : (k == D + 1 ? -kappa * nrm : 0.f));
      }
    }
    auto src = [&](int c, int uu) -> float4 {
      return uu < KF4 ? KC[(int64_t)c * KF4 + uu] : Bk[((int64_t)c * NCG + cg) * BF4 + (uu - KF4)];
    };
    float4 pre[NST];
#pragma unroll
    for (int i = 0; i < NST; ++i) {
      const int uu = t + kK32Waves * 64 * i;
      if (uu < SF4) sb[0][uu] = src(c0, uu);
    }
    __syncthreads();
    floatx16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
    for (int c = c0; c < c1; ++c) {
      {  // scalar: issue priority by the share of the run still to do, so that the
         // two workgroups of a CU finish together (the SIMDs issue for the oldest
         // ready wave first): 3 above half, then 2, 1, 0 below 20 %, 5 %
        const int64_t rem = run_len - (seg_done + (c - c0));
        if (20 * rem > 10 * run_len) __builtin_amdgcn_s_setprio(3);
        else if (20 * rem > 4 * run_len) __builtin_amdgcn_s_setprio(2);
        else if (20 * rem > run_len) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
      }
      const int buf = (c - c0) & 1;
      if (c + 1 < c1) {
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          const int uu = t + kK32Waves * 64 * i;
          pre[i] = uu < SF4 ? src(c + 1, uu) : float4{0.f, 0.f, 0.f, 0.f};
        }
      }
      const float *sK = reinterpret_cast<const float *>(sb[buf]) + h * 32 + li;
      const float4 *sB = sb[buf] + KF4 + h * 128 + li;  // row J(v, h) = 8 (v / 4) + 4 h + v % 4
      floatx16 z;
#pragma unroll
      for (int v = 0; v < 16; ++v) z[v] = 0.f;
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) z = __builtin_amdgcn_mfma_f32_32x32x2f32(sK[kk * 64], qv[kk], z, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) z[v] = __builtin_amdgcn_exp2f(z[v]);
      if (c == rb) {  // scalar branch: the self pair has Z_II = K_h(0) = 1 exactly
        asm volatile("" ::: "memory");
#pragma unroll
        for (int v = 0; v < 16; ++v) z[v] = (8 * (v >> 2) + 4 * h + (v & 3)) == li ? 1.f : z[v];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float4 b = sB[(8 * (v >> 2) + (v & 3)) * 32];
        const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(z[v], bv[nb], acc[nb], 0, 0, 0);
      }
      if (c + 1 < c1) {
#pragma unroll
        for (int i = 0; i < NST; ++i) {
          const int uu = t + kK32Waves * 64 * i;
          if (uu < SF4) sb[buf ^ 1][uu] = pre[i];
        }
      }
      // every chunk ends at a barrier, the segment's last one too: the next
      // segment's first stage overwrites buffer 0
      __syncthreads();
    }
    // output lane l, register v: row 32 rb + 8 (v / 4) + 4 h + v % 4, column 32 NB cg + 32 nb + li.
    // The output addresses are formed here: formed ahead of the chunk loop
    // (they do not depend on it) they stay live across it and spill.
    float *ybase = Y, *sbase = slots;
    int64_t ld = ldy;
    int el = lane;
    asm volatile("" : "+s"(ybase), "+s"(sbase), "+s"(ld), "+v"(el));
    const int eh = el >> 5, eli = el & 31;
    if (c0 > 0) {  // a continued item: the whole tile to this run's slot
      float *o = sbase + (int64_t)L * kgemm32_tile(NB) + (wave * 32 + 4 * eh) * (32 * NB) + eli;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) o[(8 * (v >> 2) + (v & 3)) * (32 * NB) + 32 * nb] = acc[nb][v];
    } else if (rb < nrb32) {
      float *o = ybase + ((int64_t)rb * 32 + 4 * eh) * ld + cg * 32 * NB + eli;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (cg * 32 * NB + 32 * nb + eli >= ncols) break;
#pragma unroll
        for (int v = 0; v < 16; ++v) o[(8 * (v >> 2) + (v & 3)) * ld + 32 * nb] = acc[nb][v];
      }
    }
    seg_done += c1 - c0;
  }
}

// Y += the slot of every run whose first segment continued an item (block
// (x, L): elements x 256 .. of run L's tile).  An item meets at most two runs,
// so no two slots add to the same tile.
__global__ void k_kgemm32_fixup(const float *__restrict__ slots, int nrb32, int nch, int NCG, int NB, int ncols,
                                float *__restrict__ Y, int64_t ldy) {
  const int L = (int)blockIdx.y, G = (int)gridDim.y;
  const int n_rg = (nrb32 + kK32Waves - 1) / kK32Waves;
  const int64_t U = (int64_t)NCG * n_rg * nch;
  const int64_t u0 = (int64_t)L * U / G;
  const int64_t item = u0 / nch;
  if (u0 == item * nch) return;  // the run starts its first item
  const int cg = (int)(item / n_rg), rg = (int)(item % n_rg);
  const int e = (int)blockIdx.x * 256 + threadIdx.x;
  const int tile = kgemm32_tile(NB);
  if (e >= tile) return;
  const int r = e / (32 * NB), cc = e % (32 * NB);
  const int64_t row = (int64_t)rg * 32 * kK32Waves + r;
  const int col = cg * 32 * NB + cc;
  if (row < (int64_t)nrb32 * 32 && col < ncols) Y[row * ldy + col] += slots[(int64_t)L * tile + e];
}

struct KGemm32Args {
  const float *xr;
  int nrb32;
  const float4 *KC;
  int nch;
  const float4 *Bk;
  int NCG, ncols;
  float kappa;
  float *Y;
  int64_t ldy;
  float *slots;
};

template <int D>
void launch_kgemm32(int NB, int G, const KGemm32Args &a, hipStream_t s) {
  const dim3 grid((unsigned)G), block(kK32Waves * 64);
  switch (NB) {
    case 1: k_kernel_gemm32<D, 1><<<grid, block, 0, s>>>(a.xr, a.nrb32, a.KC, a.nch, a.Bk, a.NCG, a.ncols, a.kappa, a.Y, a.ldy, a.slots); break;
    case 2: k_kernel_gemm32<D, 2><<<grid, block, 0, s>>>(a.xr, a.nrb32, a.KC, a.nch, a.Bk, a.NCG, a.ncols, a.kappa, a.Y, a.ldy, a.slots); break;
    case 3: k_kernel_gemm32<D, 3><<<grid, block, 0, s>>>(a.xr, a.nrb32, a.KC, a.nch, a.Bk, a.NCG, a.ncols, a.kappa, a.Y, a.ldy, a.slots); break;
    default: k_kernel_gemm32<D, 4><<<grid, block, 0, s>>>(a.xr, a.nrb32, a.KC, a.nch, a.Bk, a.NCG, a.ncols, a.kappa, a.Y, a.ldy, a.slots); break;
  }
}

// ---- FP16-split kernel-GEMM (used with the FP16-split pair kernels) ---------
//
// The same product with Z and B split into FP16 halves and taken on
// v_mfma_f32_16x16x32_f16 as Z_hi B_hi + Z_hi B_lo + Z_lo B_hi (about 22
// significant bits).  Z enters as 2^15 Z and B as 2^8 B' with B' = U_a for the
// w-weighted columns (uniform weights over their maximum) and (w/S) U_a for the
// others; the epilogue multiplies column col by scale0 (col < 3R) or scale1.

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
constexpr float kKgShift = 15.f;
constexpr float kKgBScale = 256.f;
constexpr int kKgFlushPairs = 4;

// BH[((cp NB16 + nbk) 64 + n + 16 g) 8 + 4 s + i] = high half of B[32 cp + 16 s + 4 g + i][16 nbk + n];
// the low halves follow after Ppad ldy halves.
__global__ void k_rom_bsw16(const float *__restrict__ Ude, const float *__restrict__ wv,
                            const float *__restrict__ invS, float wmax, int64_t P, int64_t Ppad, int R, int NB16,
                            _Float16 *__restrict__ BH) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ldy = (int64_t)NB16 * 16;
  if (t >= Ppad * ldy) return;
  const int64_t J = t / ldy;
  const int col = (int)(t % ldy);
  const int dR = 3 * R;
  float v = 0.f;
  if (J < P && col < 2 * dR) {
    const int h = col / dR, rem = col % dR, a = rem / R, tt = rem % R;
    const float wgt = h == 0 ? wv[J] / wmax : wv[J] * invS[J];
    v = kKgBScale * wgt * Ude[((int64_t)a * R + tt) * P + J];
  }
  const int jl = (int)(J & 15);
  const int64_t idx = (((J >> 5) * NB16 + (col >> 4)) * 64 + (col & 15) + 16 * (jl >> 2)) * 8 + 4 * ((J >> 4) & 1) +
                      (jl & 3);
  const _Float16 hi = (_Float16)v;
  BH[idx] = hi;
  BH[idx + Ppad * ldy] = (_Float16)(v - (float)hi);
}

__device__ inline half8 as_half8(uint4 u) {
  half8 h;
  __builtin_memcpy(&h, &u, sizeof(h));
  return h;
}

template <int KK>
__global__ __launch_bounds__(256) void k_kernel_gemm16(const float *__restrict__ QB, const float *__restrict__ KA,
                                                       int nrow_blocks, int ncol_chunks,
                                                       const uint4 *__restrict__ BH, int64_t lo_off, int NB16,
                                                       int dR, double scale0, double scale1, float one,
                                                       float *__restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rb = (int)blockIdx.x * 4 + wave;
  if (rb >= nrow_blocks) return;
  const int nb0 = (int)blockIdx.y * kNBG;
  const int nbn = min(kNBG, NB16 - nb0);
  const int diag_i = (lane & 15) - 4 * (lane >> 4);
  const int ncp = (ncol_chunks + 1) / 2;  // the last pair's second chunk lies in the zero padding
  float qv[KK];
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) qv[kk] = QB[((int64_t)rb * KK + kk) * 64 + lane];
  double tot[kNBG][4];
#pragma unroll
  for (int g = 0; g < kNBG; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[g][i] = 0.0;
  const floatx4 shift = {kKgShift, kKgShift, kKgShift, kKgShift};

  for (int cp = 0; cp < ncp;) {
    const int g_end = min(ncp, cp + kKgFlushPairs);
    floatx4 acc[kNBG];
#pragma unroll
    for (int g = 0; g < kNBG; ++g) acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (; cp < g_end; ++cp) {
      float e[8];
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
        const int c = 2 * cp + sc;
        floatx4 t = shift;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
          t = __builtin_amdgcn_mfma_f32_16x16x4f32(KA[((int64_t)c * KK + kk) * 64 + lane], qv[kk], t, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) e[4 * sc + i] = fminf(__builtin_amdgcn_exp2f(t[i]), 32768.f);
        if (c == rb) {  // the self pair has Z_II = K_h(0) = 1 exactly
#pragma unroll
          for (int i = 0; i < 4; ++i) e[4 * sc + i] = diag_i == i ? 32768.f : e[4 * sc + i];
        }
      }
      half8 eh, el;
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const half2v h = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(e[j], e[j + 1]));
        const float ra = __builtin_fmaf(-(float)h.x, one, e[j]);
        const float rb2 = __builtin_fmaf(-(float)h.y, one, e[j + 1]);
        eh[j] = h.x;
        eh[j + 1] = h.y;
        el[j] = (_Float16)ra;
        el[j + 1] = (_Float16)rb2;
      }
      const uint4 *bp = BH + ((int64_t)cp * NB16 + nb0) * 64 + lane;
#pragma unroll
      for (int g = 0; g < kNBG; ++g) {
        if (g < nbn) {
          const half8 bh = as_half8(bp[(int64_t)g * 64]);
          const half8 bl = as_half8(bp[lo_off + (int64_t)g * 64]);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh, bh, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh, bl, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(el, bh, acc[g], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kNBG; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) tot[g][i] += (double)acc[g][i];
  }
#pragma unroll
  for (int g = 0; g < kNBG; ++g) {
    if (g >= nbn) break;
    const int col = (nb0 + g) * 16 + (lane & 15);
    const double sc = col < dR ? scale0 : scale1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = (int64_t)rb * 16 + 4 * (lane >> 4) + i;
      Y[row * ldy + col] = (float)(tot[g][i] * sc);
    }
  }
}

// The same product with FP16-split distances (the pair kernels' QH/KH/RN
// operands), tiled for reuse: a workgroup of kLdsWaves waves owns
// kLdsWaves x 2 row blocks (256 rows) and kNBG column blocks (128 columns);
// per chunk pair (32 columns of Z) it stages the chunk's B highs and lows and
// its K-side distance operands in LDS once (double buffered, one barrier), and
// every wave generates its two 16 x 32 tiles of Z and multiplies them by all
// kNBG column blocks.  Each B element is thus read once per 256 rows instead
// of once per 16.  FP32 accumulation over all columns of Z (no FP64 flush: 64
// accumulators per lane already; the error stays ~1e-6 of the sums).
constexpr int kLdsWaves = 8;
constexpr int kLdsRB = 2;

// (at most 128 VGPRs, so that two workgroups share a CU: 2.5 instead of
// 3.0 ms per launch at P = 20000, 1080 columns)
template <int KQ>
__global__ __launch_bounds__(kLdsWaves * 64, 4) void k_kernel_gemm16_lds(
    const uint4 *__restrict__ QH, const uint4 *__restrict__ KH, const float *__restrict__ RN, int nrow_blocks,
    int ncp, const uint4 *__restrict__ BH, int64_t lo_off, int NB16, int dR, double scale0, double scale1,
    float one, float *__restrict__ Y, int64_t ldy) {
  __shared__ uint4 bsh[2][2 * kNBG * 64];
  __shared__ uint4 ksh[2][2 * KQ * 64];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int rb0 = ((int)blockIdx.x * kLdsWaves + wave) * kLdsRB;
  const int nb0 = (int)blockIdx.y * kNBG;
  const int nbn = min(kNBG, NB16 - nb0);
  const int diag_i = (lane & 15) - 4 * (lane >> 4);
  half8 qh[kLdsRB][KQ];
  float rinit[kLdsRB];
#pragma unroll
  for (int r = 0; r < kLdsRB; ++r) {
    const bool ok = rb0 + r < nrow_blocks;
#pragma unroll
    for (int m = 0; m < KQ; ++m)
      qh[r][m] = as_half8(ok ? QH[((int64_t)(rb0 + r) * KQ + m) * 64 + lane] : uint4{0, 0, 0, 0});
    rinit[r] = (ok ? RN[(int64_t)(rb0 + r) * 16 + (lane & 15)] : 0.f) + kKgShift;
  }
  floatx4 acc[kLdsRB][kNBG];
#pragma unroll
  for (int r = 0; r < kLdsRB; ++r)
#pragma unroll
    for (int g = 0; g < kNBG; ++g) acc[r][g] = floatx4{0.f, 0.f, 0.f, 0.f};

  // tile loads: thread t < kNBG 64 takes B high and low element t of the
  // chunk's kNBG x 64 uint4 (zero past the last column block) and, for
  // t < 2 KQ 64, distance operand t
  const int gt = t >> 6;
  static_assert(kNBG <= kLdsWaves && 2 * 2 <= kLdsWaves, "one tile element per thread");
  auto load_tile = [&](int cp, uint4 &bh, uint4 &bl, uint4 &kh) {
    const int64_t bo = ((int64_t)cp * NB16 + nb0) * 64 + t;
    bh = gt < nbn ? BH[bo] : uint4{0, 0, 0, 0};
    bl = gt < nbn ? BH[lo_off + bo] : uint4{0, 0, 0, 0};
    if (t < 2 * KQ * 64) kh = KH[(int64_t)(2 * cp) * KQ * 64 + t];
  };
  auto store_tile = [&](int buf, const uint4 &bh, const uint4 &bl, const uint4 &kh) {
    if (gt < kNBG) {
      bsh[buf][t] = bh;
      bsh[buf][kNBG * 64 + t] = bl;
    }
    if (t < 2 * KQ * 64) ksh[buf][t] = kh;
  };
  uint4 nbh = uint4{0, 0, 0, 0}, nbl = uint4{0, 0, 0, 0}, nkh = uint4{0, 0, 0, 0};
  if (ncp > 0) {
    load_tile(0, nbh, nbl, nkh);
    store_tile(0, nbh, nbl, nkh);
  }
  __syncthreads();
  const bool active = rb0 < nrow_blocks;  // wave-uniform; every wave still stages tiles
  for (int cp = 0; cp < ncp; ++cp) {
    const int cur = cp & 1;
    if (cp + 1 < ncp) load_tile(cp + 1, nbh, nbl, nkh);
    if (active) {
      half8 eh[kLdsRB], el[kLdsRB];
#pragma unroll
      for (int r = 0; r < kLdsRB; ++r) {
        float e[8];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          floatx4 tt = {rinit[r], rinit[r], rinit[r], rinit[r]};
#pragma unroll
          for (int m = 0; m < KQ; ++m)
            tt = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_half8(ksh[cur][(s2 * KQ + m) * 64 + lane]), qh[r][m], tt,
                                                        0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) e[4 * s2 + i] = __builtin_amdgcn_exp2f(tt[i]);
          if (2 * cp + s2 == rb0 + r) {  // the self pair has Z_II = K_h(0) = 1 exactly
#pragma unroll
            for (int i = 0; i < 4; ++i) e[4 * s2 + i] = diag_i == i ? 32768.f : e[4 * s2 + i];
          }
        }
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const half2v h = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(e[j], e[j + 1]));
          const float ra = __builtin_fmaf(-(float)h.x, one, e[j]);
          const float rb2 = __builtin_fmaf(-(float)h.y, one, e[j + 1]);
          eh[r][j] = h.x;
          eh[r][j + 1] = h.y;
          el[r][j] = (_Float16)ra;
          el[r][j + 1] = (_Float16)rb2;
        }
      }
#pragma unroll
      for (int g = 0; g < kNBG; ++g) {
        const half8 bh = as_half8(bsh[cur][g * 64 + lane]);
        const half8 bl = as_half8(bsh[cur][kNBG * 64 + g * 64 + lane]);
#pragma unroll
        for (int r = 0; r < kLdsRB; ++r) {
          acc[r][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh[r], bh, acc[r][g], 0, 0, 0);
          acc[r][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh[r], bl, acc[r][g], 0, 0, 0);
          acc[r][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(el[r], bh, acc[r][g], 0, 0, 0);
        }
      }
    }
    if (cp + 1 < ncp) store_tile(cur ^ 1, nbh, nbl, nkh);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int r = 0; r < kLdsRB; ++r) {
    if (rb0 + r >= nrow_blocks) break;
#pragma unroll
    for (int g = 0; g < kNBG; ++g) {
      if (g >= nbn) break;
      const int col = (nb0 + g) * 16 + (lane & 15);
      const double sc = col < dR ? scale0 : scale1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = (int64_t)(rb0 + r) * 16 + 4 * (lane >> 4) + i;
        Y[row * ldy + col] = (float)((double)acc[r][g][i] * sc);
      }
    }
  }
}

__global__ void k_fill_scaled(const float *__restrict__ src, float a, int64_t n, float *__restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) dst[t] = a * src[t];
}

__global__ void k_add(const float *__restrict__ a, const float *__restrict__ b, int64_t n, float *__restrict__ c) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) c[t] = a[t] + b[t];
}

// p <- p + a (p - prev), in place: the linear extrapolation of the reduced
// state from an earlier one
__global__ void k_extrapolate(float *__restrict__ p, const float *__restrict__ prev, float a, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = fmaf(a, p[t] - prev[t], p[t]);
}

// Explicit Euler on the reduced state p[k][s] (eq. model_DymReduced):
// dp_k/dt = X^H p_k - (kT/zeta) sum_j A_kj X^B p_j - (1/zeta) sum_j A_kj H_j p_j.
// One workgroup; p in LDS; each wavefront takes whole rows of X^H / X^B.
__global__ __launch_bounds__(1024) void k_rom_steps(const float *__restrict__ XH, const float *__restrict__ XB,
                                                    float *__restrict__ p, int nb, int R, int nsteps, EvalParams ep) {
  __shared__ float ps[kMaxNb][kMaxR];
  __shared__ float y[kMaxNb][kMaxR];
  __shared__ float z[kMaxNb][kMaxR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int t = tid; t < nb * R; t += blockDim.x) ps[t / R][t % R] = p[t];
  __syncthreads();
  const float ktz = ep.kT * ep.inv_zeta;
  for (int step = 0; step < nsteps; ++step) {
    for (int row = wave; row < 2 * R; row += nw) {
      const float *M = row < R ? XH + (int64_t)row * R : XB + (int64_t)(row - R) * R;
      float acc[kMaxNb];
#pragma unroll
      for (int k = 0; k < kMaxNb; ++k) acc[k] = 0.f;
      for (int u = lane; u < R; u += 64) {
        const float m = M[u];
#pragma unroll
        for (int k = 0; k < kMaxNb; ++k)
          if (k < nb) acc[k] = fmaf(m, ps[k][u], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < kMaxNb; ++k) {
        float v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc[k] = v;
      }
      if (lane == 0) {
        for (int k = 0; k < nb; ++k) {
          if (row < R) y[k][row] = acc[k];
          else z[k][row - R] = acc[k];
        }
      }
    }
    __syncthreads();
    float pn[kMaxNb * kMaxR / 1024 + 1];
    int cnt = 0;
    for (int t = tid; t < nb * R; t += blockDim.x, ++cnt) {
      const int k = t / R, s = t % R;
      float az = 2.f * z[k][s], ah = 2.f * ep.H[k] * ps[k][s];
      if (k > 0) {
        az -= z[k - 1][s];
        ah -= ep.H[k - 1] * ps[k - 1][s];
      }
      if (k + 1 < nb) {
        az -= z[k + 1][s];
        ah -= ep.H[k + 1] * ps[k + 1][s];
      }
      pn[cnt] = ps[k][s] + ep.dt * (y[k][s] - ktz * az - ep.inv_zeta * ah);
    }
    __syncthreads();
    cnt = 0;
    for (int t = tid; t < nb * R; t += blockDim.x, ++cnt) ps[t / R][t % R] = pn[cnt];
    __syncthreads();
  }
  for (int t = tid; t < nb * R; t += blockDim.x) p[t] = ps[t / R][t % R];
}

// The same steps with both operators held in registers for the whole window:
// thread t works on matrix row t / 2 (the rows of X^H, then those of X^B) over
// half t % 2 of its columns (halves aligned to four columns), so a step reads
// only the state, as float4 broadcasts from LDS, and combines the two halves
// with one shuffle.  The state is double-buffered: two barriers per step.
// 768 threads (three waves per SIMD leave room for the matrix slice);
// R <= 2 kHalf, NB = nb bonds known at compile time (no per-bond branches
// between the loads and their uses).
constexpr int kRegThreads = 768;
template <int kHalf, int NB>
__global__ __launch_bounds__(kRegThreads) void k_rom_steps_reg(const float *__restrict__ XH,
                                                               const float *__restrict__ XB, float *__restrict__ p,
                                                               int R, int nsteps, EvalParams ep) {
  static_assert(kHalf % 4 == 0, "halves are read as float4");
  constexpr int W = 2 * kHalf;
  constexpr int kPer = (NB * W + kRegThreads - 1) / kRegThreads;  // state entries per thread
  __shared__ float4 ps4[2][NB][W / 4];
  __shared__ float y[NB][W];
  __shared__ float z[NB][W];
  float *ps0 = reinterpret_cast<float *>(&ps4[0][0][0]);
  const int tid = threadIdx.x;
  const int row = tid >> 1, half = tid & 1;
  const int hl = (((R + 1) / 2) + 3) & ~3;  // <= kHalf
  const int u0 = half * hl;
  const int len = min(hl, R - u0);
  const bool active = row < 2 * R;
  const float *M = row < R ? XH + (int64_t)row * R : XB + (int64_t)(row - R) * R;
  float m[kHalf];
#pragma unroll
  for (int j = 0; j < kHalf; ++j) m[j] = (active && j < len) ? M[u0 + j] : 0.f;
  for (int t = tid; t < 2 * NB * W; t += kRegThreads) {  // zero padding: the unused m[j] meet zeros
    const int b = t / (NB * W), k = (t / W) % NB, s = t % W;
    ps0[t] = (b == 0 && s < R) ? p[k * R + s] : 0.f;
  }
  __syncthreads();
  const float ktz = ep.kT * ep.inv_zeta;
  int cur = 0;
  for (int step = 0; step < nsteps; ++step) {
    float acc[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = 0.f;
#pragma unroll
    for (int j4 = 0; j4 < kHalf / 4; ++j4) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const float4 v = ps4[cur][k][(u0 >> 2) + j4];
        acc[k] = fmaf(m[4 * j4], v.x, acc[k]);
        acc[k] = fmaf(m[4 * j4 + 1], v.y, acc[k]);
        acc[k] = fmaf(m[4 * j4 + 2], v.z, acc[k]);
        acc[k] = fmaf(m[4 * j4 + 3], v.w, acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] += __shfl_xor(acc[k], 1);
    if (active && half == 0) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (row < R) y[k][row] = acc[k];
        else z[k][row - R] = acc[k];
      }
    }
    __syncthreads();
    const float *pc = reinterpret_cast<const float *>(&ps4[cur][0][0]);
    float *pn = reinterpret_cast<float *>(&ps4[cur ^ 1][0][0]);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int t = tid + i * kRegThreads;
      if (t < NB * R) {
        const int k = t / R, s = t % R;
        float az = 2.f * z[k][s], ah = 2.f * ep.H[k] * pc[k * W + s];
        if (k > 0) {
          az -= z[k - 1][s];
          ah -= ep.H[k - 1] * pc[(k - 1) * W + s];
        }
        if (k + 1 < NB) {
          az -= z[k + 1][s];
          ah -= ep.H[k + 1] * pc[(k + 1) * W + s];
        }
        pn[k * W + s] = pc[k * W + s] + ep.dt * (y[k][s] - ktz * az - ep.inv_zeta * ah);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  const float *pf = reinterpret_cast<const float *>(&ps4[cur][0][0]);
  for (int t = tid; t < NB * R; t += kRegThreads) p[t] = pf[(t / R) * W + t % R];
}

template <int kHalf>
void launch_steps_reg(int nb, const float *XH, const float *XB, float *p, int R, int n, const EvalParams &ep,
                      hipStream_t s) {
  switch (nb) {
    case 1: k_rom_steps_reg<kHalf, 1><<<1, kRegThreads, 0, s>>>(XH, XB, p, R, n, ep); break;
    case 2: k_rom_steps_reg<kHalf, 2><<<1, kRegThreads, 0, s>>>(XH, XB, p, R, n, ep); break;
    case 3: k_rom_steps_reg<kHalf, 3><<<1, kRegThreads, 0, s>>>(XH, XB, p, R, n, ep); break;
    case 4: k_rom_steps_reg<kHalf, 4><<<1, kRegThreads, 0, s>>>(XH, XB, p, R, n, ep); break;
    default: k_rom_steps_reg<kHalf, 5><<<1, kRegThreads, 0, s>>>(XH, XB, p, R, n, ep); break;
  }
}

// ---- exact integration of a frozen window --------------------------------
//
// Generator of eq. model_DymReduced on vec(p) (index i = k R + s), column-major:
// L[i + l n] with l = j R + u,
//   delta_kj X^H_su - (kT/zeta) A_kj X^B_su - (1/zeta) A_kj H_j delta_su.
__global__ void k_generator(const float *__restrict__ XH, const float *__restrict__ XB, int nb, int R,
                            EvalParams ep, double *__restrict__ Lm) {
  const int64_t n = (int64_t)nb * R;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * n) return;
  const int64_t i = t % n, l = t / n;
  const int k = (int)(i / R), s = (int)(i % R), j = (int)(l / R), u = (int)(l % R);
  const double A = k == j ? 2.0 : ((k - j == 1 || j - k == 1) ? -1.0 : 0.0);
  double v = -(double)ep.kT * (double)ep.inv_zeta * A * (double)XB[(int64_t)s * R + u];
  if (k == j) v += (double)XH[(int64_t)s * R + u];
  if (s == u) v -= (double)ep.inv_zeta * A * (double)ep.H[j];
  Lm[t] = v;
}

// Largest absolute column sum of a column-major n x n matrix, per column.
__global__ void k_colabs(const double *__restrict__ Lm, int64_t n, double *__restrict__ cs) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= n) return;
  double a = 0.0;
  for (int64_t i = 0; i < n; ++i) a += fabs(Lm[i + l * n]);
  cs[l] = a;
}

__global__ void k_scale64(const double *__restrict__ a, double f, int64_t n, double *__restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) b[t] = f * a[t];
}

__global__ void k_identity64(int64_t n, double *__restrict__ M) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n * n) M[t] = (t % n == t / n) ? 1.0 : 0.0;
}

__global__ void k_f64_to_f32(const double *__restrict__ a, int64_t n, float *__restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) b[t] = (float)a[t];
}

// tau_ab = (n / P) sum_k H_k p_k^T M_ab p_k (uniform weights), FP64 sums.
__global__ __launch_bounds__(256) void k_rom_stress(const float *__restrict__ Mbig, const float *__restrict__ p, int nb,
                                                    int R, EvalParams ep, double *__restrict__ out) {
  __shared__ double sm[256];
  const int ab = blockIdx.x;  // 0..8
  const int a = ab / 3, b = ab % 3;
  const int64_t ld = 3 * (int64_t)R;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < (int64_t)R * R; t += 256) {
    const int s = (int)(t / R), u = (int)(t % R);
    const double m = Mbig[(a * (int64_t)R + s) * ld + b * R + u];
    for (int k = 0; k < nb; ++k) acc += (double)ep.H[k] * (double)p[k * R + s] * m * (double)p[k * R + u];
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[ab] = sm[0] * (double)ep.n / (double)ep.P;
}

inline unsigned nblk256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct vds_rom_s {
  vds_ctx ctx = nullptr;
  const float *U = nullptr;
  int R = 0;
  RomLayout L{};
  char *ws = nullptr;
  float *Ude, *Mbig, *XH, *I1, *XB1, *XB2, *XB, *Bsw, *Y, *qt, *T, *invS, *part, *psave, *pprev;
  double *red;
};

namespace {

vds_status rom_gemm(vds_rom r, GemmShape g, double flops) {
  timed(r->ctx, VDS_TIMER_GEMM, flops, [&] { launch_gemm(g, r->part, r->ctx->stream); });
  return VDS_OK;
}

// X^B1, X^B2 (and X^B = X^B1 + X^B2) at q~ = U p.
// q~ = U p into r->qt.
void reconstruct_qt(vds_rom r, const float *p) {
  vds_ctx c = r->ctx;
  const int64_t m = 3 * c->prob.P;
  timed(c, VDS_TIMER_PROJ, 4.0 * m * r->R,
        [&] { launch_pod_reconstruct(r->U, m, r->R, c->prob.nb, p, r->qt, c->stream); });
}

vds_status freeze(vds_rom r, const float *p) {
  vds_ctx c = r->ctx;
  const int R = r->R;
  const int64_t P = c->prob.P, Ppad = c->ep.Ppad;
  const RomLayout &L = r->L;
  hipStream_t s = c->stream;
  reconstruct_qt(r, p);
  // S and T at q~ (uniform weights), Q/K operands for Z
  eval_pass_a(c, r->qt, nullptr, nullptr);
  eval_pass_b(c, nullptr);
  k_rom_scalars<<<nblk256(Ppad), 256, 0, s>>>(c->part, c->smap, Ppad, P, c->ep.D, c->S, c->wv, r->T,
                                              r->invS);
  // Y = Z B, in the FP16-split form when the context's pair kernels use it
  if (c->ep.vhalf) {
    const float wmax = c->ep.uniform_w;  // the reduced model runs with uniform weights
    k_rom_bsw16<<<nblk256(Ppad * L.ldy), 256, 0, s>>>(r->Ude, c->wv, r->invS, wmax, P, Ppad, R, L.NB16,
                                                      reinterpret_cast<_Float16 *>(r->Bsw));
    const int nrb = (int)(Ppad / 16), ncc = (int)((P + 15) / 16);
    dim3 grid((unsigned)((nrb + 3) / 4), (unsigned)((L.NB16 + kNBG - 1) / kNBG));
    const uint4 *bh = reinterpret_cast<const uint4 *>(r->Bsw);
    const int64_t lo_off = Ppad * L.ldy / 8;  // uint4 units
    const double unscale = 1.0 / ((double)kKgBScale * 32768.0);
    const double s0 = (double)wmax * unscale, s1 = unscale;
    const double flops = 2.0 * (double)P * P * 2 * 3 * R;
    if (c->ep.qhalf) {
      const uint4 *qh = reinterpret_cast<const uint4 *>(c->f16.QH), *kh = reinterpret_cast<const uint4 *>(c->f16.KH);
      const int ncp = (ncc + 1) / 2;
      dim3 g2((unsigned)((nrb + kLdsWaves * kLdsRB - 1) / (kLdsWaves * kLdsRB)), (unsigned)((L.NB16 + kNBG - 1) / kNBG));
      timed(c, VDS_TIMER_KGEMM, flops, [&] {
        if (c->ep.KQ == 1)
          k_kernel_gemm16_lds<1><<<g2, kLdsWaves * 64, 0, s>>>(qh, kh, c->f16.RN, nrb, ncp, bh, lo_off, L.NB16, 3 * R,
                                                               s0, s1, 1.f, r->Y, L.ldy);
        else
          k_kernel_gemm16_lds<2><<<g2, kLdsWaves * 64, 0, s>>>(qh, kh, c->f16.RN, nrb, ncp, bh, lo_off, L.NB16, 3 * R,
                                                               s0, s1, 1.f, r->Y, L.ldy);
      });
    } else timed(c, VDS_TIMER_KGEMM, flops, [&] {
      switch (c->ep.KK) {
        case 2: k_kernel_gemm16<2><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, bh, lo_off, L.NB16, 3 * R, s0, s1, 1.f, r->Y, L.ldy); break;
        case 3: k_kernel_gemm16<3><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, bh, lo_off, L.NB16, 3 * R, s0, s1, 1.f, r->Y, L.ldy); break;
        case 4: k_kernel_gemm16<4><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, bh, lo_off, L.NB16, 3 * R, s0, s1, 1.f, r->Y, L.ldy); break;
        default: k_kernel_gemm16<5><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, bh, lo_off, L.NB16, 3 * R, s0, s1, 1.f, r->Y, L.ldy); break;
      }
    });
  } else if (c->ep.f32x) {
    // the 32x32 form reads the pair kernel's operands as the passes left them;
    // column blocks per workgroup and runs were fixed when the model was laid
    // out (its slots hold G tiles of that width)
    const int NB = L.kg_nb, G = L.kg_runs;
    const int NCG = (int)((2 * 3 * R + 32 * NB - 1) / (32 * NB));
    k_rom_b32<<<nblk256(Ppad * NCG * 128), 256, 0, s>>>(r->Ude, c->wv, r->invS, P, Ppad, R, NCG, NB, r->Bsw);
    const int nrb32 = (int)(Ppad / 32), nch = (int)((P + 31) / 32);
    const int ncols = 2 * 3 * R;
    const float4 *kc = reinterpret_cast<const float4 *>(c->KA), *bk = reinterpret_cast<const float4 *>(r->Bsw);
    const double flops = 2.0 * (double)P * P * 2 * 3 * R;
    float *slots = reinterpret_cast<float *>(r->part);
    timed(c, VDS_TIMER_KGEMM, flops, [&] {
      const KGemm32Args a{c->xc, nrb32, kc, nch, bk, NCG, ncols, c->ep.kappa, r->Y, L.ldy, slots};
      switch (c->ep.D) {
        case 3: launch_kgemm32<3>(NB, G, a, s); break;
        case 6: launch_kgemm32<6>(NB, G, a, s); break;
        case 9: launch_kgemm32<9>(NB, G, a, s); break;
        case 12: launch_kgemm32<12>(NB, G, a, s); break;
        default: launch_kgemm32<15>(NB, G, a, s); break;
      }
      k_kgemm32_fixup<<<dim3((unsigned)((kgemm32_tile(NB) + 255) / 256), (unsigned)G), 256, 0, s>>>(
          slots, nrb32, nch, NCG, NB, ncols, r->Y, L.ldy);
    });
  } else {
    // the 16x16 FP32 forms (VDS_PAIR_MFMA, VDS_PAIR_VALU) read the 16-row operand layout
    k_rom_bsw<<<nblk256(Ppad * L.ldy), 256, 0, s>>>(r->Ude, c->wv, r->invS, P, Ppad, R, L.NB16, r->Bsw);
    const int nrb = (int)(Ppad / 16), ncc = (int)((P + 15) / 16);
    dim3 grid((unsigned)((nrb + 3) / 4), (unsigned)((L.NB16 + kNBG - 1) / kNBG));
    const float4 *b4 = reinterpret_cast<const float4 *>(r->Bsw);
    const double flops = 2.0 * (double)P * P * 2 * 3 * R;
    timed(c, VDS_TIMER_KGEMM, flops, [&] {
      switch (c->ep.KK) {
        case 2: k_kernel_gemm<2><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, b4, L.NB16, r->Y, L.ldy); break;
        case 3: k_kernel_gemm<3><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, b4, L.NB16, r->Y, L.ldy); break;
        case 4: k_kernel_gemm<4><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, b4, L.NB16, r->Y, L.ldy); break;
        default: k_kernel_gemm<5><<<grid, 256, 0, s>>>(c->QB, c->KA, nrb, ncc, b4, L.NB16, r->Y, L.ldy); break;
      }
    });
  }
  const float ih2 = c->ep.inv_h2;
  const int64_t RR = (int64_t)R * R;
  // X^B1 = -(1/h^2) I1 + (1/h^2) sum_a U_a^T diag(1/S) Y1_a
  k_fill_scaled<<<nblk256(RR), 256, 0, s>>>(r->I1, -ih2, RR, r->XB1);
  {
    GemmShape g;
    g.M = R;
    g.N = R;
    g.K = P;
    g.nbatch = 3;
    g.A = r->Ude;
    g.lda = P;
    g.sA = (int64_t)R * P;
    g.B = r->Y;
    g.ldb = L.ldy;
    g.sB = R;
    g.b_mn = true;
    g.scale = r->invS;
    g.alpha = ih2;
    g.C = r->XB1;
    g.ldc = R;
    g.accumulate = true;
    g.splits = gemm_splits(R, R, P);
    rom_gemm(r, g, 2.0 * 3 * RR * P);
  }
  // X^B2 = -(1/h^2) sum_a U_a^T diag(T) U_a + (1/h^2) sum_a U_a^T Y2_a
  {
    GemmShape g;
    g.M = R;
    g.N = R;
    g.K = P;
    g.nbatch = 3;
    g.A = r->Ude;
    g.lda = P;
    g.sA = (int64_t)R * P;
    g.B = r->Ude;
    g.ldb = P;
    g.sB = (int64_t)R * P;
    g.scale = r->T;
    g.alpha = -ih2;
    g.C = r->XB2;
    g.ldc = R;
    g.splits = gemm_splits(R, R, P);
    rom_gemm(r, g, 2.0 * 3 * RR * P);
    g.B = r->Y + 3 * R;
    g.ldb = L.ldy;
    g.sB = R;
    g.b_mn = true;
    g.scale = nullptr;
    g.alpha = ih2;
    g.accumulate = true;
    rom_gemm(r, g, 2.0 * 3 * RR * P);
  }
  k_add<<<nblk256(RR), 256, 0, s>>>(r->XB1, r->XB2, RR, r->XB);
  return hip_check(c, hipGetLastError(), "reduced operators");
}

}  // namespace

extern "C" {

size_t vds_rom_workspace_bytes(const vds_problem *prob, int32_t R) {
  if (prob == nullptr || prob->P < 1 || prob->nb < 1 || R < 1 || R > kMaxR || R > 3 * prob->P) return 0;
  return rom_layout(*prob, R).total;
}

vds_status vds_rom_create(vds_ctx c, const float *U, int32_t R, void *ws, size_t bytes, vds_rom *out) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!U || !ws || !out || R < 1 || R > kMaxR || R > 3 * c->prob.P)
    return set_err(c, VDS_ERR_ARG, "bad arguments (1 <= R <= min(1024, 3P))");
  if (c->prob.potential != VDS_HOOKEAN)
    return set_err(c, VDS_ERR_ARG, "the reduced spring term is exact only for Hookean springs");
  const RomLayout L = rom_layout(c->prob, R);
  if (bytes < L.total) return set_err(c, VDS_ERR_NOMEM, "reduced-model workspace too small");
  vds_rom r = new (std::nothrow) vds_rom_s();
  if (r == nullptr) return set_err(c, VDS_ERR_NOMEM, "host allocation failed");
  r->ctx = c;
  r->U = U;
  r->R = R;
  r->L = L;
  r->ws = static_cast<char *>(ws);
  auto f = [&](size_t o) { return reinterpret_cast<float *>(r->ws + o); };
  r->Ude = f(L.Ude);
  r->Mbig = f(L.Mbig);
  r->XH = f(L.XH);
  r->I1 = f(L.I1);
  r->XB1 = f(L.XB1);
  r->XB2 = f(L.XB2);
  r->XB = f(L.XB);
  r->Bsw = f(L.Bsw);
  r->Y = f(L.Y);
  r->qt = f(L.qt);
  r->T = f(L.T);
  r->invS = f(L.invS);
  r->part = f(L.part);
  r->red = reinterpret_cast<double *>(r->ws + L.red);
  r->psave = f(L.psave);
  r->pprev = f(L.pprev);
  const int64_t P = c->prob.P;
  hipStream_t s = c->stream;
  k_deinterleave<<<nblk256(3 * (int64_t)R * P), 256, 0, s>>>(U, P, R, r->Ude);
  GemmShape g;
  g.M = 3 * R;
  g.N = 3 * R;
  g.K = P;
  g.A = r->Ude;
  g.lda = P;
  g.B = r->Ude;
  g.ldb = P;
  g.C = r->Mbig;
  g.ldc = 3 * R;
  g.splits = gemm_splits(3 * R, 3 * R, P);
  rom_gemm(r, g, 2.0 * 9.0 * R * R * P);
  k_hydro<<<nblk256((int64_t)R * R), 256, 0, s>>>(r->Mbig, R, c->ep, r->XH, r->I1);
  st = hip_check(c, hipGetLastError(), "reduced model setup");
  if (st != VDS_OK) {
    delete r;
    return st;
  }
  *out = r;
  return VDS_OK;
}

void vds_rom_destroy(vds_rom r) { delete r; }

vds_status vds_rom_operators(vds_rom r, const float *p, float *XH, float *XB1, float *XB2) {
  if (r == nullptr) return VDS_ERR_ARG;
  vds_ctx c = r->ctx;
  if (!p) return set_err(c, VDS_ERR_ARG, "null p");
  vds_status st = freeze(r, p);
  if (st != VDS_OK) return st;
  const size_t b = sizeof(float) * r->R * r->R;
  if (XH) st = hip_check(c, hipMemcpyAsync(XH, r->XH, b, hipMemcpyDeviceToDevice, c->stream), "copy");
  if (XB1 && st == VDS_OK) st = hip_check(c, hipMemcpyAsync(XB1, r->XB1, b, hipMemcpyDeviceToDevice, c->stream), "copy");
  if (XB2 && st == VDS_OK) st = hip_check(c, hipMemcpyAsync(XB2, r->XB2, b, hipMemcpyDeviceToDevice, c->stream), "copy");
  return st;
}

vds_status vds_rom_stress(vds_rom r, const float *p, double *tau) {
  if (r == nullptr) return VDS_ERR_ARG;
  vds_ctx c = r->ctx;
  if (!p || !tau) return set_err(c, VDS_ERR_ARG, "null argument");
  k_rom_stress<<<9, 256, 0, c->stream>>>(r->Mbig, p, c->prob.nb, r->R, c->ep, r->red);
  vds_status st = hip_check(c, hipMemcpyAsync(tau, r->red, sizeof(double) * 9, hipMemcpyDeviceToHost, c->stream), "copy");
  if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  return st;
}

size_t vds_rom_exact_workspace_bytes(const vds_problem *prob, int32_t R) {
  if (prob == nullptr || R < 1 || prob->nb < 1) return 0;
  const size_t n = (size_t)prob->nb * R;
  return sizeof(double) * (4 * n * n + 4 * n) + 8 * 256;
}

vds_status vds_rom_run_exact(vds_rom r, float *p, int32_t nsteps, int32_t freeze_every, int32_t adaptive,
                             double energy_tol, double *windows_host, int32_t max_windows, void *ws,
                             size_t ws_bytes, double *tau, vds_rom_window_stats *stats) {
  if (r == nullptr) return VDS_ERR_ARG;
  vds_ctx c = r->ctx;
  if (!p || nsteps < 0 || freeze_every < 1 || !ws || (windows_host == nullptr) != (max_windows <= 0) ||
      (adaptive && !(energy_tol > 0.0)))
    return set_err(c, VDS_ERR_ARG, "bad arguments");
  const int nb = c->prob.nb, R = r->R;
  const int64_t n = (int64_t)nb * R;
  if (ws_bytes < vds_rom_exact_workspace_bytes(&c->prob, R)) return set_err(c, VDS_ERR_NOMEM, "workspace too small");
  hipStream_t s = c->stream;
  // workspace: generator, B = scaled generator, two Horner / squaring buffers, vectors
  auto take = [&, off = size_t(0)](size_t bytes) mutable {
    char *q = static_cast<char *>(ws) + off;
    off += (bytes + 255) / 256 * 256;
    return reinterpret_cast<double *>(q);
  };
  double *Lm = take(sizeof(double) * n * n), *Bm = take(sizeof(double) * n * n);
  double *Tm = take(sizeof(double) * n * n), *Cm = take(sizeof(double) * n * n);
  double *pv = take(sizeof(double) * n), *pw = take(sizeof(double) * n), *cs = take(sizeof(double) * n);
  float *ptrial = reinterpret_cast<float *>(take(sizeof(float) * n));  // trial state of an adaptive window
  rocblas_handle hb = static_cast<rocblas_handle>(blas_handle(c));
  if (hb == nullptr) return VDS_ERR_HIP;
  rocblas_set_pointer_mode(hb, rocblas_pointer_mode_host);
  vds_status st = VDS_OK;
  const unsigned nn_blocks = (unsigned)nblk256(n * n);
  std::vector<double> hcs(n);

  // p <- exp(tw L) p with the generator L frozen at the window start (in Lm)
  auto advance = [&](double tw, float *pout) -> vds_status {
    k_colabs<<<(unsigned)nblk256(n), 256, 0, s>>>(Lm, n, cs);
    vds_status e = hip_check(c, hipMemcpyAsync(hcs.data(), cs, sizeof(double) * n, hipMemcpyDeviceToHost, s), "copy");
    if (e == VDS_OK) e = hip_check(c, hipStreamSynchronize(s), "synchronise");
    if (e != VDS_OK) return e;
    const double norm = tw * *std::max_element(hcs.begin(), hcs.end());
    // scaling: |B|_1 <= 1/2, where the degree-12 Taylor remainder is below 2e-14
    int sq = 0;
    while (norm / std::ldexp(1.0, sq) > 0.5) ++sq;
    k_scale64<<<nn_blocks, 256, 0, s>>>(Lm, tw / std::ldexp(1.0, sq), n * n, Bm);
    k_identity64<<<nn_blocks, 256, 0, s>>>(n, Tm);
    double *T = Tm, *C = Cm;
    const double one = 1.0, zero = 0.0;
    for (int k = 12; k >= 1; --k) {  // Horner: T <- I + B T / k
      k_identity64<<<nn_blocks, 256, 0, s>>>(n, C);
      const double a = 1.0 / k;
      if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, (int)n, (int)n, &a, Bm, (int)n,
                        T, (int)n, &one, C, (int)n) != rocblas_status_success)
        return set_err(c, VDS_ERR_HIP, "rocblas_dgemm");
      std::swap(T, C);
    }
    for (int i = 0; i < sq; ++i) {  // squaring: T <- T T
      if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, (int)n, (int)n, &one, T, (int)n,
                        T, (int)n, &zero, C, (int)n) != rocblas_status_success)
        return set_err(c, VDS_ERR_HIP, "rocblas_dgemm");
      std::swap(T, C);
    }
    launch_f32_to_f64(p, pv, n, s);
    if (rocblas_dgemv(hb, rocblas_operation_none, (int)n, (int)n, &one, T, (int)n, pv, 1, &zero, pw, 1) !=
        rocblas_status_success)
      return set_err(c, VDS_ERR_HIP, "rocblas_dgemv");
    k_f64_to_f32<<<(unsigned)nblk256(n), 256, 0, s>>>(pw, n, pout);
    return hip_check(c, hipGetLastError(), "window");
  };
  // F, dissipation, work of the reconstructed state q~ = U p
  auto energy = [&](const float *pp, double *F, double *Dg, double *W) {
    reconstruct_qt(r, pp);
    return vds_energy(c, r->qt, nullptr, F, Dg, W);
  };

  const double dt = c->prob.dt, t_total = nsteps * dt, tw_max = freeze_every * dt;
  double t = 0.0, tw = tw_max, max_gap = 0.0;
  int windows = 0, rejected = 0, recorded = 0, truncated = 0;
  double F0 = 0, D0 = 0, W0 = 0;
  if (adaptive && nsteps > 0) st = energy(p, &F0, &D0, &W0);
  while (st == VDS_OK && t < t_total - 0.5 * dt) {
    tw = std::min(tw, t_total - t);
    st = freeze(r, p);
    if (st != VDS_OK) break;
    k_generator<<<nn_blocks, 256, 0, s>>>(r->XH, r->XB, nb, R, c->ep, Lm);
    double gap = 0.0;
    for (;;) {
      st = advance(tw, adaptive ? ptrial : p);
      if (st != VDS_OK || !adaptive) break;
      double F1, D1, W1;
      st = energy(ptrial, &F1, &D1, &W1);
      if (st != VDS_OK) break;
      const double bound = energy_tol * tw * 0.5 * (std::fabs(W0) + D0 + std::fabs(W1) + D1);
      gap = std::fabs(F1 - F0 - tw * 0.5 * ((W0 - D0) + (W1 - D1)));
      if (gap <= bound || tw <= dt * (1.0 + 1e-9)) {
        if (gap > bound) ++truncated;  // accepted at the smallest window
        st = hip_check(c, hipMemcpyAsync(p, ptrial, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy");
        max_gap = std::max(max_gap, bound > 0 ? gap / bound * energy_tol : gap);
        F0 = F1;
        D0 = D1;
        W0 = W1;
        break;
      }
      ++rejected;
      tw = std::max(dt, 0.5 * tw);
    }
    if (st != VDS_OK) break;
    t += tw;
    ++windows;
    if (windows_host && recorded < max_windows) windows_host[recorded++] = tw;
    if (adaptive) {
      const double bound = energy_tol * tw * 0.5 * (std::fabs(W0) + D0);
      if (gap < 0.25 * bound) tw = std::min(2.0 * tw, tw_max);  // grows back, up to the requested interval
    }
  }

  if (st != VDS_OK) return st;
  if (stats) {
    stats->windows = windows;
    stats->rejected = rejected;
    stats->truncated = truncated;
    stats->recorded = recorded;
    stats->t_reached = t;
    stats->max_energy_gap = max_gap;
  }
  st = hip_check(c, hipGetLastError(), "exact windows");
  if (st != VDS_OK) return st;
  if (tau) return vds_rom_stress(r, p, tau);
  return hip_check(c, hipStreamSynchronize(s), "synchronise");
}

}  // extern "C"

namespace {

// n reduced explicit Euler steps of p with the current operators (one launch).
void rom_steps(vds_rom r, float *p, int n) {
  vds_ctx c = r->ctx;
  const int nb = c->prob.nb, R = r->R;
  if (R <= 32)
    launch_steps_reg<16>(nb, r->XH, r->XB, p, R, n, c->ep, c->stream);
  else if (R <= 64)
    launch_steps_reg<32>(nb, r->XH, r->XB, p, R, n, c->ep, c->stream);
  else if (R <= 128)
    launch_steps_reg<64>(nb, r->XH, r->XB, p, R, n, c->ep, c->stream);
  else if (R <= 192)
    launch_steps_reg<96>(nb, r->XH, r->XB, p, R, n, c->ep, c->stream);
  else
    k_rom_steps<<<1, 1024, 0, c->stream>>>(r->XH, r->XB, p, nb, R, n, c->ep);
}

// The windows of vds_rom_run / vds_rom_run_midpoint.
// Operators frozen per window of freeze_every reduced steps.  FREEZE_START:
// at the window's start state.  FREEZE_MIDPOINT: at the state half a window
// on, predicted by reduced steps with the start's operators (two operator
// builds per window).  FREEZE_EXTRAPOLATED: at the midpoint state extrapolated
// linearly from this and the previous window's start states (one build per
// window; the first window predicts as FREEZE_MIDPOINT does).  Both midpoint
// forms predict the midpoint state to O(L^2) in the window length L, so the
// frozen operators are O(L^2) from those at the true midpoint.
enum FreezeAt { FREEZE_START = 0, FREEZE_MIDPOINT = 1, FREEZE_EXTRAPOLATED = 2 };

// Stress of the reduced state p from the M_ab, copied into tau_host[9] in
// stream order (the caller synchronises before reading it).
vds_status rom_stress_async(vds_rom r, const float *p, double *tau_host) {
  vds_ctx c = r->ctx;
  k_rom_stress<<<9, 256, 0, c->stream>>>(r->Mbig, p, c->prob.nb, r->R, c->ep, r->red);
  return hip_check(c, hipMemcpyAsync(tau_host, r->red, sizeof(double) * 9, hipMemcpyDeviceToHost, c->stream),
                   "copy stress");
}

// With output_every >= 1 the stress after steps output_every, 2 output_every,
// ... and after the last step goes to tau[9 i ...]; with output_every == 0 only
// the stress after the last step (tau may be NULL).
vds_status rom_windows(vds_rom r, float *p, int nsteps, int freeze_every, FreezeAt at, double *tau,
                       int output_every = 0) {
  vds_ctx c = r->ctx;
  int nout = 0;
  // steps [k, k + n) of the run, split at the output steps
  auto steps_out = [&](int k, int n) -> vds_status {
    while (n > 0) {
      const int m = output_every > 0 ? std::min(n, output_every - k % output_every) : n;
      rom_steps(r, p, m);
      k += m;
      n -= m;
      if (tau != nullptr && ((output_every > 0 && k % output_every == 0) || k == nsteps)) {
        vds_status st = rom_stress_async(r, p, tau + 9 * nout++);
        if (st != VDS_OK) return st;
      }
    }
    return VDS_OK;
  };
  const int64_t np = (int64_t)c->prob.nb * r->R;
  const size_t pbytes = sizeof(float) * (size_t)np;
  auto copy = [&](float *dst, const float *src) {
    return hip_check(c, hipMemcpyAsync(dst, src, pbytes, hipMemcpyDeviceToDevice, c->stream), "copy");
  };
  int nprev = 0;  // length of the previous window (0: none yet)
  for (int s0 = 0; s0 < nsteps; s0 += freeze_every) {
    const int n = std::min(freeze_every, nsteps - s0), half = n / 2;
    vds_status st = VDS_OK;
    if (at == FREEZE_EXTRAPOLATED && nprev > 0 && half > 0) {
      // the midpoint state from the last two window starts; back to the start
      st = copy(r->psave, p);
      if (st != VDS_OK) return st;
      k_extrapolate<<<(unsigned)((np + 255) / 256), 256, 0, c->stream>>>(p, r->pprev, (float)half / (float)nprev, np);
      st = freeze(r, p);
      if (st == VDS_OK) st = copy(p, r->psave);
      if (st != VDS_OK) return st;
    } else {
      st = freeze(r, p);
      if (st != VDS_OK) return st;
      if (at != FREEZE_START && half > 0) {
        // operators at the state half a window on, predicted with the start's
        st = copy(r->psave, p);
        if (st != VDS_OK) return st;
        rom_steps(r, p, half);
        st = freeze(r, p);
        if (st == VDS_OK) st = copy(p, r->psave);
        if (st != VDS_OK) return st;
      }
    }
    if (at == FREEZE_EXTRAPOLATED) {
      st = copy(r->pprev, p);
      if (st != VDS_OK) return st;
      nprev = n;
    }
    vds_status so = steps_out(s0, n);
    if (so != VDS_OK) return so;
  }
  vds_status st = hip_check(c, hipGetLastError(), "reduced steps");
  if (st != VDS_OK) return st;
  if (tau != nullptr && nsteps == 0) st = rom_stress_async(r, p, tau);
  if (st != VDS_OK) return st;
  return hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
}

}  // namespace

extern "C" {

vds_status vds_rom_run(vds_rom r, float *p, int32_t nsteps, int32_t freeze_every, int32_t output_every,
                       double *tau_hist) {
  if (r == nullptr) return VDS_ERR_ARG;
  if (!p || nsteps < 0 || freeze_every < 1 || output_every < 0) return set_err(r->ctx, VDS_ERR_ARG, "bad arguments");
  return rom_windows(r, p, nsteps, freeze_every, FREEZE_START, tau_hist, output_every);
}

vds_status vds_rom_run_midpoint(vds_rom r, float *p, int32_t nsteps, int32_t freeze_every, double *tau) {
  if (r == nullptr) return VDS_ERR_ARG;
  if (!p || nsteps < 0 || freeze_every < 1) return set_err(r->ctx, VDS_ERR_ARG, "bad arguments");
  return rom_windows(r, p, nsteps, freeze_every, FREEZE_MIDPOINT, tau);
}

vds_status vds_rom_run_extrapolated(vds_rom r, float *p, int32_t nsteps, int32_t freeze_every, double *tau) {
  if (r == nullptr) return VDS_ERR_ARG;
  if (!p || nsteps < 0 || freeze_every < 1) return set_err(r->ctx, VDS_ERR_ARG, "bad arguments");
  return rom_windows(r, p, nsteps, freeze_every, FREEZE_EXTRAPOLATED, tau);
}

}  // extern "C"
