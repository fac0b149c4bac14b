// O(P D) kernels around the pair passes: centring and operand packing, the
// two finalisations (term1 and the pass-B weights; term2, drift and update,
// with the packing of the next state's operands), the implicit-iteration
// control, the FENE domain flag, and FP64 reductions of stress, energy,
// dissipation and work.  All reductions are two-stage (per-block partials in
// a fixed tree, then a fixed-order sum), so results are bitwise reproducible.
#include "vds_internal.h"

namespace vds {

// Fixed-order tree sum over the 256 threads of a block for NS values each.
template <int NS>
__device__ void block_sum(double (&v)[NS], double (*sm)[kRedBlock]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < NS; ++s) sm[s][t] = v[s];
  __syncthreads();
  for (int stride = kRedBlock / 2; stride > 0; stride >>= 1) {
    if (t < stride) {
#pragma unroll
      for (int s = 0; s < NS; ++s) sm[s][t] += sm[s][t + stride];
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = sm[s][0];
}

__device__ inline float load_weight(const float *w, int64_t I, float uniform_w) {
  return w != nullptr ? w[I] : uniform_w;
}

// Swizzled operand positions (see pair_kernels.hip):
//   QB/KA: element k of the augmented vector of particle I at
//          [((I / 16) * KK + k / 4) * 64 + (I % 16) + 16 (k % 4)]
//   VB:    element n of V_J at [((J / 16) * 64 + ((J % 16) / 4) * 16 + n) * 4 + (J % 4)]
__device__ inline int64_t qk_index(int64_t I, int k, int KK) {
  return ((I >> 4) * KK + (k >> 2)) * 64 + (I & 15) + 16 * (k & 3);
}
__device__ inline int64_t v_index(int64_t J, int n) {
  return ((J >> 4) * 64 + ((J & 15) >> 2) * 16 + n) * 4 + (J & 3);
}
//   V as FP16 halves (VDS_PAIR_MFMA_F16X2): the high half of element n of V_J
//          at [((J / 32) * 64 + n + 16 ((J % 16) / 4)) * 8 + 4 ((J / 16) % 2) + J % 4]
//          and the low half Ppad * 16 halves further on.
__device__ inline int64_t vh_index(int64_t J, int n) {
  return ((J >> 5) * 64 + n + 16 * ((J & 15) >> 2)) * 8 + 4 * ((J >> 4) & 1) + (J & 3);
}
//   QH/KH: FP16 distance slot s (0 <= s < 32 KQ) of particle I at
//          [(((I / 16) * KQ + s / 32) * 64 + I % 16 + 16 ((s % 32) / 8)) * 8 + s % 8]
__device__ inline int64_t dh_index(int64_t I, int s, int KQ) {
  return ((((I >> 4) * KQ + (s >> 5)) * 64 + (I & 15) + 16 * ((s & 31) >> 3)) << 3) + (s & 7);
}
// Row-side and column-side values of FP16 distance slot s, given the component
// y_k = cs x_k for k = s / 3 and the norm term -kappa |x|^2 (see pair_kernels.hip).
__device__ inline void dh_slot(const EvalParams &p, int s, float yk, float nterm, _Float16 &qv, _Float16 &kv) {
  const _Float16 z = (_Float16)0.f;
  qv = z;
  kv = z;
  if (s < 3 * p.D) {
    const int ty = s % 3;
    const _Float16 hi = (_Float16)yk;
    const _Float16 lo = (_Float16)(yk - (float)hi);
    qv = ty == 2 ? lo : hi;
    kv = ty == 1 ? lo : hi;
  } else if (s < 3 * p.D + 2) {
    const float v = nterm * 0.0625f;
    const _Float16 hi = (_Float16)v;
    qv = (_Float16)16.f;
    kv = s == 3 * p.D ? hi : (_Float16)(v - (float)hi);
  }
}
__device__ inline void store_v(const EvalParams &p, float *V, int64_t J, int n, float v) {
  if (p.vhalf) {
    _Float16 *h = reinterpret_cast<_Float16 *>(V);
    const _Float16 hi = (_Float16)v;
    const int64_t i = vh_index(J, n);
    h[i] = hi;
    h[i + p.Ppad * 16] = (_Float16)(v - (float)hi);
  } else if (p.f32x) {
    V[vc_index(J, n)] = v;
  } else {
    V[v_index(J, n)] = v;
  }
}

// Partial sums of w_I x_I (FP64) per block, for the weighted centring.
// Bodies take the block index `lb` within the problem (one ensemble) so that
// the batched step can run them per ensemble.
__device__ void mean_partials_body(const EvalParams &p, int64_t lb, const float *__restrict__ q,
                                   const float *__restrict__ w, double *__restrict__ meanp) {
  __shared__ double sm[kMaxD][kRedBlock];
  const int64_t I = lb * kRedBlock + threadIdx.x;
  double v[kMaxD];
  const double wi = I < p.P ? (double)load_weight(w, I, p.uniform_w) : 0.0;
#pragma unroll
  for (int a = 0; a < kMaxD; ++a) {
    const int k = a / 3, al = a % 3;
    v[a] = (I < p.P && a < p.D) ? wi * (double)q[((int64_t)k * p.P + I) * 3 + al] : 0.0;
  }
  block_sum<kMaxD>(v, sm);
  if (threadIdx.x < kMaxD) meanp[lb * 16 + threadIdx.x] = v[threadIdx.x];
  // slot 15: the block's largest weight
  __shared__ float wm[kRedBlock / 64];
  float m = I < p.P ? load_weight(w, I, p.uniform_w) : 0.f;
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kRedBlock / 64; ++i) m = fmaxf(m, wm[i]);
    meanp[lb * 16 + 15] = (double)m;
  }
}

__global__ __launch_bounds__(kRedBlock) void k_mean_partials(EvalParams p, const float *__restrict__ q,
                                                             const float *__restrict__ w, double *__restrict__ meanp,
                                                             const int *done, Ctrl *begin) {
  if (done != nullptr && *done) return;
  if (begin != nullptr) {
    // opens a queued implicit step (no other block of this launch reads
    // the fields that block 0 clears)
    if (begin->halted) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      begin->done = 0;
      begin->conv_iter = -1;
      begin->checked = 0;
    }
  }
  mean_partials_body(p, blockIdx.x, q, w, meanp);
}

// Sum of the centring partials (mean_sh[0..D)) and the largest weight
// (mean_sh[15]), computed identically by every block: thread (c, j) = (t % 16,
// t / 16) folds the partials of blocks j, j + 16, ... of slot c, then one
// thread per slot combines the sixteen results in order.
__device__ void load_mean(const EvalParams &p, const double *meanp, int nmeanp, float *mean_sh) {
  __shared__ double part[16][17];
  const int c = threadIdx.x & 15, j = threadIdx.x >> 4;  // blockDim.x == 256
  double v = 0.0;
  const int nj = strided_count(j, nmeanp, 16);
  if (c == 15) v = strided_max(meanp + (int64_t)j * 16 + 15, nj, 256, 0.0);
  else if (c < p.D) v = ordered_sum<double>(meanp + (int64_t)j * 16 + c, nj, 256);
  part[c][j] = v;
  __syncthreads();
  if (threadIdx.x < 16 && (threadIdx.x < p.D || threadIdx.x == 15)) {
    double r = 0.0;
    for (int i = 0; i < 16; ++i) r = threadIdx.x == 15 ? fmax(r, part[threadIdx.x][i]) : r + part[threadIdx.x][i];
    mean_sh[threadIdx.x] = (float)r;
  }
  __syncthreads();
}

// The per-particle kernels below use 16 lanes per particle: lane n owns
// component n of the configuration vector (n < D <= 15), so loads and stores
// of a wave cover four particles' contiguous records and P/16 blocks fill the
// chip.  Cross-component terms (norms, the 3x3 flow, bond neighbours) are
// 16-wide shuffles.
__device__ inline int64_t group_particle(int64_t lb) { return (lb * kRedBlock + threadIdx.x) >> 4; }
__device__ inline int group_lane() { return threadIdx.x & 15; }
__device__ inline float gshfl(float v, int n) { return __shfl(v, n, 16); }
__device__ inline double gshfl(double v, int n) { return __shfl(v, n, 16); }
__device__ inline float gsum(float v) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
  return v;
}

// Convergence test of fixed-point iteration chk.iter from the combine kernel's
// block maxima of |dx| and |x|: max|dx| <= rtol * max(1, max|x|).  Every block
// of the calling launch evaluates it (the maxima are the previous kernel's
// output, so the launch boundary orders them) and gets the same answer;
// *resid receives max|dx|.
__device__ bool picard_converged(const PicardCheck &chk, const float *__restrict__ blockmax, int nblk,
                                 float *resid) {
  __shared__ float sr[kRedBlock / 64], sx[kRedBlock / 64];
  __shared__ int conv;
  __shared__ float rr;
  const int nt = strided_count(threadIdx.x, nblk, kRedBlock);
  float r = strided_max(blockmax + 2 * threadIdx.x, nt, 2 * kRedBlock, 0.f);
  float x = strided_max(blockmax + 2 * threadIdx.x + 1, nt, 2 * kRedBlock, 0.f);
  for (int off = 32; off > 0; off >>= 1) {
    r = fmaxf(r, __shfl_xor(r, off));
    x = fmaxf(x, __shfl_xor(x, off));
  }
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x >> 6] = r;
    sx[threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kRedBlock / 64; ++i) {
      r = fmaxf(r, sr[i]);
      x = fmaxf(x, sx[i]);
    }
    rr = r;
    conv = r <= chk.rtol * fmaxf(1.f, x) ? 1 : 0;
  }
  __syncthreads();
  *resid = rr;
  return conv != 0;
}

// Centre, pack Q/K operands and the pass-A V operand (weights w; over their
// maximum, which goes to *wscale, when V is written in FP16 halves).
// Lane n of particle I's raw coordinate (0 past the particles or D).
__device__ inline float prep_coord(const EvalParams &p, const float *__restrict__ q, int64_t I, int n) {
  return (I < p.P && n < p.D) ? q[((int64_t)(n / 3) * p.P + I) * 3 + (n % 3)] : 0.f;
}

// Operand packing of particle I (lane n) from its centred coordinate x and
// weight wi; mean_sh[15] is the largest weight.
__device__ void prep_write(const EvalParams &p, int64_t I, int n, float x, float wi, const float *mean_sh,
                           float *__restrict__ xc, float *__restrict__ wv, float *__restrict__ QB,
                           float *__restrict__ KA, float *__restrict__ VA, F16Operands f16) {
  const bool real = I < p.P;
  const float nrm = gsum(x * x);
  if (n == 0) wv[I] = wi;
  if (n < p.D) xc[I * p.D + n] = x;
  // the FP32 distance operands are read only by the FP32-distance pair forms
  // (KP can exceed the sixteen lanes: slots k = n, n + 16)
  for (int k = n; k < (p.f32x ? p.KP : 0); k += 16) {
    float ka = 0.f;
    if (real) {
      if (k < p.D) ka = 2.f * p.kappa * x;  // k < D <= 15 only for k == n
      else if (k == p.D) ka = -p.kappa * nrm;
      else if (k == p.D + 1) ka = 1.f;
    }
    KA[kc_index(I, k, p.KP)] = ka;
  }
  for (int k = n; k < ((p.qhalf || p.f32x) ? 0 : 4 * p.KK); k += 16) {
    float qa = 0.f, ka = 0.f;
    if (real) {
      if (k < p.D) {
        qa = x;
        ka = 2.f * p.kappa * x;
      } else if (k == p.D) {
        qa = -p.kappa * nrm;
        ka = 1.f;
      } else if (k == p.D + 1) {
        qa = 1.f;
        ka = -p.kappa * nrm;
      }
    }
    QB[qk_index(I, k, p.KK)] = qa;
    KA[qk_index(I, k, p.KK)] = ka;
  }
  if (p.qhalf) {
    // slots 2 m and 2 m + 1 are adjacent: one 32-bit store each for QH and KH
    uint32_t *qh = reinterpret_cast<uint32_t *>(f16.QH);
    uint32_t *kh = reinterpret_cast<uint32_t *>(f16.KH);
    const float y = p.cs * x;
    const float nt = real ? -p.kappa * nrm : 0.f;
    for (int sp = n; sp < 16 * p.KQ; sp += 16) {  // the same trip count on every lane
      const int s0 = 2 * sp, k0 = s0 / 3, k1 = (s0 + 1) / 3;
      const float y0 = gshfl(y, k0 < 16 ? k0 : 0), y1 = gshfl(y, k1 < 16 ? k1 : 0);
      _Float16 q0, c0, q1, c1;
      dh_slot(p, s0, y0, nt, q0, c0);
      dh_slot(p, s0 + 1, y1, nt, q1, c1);
      const int64_t di = dh_index(I, s0, p.KQ) >> 1;
      qh[di] = (uint32_t)__builtin_bit_cast(uint16_t, q0) | ((uint32_t)__builtin_bit_cast(uint16_t, q1) << 16);
      kh[di] = (uint32_t)__builtin_bit_cast(uint16_t, c0) | ((uint32_t)__builtin_bit_cast(uint16_t, c1) << 16);
    }
    if (n == 0) f16.RN[I] = nt;
  }
  const float wn = p.vhalf ? (real ? wi / mean_sh[15] : 0.f) : wi;
  float v = 0.f;
  if (n < p.D) v = wn * x;
  else if (n == p.D) v = wn;
  store_v(p, VA, I, n, v);
}

__device__ void prep_body(const EvalParams &p, int64_t lb, const float *__restrict__ q, const float *__restrict__ w,
                          const double *__restrict__ meanp, int nmeanp, float *__restrict__ xc,
                          float *__restrict__ wv, float *__restrict__ QB, float *__restrict__ KA,
                          float *__restrict__ VA, float *__restrict__ wscale, F16Operands f16,
                          float *__restrict__ cmean = nullptr) {
  __shared__ float mean_sh[16];
  load_mean(p, meanp, nmeanp, mean_sh);
  if (p.vhalf && wscale != nullptr && lb == 0 && threadIdx.x == 0) *wscale = mean_sh[15];
  if (cmean != nullptr && lb == 0 && threadIdx.x < 16) cmean[threadIdx.x] = mean_sh[threadIdx.x];
  const int64_t I = group_particle(lb);
  const int n = group_lane();
  if (I >= p.Ppad) return;
  const float x = I < p.P && n < p.D ? prep_coord(p, q, I, n) - mean_sh[n] : 0.f;
  const float wi = I < p.P ? load_weight(w, I, p.uniform_w) : 0.f;
  prep_write(p, I, n, x, wi, mean_sh, xc, wv, QB, KA, VA, f16);
}

__global__ __launch_bounds__(kRedBlock) void k_prep(EvalParams p, const float *__restrict__ q,
                                                    const float *__restrict__ w, const double *__restrict__ meanp,
                                                    int nmeanp, float *__restrict__ xc, float *__restrict__ wv,
                                                    float *__restrict__ QB, float *__restrict__ KA,
                                                    float *__restrict__ VA, float *__restrict__ wscale,
                                                    F16Operands f16, const int *done, float *__restrict__ cmean,
                                                    Ctrl *begin) {
  if (begin != nullptr) {
    // opens a queued implicit step (no other block of this launch reads the
    // fields that block 0 clears)
    if (begin->halted) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      begin->done = 0;
      begin->conv_iter = -1;
      begin->checked = 0;
    }
  } else if (done != nullptr && *done) {
    return;
  }
  prep_body(p, blockIdx.x, q, w, meanp, nmeanp, xc, wv, QB, KA, VA, wscale, f16, cmean);
}

// Component n of row I summed over its partial-sum slots in slot order, in FP64.
__device__ inline double sum_splits(const EvalParams &p, const float *__restrict__ partial, const SplitMap &splits,
                                    int64_t I, int n) {
  return ordered_sum<double>(partial + I * splits.width + n, splits.count(I), p.Ppad * splits.width);
}

// Pass-A finalisation: S_I = w_I + sum_{J != I} w_J e_IJ,
// term1_I = -(1/h^2) sum_J w_J e_IJ (x_I - x_J) / S_I, and the pass-B operand
// with weights w_J / S_J.
__device__ void finalize_a_body(const EvalParams &p, int64_t lb, const float *__restrict__ partial, const SplitMap &splits,
                                const float *__restrict__ xc, const float *__restrict__ wv, float *__restrict__ S,
                                float *__restrict__ t1, float *__restrict__ VB) {
  const int64_t I = group_particle(lb);
  const int n = group_lane();
  if (I >= p.Ppad) return;
  if (I >= p.P) {  // padding columns carry zero weight in pass B too
    store_v(p, VB, I, n, 0.f);
    return;
  }
  const double o = n <= p.D ? sum_splits(p, partial, splits, I, n) : 0.0;
  const double wI = (double)wv[I];
  const double Si = gshfl(o, p.D) + wI;  // the pass left out the self term w_I e_II = w_I
  const float wb = (float)(wI / Si);
  float v = 0.f;
  if (n < p.D) {
    t1[I * p.D + n] = (float)(-(double)p.inv_h2 * o / Si);
    v = wb * xc[I * p.D + n];
  } else if (n == p.D) {
    S[I] = (float)Si;
    v = wb;
  }
  store_v(p, VB, I, n, v);  // wb <= 1, so the FP16 form needs no normalisation
}

__global__ __launch_bounds__(kRedBlock) void k_finalize_a(EvalParams p, const float *__restrict__ partial, SplitMap splits,
                                                          const float *__restrict__ xc, const float *__restrict__ wv,
                                                          float *__restrict__ S, float *__restrict__ t1,
                                                          float *__restrict__ VB, const int *__restrict__ done) {
  if (done != nullptr && *done) return;
  finalize_a_body(p, blockIdx.x, partial, splits, xc, wv, S, t1, VB);
}

// Pass-B finalisation and everything local: term2, b = term1 + term2,
// g = kT b + grad Psi, u = -(1/zeta)(A (x) I) g, flow G q, and by mode the
// terms, the velocity, an explicit update or a fixed-point update (whose flow
// term is taken at the step's start state qs).  With `obs` it also
// accumulates F_h, dissipation, work and stress in FP64.  With pack.VA set
// (fixed-point or explicit mode) it packs the new iterate's or state's pair
// operands as the prep kernel would: the same lanes hold the same coordinates
// there.
__device__ void combine_body(const EvalParams &p, int64_t lb, int mode, int obs, const float *__restrict__ partial,
                             const SplitMap &splits, const float *xc, const float *__restrict__ t1,
                             const float *__restrict__ S, const float *wv, const float *qin,
                             const float *__restrict__ qs, float *out, float *out2, double *__restrict__ redp,
                             float *__restrict__ blockmax, const PackOps &pack, int *fene_out) {
  __shared__ double sm[12][kRedBlock];
  const int64_t I = group_particle(lb);
  const int n = group_lane();
  const bool real = I < p.P;          // uniform over the 16 lanes of a particle
  const bool comp = real && n < p.D;  // this lane owns a component
  const int k = n / 3, al = n % 3, base = 3 * k;
  const int64_t idx = ((int64_t)k * p.P + I) * 3 + al;
  double red[12];
#pragma unroll
  for (int s = 0; s < 12; ++s) red[s] = 0.0;
  float resid = 0.f, xmax = 0.f, xnew = 0.f;

  const double o = comp ? sum_splits(p, partial, splits, I, n) : 0.0;
  const float t2v = (float)(-(double)p.inv_h2 * o);
  const float t1v = comp ? t1[I * p.D + n] : 0.f;
  const float b = t1v + t2v;
  if (mode == MODE_TERMS) {
    if (comp) {
      out[idx] = t1v;
      out2[idx] = t2v;
    }
  } else {
    const float qv = comp ? qin[idx] : 0.f;
    // the three components of this lane's bond
    const float q0 = gshfl(qv, base), q1 = gshfl(qv, base + 1), q2 = gshfl(qv, base + 2);
    const float r2 = q0 * q0 + q1 * q1 + q2 * q2;
    const float H = k < p.nb ? p.H[k < kMaxNb ? k : 0] : 0.f;
    float fac = H, psi = 0.f;
    if (p.potential == VDS_FENE) {
      const float sb = 1.f - r2 / p.b_max;
      // outside the domain (or not finite): every such lane stores the same flag
      if (fene_out != nullptr && comp && !(sb > 0.f)) *fene_out = 1;
      fac = H / sb;
      psi = comp && al == 0 ? -0.5f * H * p.b_max * logf(sb) : 0.f;
    } else {
      psi = comp && al == 0 ? 0.5f * H * r2 : 0.f;
    }
    const float gp = comp ? fac * qv : 0.f;
    const float g = comp ? p.kT * b + gp : 0.f;
    // (A (x) I) g with A = tridiag(-1, 2, -1) over bonds
    const float gm = gshfl(g, n >= 3 ? n - 3 : n), gpl = gshfl(g, n + 3 < 16 ? n + 3 : n);
    float Ag = 2.f * g;
    if (k > 0) Ag -= gm;
    if (k + 1 < p.nb) Ag -= gpl;
    const float flow = p.G[3 * (al % 3)] * q0 + p.G[3 * (al % 3) + 1] * q1 + p.G[3 * (al % 3) + 2] * q2;
    float qstart = 0.f, flow0 = 0.f;
    if (mode == MODE_PICARD) {
      qstart = comp ? qs[idx] : 0.f;
      const float s0 = gshfl(qstart, base), s1 = gshfl(qstart, base + 1), s2 = gshfl(qstart, base + 2);
      flow0 = p.G[3 * (al % 3)] * s0 + p.G[3 * (al % 3) + 1] * s1 + p.G[3 * (al % 3) + 2] * s2;
    }
    const float u = -p.inv_zeta * Ag;
    if (comp) {
      if (mode == MODE_VELOCITY) {
        out[idx] = flow + u;
      } else if (mode == MODE_EXPLICIT) {
        xnew = qv + p.dt * (flow + u);
        out[idx] = xnew;
      } else if (mode == MODE_PICARD) {
        const float xn = qstart + p.dt * (flow0 + u);
        out[idx] = xn;
        resid = fabsf(xn - qv);
        xmax = fabsf(xn);
        xnew = xn;
      }
    }
    if ((mode == MODE_PICARD || mode == MODE_EXPLICIT) && pack.VA != nullptr) {
      // the prep kernel's work for the new iterate or state: wv already holds
      // the weights (zero past the particles)
      const float x = comp ? xnew - pack.cmean[n] : 0.f;
      const float wi = real ? wv[I] : 0.f;
      prep_write(p, I, n, x, wi, pack.cmean, pack.xc, pack.wv, pack.QB, pack.KA, pack.VA, pack.f16);
    }
    if (obs) {
      // stress column beta needs grad Psi of this bond's component beta
      const float gp0 = gshfl(gp, base), gp1 = gshfl(gp, base + 1), gp2 = gshfl(gp, base + 2);
      if (comp) {
        const double wi = (double)wv[I];
        red[RED_DISS] = wi * (double)g * (double)Ag * (double)p.inv_zeta;
        red[RED_WORK] = wi * (double)g * (double)flow;
        red[RED_TAU + 3 * al + 0] = (double)p.n * wi * (double)qv * (double)gp0;
        red[RED_TAU + 3 * al + 1] = (double)p.n * wi * (double)qv * (double)gp1;
        red[RED_TAU + 3 * al + 2] = (double)p.n * wi * (double)qv * (double)gp2;
        red[RED_F] = wi * (double)psi;
        if (n == 0) red[RED_F] += wi * (double)p.kT * (log((double)S[I]) - (double)p.log_norm);
      }
    }
  }
  if (obs) {
    block_sum<12>(red, sm);
    if (threadIdx.x < 12) redp[lb * 16 + threadIdx.x] = red[threadIdx.x];
  }
  if (mode == MODE_PICARD) {
    // block maxima of |dx| and |x| into per-block slots; the check kernel
    // takes the max over blocks (no contended atomics)
    __shared__ float smax[2][kRedBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
      resid = fmaxf(resid, __shfl_xor(resid, off));
      xmax = fmaxf(xmax, __shfl_xor(xmax, off));
    }
    if ((threadIdx.x & 63) == 0) {
      smax[0][threadIdx.x >> 6] = resid;
      smax[1][threadIdx.x >> 6] = xmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float r = 0.f, x = 0.f;
      for (int i = 0; i < kRedBlock / 64; ++i) {
        r = fmaxf(r, smax[0][i]);
        x = fmaxf(x, smax[1][i]);
      }
      blockmax[2 * lb] = r;
      blockmax[2 * lb + 1] = x;
    }
  }
}

__global__ __launch_bounds__(kRedBlock) void k_combine(EvalParams p, int mode, int obs,
                                                       const float *__restrict__ partial, SplitMap splits,
                                                       const float *xc, const float *__restrict__ t1,
                                                       const float *__restrict__ S, const float *wv,
                                                       const float *qin, const float *__restrict__ qs,
                                                       float *out, float *out2, double *__restrict__ redp,
                                                       float *__restrict__ blockmax, const int *__restrict__ done,
                                                       PackOps pack, int *fene_out) {
  if (done != nullptr && *done) return;
  combine_body(p, blockIdx.x, mode, obs, partial, splits, xc, t1, S, wv, qin, qs, out, out2, redp, blockmax, pack,
               fene_out);
}

// Sum over blocks of the FP64 block partials, slot by slot: wave s takes slot s,
// lane l folds blocks l, l + 64, ... in order, then a fixed butterfly over the
// wave (deterministic; the latency is that of nblk / 64 loads, not nblk).
__global__ __launch_bounds__(1024) void k_reduce_final(const double *__restrict__ redp, int nblk, int nslots,
                                                       double *__restrict__ out, const int *__restrict__ done) {
  if (done != nullptr && *done) return;
  const int s = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (s >= nslots) return;
  double a0 = 0.0, a1 = 0.0;
  int b = lane;
  for (; b + 64 < nblk; b += 128) {
    a0 += redp[(int64_t)b * 16 + s];
    a1 += redp[(int64_t)(b + 64) * 16 + s];
  }
  if (b < nblk) a0 += redp[(int64_t)b * 16 + s];
  double acc = a0 + a1;
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[s] = acc;
}

// Stand-alone convergence test: between the fixed-point iterations of a
// queued step (after a combine that packed the next iterate) and in the
// host-driven iterations.
__global__ __launch_bounds__(kRedBlock) void k_picard_check(PicardCheck chk, const float *__restrict__ blockmax,
                                                            int nblk_chk) {
  Ctrl *ctrl = chk.ctrl;
  // the flag and the block maxima are loaded together (one block: nothing
  // else writes the flag during this launch)
  const int done = ctrl->done;
  float r;
  const bool conv = picard_converged(chk, blockmax, nblk_chk, &r);
  if (done || threadIdx.x != 0) return;
  ctrl->last_resid = r;
  ctrl->checked = chk.iter + 1;
  if (conv) {
    ctrl->conv_iter = chk.iter;
    ctrl->done = 1;
  }
}

__global__ void k_ctrl_reset(Ctrl *ctrl) {
  if (threadIdx.x != 0) return;
  ctrl->done = 0;
  ctrl->conv_iter = -1;
  ctrl->last_resid = 0.f;
  ctrl->checked = 0;
  ctrl->halted = 0;
  ctrl->steps_done = 0;
  ctrl->last_iters = 0;
  ctrl->total_iters = 0;
  ctrl->fene_out = 0;
}

// End of a queued implicit step (see launch_step_end), one thread per
// particle.  Only block 0 writes *ctrl.  If another block sees its `halted` or
// `done` of this launch, the step did not converge (conv_iter is still -1
// then) and it returns as block 0 does.
__global__ __launch_bounds__(kRedBlock) void k_step_end(EvalParams p, Ctrl *ctrl, PicardCheck chk,
                                                        const float *__restrict__ blockmax, int nblk_chk,
                                                        const float *__restrict__ xb0, const float *__restrict__ xb1,
                                                        float *__restrict__ q, float *__restrict__ xpred,
                                                        const float *__restrict__ w, double *__restrict__ meanp) {
  // block 0 may set `halted` and `done` during this launch: one read per
  // block keeps the block's waves together
  __shared__ int st[3];
  if (threadIdx.x == 0) {
    st[0] = ctrl->halted;
    st[1] = ctrl->done;
    st[2] = ctrl->conv_iter;
  }
  // the copy's loads for the tested iteration (the usual outcome) go out
  // before the test, so that their latency overlaps it
  const int64_t I = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  const bool real = I < p.P;
  float qn[kMaxD], qo[kMaxD];
  auto at = [&](int a) { return ((int64_t)(a / 3) * p.P + I) * 3 + a % 3; };
  const float *src = (chk.iter & 1) ? xb1 : xb0;
#pragma unroll
  for (int a = 0; a < kMaxD; ++a) {
    qn[a] = 0.f;
    qo[a] = 0.f;
    if (real && a < p.D) {
      qn[a] = src[at(a)];
      if (xpred != nullptr) qo[a] = q[at(a)];
    }
  }
  __syncthreads();
  if (st[0]) return;
  int it;
  if (st[1]) {
    it = st[2];  // converged at an earlier test of this step
    if (it < 0) return;
    if ((it ^ chk.iter) & 1) {
      const float *alt = (it & 1) ? xb1 : xb0;
#pragma unroll
      for (int a = 0; a < kMaxD; ++a)
        if (real && a < p.D) qn[a] = alt[at(a)];
    }
  } else {
    float r;
    const bool conv = picard_converged(chk, blockmax, nblk_chk, &r);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->last_resid = r;
      ctrl->checked = chk.iter + 1;
      if (!conv) {
        ctrl->halted = 1;
        ctrl->done = 1;
      }
    }
    if (!conv) return;
    it = chk.iter;
  }
#pragma unroll
  for (int a = 0; a < kMaxD; ++a) {
    if (real && a < p.D) {
      if (xpred != nullptr) xpred[at(a)] = 2.f * qn[a] - qo[a];
      q[at(a)] = qn[a];
    }
  }
  // the next step's centring partials from the new state, as k_mean_partials
  // computes them (each thread reads back what it wrote)
  if (meanp != nullptr) mean_partials_body(p, blockIdx.x, q, w, meanp);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->steps_done += 1;
    ctrl->last_iters = it + 1;
    ctrl->total_iters += it + 1;
  }
}

__device__ void stress_body(const EvalParams &p, int64_t lb, const float *__restrict__ q, const float *__restrict__ w,
                            double *__restrict__ redp) {
  __shared__ double sm[9][kRedBlock];
  const int64_t I = lb * kRedBlock + threadIdx.x;
  double t[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) t[s] = 0.0;
  if (I < p.P) {
    const double wi = (double)load_weight(w, I, p.uniform_w) * (double)p.n;
    for (int k = 0; k < p.nb; ++k) {
      const float *qk = q + ((int64_t)k * p.P + I) * 3;
      const float r2 = qk[0] * qk[0] + qk[1] * qk[1] + qk[2] * qk[2];
      const float fac = p.potential == VDS_FENE ? p.H[k] / (1.f - r2 / p.b_max) : p.H[k];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t[3 * a + b] += wi * (double)qk[a] * (double)(fac * qk[b]);
    }
  }
  block_sum<9>(t, sm);
  if (threadIdx.x < 9) redp[lb * 16 + threadIdx.x] = t[threadIdx.x];
}

__global__ __launch_bounds__(kRedBlock) void k_stress(EvalParams p, const float *__restrict__ q,
                                                      const float *__restrict__ w, double *__restrict__ redp) {
  stress_body(p, blockIdx.x, q, w, redp);
}

// Foreign rows y[ny][D] (particle-major) as Q operands, centred like the particles.
__global__ __launch_bounds__(kRedBlock) void k_density_rows(EvalParams p, const float *__restrict__ y, int64_t ny,
                                                            const double *__restrict__ meanp, int nmeanp,
                                                            float *__restrict__ QB, F16Operands f16,
                                                            int64_t nrows_pad) {
  __shared__ float mean_sh[16];
  load_mean(p, meanp, nmeanp, mean_sh);
  const int64_t I = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  if (I >= nrows_pad) return;
  float x[kMaxD];
  float nrm = 0.f;
  for (int a = 0; a < p.D; ++a) {
    x[a] = I < ny ? y[I * p.D + a] - mean_sh[a] : 0.f;
    nrm = fmaf(x[a], x[a], nrm);
  }
  if (p.f32x) {  // plain centred coordinates, read by VDS_PAIR_MFMA32
    for (int a = 0; a < p.D; ++a) QB[I * p.D + a] = x[a];
    return;
  }
  for (int k = 0; k < 4 * p.KK; ++k) {
    float qa = 0.f;
    if (I < ny) {
      if (k < p.D) qa = x[k];
      else if (k == p.D) qa = -p.kappa * nrm;
      else if (k == p.D + 1) qa = 1.f;
    }
    QB[qk_index(I, k, p.KK)] = qa;
  }
  if (p.qhalf) {
    _Float16 *qh = reinterpret_cast<_Float16 *>(f16.QH);
    for (int sl = 0; sl < 32 * p.KQ; ++sl) {
      const int k = sl / 3;
      _Float16 qv, kv;
      dh_slot(p, sl, I < ny && k < p.D ? p.cs * x[k] : 0.f, 0.f, qv, kv);
      qh[dh_index(I, sl, p.KQ)] = qv;
    }
    f16.RN[I] = I < ny ? -p.kappa * nrm : 0.f;
  }
}

// QB/KA in the 16-row FP32 layout (qk_index) from the centred coordinates,
// one thread per particle (padding rows: zeros).
__global__ __launch_bounds__(kRedBlock) void k_pack_qk(EvalParams p, const float *__restrict__ xc,
                                                       float *__restrict__ QB, float *__restrict__ KA) {
  const int64_t I = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  if (I >= p.Ppad) return;
  const bool real = I < p.P;
  float x[kMaxD];
  float nrm = 0.f;
  for (int a = 0; a < p.D; ++a) {
    x[a] = real ? xc[I * p.D + a] : 0.f;
    nrm = fmaf(x[a], x[a], nrm);
  }
  for (int k = 0; k < 4 * p.KK; ++k) {
    float qa = 0.f, ka = 0.f;
    if (real) {
      if (k < p.D) {
        qa = x[k];
        ka = 2.f * p.kappa * x[k];
      } else if (k == p.D) {
        qa = -p.kappa * nrm;
        ka = 1.f;
      } else if (k == p.D + 1) {
        qa = 1.f;
        ka = -p.kappa * nrm;
      }
    }
    QB[qk_index(I, k, p.KK)] = qa;
    KA[qk_index(I, k, p.KK)] = ka;
  }
}

__global__ __launch_bounds__(kRedBlock) void k_density_out(const float *__restrict__ partial, SplitMap splits,
                                                           int64_t stride_rows, int64_t ny, int D, float norm,
                                                           float *__restrict__ f) {
  const int64_t I = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  if (I >= ny) return;
  f[I] = ordered_sum<float>(partial + I * splits.width + D, splits.count(I), stride_rows * splits.width) * norm;
}

// ---- batched ensembles: the same bodies, per ensemble ----

__global__ __launch_bounds__(kRedBlock) void k_batch_mean(BatchView b, const float *__restrict__ q,
                                                          double *__restrict__ meanp) {
  const EnsDesc &d = b.ens[b.blk256_ens[blockIdx.x]];
  mean_partials_body(d.p, blockIdx.x - d.blk256, q + d.q_off, nullptr, meanp + (int64_t)d.blk256 * 16);
}

// Ensemble d's slice of the concatenated FP16 distance operands.
__device__ inline F16Operands batch_f16(const BatchView &b, const EnsDesc &d) {
  if (!d.p.qhalf) return F16Operands{nullptr, nullptr, nullptr};
  const int64_t halves = d.pad_off * 32 * d.p.KQ;
  return F16Operands{reinterpret_cast<_Float16 *>(b.f16.QH) + halves, reinterpret_cast<_Float16 *>(b.f16.KH) + halves,
                     b.f16.RN + d.pad_off};
}

__global__ __launch_bounds__(kRedBlock) void k_batch_prep(BatchView b, const float *__restrict__ q,
                                                          const double *__restrict__ meanp, float *__restrict__ xc,
                                                          float *__restrict__ wv, float *__restrict__ QB,
                                                          float *__restrict__ KA, float *__restrict__ VA) {
  const EnsDesc &d = b.ens[b.blk16_ens[blockIdx.x]];
  const int64_t o = d.pad_off;
  prep_body(d.p, blockIdx.x - d.blk16, q + d.q_off, nullptr, meanp + (int64_t)d.blk256 * 16,
            (int)(d.p.Ppad / kRedBlock), xc + o * b.D, wv + o, QB + o * b.KK * 4, KA + o * b.KK * 4, VA + o * 16,
            nullptr, batch_f16(b, d));
}

__global__ __launch_bounds__(kRedBlock) void k_batch_finalize_a(BatchView b, const float *__restrict__ partial,
                                                                const float *__restrict__ xc,
                                                                const float *__restrict__ wv, float *__restrict__ S,
                                                                float *__restrict__ t1, float *__restrict__ VB) {
  const EnsDesc &d = b.ens[b.blk16_ens[blockIdx.x]];
  const int64_t o = d.pad_off;
  finalize_a_body(d.p, blockIdx.x - d.blk16, partial + o * 16, SplitMap{}, xc + o * b.D, wv + o, S + o, t1 + o * b.D,
                  VB + o * 16);
}

__global__ __launch_bounds__(kRedBlock) void k_batch_explicit(BatchView b, const float *__restrict__ partial,
                                                              const float *__restrict__ xc,
                                                              const float *__restrict__ t1,
                                                              const float *__restrict__ S,
                                                              const float *__restrict__ wv, float *q) {
  const EnsDesc &d = b.ens[b.blk16_ens[blockIdx.x]];
  const int64_t o = d.pad_off;
  combine_body(d.p, blockIdx.x - d.blk16, MODE_EXPLICIT, 0, partial + o * 16, SplitMap{}, xc + o * b.D, t1 + o * b.D, S + o,
               wv + o, q + d.q_off, nullptr, q + d.q_off, nullptr, nullptr, nullptr, PackOps{}, nullptr);
}

__global__ __launch_bounds__(kRedBlock) void k_batch_stress(BatchView b, const float *__restrict__ q,
                                                            double *__restrict__ redp) {
  const EnsDesc &d = b.ens[b.blk256_ens[blockIdx.x]];
  stress_body(d.p, blockIdx.x - d.blk256, q + d.q_off, nullptr, redp + (int64_t)d.blk256 * 16);
}

__global__ void k_batch_stress_sum(const EnsDesc *__restrict__ ens, const double *__restrict__ redp,
                                   double *__restrict__ tau) {
  const EnsDesc &d = ens[blockIdx.x];
  const int s = threadIdx.x;
  if (s >= 9) return;
  const int nb = (int)(d.p.Ppad / kRedBlock);
  double acc = 0.0;
  for (int i = 0; i < nb; ++i) acc += redp[((int64_t)d.blk256 + i) * 16 + s];
  tau[(int64_t)blockIdx.x * 9 + s] = acc;
}

// ---- launchers ----

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + kRedBlock - 1) / kRedBlock); }

void launch_mean_partials(const EvalParams &p, const float *q, const float *w, double *meanp, const int *done,
                          Ctrl *begin, hipStream_t s) {
  k_mean_partials<<<nblocks(p.P), kRedBlock, 0, s>>>(p, q, w, meanp, done, begin);
}
void launch_prep(const EvalParams &p, const float *q, const float *w, const double *meanp, int nmeanp, float *xc,
                 float *wv, float *QB, float *KA, float *VA, float *wscale, const F16Operands *f16, const int *done,
                 hipStream_t s, float *cmean, Ctrl *begin) {
  const F16Operands ops = f16 != nullptr ? *f16 : F16Operands{nullptr, nullptr, nullptr};
  k_prep<<<nblocks(p.Ppad * 16), kRedBlock, 0, s>>>(p, q, w, meanp, nmeanp, xc, wv, QB, KA, VA, wscale, ops, done,
                                                    cmean, begin);
}
void launch_finalize_a(const EvalParams &p, const float *partial, const SplitMap &splits, const float *xc, const float *wv,
                       float *S, float *t1, float *VB, const int *done, hipStream_t s) {
  k_finalize_a<<<nblocks(p.Ppad * 16), kRedBlock, 0, s>>>(p, partial, splits, xc, wv, S, t1, VB, done);
}
void launch_combine(const EvalParams &p, int mode, bool obs, const float *partial, const SplitMap &splits, const float *xc,
                    const float *t1, const float *S, const float *wv, const float *qin, const float *q0,
                    float *out, float *out2, double *redp, float *blockmax, const int *done, hipStream_t s,
                    const PackOps *pack, int *fene_out) {
  const PackOps pk = pack != nullptr ? *pack : PackOps{};
  k_combine<<<nblocks(p.P * 16), kRedBlock, 0, s>>>(p, mode, obs ? 1 : 0, partial, splits, xc, t1, S, wv, qin, q0,
                                                    out, out2, redp, blockmax, done, pk, fene_out);
}
void launch_reduce_final(const double *redp, int nblk, int nslots, double *out, const int *done, hipStream_t s) {
  k_reduce_final<<<1, 1024, 0, s>>>(redp, nblk, nslots, out, done);
}
void launch_ctrl_reset(Ctrl *ctrl, hipStream_t s) { k_ctrl_reset<<<1, 64, 0, s>>>(ctrl); }
void launch_step_end(const EvalParams &p, Ctrl *ctrl, const PicardCheck &chk, const float *blockmax, int nblk_chk,
                     const float *xb0, const float *xb1, float *q, float *xpred, const float *w, double *meanp,
                     hipStream_t s) {
  k_step_end<<<nblocks(p.P), kRedBlock, 0, s>>>(p, ctrl, chk, blockmax, nblk_chk, xb0, xb1, q, xpred, w, meanp);
}
void launch_picard_check(const PicardCheck &chk, const float *blockmax, int nblk_chk, hipStream_t s) {
  k_picard_check<<<1, kRedBlock, 0, s>>>(chk, blockmax, nblk_chk);
}
void launch_stress(const EvalParams &p, const float *q, const float *w, double *redp, hipStream_t s) {
  k_stress<<<nblocks(p.P), kRedBlock, 0, s>>>(p, q, w, redp);
}
void launch_density_rows(const EvalParams &p, const float *y, int64_t ny, const double *meanp, int nmeanp,
                         float *QB, const F16Operands *f16, hipStream_t s) {
  const F16Operands ops = f16 != nullptr ? *f16 : F16Operands{nullptr, nullptr, nullptr};
  // rows are padded to a multiple of 256 within the Ppad-row operand buffer
  const int64_t nrows_pad = round_up(ny, kRowAlign);
  k_density_rows<<<nblocks(nrows_pad), kRedBlock, 0, s>>>(p, y, ny, meanp, nmeanp, QB, ops, nrows_pad);
}
void launch_pack_qk(const EvalParams &p, const float *xc, float *QB, float *KA, hipStream_t s) {
  k_pack_qk<<<nblocks(p.Ppad), kRedBlock, 0, s>>>(p, xc, QB, KA);
}
void launch_density_out(const EvalParams &p, const float *partial, const SplitMap &splits, int64_t ny, float norm, float *f,
                        hipStream_t s) {
  k_density_out<<<nblocks(ny), kRedBlock, 0, s>>>(partial, splits, p.Ppad, ny, p.D, norm, f);
}

void launch_batch_mean(const BatchView &b, const float *q, double *meanp, hipStream_t s) {
  k_batch_mean<<<b.nblk256, kRedBlock, 0, s>>>(b, q, meanp);
}
void launch_batch_prep(const BatchView &b, const float *q, const double *meanp, float *xc, float *wv, float *QB,
                       float *KA, float *VA, hipStream_t s) {
  k_batch_prep<<<b.nblk16, kRedBlock, 0, s>>>(b, q, meanp, xc, wv, QB, KA, VA);
}
void launch_batch_finalize_a(const BatchView &b, const float *partial, const float *xc, const float *wv, float *S,
                             float *t1, float *VB, hipStream_t s) {
  k_batch_finalize_a<<<b.nblk16, kRedBlock, 0, s>>>(b, partial, xc, wv, S, t1, VB);
}
void launch_batch_explicit(const BatchView &b, const float *partial, const float *xc, const float *t1,
                           const float *S, const float *wv, float *q, hipStream_t s) {
  k_batch_explicit<<<b.nblk16, kRedBlock, 0, s>>>(b, partial, xc, t1, S, wv, q);
}
void launch_batch_stress(const BatchView &b, const float *q, double *redp, hipStream_t s) {
  k_batch_stress<<<b.nblk256, kRedBlock, 0, s>>>(b, q, redp);
}
void launch_batch_stress_sum(const EnsDesc *ens, int nens, const double *redp, double *tau, hipStream_t s) {
  k_batch_stress_sum<<<nens, 64, 0, s>>>(ens, redp, tau);
}

__global__ void k_copy(const float *__restrict__ src, float *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
void launch_copy(const float *src, float *dst, int64_t n, const int *, hipStream_t s) {
  k_copy<<<nblocks(n), kRedBlock, 0, s>>>(src, dst, n);
}

}  // namespace vds
