// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vds.h"

namespace vds {

constexpr int kMaxNb = 5;          // D = 3 nb <= 15 keeps D + 1 within one 16-wide MFMA tile
constexpr int kMaxD = 3 * kMaxNb;
constexpr int kMaxSplits = 32;     // column splits the partial-sum buffer is sized for
constexpr int kRowAlign = 256;     // particle padding: rows and columns come in multiples of this
constexpr int kHistBins = 4096;   // bins per target of the median-bandwidth selection
constexpr int kRedBlock = 256;     // threads per block of the O(P) kernels
constexpr int kNumRed = 16;        // FP64 reduction slots: F, diss, work, tau[9], spare

// Reduction slot indices.
enum { RED_F = 0, RED_DISS = 1, RED_WORK = 2, RED_TAU = 3 };

// Device control block of the implicit iteration.  Every kernel of a step
// returns at once while `done` is set, so iterations queued past convergence
// cost a launch each and nothing more.
struct Ctrl {
  int done;               // the current step converged, or the queue halted
  int conv_iter;          // iteration (0-based) that converged in this step, -1 before
  float last_resid;       // max |x_new - x_old| of the last checked iteration
  int checked;            // iterations checked so far in this step
  int halted;             // a queued step used its iterations without converging
  int steps_done;         // queued steps written back since the last reset
  int last_iters;         // iterations of the last step written back
  long long total_iters;  // iterations of the steps written back since the last reset
  int fene_out;           // a combine kernel saw a FENE bond with |q|^2 >= b_max (or not finite)
};

// Convergence test of one fixed-point iteration, taken from the combine
// kernel's block maxima by the next kernel in stream order.
struct PicardCheck {
  Ctrl *ctrl;
  float rtol;     // converged when max|dx| <= rtol * max(1, max|x|)
  int iter;    // index of the tested iteration within the step
};

// Kernel-side description of one evaluation.
struct EvalParams {
  int64_t P;          // particles
  int64_t Ppad;       // padded particles (multiple of kRowAlign)
  int nb, D, KK;      // bonds, D = 3 nb, MFMA k-steps (augmented length 4 KK)
  float kappa;        // log2(e) / (2 h^2)
  float inv_h2;       // 1 / h^2
  float kT, inv_zeta, dt, n;
  float G[9];
  float H[kMaxNb];
  float b_max;
  int potential;
  float uniform_w;    // 1 / P
  float log_norm;     // (D/2) log(2 pi h^2)
  int vhalf;          // V operands as FP16 high/low halves (FP16-split products), weights over their maximum
  int qhalf;          // FP16 distance operands QH/KH and row norms RN written too (VDS_PAIR_MFMA_F16X2_ALL)
  int KQ;             // FP16 distance slices of 32 products: f16_slices(D)
  float cs;           // sqrt(2 kappa): the distance operands are cs x
  int f32x;           // FP32 operands in the per-chunk layout of VDS_PAIR_MFMA32 (KC in the KA buffer,
                      // V in VA/VB at vc_index); QB/KA in the 16-row layout are then not written
  int KP;             // K slots of that kernel's distance product: D + 2 rounded up to even
};

// FP32 operands of VDS_PAIR_MFMA32, per chunk of 32 columns (see pair_kernels.hip):
//   KC: slot k < KP of column J at [((J / 32) * KP + k) * 32 + J % 32], slot k < D holding
//       2 kappa x_J[k], slot D the column norm term -kappa |x_J|^2, slot D + 1 one (the row
//       side holds x_I, 1 and the row norm term there), zero beyond;
//   V:  element n < 16 of V_J at [J * 16 + (n % 4) * 4 + n / 4], so that the float4 at
//       J * 4 + j holds elements j, 4 + j, 8 + j, 12 + j.
__host__ __device__ constexpr int mfma32_kslots(int D) { return (D + 3) & ~1; }
__host__ __device__ inline int64_t kc_index(int64_t J, int k, int KP) { return ((J >> 5) * KP + k) * 32 + (J & 31); }
__host__ __device__ inline int64_t vc_index(int64_t J, int n) { return J * 16 + (n & 3) * 4 + (n >> 2); }

// FP16 MFMA slices (32 products each) of the split distance product: three
// per configuration component and two for the column norm.
__host__ __device__ constexpr int f16_slices(int D) { return (3 * D + 2 + 31) / 32; }

// Workspace of the FP16 distance operands (see pair_kernels.hip).
struct F16Operands {
  void *QH;   // [Ppad / 16][KQ][64 lanes][8] halves, row side
  void *KH;   // same layout, column side
  float *RN;  // [Ppad] -kappa |x_I|^2
};

// One ensemble of a batch: its problem parameters and where its particles sit
// in the concatenated arrays.  Every ensemble is padded to a multiple of
// kRowAlign particles, so each 16- or 256-particle block belongs to one ensemble.
struct EnsDesc {
  EvalParams p;
  int64_t pad_off;  // first padded particle in the operand arrays
  int64_t q_off;    // first float of the ensemble's state [nb][P][3] in the packed state
  int blk16;        // first 16-particle block of the ensemble
  int blk256;       // first 256-particle block of the ensemble
};

// sum_{k < n} src[k stride], added in the order of k into Acc.  The loads of
// eight terms are issued together, so a sum over column splits or block
// partials waits for one memory latency per eight terms rather than one per
// term (a plain loop waits for each load before its add).  Terms past n are
// read as zero, which leaves every sum unchanged.
template <typename Acc, typename T>
__device__ inline Acc ordered_sum(const T *__restrict__ src, int n, int64_t stride) {
  Acc o = Acc(0);
  for (int k0 = 0; k0 < n; k0 += 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k0 + j < n ? src[(int64_t)(k0 + j) * stride] : T(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) o += (Acc)v[j];
  }
  return o;
}

// fmax(init, src[k stride]) over k < n (NaN terms ignored, as fmax does),
// the loads issued eight at a time.
template <typename T>
__device__ inline T strided_max(const T *__restrict__ src, int n, int64_t stride, T init) {
  T m = init;
  for (int k0 = 0; k0 < n; k0 += 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k0 + j < n ? src[(int64_t)(k0 + j) * stride] : init;
#pragma unroll
    for (int j = 0; j < 8; ++j) m = fmax(m, v[j]);
  }
  return m;
}

// Terms of a strided loop b = first, first + step, ... < end.
__host__ __device__ inline int strided_count(int first, int end, int step) {
  return first < end ? (end - first + step - 1) / step : 0;
}

// Where a pair pass leaves its partial sums: partial[slot][row][width] for the
// slots 0 .. count(row) - 1, which the consuming kernels add in slot order
// (width 16, or D + 1 where the pass writes only the D + 1 sums of a row).
// Fixed splits (G == 0): every row has `splits` slots, one per column range.
// Balanced grid (VDS_PAIR_MFMA32): the row-group-major sequence of
// (row group, column chunk) units is cut into G runs of equal length, one per
// workgroup; a run leaves one slot in every row group it covers, and the runs
// covering a row group fill its slots in run order.
struct SplitMap {
  int width = 16;          // floats per row of a slot: 16, or D + 1 for the compact layout
  int splits = 1;          // fixed splits; with G > 0, a bound on count()
  int G = 0;               // runs (workgroups) of the balanced grid, 0 for fixed splits
  int rows_per_group = 0;  // rows of one row group
  int64_t nch = 0;         // column chunks per row group
  int64_t n_rg = 0;        // row groups
  __host__ __device__ int64_t units() const { return n_rg * nch; }
  // first unit of run L, and the run holding unit u
  __host__ __device__ int64_t run_start(int64_t L) const { return L * units() / G; }
  __host__ __device__ int64_t run_of(int64_t u) const { return ((u + 1) * G - 1) / units(); }
  __host__ __device__ int count(int64_t row) const {
    if (G == 0) return splits;
    const int64_t rg = row / rows_per_group;
    return (int)(run_of((rg + 1) * nch - 1) - run_of(rg * nch) + 1);
  }
};

// Operands the combine kernel packs for the next fixed-point iterate, as the
// prep kernel would (VA == nullptr: no packing).  cmean holds the step's
// centre in slots 0..D-1 and the weight maximum in slot 15, as the prep
// kernel of the step's first iteration wrote them.
struct PackOps {
  float *xc, *wv, *QB, *KA, *VA;
  F16Operands f16;
  const float *cmean;
};

// Modes of the combine kernel.
enum CombineMode { MODE_TERMS = 0, MODE_VELOCITY = 1, MODE_EXPLICIT = 2, MODE_PICARD = 3, MODE_OBS_ONLY = 4 };

// ---- launchers (pair_kernels.hip) ----
// Writes partial[slot][row][0..D) = sum_J e wh (x_row - x_J) and [D] = sum_J e wh
// in the layout pair_split_map gives for the pass (slot width 16, or D + 1 for
// VDS_PAIR_MFMA32), J = row left out when exclude_self (rows are the particles
// themselves).
// `xc` holds the centred row coordinates the difference sums use; ncol_pad is
// the padded column count the V operand was written for.  With the FP16-split
// implementation the V weights were divided by *wscale (NULL: by one), which
// the pass multiplies back.
// VDS_PAIR_MFMA32 reads its rows from QB as plain coordinates [nrow_blocks * 16][D] (the
// centred particles, or centred foreign rows), KC from KA and V from VB in the per-chunk
// layout above; kappa = log2(e) / 2h^2.
void launch_pair_pass(const vds_tuning &t, int KK, int D, const float *QB, int64_t nrow_blocks,
                      const float *KA, const float *VB, int64_t ncol_chunks, int64_t ncol_pad, const float *xc,
                      bool exclude_self, const float *wscale, const F16Operands &f16, float *partial,
                      int64_t part_stride_rows, const int *done, hipStream_t s, float kappa = 0.f);
bool pair_shape_ok(const vds_tuning &t, int D);
// Compute units of the current device (256 on MI355X; 256 if the query fails).
int device_cu_count();
// The slots a pass of tuning t over nrow_blocks 16-row blocks and ncol_chunks
// 16-column chunks writes (launch_pair_pass takes its grid from the same map).
SplitMap pair_split_map(const vds_tuning &t, int D, int64_t nrow_blocks, int64_t ncol_chunks);
// Batched pair pass over the (ensemble, row tile) work list `items` with a
// persistent grid of `grid` workgroups; rb = row blocks per wavefront.
// impl selects the pair implementation (VDS_PAIR_MFMA or one of the FP16-split
// ones, whose operand formats the ensembles' vhalf / qhalf flags must match);
// pass_a tells the FP16-split kernels that V holds the uniform weights 1/P_e.
void launch_batch_pair(int impl, int rb, int grid, int KK, int D, const int2 *items, int nitems, const EnsDesc *ens,
                       const float *QB, const float *KA, const float *VB, const F16Operands &f16, bool pass_a,
                       const float *xc, float *partial, hipStream_t s);

// ---- launchers (local_kernels.hip) ----
// With `begin`, the launch also opens a queued implicit step: it does nothing
// once the queue has halted, and otherwise clears the step's fields of *begin.
void launch_mean_partials(const EvalParams &p, const float *q, const float *w, double *meanp, const int *done,
                          Ctrl *begin, hipStream_t s);
// With p.vhalf, VA is written as FP16 halves (see pair_kernels.hip) with the
// weights divided by their maximum, which goes to *wscale; with p.qhalf the
// FP16 distance operands and row norms too (f16 may be null otherwise).
// cmean (may be null) receives the centre and weight maximum (see PackOps).
// With `begin`, the launch opens a queued implicit step as
// launch_mean_partials does (and ignores `done`).
void launch_prep(const EvalParams &p, const float *q, const float *w, const double *meanp, int nmeanp,
                 float *xc, float *wv, float *QB, float *KA, float *VA, float *wscale, const F16Operands *f16,
                 const int *done, hipStream_t s, float *cmean = nullptr, Ctrl *begin = nullptr);
void launch_finalize_a(const EvalParams &p, const float *partial, const SplitMap &splits, const float *xc, const float *wv,
                       float *S, float *t1, float *VB, const int *done, hipStream_t s);
// In MODE_PICARD, q0 is the state at the start of the step (the flow term is
// taken there) and each block leaves its maxima of |dx| and |x| in blockmax.
// With `pack` (MODE_PICARD or MODE_EXPLICIT), it also writes the pair operands
// of the new iterate or state from `out`, centred at pack->cmean (the prep
// kernel's work for it).
// With fene_out (FENE springs), a bond of qin outside the spring's domain sets
// *fene_out to 1.
void launch_combine(const EvalParams &p, int mode, bool obs, const float *partial, const SplitMap &splits, const float *xc,
                    const float *t1, const float *S, const float *wv, const float *qin, const float *q0,
                    float *out, float *out2, double *redp, float *blockmax, const int *done, hipStream_t s,
                    const PackOps *pack = nullptr, int *fene_out = nullptr);
void launch_reduce_final(const double *redp, int nblk, int nslots, double *out, const int *done, hipStream_t s);
void launch_ctrl_reset(Ctrl *ctrl, hipStream_t s);
// Closes a queued implicit step whose last queued iteration is chk.iter: tests
// it unless an earlier test converged, then copies the converged iterate
// (xb[conv_iter & 1]) into q and counts the step, or halts the queue.  With
// xpred it also writes the next step's starting point 2 q^(n+1) - q^n there.
// With meanp it also leaves the centring partials of the new q there, as
// launch_mean_partials would.
void launch_step_end(const EvalParams &p, Ctrl *ctrl, const PicardCheck &chk, const float *blockmax, int nblk_chk,
                     const float *xb0, const float *xb1, float *q, float *xpred, const float *w, double *meanp,
                     hipStream_t s);
// Stand-alone test of iteration chk.iter, one block (queued steps after a
// packing combine; host-driven iterations).
void launch_picard_check(const PicardCheck &chk, const float *blockmax, int nblk_chk, hipStream_t s);
void launch_stress(const EvalParams &p, const float *q, const float *w, double *redp, hipStream_t s);
// With p.f32x the centred rows go to QB as plain coordinates [rows][D] (VDS_PAIR_MFMA32).
void launch_density_rows(const EvalParams &p, const float *y, int64_t ny, const double *meanp, int nmeanp,
                         float *QB, const F16Operands *f16, hipStream_t s);
// QB/KA in the 16-row FP32 layout from the centred coordinates xc (the FP32 kernel GEMM of
// the reduced model reads them; under p.f32x the prep kernels write the per-chunk layout).
void launch_pack_qk(const EvalParams &p, const float *xc, float *QB, float *KA, hipStream_t s);
void launch_density_out(const EvalParams &p, const float *partial, const SplitMap &splits, int64_t ny, float norm,
                        float *f, hipStream_t s);
void launch_copy(const float *src, float *dst, int64_t n, const int *done_flag_or_null, hipStream_t s);
// q[k][i] = sum_r U[r][i] p[k][r] for i < m, k < nb (U is m x R column-major; pod.hip).
void launch_pod_reconstruct(const float *U, int64_t m, int R, int nb, const float *p, float *q, hipStream_t s);

// ---- batched per-particle kernels (local_kernels.hip) ----
// Block tables: blk16_ens[b] / blk256_ens[b] = ensemble of 16- / 256-particle block b.
struct BatchView {
  const EnsDesc *ens;
  const int *blk16_ens;
  const int *blk256_ens;
  int nblk16, nblk256;  // total blocks over all ensembles (padded particles)
  int D, KK;
  F16Operands f16;      // concatenated FP16 distance operands (used when the ensembles' qhalf is set)
};
void launch_batch_mean(const BatchView &b, const float *q, double *meanp, hipStream_t s);
void launch_batch_prep(const BatchView &b, const float *q, const double *meanp, float *xc, float *wv, float *QB,
                       float *KA, float *VA, hipStream_t s);
void launch_batch_finalize_a(const BatchView &b, const float *partial, const float *xc, const float *wv, float *S,
                             float *t1, float *VB, hipStream_t s);
void launch_batch_explicit(const BatchView &b, const float *partial, const float *xc, const float *t1,
                           const float *S, const float *wv, float *q, hipStream_t s);
void launch_batch_stress(const BatchView &b, const float *q, double *redp, hipStream_t s);
// tau[e][9] = sum of the stress block partials of ensemble e (one block per ensemble).
void launch_batch_stress_sum(const EnsDesc *ens, int nens, const double *redp, double *tau, hipStream_t s);

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

}  // namespace vds
