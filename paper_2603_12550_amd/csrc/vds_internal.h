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
constexpr int kRedBlock = 256;     // threads per block of the O(P) kernels
constexpr int kNumRed = 16;        // FP64 reduction slots: F, diss, work, tau[9], spare

// Reduction slot indices.
enum { RED_F = 0, RED_DISS = 1, RED_WORK = 2, RED_TAU = 3 };

// Device control block of the implicit iteration.
struct Ctrl {
  int done;           // set once the iteration has converged
  int conv_iter;      // iteration index (0-based) that converged
  float last_resid;   // max |x_new - x_old| of the last checked iteration
  int checked;        // iterations checked so far in this step
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
};

// Modes of the combine kernel.
enum CombineMode { MODE_TERMS = 0, MODE_VELOCITY = 1, MODE_EXPLICIT = 2, MODE_PICARD = 3, MODE_OBS_ONLY = 4 };

// ---- launchers (pair_kernels.hip) ----
// Writes partial[split][row][0..D) = sum_J e wh (x_row - x_J) and [D] = sum_J e wh,
// J = row left out when exclude_self (rows are the particles themselves).
// `xc` holds the centred row coordinates the difference sums use.
void launch_pair_pass(const vds_tuning &t, int KK, int D, const float *QB, int64_t nrow_blocks,
                      const float *KA, const float *VB, int64_t ncol_chunks, const float *xc, bool exclude_self,
                      float *partial,
                      int64_t part_stride_rows, const int *done, hipStream_t s);
bool pair_shape_ok(const vds_tuning &t, int D);

// ---- launchers (local_kernels.hip) ----
void launch_mean_partials(const EvalParams &p, const float *q, const float *w, double *meanp, const int *done, hipStream_t s);
void launch_prep(const EvalParams &p, const float *q, const float *w, const double *meanp, int nmeanp,
                 float *xc, float *wv, float *QB, float *KA, float *VA, const int *done, hipStream_t s);
void launch_finalize_a(const EvalParams &p, const float *partial, int splits, const float *xc, const float *wv,
                       float *S, float *t1, float *VB, const int *done, hipStream_t s);
void launch_combine(const EvalParams &p, int mode, bool obs, const float *partial, int splits, const float *xc,
                    const float *t1, const float *S, const float *wv, const float *qin, const float *qstar,
                    float *out, float *out2, double *redp, float *blockmax, const int *done, hipStream_t s);
void launch_reduce_final(const double *redp, int nblk, int nslots, double *out, const int *done, hipStream_t s);
void launch_qstar(const EvalParams &p, const float *q, float *qstar, hipStream_t s);
void launch_picard_check(Ctrl *ctrl, const float *blockmax, int nblk, float rtol, int iter, hipStream_t s);
void launch_ctrl_reset(Ctrl *ctrl, hipStream_t s);
void launch_stress(const EvalParams &p, const float *q, const float *w, double *redp, hipStream_t s);
void launch_density_rows(const EvalParams &p, const float *y, int64_t ny, const double *meanp, int nmeanp,
                         float *QB, hipStream_t s);
void launch_density_out(const EvalParams &p, const float *partial, int splits, int64_t ny, float norm,
                        float *f, hipStream_t s);
void launch_copy(const float *src, float *dst, int64_t n, const int *done_flag_or_null, hipStream_t s);

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

}  // namespace vds
