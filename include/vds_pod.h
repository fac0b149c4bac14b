/*
 * vds_pod.h - POD offline phase, POD maps and the Galerkin reduced model of
 * the particle scheme (paper Sections 1.3, 2.3, 2.4 and 3.1).
 *
 * Conventions of vds.h apply (device pointers *_dev owned by the caller,
 * stream-ordered calls on the context's stream, status codes, host-side
 * validation before any launch).  The snapshot matrix and the basis are FP32
 * and column-major; the symmetric eigensolve runs in FP64.
 */
#ifndef VDS_POD_H
#define VDS_POD_H

#include "vds.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- POD offline phase (Section 1.3; method of snapshots, Section 3.1) ---- */

/* Device workspace (bytes) for vds_pod_gram / vds_pod_basis on an m x ncols
 * snapshot matrix and rank R. */
size_t vds_pod_workspace_bytes(int64_t m, int32_t ncols, int32_t R);

/* Gram matrix gram_dev[ncols][ncols] (row-major, symmetric) = X^T X of the
 * column-major snapshot matrix X_dev (m rows, leading dimension m): column
 * (l, k) is the bond-k slice q_{k:}(t_l) of snapshot l, so a run of snapshots
 * stored back to back in the state layout [nb][P][3] is X with m = 3P and
 * ncols = snapshots * nb.  FP32 MFMA products, fixed-order split-K sums. */
vds_status vds_pod_gram(vds_ctx ctx, const float *X_dev, int64_t m, int32_t ncols, float *gram_dev,
                        void *ws_dev, size_t ws_bytes);

/* POD basis U_dev[R][m] (column-major m x R, orthonormal columns) from the
 * eigenvectors of the Gram matrix (method of snapshots): X^T X = V L V^T in
 * FP64 (descending), U = X V_R L_R^{-1/2}, then re-orthonormalised by three
 * Cholesky-QR passes (the first with a small diagonal shift).  eig_host[ncols]
 * receives all eigenvalues, descending (= squared singular values of X).
 * Requires 1 <= R <= min(m, ncols).  Synchronises. */
vds_status vds_pod_basis(vds_ctx ctx, const float *X_dev, int64_t m, int32_t ncols, int32_t R, float *U_dev,
                         double *eig_host, void *ws_dev, size_t ws_bytes);

/* p_dev[nb][R] = U^T q_{k:} for every bond of q_dev[nb][P][3] (eq. model_pq);
 * U is 3P x R column-major.  Uses the context's nb and P.  ws as for
 * vds_pod_map_workspace_bytes. */
size_t vds_pod_map_workspace_bytes(const vds_problem *prob, int32_t R);
vds_status vds_pod_project(vds_ctx ctx, const float *U_dev, int32_t R, const float *q_dev, float *p_dev,
                           void *ws_dev, size_t ws_bytes);
/* q_dev[nb][P][3] = U p_{k:} for every bond (eq. model_pq). */
vds_status vds_pod_reconstruct(vds_ctx ctx, const float *U_dev, int32_t R, const float *p_dev, float *q_dev,
                               void *ws_dev, size_t ws_bytes);

/* ---- Galerkin reduced model (Section 2.4, eq. model_DymReduced) ---------- */

typedef struct vds_rom_s *vds_rom;

/* Workspace for a reduced model of rank R on the context's problem.  The
 * kernel-GEMM's launch shape, and so the size, follows the compute-unit count
 * of the current device: query it with the device current that the model
 * will run on (vds_rom_create checks the size and fails with VDS_ERR_NOMEM
 * when it is short). */
size_t vds_rom_workspace_bytes(const vds_problem *prob, int32_t R);

/* Builds the reduced model of basis U_dev (3P x R column-major, orthonormal
 * columns) on the Hookean problem of `ctx` with uniform weights (the paper's
 * setting): the mode blocks U_alpha (rows (I, alpha) of U), their products
 * M_ab = U_a^T U_b, and the hydrodynamic operator X^H = sum_ab G_ab M_ab.
 * Keeps U_dev (not copied).  The context must stay alive. */
vds_status vds_rom_create(vds_ctx ctx, const float *U_dev, int32_t R, void *ws_dev, size_t ws_bytes, vds_rom *out);
void vds_rom_destroy(vds_rom rom);

/* Reduced operators at the reconstruction q~ = U p of p_dev[nb][R]: the
 * Brownian operators X^B1, X^B2 from the kernel matrix Z_IK = K_h(q~_I - q~_K)
 * (frozen nonlinearity, Section 2.4), and X^H; outputs R x R row-major device
 * arrays (any may be NULL).  Evaluated as products of the mode blocks with
 * Z (applied on the fly, never stored): X^B1 = -(1/h^2)(sum_a U_a^T U_a -
 * sum_a U_a^T diag(1/S) Z diag(w) U_a), X^B2 = -(1/h^2)(sum_a U_a^T diag(T) U_a
 * - sum_a U_a^T Z diag(w/S) U_a), S = Z w, T = Z (w/S). */
vds_status vds_rom_operators(vds_rom rom, const float *p_dev, float *XH_dev, float *XB1_dev, float *XB2_dev);

/* Advances p_dev[nb][R] by nsteps explicit Euler steps of eq.
 * model_DymReduced (Section 3.1), rebuilding X^B1 and X^B2 at q~ = U p before
 * steps 0, M, 2M, ... (M = freeze_every >= 1) and keeping p.
 * tau_hist_host (may be NULL) receives the stress history of the reconstructed
 * states (Section 2.1; the quantity of the stress comparisons of Section 3),
 * each evaluated from p and the M_ab without reconstruction, row-major 3 x 3
 * per entry: with output_every >= 1, entry i holds the stress after step
 * min((i + 1) output_every, nsteps), so ceil(nsteps / output_every) entries
 * (the last one after the final step); with output_every == 0, one entry, the
 * stress after the final step (also for nsteps == 0).  The host buffer must
 * hold that many entries of 9 doubles.  VDS_ERR_ARG for nsteps < 0,
 * freeze_every < 1 or output_every < 0.  Synchronises. */
vds_status vds_rom_run(vds_rom rom, float *p_dev, int32_t nsteps, int32_t freeze_every, int32_t output_every,
                       double *tau_hist_host);

/* As vds_rom_run, with the operators of each window (n steps) rebuilt at the
 * state predicted for its midpoint (not in the paper): after the freeze at the
 * window's start, n / 2 steps from there give q~ for a second freeze, and the
 * window then runs from its start with those operators (a window of one step
 * has no midpoint and keeps the start's).  The freeze error of a window falls
 * from first to second order in its length, at two freezes and 1.5 n steps
 * per window.  Synchronises. */
vds_status vds_rom_run_midpoint(vds_rom rom, float *p_dev, int32_t nsteps, int32_t freeze_every,
                                double *tau_host);

/* As vds_rom_run_midpoint (not in the paper either), with one freeze per
 * window after the first: a window of n steps whose predecessor had n_prev
 * steps and started at p_prev takes its operators at
 * p + (n / 2) / n_prev (p - p_prev), the midpoint state extrapolated on the
 * line through the two window starts.  The first window, and any window of
 * one step, behaves as in vds_rom_run_midpoint.  The extrapolated state is
 * second order in the window length, as the predicted one is, so the freeze
 * error stays second order at half the freezes and n steps per window.
 * Uses the reduced model's own workspace (two nb x R buffers).  Arguments and
 * errors as vds_rom_run.  Synchronises. */
vds_status vds_rom_run_extrapolated(vds_rom rom, float *p_dev, int32_t nsteps, int32_t freeze_every,
                                    double *tau_host);

/* Stress of q~ = U p from p_dev and the M_ab: tau_ab = (n/P) sum_j H_j p_j^T M_ab p_j. */
vds_status vds_rom_stress(vds_rom rom, const float *p_dev, double *tau_host);

/* ---- exact integration of the frozen windows (beyond the paper) ----------- */

/* Between freezes eq. model_DymReduced is linear with constant coefficients,
 * so a window of length t_w advances vec(p) (index k R + s) exactly by
 * exp(t_w L), L the (nb R) x (nb R) generator of the reduced equation with X^B
 * frozen at the window start (FP64: scaling so that |t_w L / 2^s|_1 <= 1/2, a
 * degree-12 Taylor polynomial, s squarings; rocBLAS FP64 GEMMs).  The windows
 * cover nsteps dt; the first is freeze_every dt long.
 *   adaptive = 0: every window has that length (the last one may be shorter).
 *   adaptive != 0: after each window the energy law of the reconstructed
 *   states q~ = U p is checked with the trapezoid rule,
 *     |F(e) - F(s) - t_w ((W - D)(s) + (W - D)(e)) / 2|
 *         <= energy_tol t_w ((|W| + D)(s) + (|W| + D)(e)) / 2,
 *   a window that fails is halved and redone (down to dt, where it is accepted
 *   and counted as truncated), and one whose gap is under a quarter of its
 *   bound doubles the next, up to freeze_every dt: the check only ever shortens
 *   the requested freeze interval.  (The energy law bounds the freeze error of a
 *   window, not the truncation error of the basis, which grows when a long
 *   window runs into the part of the trajectory the snapshots did not cover.)
 * windows_host[max_windows] (NULL with max_windows = 0) receives the accepted
 * window lengths in order, so the run can be replayed; stats (may be NULL) the
 * counts.  ws_dev: vds_rom_exact_workspace_bytes bytes of device scratch.
 * tau_host (may be NULL) as for vds_rom_run.  Synchronises. */
typedef struct vds_rom_window_stats {
  int32_t windows;        /* accepted windows */
  int32_t rejected;       /* windows halved and redone */
  int32_t truncated;      /* windows accepted at the smallest length dt despite the check */
  int32_t recorded;       /* entries written to windows_host */
  double t_reached;       /* time covered */
  double max_energy_gap;  /* largest accepted gap relative to its bound, times energy_tol */
} vds_rom_window_stats;

size_t vds_rom_exact_workspace_bytes(const vds_problem *prob, int32_t R);
vds_status vds_rom_run_exact(vds_rom rom, float *p_dev, int32_t nsteps, int32_t freeze_every, int32_t adaptive,
                             double energy_tol, double *windows_host, int32_t max_windows, void *ws_dev,
                             size_t ws_bytes, double *tau_host, vds_rom_window_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* VDS_POD_H */
