/*
 * vds_mlp.h - a learned reduced step on top of the POD reduction (not in the
 * paper): a multilayer perceptron maps the reduced state (every bond's POD
 * coefficients and the log shear rate) to the coefficient increment of one
 * time step, trained on trajectories of the particle scheme itself, and a
 * rollout that checks it against the plain scheme and falls back to it.
 *
 * Network: nin -> width -> width -> nout, SiLU after both hidden layers, FP32
 * master parameters stored flat as [W1 (width x nin), b1, W2 (width x width),
 * b2, W3 (nout x width), b3], row-major.  Loss: mean squared error over every
 * output entry.  Optimiser: Adam with bias correction.  Training products run
 * on FP32 MFMA; inference products on BF16 MFMA with FP32 accumulation.
 * Conventions of vds.h apply.
 */
#ifndef VDS_MLP_H
#define VDS_MLP_H

#include "vds.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vds_mlp_s *vds_mlp;

/* Device workspace (bytes) for the network and batches of up to max_batch rows. */
size_t vds_mlp_workspace_bytes(int32_t nin, int32_t width, int32_t nout, int32_t max_batch);
vds_status vds_mlp_create(int32_t nin, int32_t width, int32_t nout, int32_t max_batch, void *hip_stream,
                          vds_mlp *out);
vds_status vds_mlp_bind_workspace(vds_mlp m, void *ws_dev, size_t bytes);
void vds_mlp_destroy(vds_mlp m);
const char *vds_mlp_last_error(vds_mlp m);
int64_t vds_mlp_param_count(vds_mlp m);

/* Copies the flat FP32 parameters in / out (device arrays of vds_mlp_param_count
 * floats).  Setting parameters resets the Adam moments and step count. */
vds_status vds_mlp_set_params(vds_mlp m, const float *params_dev);
vds_status vds_mlp_get_params(vds_mlp m, float *params_dev);
/* Gradient of the last vds_mlp_loss_grad call, flat like the parameters. */
vds_status vds_mlp_get_grads(vds_mlp m, float *grads_dev);

/* Y_dev[n][nout] = network(X_dev[n][nin]); bf16 != 0 uses the BF16 weights
 * (refreshed from the FP32 parameters whenever they change). n <= max_batch. */
vds_status vds_mlp_forward(vds_mlp m, const float *X_dev, int32_t n, float *Y_dev, int32_t bf16);

/* nsteps learned reduced steps in place (the step of the learned reduced model
 * that replaces the POD-Galerkin step of Section 3): p_dev[nout] +=
 * network((p_dev, log_rate)) through the scaling, nsteps times, in the BF16
 * inference arithmetic of vds_mlp_forward (inputs and hidden activations
 * rounded to BF16, FP32 sums).  Needs nin = nout + 1.  Runs as one launch of
 * one workgroup that keeps the state and activations in LDS while
 * nin + 2 width + 2 nout <= 16384 floats, else layer by layer.  Asynchronous. */
vds_status vds_mlp_predict_steps(vds_mlp m, float *p_dev, float log_rate, int32_t nsteps);

/* FP32 forward and backward pass of the mean squared error against T_dev[n][nout];
 * keeps the gradient; loss_host (may be NULL) gets the loss (FP64 sum).  Synchronises
 * when loss_host is given. */
vds_status vds_mlp_loss_grad(vds_mlp m, const float *X_dev, const float *T_dev, int32_t n, double *loss_host);

/* One Adam update with the kept gradient (step count t incremented first):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
vds_status vds_mlp_adam_step(vds_mlp m, float lr, float beta1, float beta2, float eps);

/* Affine maps around the network: it sees x = (input - x_shift) / x_scale and its
 * output y means target = y * y_scale + y_shift (device arrays of nin, nin, nout,
 * nout floats; copied).  Identity until set. */
vds_status vds_mlp_set_scaling(vds_mlp m, const float *x_shift_dev, const float *x_scale_dev,
                               const float *y_shift_dev, const float *y_scale_dev);
/* Sets the scaling to the per-column means and standard deviations (FP64 sums)
 * of the inputs X_dev[n][nin] and targets T_dev[n][nout]. */
vds_status vds_mlp_fit_scaling(vds_mlp m, const float *X_dev, const float *T_dev, int32_t n);

/* Training pairs from a reduced trajectory traj_dev[nt][nout] at one shear
 * rate: X_dev[i] = (traj[i], log_rate), T_dev[i] = traj[i+1] - traj[i] for
 * i < nt - 1 (requires nin = nout + 1). */
vds_status vds_mlp_make_pairs(vds_mlp m, const float *traj_dev, int32_t nt, float log_rate, float *X_dev,
                              float *T_dev);

/* Input-noise regularisation of vds_mlp_train_epoch (for learned steps, nin =
 * nout + 1): each gathered input coefficient c < nout gets sigma * y_scale[c]
 * * xi in raw units, xi standard normal (SplitMix64 counters and the
 * Box-Muller transform, stream `seed`, restarted by this call), the target
 * unchanged, so that the network's increment varies little off the training
 * trajectories.  sigma = 0 (the default) turns it off. */
vds_status vds_mlp_set_input_noise(vds_mlp m, float sigma, uint64_t seed);

/* One pass over n raw samples in minibatches of `batch` rows: each minibatch
 * gathers rows order_dev[i] (a permutation of 0..n-1 supplied by the caller;
 * NULL = in order), applies the scaling, then loss_grad + adam_step (beta1 0.9,
 * beta2 0.999, eps 1e-8).  loss_host (may be NULL) receives the mean minibatch
 * loss in scaled units.  Synchronises. */
vds_status vds_mlp_train_epoch(vds_mlp m, const float *X_dev, const float *T_dev, int32_t n, int32_t batch, float lr,
                               const int32_t *order_dev, double *loss_host);

/* Rollout statistics. */
typedef struct vds_mlp_rollout {
  int32_t steps;          /* steps taken */
  int32_t checks;         /* windows checked */
  int32_t fallbacks;      /* windows redone with the plain scheme */
  int32_t reserved;
  double max_resid;       /* largest full-step residual seen */
  double max_energy_gap;  /* largest relative energy-law gap seen */
  double tau[9];          /* stress of the final reconstructed state */
} vds_mlp_rollout;

/* Workspace of a rollout on the problem of `ctx` with a rank-R basis. */
size_t vds_mlp_rollout_workspace_bytes(const vds_problem *prob, int32_t R);

/* Advances the reduced state p_dev[nb][R] (nin = nb R + 1, nout = nb R) by
 * nsteps learned steps p += network increment, in windows of check_every steps.
 * After each window, at q~ = U p: (a) the energy law over the window,
 * |F_h(end) - F_h(start) - dt sum (work - dissipation)| <= energy_tol
 * dt sum (|work| + dissipation) (trapezoid rule), and (b) the full-step
 * residual |dp_net - U^T dt v(q~)| / |U^T dt v(q~)| <= resid_tol, with v the
 * particle scheme's velocity.  A window that fails either check is redone from
 * its start with the plain scheme of `ctx` (check_every steps) and re-projected.
 * U_dev is 3P x R column-major.  Synchronises. */
vds_status vds_mlp_rollout_run(vds_mlp m, vds_ctx ctx, const float *U_dev, int32_t R, float *p_dev, float log_rate,
                               int32_t nsteps, int32_t check_every, double resid_tol, double energy_tol,
                               void *ws_dev, size_t ws_bytes, vds_mlp_rollout *stats);

#ifdef __cplusplus
}
#endif

#endif /* VDS_MLP_H */
