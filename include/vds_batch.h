/*
 * vds_batch.h - many independent particle ensembles (one per macroscopic
 * point of a micro-macro coupling, Section 1.1 of the paper) advanced together:
 * every ensemble has its own particle count P_b, bandwidth h_b and velocity
 * gradient G_b, and shares the chain model (bonds, springs, friction, kT, dt).
 *
 * Conventions of vds.h apply.  Each step is the explicit Euler step of the
 * particle scheme (Appendix A; the scheme of the paper's experiments) applied
 * to every ensemble; a step is five launches captured once into a hipGraph and
 * replayed, and each kernel pass covers all ensembles (the pair pass is one
 * persistent launch over a work list of (ensemble, row tile) items sorted by
 * decreasing cost).  Weights are uniform within each ensemble.
 */
#ifndef VDS_BATCH_H
#define VDS_BATCH_H

#include "vds.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vds_batch_s *vds_batch;

/* Device workspace (bytes) for nens ensembles of P_host[nens] particles and
 * nb bonds (0 if invalid). */
size_t vds_batch_workspace_bytes(int32_t nens, const int64_t *P_host, int32_t nb);

/* Validates and creates a batch.  h_host[nens] > 0; G_host[nens][9] row-major;
 * `common` supplies nb, potential, kT, zeta, n, dt, b_max (its P, h, G and
 * scheme are ignored); H_host[nb] > 0.  Launches on `hip_stream` (a
 * hipStream_t, NULL = null stream); graph capture uses a private stream that
 * is ordered after it with events. */
vds_status vds_batch_create(int32_t nens, const int64_t *P_host, const double *h_host, const double *G_host,
                            const vds_problem *common, const double *H_host, void *hip_stream, vds_batch *out);
/* Binds caller-owned device memory (>= vds_batch_workspace_bytes, 256-byte
 * aligned) and uploads the ensemble tables (synchronises). */
vds_status vds_batch_bind_workspace(vds_batch b, void *ws_dev, size_t bytes);
void vds_batch_destroy(vds_batch b);
const char *vds_batch_last_error(vds_batch b);

/* Float offset of ensemble e's state [nb][P_e][3] in the packed state array
 * (ensembles stored back to back in order); e = nens gives the total length. */
int64_t vds_batch_state_offset(vds_batch b, int32_t e);

/* Pair-pass implementation (VDS_PAIR_MFMA32, VDS_PAIR_MFMA, VDS_PAIR_MFMA_F16X2
 * or VDS_PAIR_MFMA_F16X2_ALL; see vds.h) and launch shape: row blocks per
 * wavefront (1, 2, 4; 1 or 2 for VDS_PAIR_MFMA32, whose blocks hold 32 rows)
 * and persistent grid size (workgroups, >= 1);
 * use_graph = 0 launches each step eagerly.  Changing the implementation
 * synchronises (the ensemble table is re-uploaded). */
vds_status vds_batch_set_tuning(vds_batch b, int32_t impl, int32_t rows_per_wave, int32_t grid, int32_t use_graph);
vds_status vds_batch_get_tuning(vds_batch b, int32_t *impl, int32_t *rows_per_wave, int32_t *grid,
                                int32_t *use_graph);
/* Times the admissible launch shapes (row blocks per wavefront, grid) of the
 * current implementation on the packed state q_dev and keeps the fastest; the
 * implementation, and so the arithmetic, is left as set (synchronises).  A new
 * batch starts with VDS_PAIR_MFMA32 (FP32), 2 row blocks per wavefront and
 * 1024 workgroups. */
vds_status vds_batch_autotune(vds_batch b, const float *q_dev);

/* Advances every ensemble of the packed state q_dev by nsteps explicit Euler
 * steps.  tau_host[nens][9] (may be NULL) receives each ensemble's stress
 * (FP64 sums) after the last step; then the call synchronises. */
vds_status vds_batch_step(vds_batch b, float *q_dev, int32_t nsteps, double *tau_host);

#ifdef __cplusplus
}
#endif

#endif /* VDS_BATCH_H */
