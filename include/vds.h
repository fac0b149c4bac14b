/*
 * vds.h - C ABI of the MI355X (gfx950) library for the variational
 * deterministic-particle scheme (VDS) for the microscopic Fokker-Planck
 * equation of bead-spring chains, and its POD model-order reduction.
 *
 * Paper: "Reduced-order variational deterministic-particle scheme", arXiv
 * 2603.12550.  Section numbers and equation labels below are the paper's.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Plain C types only.  Array arguments named *_dev are device pointers
 *   (HIP global memory) owned by the caller; *_host are host pointers.
 * - Particle states use the paper's bond-major index k(I alpha) (Section 2.2):
 *   float q[nb][P][3], bond k, particle I, spatial component alpha, contiguous.
 * - Weights w_dev[P] are positive and sum to one; NULL means the paper's
 *   uniform 1/P (eq. model_DeteParAppr).  The kernel terms only use weight
 *   ratios; stress and energy use the weights as given.
 * - Every call is ordered on the HIP stream given at creation.  Calls that
 *   return host values synchronise that stream; the others are asynchronous.
 * - The library allocates no device memory for contexts: the caller binds a
 *   device workspace of the size the *_workspace_bytes query returns.  The one
 *   exception is rocBLAS: the FP64 eigensolve of vds_pod_basis and the exact
 *   window integrator vds_rom_run_exact use a rocBLAS handle that the context
 *   creates on its first such call and keeps until vds_destroy; rocBLAS
 *   allocates that handle's own device workspace.
 * - Errors: every call returns a vds_status.  Arguments are validated on the
 *   host before anything is launched; on error nothing is launched and
 *   vds_last_error() describes it.  Asynchronous device faults surface as
 *   VDS_ERR_HIP at the next synchronising call.  No C++ exception crosses the
 *   ABI.  A context is not thread-safe.
 */
#ifndef VDS_H
#define VDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vds_status {
  VDS_OK = 0,
  VDS_ERR_ARG = 1,            /* bad size, null pointer, non-positive h/dt/zeta, ... */
  VDS_ERR_HIP = 2,            /* a HIP runtime or library call failed */
  VDS_ERR_NOMEM = 3,          /* bound workspace smaller than required */
  VDS_ERR_NOT_CONVERGED = 4,  /* implicit step: fixed-point iteration hit its cap */
  VDS_ERR_STATE = 5           /* call-order violation (e.g. no workspace bound) */
} vds_status;

enum { VDS_HOOKEAN = 0, VDS_FENE = 1 };
enum { VDS_EXPLICIT = 0, VDS_IMPLICIT = 1 };
/* Pair-kernel implementations (all compute the same sums):
 *   VDS_PAIR_MFMA32     FP32 throughout (the default): distances on FP32 32x32x2 matrix
 *                       instructions over augmented vectors with both squared norms in the
 *                       contraction, kernel-weighted sums on FP32 4x4x1 matrix instructions
 *                       (outputs in groups of four), FP32 exponentials;
 *   VDS_PAIR_MFMA       FP32 matrix cores for both products on 16x16x4 tiles;
 *   VDS_PAIR_VALU       FP32 vector FMAs;
 *   VDS_PAIR_MFMA_F16X2 FP32 matrix cores for the distances, the kernel-weighted sums on FP16
 *                       matrix cores with both factors split into high and low halves (about
 *                       22 significant bits, against 24 for FP32; sums beyond 128 columns
 *                       in FP64 as for the others);
 *   VDS_PAIR_MFMA_F16X2_ALL  both products on FP16 matrix cores with split factors; the
 *                       squared norms enter in FP32.
 * The FP16-split forms are valid while every centred particle lies within about 1e3 h of
 * the weighted mean; further out the rounding of the expanded squared distance can exceed
 * the FP16 range (the FP32 forms have lost all accuracy there too). */
enum { VDS_PAIR_MFMA = 0, VDS_PAIR_VALU = 1, VDS_PAIR_MFMA_F16X2 = 2, VDS_PAIR_MFMA_F16X2_ALL = 3,
       VDS_PAIR_MFMA32 = 4 };

/* Problem description (Sections 2.1, 2.2, 3.1; Appendix A).
 * Drift of bond k of particle I (eq. model_DymRepPar, convection dropped):
 *   dq_{k,I}/dt = G q_{k,I}
 *                 - (1/zeta) sum_j A_kj [kT (term1 + term2)_{j,I} + grad_{q_j} Psi(q_I)]
 * with the Rouse matrix A_jk = 2[j=k] - [|j-k|=1] and the Gaussian kernel of
 * bandwidth h.  Hookean grad Psi_j = H_j q_j (eq. model_Hookean); FENE (not in
 * the paper, the standard law) H_j q_j / (1 - |q_j|^2 / b_max). */
typedef struct vds_problem {
  int32_t nb;            /* bonds N-1, 1..5 (configuration dimension D = 3 nb <= 15) */
  int32_t potential;     /* VDS_HOOKEAN or VDS_FENE */
  int64_t P;             /* representative particles, >= 1 */
  double kT;             /* k_B T >= 0 */
  double zeta;           /* friction > 0 */
  double n;              /* number density in the stress */
  double h;              /* kernel bandwidth > 0 */
  double dt;             /* time step > 0 */
  double G[9];           /* G = (grad u)^T, row-major; drift G q */
  double b_max;          /* FENE extensibility (> 0 when potential == VDS_FENE) */
  int32_t scheme;        /* VDS_EXPLICIT (q+ = q + dt v(q)) or VDS_IMPLICIT */
  int32_t picard_max;    /* implicit: iteration cap (>= 1) */
  double picard_rtol;    /* implicit: stop when max|dx| <= rtol * max(1, max|x|) */
  int32_t picard_batch;  /* implicit: iterations queued per step before the host checks (>= 1) */
  int32_t picard_predictor; /* implicit: 0 iterate from q^n; 1 from 2 q^n - q^(n-1) where the
                             * previous step of the same vds_step call is at hand (same fixed
                             * point, about one iteration fewer per step) */
} vds_problem;

/* Diagnostics of a step or an evaluation (host struct). */
typedef struct vds_diag {
  int32_t steps;         /* steps taken */
  int32_t iters;         /* fixed-point iterations summed over the steps */
  int32_t last_iters;    /* iterations of the last step */
  int32_t energy_valid;  /* 1 if F/dissipation/work below were computed */
  double resid;          /* last max|dx| of the implicit iteration */
  double F;              /* F_h = sum_I w_I [kT log f_h(q_I) + Psi(q_I)] */
  double dissipation;    /* (1/zeta) sum_I w_I g_I^T (A (x) I) g_I, g = kT b + grad Psi */
  double work;           /* sum_I w_I g_I . (G q_I) */
  double tau[9];         /* stress n sum_I w_I sum_j q_j (x) grad Psi_j, row-major */
} vds_diag;

/* Pair-kernel launch shape (chosen by vds_autotune or set by hand; a new
 * context starts with VDS_PAIR_MFMA32, 2 row blocks per wave, 4 workgroups per
 * compute unit).  The FP16-split forms are opt-in: they keep about 22 bits, not
 * FP32's 24. */
typedef struct vds_tuning {
  int32_t impl;          /* one of the VDS_PAIR_* implementations */
  int32_t rows_per_wave; /* MFMA forms: row blocks per wavefront (16 rows each: 1, 2 or 4;
                          * VDS_PAIR_MFMA32: 32 rows each, 1 or 2) */
  int32_t col_splits;    /* 1..32.  Column ranges summed separately, then reduced; for
                          * VDS_PAIR_MFMA32 the workgroups per compute unit of its balanced
                          * grid, whose workgroups take equal runs of (row group, column
                          * chunk) work and leave one partial sum per row group they cover */
  int32_t reserved;
} vds_tuning;

typedef struct vds_ctx_s *vds_ctx;

/* ---- lifecycle ---------------------------------------------------------- */

/* Validates `prob` (see vds_status) and H_host[nb] (> 0), and creates a
 * context that launches on `hip_stream` (a hipStream_t; NULL = null stream). */
vds_status vds_create(const vds_problem *prob, const double *H_host, void *hip_stream, vds_ctx *out);
void vds_destroy(vds_ctx ctx);
/* Device workspace the context needs, in bytes (0 if `prob` is invalid). */
size_t vds_workspace_bytes(const vds_problem *prob);
/* Binds caller-owned device memory (>= vds_workspace_bytes, 256-byte aligned). */
vds_status vds_bind_workspace(vds_ctx ctx, void *ws_dev, size_t bytes);
/* Last error message of `ctx` (or of the last failed create when ctx is NULL). */
const char *vds_last_error(vds_ctx ctx);
vds_status vds_set_tuning(vds_ctx ctx, const vds_tuning *t);
vds_status vds_get_tuning(vds_ctx ctx, vds_tuning *t);
/* Times every admissible launch shape (row blocks per wave, column splits) of
 * the current implementation on the state q_dev (a pair pass with the
 * finalisation that sums its column splits) and keeps the fastest; the
 * implementation, and so the arithmetic, is left as set (synchronises). */
vds_status vds_autotune(vds_ctx ctx, const float *q_dev, const float *w_dev);

/* ---- the particle scheme (Sections 2.1-2.2, Appendix A) ----------------- */

/* Kernel sums at the particles (eq. model_DeteParAppr, eq. model_DymRepPar):
 *   S_I     = sum_J w_J exp(-|q_I - q_J|^2 / 2h^2)           (J = I included)
 *   term1_I = -(1/h^2) sum_J w_J e_IJ (q_I - q_J) / S_I
 *   term2_I = -(1/h^2) sum_K (w_K / S_K) e_IK (q_I - q_K)
 * Outputs: S_dev[P]; term1_dev, term2_dev in the state layout [nb][P][3]. */
vds_status vds_pair_sums(vds_ctx ctx, const float *q_dev, const float *w_dev,
                         float *S_dev, float *term1_dev, float *term2_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): vds_pair_sums
 * with the same arguments and results (the same kernels, bit for bit), on a
 * context with or without a bound workspace, using instead a static device
 * scratch of 64 MiB that the library holds on every GPU it runs on until the
 * process ends.  It allocates nothing: no hipMalloc or hipFree, no library
 * routine that allocates, no kernel timing.  VDS_ERR_ARG (nothing launched)
 * when vds_workspace_bytes of the context's problem exceeds 64 MiB (e.g. the
 * 4-bead chain fits up to P = 25600).  Every call on a GPU shares that
 * GPU's scratch, so calls that overlap on one GPU (concurrent streams or
 * threads) race; the scratch keeps the last call's contents, and this path
 * reads none of them before writing.  A workspace bound to the context is left
 * bound and untouched.  Asynchronous, as vds_pair_sums. */
vds_status vds_pair_sums_noalloc(vds_ctx ctx, const float *q_dev, const float *w_dev,
                                 float *S_dev, float *term1_dev, float *term2_dev);

/* Particle velocity v = dq/dt of eq. model_DymRepPar into v_dev[nb][P][3].
 * `diag` (host, may be NULL) receives the stress and, at no extra kernel
 * cost, F_h, dissipation and work at q.
 * FENE domain: with FENE springs, every call that evaluates the spring force
 * (vds_velocity, vds_step, vds_energy) returns VDS_ERR_ARG when a bond of an
 * evaluated state has |q_j|^2 >= b_max or is not finite.  The kernels flag
 * such bonds on the device and the call synchronises to read the flag.  The
 * outputs are then meaningless, and vds_step leaves q_dev at the steps taken
 * so far. */
vds_status vds_velocity(vds_ctx ctx, const float *q_dev, const float *w_dev, float *v_dev, vds_diag *diag);

/* Advances q_dev in place by `nsteps` steps of the problem's scheme
 * (explicit Euler of Appendix A, or the implicit Euler of Appendix A with the
 * flow term at t and the kernel and spring terms at t+, solved by fixed-point
 * iteration from q).  Implicit steps are queued on the device with
 * picard_batch iterations each: the convergence test runs in the kernels, the
 * iterations queued past convergence return at once, and the host
 * synchronises once per 64 steps, plus once per picard_batch further
 * iterations for a step that needs more than picard_batch.  The iterates, and
 * so the result, do not depend on picard_batch.  Explicit steps do not
 * synchronise (FENE springs: once per call, see vds_velocity); their pair
 * operands are centred at the state of every 64th step (the sums are
 * differences: only rounding depends on the centre).  On
 * VDS_ERR_NOT_CONVERGED q_dev holds the last iterate of the failing step.
 * `diag` (host, may be NULL) gets iteration counts, the last residual and the
 * stress after the last step. */
vds_status vds_step(vds_ctx ctx, float *q_dev, const float *w_dev, int32_t nsteps, vds_diag *diag);

/* Stress tau (Section 2.1; discrete form of Appendix A), FP64 accumulation,
 * into tau_host[9] row-major.  Synchronises. */
vds_status vds_stress(vds_ctx ctx, const float *q_dev, const float *w_dev, double *tau_host);

/* F_h, dissipation and work at q (FP64 accumulation).  Synchronises. */
vds_status vds_energy(vds_ctx ctx, const float *q_dev, const float *w_dev,
                      double *F_host, double *diss_host, double *work_host);

/* Mollified density f_h(y) = sum_I w_I K_h(y - q_I) (normalised Gaussian) at
 * ny foreign points y_dev[ny][3 nb] (particle-major), into f_dev[ny]
 * (Appendix A density errors).  Uses the same pair kernel. */
vds_status vds_density_at(vds_ctx ctx, const float *q_dev, const float *w_dev,
                          const float *y_dev, int64_t ny, float *f_dev);

/* Median-heuristic bandwidth (eq. model_bandwidth): med = the median of
 * |q_J - q_K| (configuration-space distance) over all P^2 ordered pairs, J = K
 * included (for an even count, the mean of the two middle values), and
 * h = med / sqrt(2 log P).  Unweighted.  Exact selection over the FP32 squared
 * distances of the state q_dev ([nb][P][3]); med_host, h_host (either may be
 * NULL) receive the FP64 results.  Needs 2 <= P <= 2^24.  Synchronises (three passes over
 * the pairs).  The context's h is not changed: create a context with the result. */
vds_status vds_median_bandwidth(vds_ctx ctx, const float *q_dev, double *med_host, double *h_host);

/* ---- per-kernel timing (HIP events on the context's stream) ------------- */

enum { VDS_TIMER_PAIR = 0, VDS_TIMER_GEMM = 1, VDS_TIMER_KGEMM = 2, VDS_TIMER_PROJ = 3, VDS_TIMER_COUNT = 4 };
/* enable = N >= 1 starts recording an event pair around every N-th launch of
 * each timed kernel (1: every launch) and clears the totals; 0 stops.  The
 * events carry no system-scope fence (timing only).  Launches that return at
 * once (fixed-point iterations queued past convergence) are counted too when
 * sampled. */
vds_status vds_timing_enable(vds_ctx ctx, int32_t enable);
/* Synchronises and returns the summed kernel time (ms), the launch count and
 * the pair-evaluations (pair kernel) or flops (GEMMs) of timer `which`. */
vds_status vds_timing_read(vds_ctx ctx, int32_t which, double *ms_host, int64_t *launches_host, double *work_host);

#ifdef __cplusplus
}
#endif

#endif /* VDS_H */
