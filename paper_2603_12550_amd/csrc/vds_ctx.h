// The particle-scheme context, shared by the library's host translation units.
#pragma once

#include <string>
#include <vector>

#include "vds_internal.h"

namespace vds {

struct Layout {
  size_t QB, KA, VA, VB, part, xc, t1, S, wv, meanp, redp, redout, ctrl, blockmax, wscale, cmean, QH, KH, RN, hist, xb0,
      xb1, xpred, total;
};

struct TimerAcc {
  double ms = 0.0;
  int64_t launches = 0;
  double work = 0.0;
  int64_t seen = 0;  // launches since timing was enabled, sampled or not
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<double> pending_work;
};

}  // namespace vds

struct vds_ctx_s {
  vds_problem prob{};
  std::vector<double> H;
  hipStream_t stream = nullptr;
  vds::EvalParams ep{};
  vds_tuning tune{VDS_PAIR_MFMA32, 2, 4, 0};
  vds::SplitMap smap{};  // partial-sum slots of a pass over the particle rows under `tune`
  vds::Layout lay{};
  char *ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  bool timing = false;
  int timing_stride = 1;  // time every timing_stride-th launch of each timer
  vds::TimerAcc timers[VDS_TIMER_COUNT];
  std::vector<hipEvent_t> event_pool;

  // workspace views
  float *QB, *KA, *VA, *VB, *part, *xc, *t1, *S, *wv, *xb[2], *xpred, *blockmax, *wscale;
  float *cmean;  // a step's centre and weight maximum (see vds::PackOps)
  vds::F16Operands f16{};
  unsigned long long *hist;  // median-bandwidth histograms [2][kHistBins]
  double *meanp, *redp, *redout;
  vds::Ctrl *ctrl;
  int nblk;       // blocks of the one-thread-per-particle kernels
  int nblk_comb;  // blocks of the sixteen-lanes-per-particle combine kernel
  void *blas = nullptr;  // rocblas_handle of the FP64 eigensolve and exact windows, made on first use
};

namespace vds {

vds_status set_err(vds_ctx c, vds_status st, const std::string &m);
vds_status hip_check(vds_ctx c, hipError_t e, const char *what);
vds_status ready(vds_ctx c);
hipEvent_t get_event(vds_ctx c);
// The context's rocBLAS handle on the context's stream, created on the first call
// (NULL on failure, with the error set).  Destroyed with the context.
void *blas_handle(vds_ctx c);

// Runs `fn` (which launches work on the context stream), bracketed by an event
// pair when timing is on; `work` is the pair-evaluations or FLOP it performs.
template <class F>
void timed(vds_ctx c, int which, double work, F &&fn) {
  if (!c->timing || c->timers[which].seen++ % c->timing_stride != 0) {
    fn();
    return;
  }
  hipEvent_t a = get_event(c), b = get_event(c);
  (void)hipEventRecord(a, c->stream);
  fn();
  (void)hipEventRecord(b, c->stream);
  c->timers[which].pending.emplace_back(a, b);
  c->timers[which].pending_work.push_back(work);
}
// Centring, operand packing and pass A at the state q (weights w or uniform):
// leaves S, term1 and the pass-B operand in the workspace.  Without `centre`
// the centring partials already in the workspace are reused.
void eval_pass_a(vds_ctx c, const float *q, const float *w, const int *done, bool centre = true);
// Pass B with the operand eval_pass_a left; partial sums stay in c->part.
void eval_pass_b(vds_ctx c, const int *done);

}  // namespace vds
