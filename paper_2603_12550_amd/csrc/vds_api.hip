// C ABI of the particle scheme: context, workspace binding, evaluation
// sequences, the queued explicit and implicit steps, the FENE domain check,
// observables and kernel timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include <rocblas/rocblas.h>

#include "vds_ctx.h"
#include "vds_internal.h"

using namespace vds;

// Device scratch of vds_pair_sums_noalloc: one copy per GPU, held until the
// process ends.  Its name is a host-side stand-in; device addresses come from
// hipGetSymbolAddress (scratch_base below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};  // address of `scratch` on each device, once resolved
}  // namespace

namespace vds {

vds_status set_err(vds_ctx c, vds_status st, const std::string &m) {
  if (c) c->err = m;
  return st;
}

vds_status hip_check(vds_ctx c, hipError_t e, const char *what) {
  if (e == hipSuccess) return VDS_OK;
  return set_err(c, VDS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

vds_status ready(vds_ctx c) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (c->ws == nullptr) return set_err(c, VDS_ERR_STATE, "no workspace bound");
  return VDS_OK;
}

hipEvent_t get_event(vds_ctx c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (its cache writeback and invalidation
  // would slow the kernels between the events); elapsed times are read after
  // a stream synchronisation
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
  return e;
}

void *blas_handle(vds_ctx c) {
  if (c->blas == nullptr) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
      set_err(c, VDS_ERR_HIP, "rocblas_create_handle");
      return nullptr;
    }
    c->blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(c->blas);
  rocblas_set_stream(h, c->stream);
  return h;
}

int64_t ncol_chunks(const vds_ctx c) { return (c->prob.P + 15) / 16; }

// Where the combine kernel flags FENE bonds outside the spring's domain (NULL
// for Hookean springs).
int *fene_flag(vds_ctx c) { return c->prob.potential == VDS_FENE ? &c->ctrl->fene_out : nullptr; }

// One pair pass over all particle rows with the V operand `V`.
// `wscale` is the weight maximum the FP16-split V operand was divided by
// (pass A), or NULL (pass B: its weights w_J / S_J are at most one already).
void pair_pass(vds_ctx c, const float *V, const float *wscale, const int *done) {
  const int64_t nrb = c->ep.Ppad / 16;
  const double pairs = (double)c->prob.P * (double)c->prob.P;
  timed(c, VDS_TIMER_PAIR, pairs, [&] {
    // VDS_PAIR_MFMA32 takes its rows straight from the centred coordinates
    launch_pair_pass(c->tune, c->ep.KK, c->ep.D, c->ep.f32x ? c->xc : c->QB, nrb, c->KA, V, ncol_chunks(c),
                     c->ep.Ppad, c->xc, true, wscale, c->f16, c->part, c->ep.Ppad, done, c->stream, c->ep.kappa);
  });
}

// Keeps the operand format the prep and finalisation kernels write in step
// with the pair implementation.
void apply_tuning(vds_ctx c, const vds_tuning &t) {
  c->tune = t;
  c->smap = pair_split_map(t, c->ep.D, c->ep.Ppad / 16, ncol_chunks(c));
  c->ep.vhalf = (t.impl == VDS_PAIR_MFMA_F16X2 || t.impl == VDS_PAIR_MFMA_F16X2_ALL) ? 1 : 0;
  c->ep.qhalf = t.impl == VDS_PAIR_MFMA_F16X2_ALL ? 1 : 0;
  c->ep.f32x = t.impl == VDS_PAIR_MFMA32 ? 1 : 0;
}

void eval_pass_a(vds_ctx c, const float *q, const float *w, const int *done, bool centre) {
  const EvalParams &e = c->ep;
  if (centre) launch_mean_partials(e, q, w, c->meanp, done, nullptr, c->stream);
  launch_prep(e, q, w, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16, done, c->stream);
  pair_pass(c, c->VA, c->wscale, done);
  launch_finalize_a(e, c->part, c->smap, c->xc, c->wv, c->S, c->t1, c->VB, done, c->stream);
}

void eval_pass_b(vds_ctx c, const int *done) { pair_pass(c, c->VB, nullptr, done); }

}  // namespace vds

namespace {

bool problem_valid(const vds_problem *p, std::string *why) {
  auto fail = [&](const char *m) {
    if (why) *why = m;
    return false;
  };
  if (p == nullptr) return fail("problem is NULL");
  if (p->nb < 1 || p->nb > kMaxNb) return fail("nb must be in 1..5 (D = 3 nb <= 15)");
  if (p->P < 1) return fail("P must be >= 1");
  if (p->P > (int64_t)1 << 28) return fail("P too large");
  if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail("h must be positive and finite");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail("dt must be positive and finite");
  if (!(p->zeta > 0.0) || !std::isfinite(p->zeta)) return fail("zeta must be positive and finite");
  if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return fail("kT must be >= 0 and finite");
  if (!std::isfinite(p->n)) return fail("n must be finite");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(p->G[i])) return fail("G must be finite");
  if (p->potential != VDS_HOOKEAN && p->potential != VDS_FENE) return fail("unknown potential");
  if (p->potential == VDS_FENE && !(p->b_max > 0.0)) return fail("FENE needs b_max > 0");
  if (p->scheme != VDS_EXPLICIT && p->scheme != VDS_IMPLICIT) return fail("unknown scheme");
  if (p->scheme == VDS_IMPLICIT) {
    if (p->picard_max < 1) return fail("picard_max must be >= 1");
    if (!(p->picard_rtol > 0.0)) return fail("picard_rtol must be > 0");
    if (p->picard_batch < 1) return fail("picard_batch must be >= 1");
    if (p->picard_predictor != 0 && p->picard_predictor != 1) return fail("picard_predictor must be 0 or 1");
  }
  return true;
}

Layout make_layout(const vds_problem &p) {
  const int64_t Ppad = round_up(p.P, kRowAlign);
  const int D = 3 * p.nb;
  const int KK = (D + 2 + 3) / 4;
  // per-particle kernels run either one thread or 16 lanes per particle
  const int64_t nblk = (p.P * 16 + kRedBlock - 1) / kRedBlock;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += round_up((int64_t)bytes, 256);
    return o;
  };
  L.QB = take(sizeof(float) * Ppad * KK * 4);
  L.KA = take(sizeof(float) * Ppad * KK * 4);
  L.VA = take(sizeof(float) * Ppad * 16);
  L.VB = take(sizeof(float) * Ppad * 16);
  L.part = take(sizeof(float) * (size_t)kMaxSplits * Ppad * 16);
  L.xc = take(sizeof(float) * Ppad * D);
  L.t1 = take(sizeof(float) * Ppad * D);
  L.S = take(sizeof(float) * Ppad);
  L.wv = take(sizeof(float) * Ppad);
  L.meanp = take(sizeof(double) * nblk * 16);
  L.redp = take(sizeof(double) * nblk * 16);
  L.redout = take(sizeof(double) * 16);
  L.ctrl = take(sizeof(Ctrl));
  L.blockmax = take(sizeof(float) * 2 * nblk);
  L.wscale = take(sizeof(float) * 4);
  L.cmean = take(sizeof(float) * 16);
  L.QH = take(sizeof(uint16_t) * Ppad * 32 * f16_slices(D));
  L.KH = take(sizeof(uint16_t) * Ppad * 32 * f16_slices(D));
  L.RN = take(sizeof(float) * Ppad);
  L.hist = take(sizeof(unsigned long long) * 2 * kHistBins);
  L.xb0 = take(sizeof(float) * p.P * D);
  L.xb1 = take(sizeof(float) * p.P * D);
  L.xpred = take(sizeof(float) * p.P * D);
  L.total = off;
  return L;
}

void fill_params(vds_ctx c) {
  const vds_problem &p = c->prob;
  EvalParams &e = c->ep;
  e.P = p.P;
  e.Ppad = round_up(p.P, kRowAlign);
  e.nb = p.nb;
  e.D = 3 * p.nb;
  e.KK = (e.D + 2 + 3) / 4;
  e.kappa = (float)(1.4426950408889634 / (2.0 * p.h * p.h));
  e.inv_h2 = (float)(1.0 / (p.h * p.h));
  e.kT = (float)p.kT;
  e.inv_zeta = (float)(1.0 / p.zeta);
  e.dt = (float)p.dt;
  e.n = (float)p.n;
  for (int i = 0; i < 9; ++i) e.G[i] = (float)p.G[i];
  for (int k = 0; k < kMaxNb; ++k) e.H[k] = k < p.nb ? (float)c->H[k] : 0.f;
  e.b_max = (float)p.b_max;
  e.potential = p.potential;
  e.uniform_w = (float)(1.0 / (double)p.P);
  e.log_norm = (float)(0.5 * e.D * std::log(2.0 * M_PI * p.h * p.h));
  e.KQ = f16_slices(e.D);
  e.cs = (float)std::sqrt(2.0 * 1.4426950408889634 / (2.0 * p.h * p.h));
  e.KP = mfma32_kslots(e.D);
  c->nblk = (int)((p.P + kRedBlock - 1) / kRedBlock);
  c->nblk_comb = (int)((p.P * 16 + kRedBlock - 1) / kRedBlock);
  apply_tuning(c, c->tune);  // operand formats of the default implementation
}

void drain_timers(vds_ctx c) {
  for (auto &t : c->timers) {
    for (size_t i = 0; i < t.pending.size(); ++i) {
      float ms = 0.f;
      (void)hipEventSynchronize(t.pending[i].second);
      (void)hipEventElapsedTime(&ms, t.pending[i].first, t.pending[i].second);
      t.ms += ms;
      t.launches += 1;
      t.work += t.pending_work[i];
      c->event_pool.push_back(t.pending[i].first);
      c->event_pool.push_back(t.pending[i].second);
    }
    t.pending.clear();
    t.pending_work.clear();
  }
}

// Prep + pass A + finalize A + pass B + combine(mode).  Without `centre` the
// centring partials already in the workspace are used (the fixed-point
// iterations of a step all centre at the step's start state: the sums are
// differences, so any centre near the particles gives the same result).
void evaluate(vds_ctx c, const float *q, const float *w, int mode, bool obs, const float *q0, float *out,
              float *out2, const int *done, bool centre = true) {
  const EvalParams &e = c->ep;
  eval_pass_a(c, q, w, done, centre);
  eval_pass_b(c, done);
  launch_combine(e, mode, obs, c->part, c->smap, c->xc, c->t1, c->S, c->wv, q, q0, out, out2, c->redp,
                 c->blockmax, done, c->stream, nullptr, fene_flag(c));
  if (obs) launch_reduce_final(c->redp, c->nblk_comb, 12, c->redout, done, c->stream);
}

// Reads and clears the FENE domain flag (FENE problems only; synchronises).
vds_status fene_domain_check(vds_ctx c) {
  if (c->prob.potential != VDS_FENE) return VDS_OK;
  int out = 0;
  vds_status st = hip_check(c, hipMemcpyAsync(&out, fene_flag(c), sizeof(int), hipMemcpyDeviceToHost, c->stream),
                            "copy flag");
  if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  if (st != VDS_OK) return st;
  if (out == 0) return VDS_OK;
  launch_ctrl_reset(c->ctrl, c->stream);
  return set_err(c, VDS_ERR_ARG, "a FENE bond reached |q|^2 >= b_max (outside the spring's domain) or is not finite");
}

vds_status fetch_obs(vds_ctx c, vds_diag *d) {
  double r[16];
  vds_status st = hip_check(c, hipMemcpyAsync(r, c->redout, sizeof(double) * 12, hipMemcpyDeviceToHost, c->stream),
                            "copy observables");
  if (st != VDS_OK) return st;
  st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  if (st != VDS_OK) return st;
  d->F = r[RED_F];
  d->dissipation = r[RED_DISS];
  d->work = r[RED_WORK];
  for (int i = 0; i < 9; ++i) d->tau[i] = r[RED_TAU + i];
  d->energy_valid = 1;
  return VDS_OK;
}

vds_status stress_into(vds_ctx c, const float *q, const float *w, double *tau) {
  launch_stress(c->ep, q, w, c->redp, c->stream);
  launch_reduce_final(c->redp, c->nblk, 9, c->redout, nullptr, c->stream);
  double r[9];
  vds_status st =
      hip_check(c, hipMemcpyAsync(r, c->redout, sizeof(double) * 9, hipMemcpyDeviceToHost, c->stream), "copy stress");
  if (st != VDS_OK) return st;
  st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  if (st != VDS_OK) return st;
  std::memcpy(tau, r, sizeof(r));
  return VDS_OK;
}

}  // namespace

extern "C" {

size_t vds_workspace_bytes(const vds_problem *prob) {
  if (!problem_valid(prob, nullptr)) return 0;
  return make_layout(*prob).total;
}

vds_status vds_create(const vds_problem *prob, const double *H_host, void *hip_stream, vds_ctx *out) {
  std::string why;
  if (out == nullptr) {
    g_create_error = "out is NULL";
    return VDS_ERR_ARG;
  }
  *out = nullptr;
  if (!problem_valid(prob, &why)) {
    g_create_error = why;
    return VDS_ERR_ARG;
  }
  if (H_host == nullptr) {
    g_create_error = "H is NULL";
    return VDS_ERR_ARG;
  }
  for (int k = 0; k < prob->nb; ++k)
    if (!(H_host[k] > 0.0) || !std::isfinite(H_host[k])) {
      g_create_error = "spring constants H must be positive and finite";
      return VDS_ERR_ARG;
    }
  vds_ctx c = new (std::nothrow) vds_ctx_s();
  if (c == nullptr) {
    g_create_error = "host allocation failed";
    return VDS_ERR_NOMEM;
  }
  c->prob = *prob;
  c->H.assign(H_host, H_host + prob->nb);
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->lay = make_layout(*prob);
  fill_params(c);
  *out = c;
  return VDS_OK;
}

void vds_destroy(vds_ctx c) {
  if (c == nullptr) return;
  for (auto &t : c->timers)
    for (auto &pr : t.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->blas != nullptr) rocblas_destroy_handle(static_cast<rocblas_handle>(c->blas));
  delete c;
}

const char *vds_last_error(vds_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

namespace {

// Points the context's workspace views into `base` (bytes >= c->lay.total).
void bind_views(vds_ctx c, char *base, size_t bytes) {
  c->ws = base;
  c->ws_bytes = bytes;
  const Layout &L = c->lay;
  c->QB = reinterpret_cast<float *>(c->ws + L.QB);
  c->KA = reinterpret_cast<float *>(c->ws + L.KA);
  c->VA = reinterpret_cast<float *>(c->ws + L.VA);
  c->VB = reinterpret_cast<float *>(c->ws + L.VB);
  c->part = reinterpret_cast<float *>(c->ws + L.part);
  c->xc = reinterpret_cast<float *>(c->ws + L.xc);
  c->t1 = reinterpret_cast<float *>(c->ws + L.t1);
  c->S = reinterpret_cast<float *>(c->ws + L.S);
  c->wv = reinterpret_cast<float *>(c->ws + L.wv);
  c->meanp = reinterpret_cast<double *>(c->ws + L.meanp);
  c->redp = reinterpret_cast<double *>(c->ws + L.redp);
  c->redout = reinterpret_cast<double *>(c->ws + L.redout);
  c->ctrl = reinterpret_cast<Ctrl *>(c->ws + L.ctrl);
  c->blockmax = reinterpret_cast<float *>(c->ws + L.blockmax);
  c->wscale = reinterpret_cast<float *>(c->ws + L.wscale);
  c->cmean = reinterpret_cast<float *>(c->ws + L.cmean);
  c->f16 = F16Operands{c->ws + L.QH, c->ws + L.KH, reinterpret_cast<float *>(c->ws + L.RN)};
  c->hist = reinterpret_cast<unsigned long long *>(c->ws + L.hist);
  c->xb[0] = reinterpret_cast<float *>(c->ws + L.xb0);
  c->xb[1] = reinterpret_cast<float *>(c->ws + L.xb1);
  c->xpred = reinterpret_cast<float *>(c->ws + L.xpred);
}

}  // namespace

extern "C" {

vds_status vds_bind_workspace(vds_ctx c, void *ws, size_t bytes) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (ws == nullptr) return set_err(c, VDS_ERR_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return set_err(c, VDS_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < c->lay.total) return set_err(c, VDS_ERR_NOMEM, "workspace smaller than vds_workspace_bytes()");
  bind_views(c, static_cast<char *>(ws), bytes);
  return VDS_OK;
}

vds_status vds_set_tuning(vds_ctx c, const vds_tuning *t) {
  if (c == nullptr || t == nullptr) return VDS_ERR_ARG;
  if (!pair_shape_ok(*t, c->ep.D)) return set_err(c, VDS_ERR_ARG, "invalid tuning");
  apply_tuning(c, *t);
  return VDS_OK;
}

vds_status vds_get_tuning(vds_ctx c, vds_tuning *t) {
  if (c == nullptr || t == nullptr) return VDS_ERR_ARG;
  *t = c->tune;
  return VDS_OK;
}

vds_status vds_pair_sums(vds_ctx c, const float *q, const float *w, float *S, float *t1, float *t2) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q || !S || !t1 || !t2) return set_err(c, VDS_ERR_ARG, "null array");
  evaluate(c, q, w, MODE_TERMS, false, nullptr, t1, t2, nullptr);
  return hip_check(c, hipMemcpyAsync(S, c->S, sizeof(float) * c->prob.P, hipMemcpyDeviceToDevice, c->stream),
                   "copy S");
}

}  // extern "C"

namespace {

// This device's copy of `scratch`: resolved once per device, with that device
// current, and kept.
vds_status scratch_base(vds_ctx c, char **out) {
  int dev = 0;
  vds_status st = hip_check(c, hipGetDevice(&dev), "hipGetDevice");
  if (st != VDS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return set_err(c, VDS_ERR_HIP, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void *p = nullptr;
    st = hip_check(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != VDS_OK) return st;
    if (p == nullptr) return set_err(c, VDS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_dev[dev];
  return VDS_OK;
}

}  // namespace

extern "C" {

vds_status vds_pair_sums_noalloc(vds_ctx c, const float *q, const float *w, float *S, float *t1, float *t2) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (!q || !S || !t1 || !t2) return set_err(c, VDS_ERR_ARG, "null array");
  if (c->lay.total > kScratchBytes)
    return set_err(c, VDS_ERR_ARG,
                   "problem too large for the static scratch: it needs " + std::to_string(c->lay.total) +
                       " bytes (vds_workspace_bytes) and the scratch holds " + std::to_string(kScratchBytes) +
                       "; vds_pair_sums with a bound workspace has no such limit");
  char *base = nullptr;
  vds_status st = scratch_base(c, &base);
  if (st != VDS_OK) return st;
  // the evaluation of vds_pair_sums on views into the scratch; every scratch
  // element it reads is written earlier in the same call, so nothing needs
  // clearing.  No kernel timing (its events would be created on demand).
  char *old = c->ws;
  const size_t old_bytes = c->ws_bytes;
  const bool was_timing = c->timing;
  c->timing = false;
  bind_views(c, base, kScratchBytes);
  evaluate(c, q, w, MODE_TERMS, false, nullptr, t1, t2, nullptr);
  st = hip_check(c, hipMemcpyAsync(S, c->S, sizeof(float) * c->prob.P, hipMemcpyDeviceToDevice, c->stream),
                 "copy S");
  if (old != nullptr) {
    bind_views(c, old, old_bytes);
  } else {
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  c->timing = was_timing;
  if (st == VDS_OK) st = hip_check(c, hipGetLastError(), "launch");
  return st;
}

vds_status vds_velocity(vds_ctx c, const float *q, const float *w, float *v, vds_diag *d) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q || !v) return set_err(c, VDS_ERR_ARG, "null array");
  if (c->prob.potential == VDS_FENE) launch_ctrl_reset(c->ctrl, c->stream);
  evaluate(c, q, w, MODE_VELOCITY, d != nullptr, nullptr, v, nullptr, nullptr);
  st = hip_check(c, hipGetLastError(), "launch");
  if (st == VDS_OK) st = fene_domain_check(c);
  if (st != VDS_OK || d == nullptr) return st;
  std::memset(d, 0, sizeof(*d));
  return fetch_obs(c, d);
}

}  // extern "C"

namespace {

// Implicit steps queued on the stream between two host synchronisations.
constexpr int kQueueSteps = 64;

// Explicit steps: every kQueueSteps steps the centring partials and the pair
// operands come from the prep kernels; in between, each step's combine kernel
// packs the next step's operands centred where the last prep centred (the
// sums are differences, so a centre near the particles serves).
void explicit_steps(vds_ctx c, float *q, const float *w, int nsteps) {
  const PackOps pk{c->xc, c->wv, c->QB, c->KA, c->VA, c->f16, c->cmean};
  for (int s = 0; s < nsteps; ++s) {
    if (s % kQueueSteps == 0) {
      launch_mean_partials(c->ep, q, w, c->meanp, nullptr, nullptr, c->stream);
      launch_prep(c->ep, q, w, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16, nullptr,
                  c->stream, c->cmean);
    }
    pair_pass(c, c->VA, c->wscale, nullptr);
    launch_finalize_a(c->ep, c->part, c->smap, c->xc, c->wv, c->S, c->t1, c->VB, nullptr, c->stream);
    eval_pass_b(c, nullptr);
    const bool pack = s + 1 < nsteps && (s + 1) % kQueueSteps != 0;
    launch_combine(c->ep, MODE_EXPLICIT, false, c->part, c->smap, c->xc, c->t1, c->S, c->wv, q, nullptr,
                   q, nullptr, c->redp, c->blockmax, nullptr, c->stream, pack ? &pk : nullptr, fene_flag(c));
  }
}

struct StepCounts {
  int total_iters = 0, last_iters = 0;
  float last_resid = 0.f;
};

// Finishes the fixed-point iteration of one implicit step from iteration m0
// (xb[(m0 - 1) & 1] holds iterate m0 - 1 when m0 > 0; q holds the step's start
// state), checking convergence on the host every picard_batch iterations, and
// writes the converged iterate to q.
vds_status finish_step(vds_ctx c, float *q, const float *w, int m0, StepCounts &n) {
  const vds_problem &p = c->prob;
  const int64_t nq = (int64_t)p.P * c->ep.D;
  launch_ctrl_reset(c->ctrl, c->stream);
  launch_mean_partials(c->ep, q, w, c->meanp, nullptr, nullptr, c->stream);
  const int *done = &c->ctrl->done;
  int m = m0;
  Ctrl h{};
  h.last_resid = n.last_resid;  // the residual of iteration m0 - 1, if no further one runs
  bool converged = false;
  while (m < p.picard_max) {
    const int batch = std::min(p.picard_batch, p.picard_max - m);
    for (int b = 0; b < batch; ++b, ++m) {
      const float *xin = (m == 0) ? q : c->xb[(m - 1) & 1];
      evaluate(c, xin, w, MODE_PICARD, false, q, c->xb[m & 1], nullptr, done, false);
      launch_picard_check(PicardCheck{c->ctrl, (float)p.picard_rtol, m}, c->blockmax, c->nblk_comb, c->stream);
    }
    vds_status st = hip_check(c, hipMemcpyAsync(&h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream),
                              "copy ctrl");
    if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
    if (st != VDS_OK) return st;
    if (h.fene_out)
      return set_err(c, VDS_ERR_ARG, "a FENE bond reached |q|^2 >= b_max (outside the spring's domain) or is not finite");
    if (h.done) {
      converged = true;
      break;
    }
  }
  const int final_iter = converged ? h.conv_iter : m - 1;
  if (final_iter >= 0) {
    vds_status st = hip_check(
        c, hipMemcpyAsync(q, c->xb[final_iter & 1], sizeof(float) * nq, hipMemcpyDeviceToDevice, c->stream),
        "copy state");
    if (st != VDS_OK) return st;
  }
  n.last_iters = final_iter + 1;
  n.total_iters += n.last_iters;
  n.last_resid = h.last_resid;
  if (!converged) return set_err(c, VDS_ERR_NOT_CONVERGED, "fixed-point iteration reached picard_max");
  return VDS_OK;
}

// Implicit Euler steps (eq. implicit) with the fixed-point iteration run from
// the device: each step is queued with picard_batch iterations, the prep
// kernel of each iteration tests the one before (the step-end kernel tests
// the last), the iterations queued past convergence return at once, and the
// step-end kernel writes the converged iterate back.  A step
// that has not converged after its queued iterations halts the queue (every
// later kernel returns at once); the host then finishes that step and queues
// the rest.  The host synchronises once per kQueueSteps steps.
vds_status implicit_steps(vds_ctx c, float *q, const float *w, int nsteps, StepCounts &n, int &steps_taken) {
  const vds_problem &p = c->prob;
  const int batch = std::min(p.picard_batch, p.picard_max);
  const int *done = &c->ctrl->done;
  steps_taken = 0;
  while (steps_taken < nsteps) {
    const int chunk = std::min(nsteps - steps_taken, kQueueSteps);
    launch_ctrl_reset(c->ctrl, c->stream);
    for (int j = 0; j < chunk; ++j) {
      // the first step of the queue computes its centring partials; the step
      // end of every other step left them behind, and its prep kernel opens
      // the step in the control block
      if (j == 0) launch_mean_partials(c->ep, q, w, c->meanp, nullptr, c->ctrl, c->stream);
      // with the predictor, steps after the first of the queue start from
      // the extrapolation the previous step end wrote
      const float *x0 = (p.picard_predictor && j > 0) ? c->xpred : q;
      for (int m = 0; m < batch; ++m) {
        const float *xin = (m == 0) ? x0 : c->xb[(m - 1) & 1];
        if (m == 0) {
          launch_prep(c->ep, x0, w, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16,
                      j == 0 ? done : nullptr, c->stream, c->cmean, j > 0 ? c->ctrl : nullptr);
        } else {
          // the previous combine packed this iterate's operands; one block
          // tests the previous iteration
          launch_picard_check(PicardCheck{c->ctrl, (float)p.picard_rtol, m - 1}, c->blockmax, c->nblk_comb,
                              c->stream);
        }
        pair_pass(c, c->VA, c->wscale, done);
        launch_finalize_a(c->ep, c->part, c->smap, c->xc, c->wv, c->S, c->t1, c->VB, done, c->stream);
        eval_pass_b(c, done);
        const PackOps pk{c->xc, c->wv, c->QB, c->KA, c->VA, c->f16, c->cmean};
        launch_combine(c->ep, MODE_PICARD, false, c->part, c->smap, c->xc, c->t1, c->S, c->wv, xin, q,
                       c->xb[m & 1], nullptr, c->redp, c->blockmax, done, c->stream, m + 1 < batch ? &pk : nullptr,
                       fene_flag(c));
      }
      launch_step_end(c->ep, c->ctrl, PicardCheck{c->ctrl, (float)p.picard_rtol, batch - 1}, c->blockmax,
                      c->nblk_comb, c->xb[0], c->xb[1], q, p.picard_predictor ? c->xpred : nullptr, w,
                      j + 1 < chunk ? c->meanp : nullptr, c->stream);
    }
    Ctrl h{};
    vds_status st = hip_check(c, hipMemcpyAsync(&h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream),
                              "copy ctrl");
    if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
    if (st != VDS_OK) return st;
    if (h.fene_out)
      return set_err(c, VDS_ERR_ARG, "a FENE bond reached |q|^2 >= b_max (outside the spring's domain) or is not finite");
    n.total_iters += (int)h.total_iters;
    if (h.steps_done > 0) n.last_iters = h.last_iters;
    n.last_resid = h.last_resid;  // of the last iteration checked
    steps_taken += h.steps_done;
    if (h.halted) {
      st = finish_step(c, q, w, batch, n);
      steps_taken += 1;
      if (st != VDS_OK) return st;
    } else if (h.steps_done != chunk) {
      return set_err(c, VDS_ERR_HIP, "queued implicit steps lost count");
    }
  }
  return VDS_OK;
}

}  // namespace

extern "C" {

vds_status vds_step(vds_ctx c, float *q, const float *w, int32_t nsteps, vds_diag *d) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q) return set_err(c, VDS_ERR_ARG, "null state");
  if (nsteps < 0) return set_err(c, VDS_ERR_ARG, "nsteps < 0");
  const vds_problem &p = c->prob;
  StepCounts n;
  if (p.scheme == VDS_EXPLICIT) {
    if (p.potential == VDS_FENE && nsteps > 0) launch_ctrl_reset(c->ctrl, c->stream);
    explicit_steps(c, q, w, nsteps);
    if (nsteps > 0) st = fene_domain_check(c);
    if (st != VDS_OK) return st;
  } else if (nsteps > 0) {
    int taken = 0;
    st = implicit_steps(c, q, w, nsteps, n, taken);
    if (st == VDS_ERR_NOT_CONVERGED && d != nullptr) {
      std::memset(d, 0, sizeof(*d));
      d->steps = taken;
      d->iters = n.total_iters;
      d->last_iters = n.last_iters;
      d->resid = n.last_resid;
    }
    if (st != VDS_OK) return st;
  }
  st = hip_check(c, hipGetLastError(), "launch");
  if (st != VDS_OK) return st;
  if (d != nullptr) {
    std::memset(d, 0, sizeof(*d));
    d->steps = nsteps;
    d->iters = n.total_iters;
    d->last_iters = n.last_iters;
    d->resid = n.last_resid;
    return stress_into(c, q, w, d->tau);
  }
  return VDS_OK;
}

vds_status vds_stress(vds_ctx c, const float *q, const float *w, double *tau) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q || !tau) return set_err(c, VDS_ERR_ARG, "null array");
  return stress_into(c, q, w, tau);
}

vds_status vds_energy(vds_ctx c, const float *q, const float *w, double *F, double *diss, double *work) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q) return set_err(c, VDS_ERR_ARG, "null state");
  if (c->prob.potential == VDS_FENE) launch_ctrl_reset(c->ctrl, c->stream);
  evaluate(c, q, w, MODE_OBS_ONLY, true, nullptr, nullptr, nullptr, nullptr);
  st = fene_domain_check(c);
  if (st != VDS_OK) return st;
  vds_diag d{};
  st = fetch_obs(c, &d);
  if (st != VDS_OK) return st;
  if (F) *F = d.F;
  if (diss) *diss = d.dissipation;
  if (work) *work = d.work;
  return VDS_OK;
}

vds_status vds_density_at(vds_ctx c, const float *q, const float *w, const float *y, int64_t ny, float *f) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q || !y || !f || ny < 0) return set_err(c, VDS_ERR_ARG, "bad arguments");
  if (ny == 0) return VDS_OK;
  const EvalParams &e = c->ep;
  launch_mean_partials(e, q, w, c->meanp, nullptr, nullptr, c->stream);
  launch_prep(e, q, w, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16, nullptr, c->stream);
  const float norm = (float)std::pow(2.0 * M_PI * c->prob.h * c->prob.h, -0.5 * e.D);
  // foreign rows go through the Q-operand buffer in blocks of Ppad rows
  for (int64_t r0 = 0; r0 < ny; r0 += e.Ppad) {
    const int64_t nr = std::min<int64_t>(e.Ppad, ny - r0);
    launch_density_rows(e, y + r0 * e.D, nr, c->meanp, c->nblk, c->QB, &c->f16, c->stream);
    const int64_t nrb = round_up(nr, kRowAlign) / 16;
    timed(c, VDS_TIMER_PAIR, (double)nr * (double)c->prob.P, [&] {
      launch_pair_pass(c->tune, e.KK, e.D, c->QB, nrb, c->KA, c->VA, ncol_chunks(c), e.Ppad, c->xc, false,
                       c->wscale, c->f16, c->part, e.Ppad, nullptr, c->stream, e.kappa);
    });
    launch_density_out(e, c->part, pair_split_map(c->tune, e.D, nrb, ncol_chunks(c)), nr, norm, f + r0, c->stream);
  }
  return hip_check(c, hipGetLastError(), "launch");
}

vds_status vds_timing_enable(vds_ctx c, int32_t enable) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (enable < 0) return set_err(c, VDS_ERR_ARG, "timing stride < 0");
  drain_timers(c);
  for (auto &t : c->timers) {
    t.ms = 0.0;
    t.launches = 0;
    t.work = 0.0;
    t.seen = 0;
  }
  c->timing = enable != 0;
  c->timing_stride = enable > 0 ? enable : 1;
  return VDS_OK;
}

vds_status vds_timing_read(vds_ctx c, int32_t which, double *ms, int64_t *launches, double *work) {
  if (c == nullptr || which < 0 || which >= VDS_TIMER_COUNT) return VDS_ERR_ARG;
  drain_timers(c);
  if (ms) *ms = c->timers[which].ms;
  if (launches) *launches = c->timers[which].launches;
  if (work) *work = c->timers[which].work;
  return VDS_OK;
}

vds_status vds_autotune(vds_ctx c, const float *q, const float *w) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q) return set_err(c, VDS_ERR_ARG, "null state");
  hipEvent_t a = get_event(c), b = get_event(c);
  vds_tuning best = c->tune;
  float best_ms = 1e30f;
  // column splits, or for VDS_PAIR_MFMA32 workgroups per compute unit of its balanced grid
  const std::vector<int> splits_list = c->tune.impl == VDS_PAIR_MFMA32
                                           ? std::vector<int>{1, 2, 3, 4, 5, 6, 8, 12, 16}
                                           : std::vector<int>{1, 2, 4, 6, 8, 12, 16, 20, 24, 32};
  const int rb_list[] = {1, 2, 4};
  std::vector<vds_tuning> cands;
  // the launch shape only: the implementation, and so the arithmetic, stays the caller's choice
  for (int rb : rb_list)
    for (int sp : splits_list) cands.push_back(vds_tuning{c->tune.impl, rb, sp, 0});
  const bool was_timing = c->timing;
  c->timing = false;
  int prepared = -1;
  for (const vds_tuning &t : cands) {
    if (!pair_shape_ok(t, c->ep.D)) continue;
    apply_tuning(c, t);
    if (c->ep.vhalf + 2 * c->ep.qhalf + 4 * c->ep.f32x != prepared) {  // operand formats follow the implementation
      launch_mean_partials(c->ep, q, w, c->meanp, nullptr, nullptr, c->stream);
      launch_prep(c->ep, q, w, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16, nullptr,
                  c->stream);
      prepared = c->ep.vhalf + 2 * c->ep.qhalf + 4 * c->ep.f32x;
    }
    // each candidate is timed with the finalisation that sums its column splits
    auto pass = [&] {
      pair_pass(c, c->VA, c->wscale, nullptr);
      launch_finalize_a(c->ep, c->part, c->smap, c->xc, c->wv, c->S, c->t1, c->VB, nullptr, c->stream);
    };
    pass();  // warm-up
    (void)hipEventRecord(a, c->stream);
    const int reps = 3;
    for (int r = 0; r < reps; ++r) pass();
    (void)hipEventRecord(b, c->stream);
    st = hip_check(c, hipEventSynchronize(b), "autotune");
    if (st != VDS_OK) break;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  c->timing = was_timing;
  c->event_pool.push_back(a);
  c->event_pool.push_back(b);
  apply_tuning(c, best);
  return st;
}

}  // extern "C"
