// Batched ensembles (C ABI of include/vds_batch.h): concatenated, padded
// operand arrays; per-ensemble parameters in a device table; one explicit
// Euler step = centring, packing, pass A, finalisation, pass B, update, captured
// once into a hipGraph on a private stream and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "vds_batch.h"
#include "vds_internal.h"

using namespace vds;

namespace {

thread_local std::string g_batch_create_error;

struct BatchLayout {
  size_t ens, blk16, blk256, items, QB, KA, VA, VB, QH, KH, RN, xc, t1, S, wv, part, meanp, redp, tau, total;
};

}  // namespace

struct vds_batch_s {
  int nens = 0, nb = 0, D = 0, KK = 0;
  std::vector<int64_t> P;
  std::vector<EnsDesc> ens;
  std::vector<int> blk16, blk256;
  int64_t Ptot_pad = 0, qlen = 0;
  BatchLayout L{};
  char *ws = nullptr;
  hipStream_t user = nullptr, priv = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int impl = VDS_PAIR_MFMA32, rb = 2, grid = 1024, use_graph = 1;
  int nitems = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float *graph_q = nullptr;  // state pointer the graph was captured for
  int graph_impl = -1, graph_rb = 0, graph_grid = 0;
  std::string err;

  EnsDesc *d_ens;
  int *d_blk16, *d_blk256;
  int2 *d_items;
  float *QB, *KA, *VA, *VB, *xc, *t1, *S, *wv, *part;
  F16Operands f16{};
  double *meanp, *redp, *tau;
};

namespace {

vds_status berr(vds_batch b, vds_status st, const std::string &m) {
  if (b) b->err = m;
  return st;
}

vds_status bhip(vds_batch b, hipError_t e, const char *what) {
  if (e == hipSuccess) return VDS_OK;
  return berr(b, VDS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t pad(int64_t P) { return round_up(P, kRowAlign); }

BatchLayout batch_layout(int nens, const int64_t *P, int nb) {
  const int D = 3 * nb, KK = (D + 2 + 3) / 4;
  int64_t Ptot = 0;
  int64_t items_max = 0;
  for (int e = 0; e < nens; ++e) {
    Ptot += pad(P[e]);
    items_max += pad(P[e]) / 64;  // rows_per_wave = 1: 64 rows per item
  }
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  L.ens = take(sizeof(EnsDesc) * nens);
  L.blk16 = take(sizeof(int) * (Ptot / 16));
  L.blk256 = take(sizeof(int) * (Ptot / 256));
  L.items = take(sizeof(int2) * items_max);
  L.QB = take(sizeof(float) * Ptot * KK * 4);
  L.KA = take(sizeof(float) * Ptot * KK * 4);
  L.VA = take(sizeof(float) * Ptot * 16);
  L.VB = take(sizeof(float) * Ptot * 16);
  L.QH = take(sizeof(uint16_t) * Ptot * 32 * f16_slices(D));
  L.KH = take(sizeof(uint16_t) * Ptot * 32 * f16_slices(D));
  L.RN = take(sizeof(float) * Ptot);
  L.xc = take(sizeof(float) * Ptot * D);
  L.t1 = take(sizeof(float) * Ptot * D);
  L.S = take(sizeof(float) * Ptot);
  L.wv = take(sizeof(float) * Ptot);
  L.part = take(sizeof(float) * Ptot * 16);
  L.meanp = take(sizeof(double) * (Ptot / 256) * 16);
  L.redp = take(sizeof(double) * (Ptot / 256) * 16);
  L.tau = take(sizeof(double) * nens * 9);
  L.total = off;
  return L;
}

// (ensemble, row tile) items, costliest ensembles first.  A row tile is the
// 4 rb 16-row blocks of the 16x16 forms, or the 4 rb 32-row blocks of
// VDS_PAIR_MFMA32.
std::vector<int2> make_items(const vds_batch b, int rb) {
  const int64_t rows_per_block = b->impl == VDS_PAIR_MFMA32 ? 32 : 16;
  std::vector<int> order(b->nens);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->P[x] > b->P[y]; });
  std::vector<int2> items;
  for (int e : order) {
    const int64_t tiles = (pad(b->P[e]) / rows_per_block + 4 * rb - 1) / (4 * rb);
    for (int64_t t = 0; t < tiles; ++t) items.push_back(make_int2(e, (int)t));
  }
  return items;
}

vds_status upload_items(vds_batch b) {
  std::vector<int2> items = make_items(b, b->rb);
  b->nitems = (int)items.size();
  vds_status st = bhip(b, hipMemcpyAsync(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice,
                                         b->priv), "upload items");
  if (st == VDS_OK) st = bhip(b, hipStreamSynchronize(b->priv), "synchronise");
  return st;
}

BatchView view(vds_batch b) {
  BatchView v;
  v.ens = b->d_ens;
  v.blk16_ens = b->d_blk16;
  v.blk256_ens = b->d_blk256;
  v.nblk16 = (int)(b->Ptot_pad / 16);
  v.nblk256 = (int)(b->Ptot_pad / 256);
  v.D = b->D;
  v.KK = b->KK;
  v.f16 = b->f16;
  return v;
}

// Operand formats of the ensembles follow the pair implementation.
void set_formats(vds_batch b) {
  for (EnsDesc &d : b->ens) {
    d.p.vhalf = (b->impl == VDS_PAIR_MFMA_F16X2 || b->impl == VDS_PAIR_MFMA_F16X2_ALL) ? 1 : 0;
    d.p.qhalf = b->impl == VDS_PAIR_MFMA_F16X2_ALL ? 1 : 0;
    d.p.f32x = b->impl == VDS_PAIR_MFMA32 ? 1 : 0;  // its per-chunk operand layout
  }
}

vds_status upload_ens(vds_batch b) {
  set_formats(b);
  vds_status st = bhip(b, hipMemcpyAsync(b->d_ens, b->ens.data(), sizeof(EnsDesc) * b->nens, hipMemcpyHostToDevice,
                                         b->priv), "upload ensembles");
  if (st == VDS_OK) st = bhip(b, hipStreamSynchronize(b->priv), "synchronise");
  return st;
}

void pair_pass(vds_batch b, const float *V, bool pass_a, hipStream_t s) {
  launch_batch_pair(b->impl, b->rb, b->grid, b->KK, b->D, b->d_items, b->nitems, b->d_ens, b->QB, b->KA, V, b->f16,
                    pass_a, b->xc, b->part, s);
}

// Centring, packing and pass A (through its finalisation) of every ensemble.
void pass_a(vds_batch b, const float *q, hipStream_t s) {
  const BatchView v = view(b);
  launch_batch_mean(v, q, b->meanp, s);
  launch_batch_prep(v, q, b->meanp, b->xc, b->wv, b->QB, b->KA, b->VA, s);
  pair_pass(b, b->VA, true, s);
  launch_batch_finalize_a(v, b->part, b->xc, b->wv, b->S, b->t1, b->VB, s);
}

void one_step(vds_batch b, float *q, hipStream_t s) {
  pass_a(b, q, s);
  pair_pass(b, b->VB, false, s);
  launch_batch_explicit(view(b), b->part, b->xc, b->t1, b->S, b->wv, q, s);
}

void drop_graph(vds_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_q = nullptr;
}

vds_status capture(vds_batch b, float *q) {
  drop_graph(b);
  vds_status st = bhip(b, hipStreamBeginCapture(b->priv, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st != VDS_OK) return st;
  one_step(b, q, b->priv);
  st = bhip(b, hipStreamEndCapture(b->priv, &b->graph), "end capture");
  if (st != VDS_OK) return st;
  st = bhip(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
  if (st != VDS_OK) return st;
  b->graph_q = q;
  b->graph_impl = b->impl;
  b->graph_rb = b->rb;
  b->graph_grid = b->grid;
  return VDS_OK;
}

}  // namespace

extern "C" {

size_t vds_batch_workspace_bytes(int32_t nens, const int64_t *P, int32_t nb) {
  if (nens < 1 || P == nullptr || nb < 1 || nb > kMaxNb) return 0;
  for (int e = 0; e < nens; ++e)
    if (P[e] < 1 || P[e] > ((int64_t)1 << 26)) return 0;
  return batch_layout(nens, P, nb).total;
}

vds_status vds_batch_create(int32_t nens, const int64_t *P, const double *h, const double *G,
                            const vds_problem *common, const double *H, void *hip_stream, vds_batch *out) {
  auto fail = [&](const char *m) {
    g_batch_create_error = m;
    return VDS_ERR_ARG;
  };
  if (out == nullptr) return fail("out is NULL");
  *out = nullptr;
  if (nens < 1 || !P || !h || !G || !common || !H) return fail("null argument or nens < 1");
  const vds_problem &c = *common;
  if (c.nb < 1 || c.nb > kMaxNb) return fail("nb must be in 1..5");
  if (!(c.dt > 0.0) || !(c.zeta > 0.0) || !(c.kT >= 0.0)) return fail("dt, zeta must be > 0 and kT >= 0");
  if (c.potential != VDS_HOOKEAN && c.potential != VDS_FENE) return fail("unknown potential");
  if (c.potential == VDS_FENE && !(c.b_max > 0.0)) return fail("FENE needs b_max > 0");
  for (int k = 0; k < c.nb; ++k)
    if (!(H[k] > 0.0) || !std::isfinite(H[k])) return fail("spring constants must be positive");
  for (int e = 0; e < nens; ++e) {
    if (P[e] < 1 || P[e] > ((int64_t)1 << 26)) return fail("each P must be in 1..2^26");
    if (!(h[e] > 0.0) || !std::isfinite(h[e])) return fail("each h must be positive and finite");
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(G[9 * e + i])) return fail("G must be finite");
  }
  vds_batch b = new (std::nothrow) vds_batch_s();
  if (b == nullptr) {
    g_batch_create_error = "host allocation failed";
    return VDS_ERR_NOMEM;
  }
  b->nens = nens;
  b->nb = c.nb;
  b->D = 3 * c.nb;
  b->KK = (b->D + 2 + 3) / 4;
  b->P.assign(P, P + nens);
  b->user = reinterpret_cast<hipStream_t>(hip_stream);
  int64_t pad_off = 0, q_off = 0;
  for (int e = 0; e < nens; ++e) {
    EnsDesc d{};
    EvalParams &p = d.p;
    p.P = P[e];
    p.Ppad = pad(P[e]);
    p.nb = c.nb;
    p.D = b->D;
    p.KK = b->KK;
    p.kappa = (float)(1.4426950408889634 / (2.0 * h[e] * h[e]));
    p.inv_h2 = (float)(1.0 / (h[e] * h[e]));
    p.kT = (float)c.kT;
    p.inv_zeta = (float)(1.0 / c.zeta);
    p.dt = (float)c.dt;
    p.n = (float)c.n;
    for (int i = 0; i < 9; ++i) p.G[i] = (float)G[9 * e + i];
    for (int k = 0; k < kMaxNb; ++k) p.H[k] = k < c.nb ? (float)H[k] : 0.f;
    p.b_max = (float)c.b_max;
    p.potential = c.potential;
    p.uniform_w = (float)(1.0 / (double)P[e]);
    p.log_norm = (float)(0.5 * b->D * std::log(2.0 * M_PI * h[e] * h[e]));
    p.KQ = f16_slices(b->D);
    p.cs = (float)std::sqrt(2.0 * 1.4426950408889634 / (2.0 * h[e] * h[e]));
    p.KP = mfma32_kslots(b->D);
    d.pad_off = pad_off;
    d.q_off = q_off;
    d.blk16 = (int)(pad_off / 16);
    d.blk256 = (int)(pad_off / 256);
    for (int64_t i = 0; i < p.Ppad / 16; ++i) b->blk16.push_back(e);
    for (int64_t i = 0; i < p.Ppad / 256; ++i) b->blk256.push_back(e);
    b->ens.push_back(d);
    pad_off += p.Ppad;
    q_off += (int64_t)c.nb * P[e] * 3;
  }
  b->Ptot_pad = pad_off;
  b->qlen = q_off;
  b->L = batch_layout(nens, P, c.nb);
  *out = b;
  return VDS_OK;
}

vds_status vds_batch_bind_workspace(vds_batch b, void *ws, size_t bytes) {
  if (b == nullptr) return VDS_ERR_ARG;
  if (ws == nullptr || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return berr(b, VDS_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (bytes < b->L.total) return berr(b, VDS_ERR_NOMEM, "workspace smaller than vds_batch_workspace_bytes()");
  b->ws = static_cast<char *>(ws);
  const BatchLayout &L = b->L;
  auto f = [&](size_t o) { return reinterpret_cast<float *>(b->ws + o); };
  b->d_ens = reinterpret_cast<EnsDesc *>(b->ws + L.ens);
  b->d_blk16 = reinterpret_cast<int *>(b->ws + L.blk16);
  b->d_blk256 = reinterpret_cast<int *>(b->ws + L.blk256);
  b->d_items = reinterpret_cast<int2 *>(b->ws + L.items);
  b->QB = f(L.QB);
  b->KA = f(L.KA);
  b->VA = f(L.VA);
  b->VB = f(L.VB);
  b->xc = f(L.xc);
  b->t1 = f(L.t1);
  b->S = f(L.S);
  b->wv = f(L.wv);
  b->part = f(L.part);
  b->f16 = F16Operands{b->ws + L.QH, b->ws + L.KH, f(L.RN)};
  b->meanp = reinterpret_cast<double *>(b->ws + L.meanp);
  b->redp = reinterpret_cast<double *>(b->ws + L.redp);
  b->tau = reinterpret_cast<double *>(b->ws + L.tau);
  vds_status st = VDS_OK;
  if (b->priv == nullptr) {
    st = bhip(b, hipStreamCreateWithFlags(&b->priv, hipStreamNonBlocking), "create stream");
    if (st == VDS_OK) st = bhip(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "event");
    if (st == VDS_OK) st = bhip(b, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "event");
    if (st != VDS_OK) return st;
  }
  drop_graph(b);
  set_formats(b);
  st = bhip(b, hipMemcpyAsync(b->d_ens, b->ens.data(), sizeof(EnsDesc) * b->nens, hipMemcpyHostToDevice, b->priv),
            "upload ensembles");
  if (st == VDS_OK)
    st = bhip(b, hipMemcpyAsync(b->d_blk16, b->blk16.data(), sizeof(int) * b->blk16.size(), hipMemcpyHostToDevice,
                                b->priv), "upload tables");
  if (st == VDS_OK)
    st = bhip(b, hipMemcpyAsync(b->d_blk256, b->blk256.data(), sizeof(int) * b->blk256.size(),
                                hipMemcpyHostToDevice, b->priv), "upload tables");
  if (st == VDS_OK) st = upload_items(b);
  return st;
}

void vds_batch_destroy(vds_batch b) {
  if (b == nullptr) return;
  drop_graph(b);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->priv) (void)hipStreamDestroy(b->priv);
  delete b;
}

const char *vds_batch_last_error(vds_batch b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

int64_t vds_batch_state_offset(vds_batch b, int32_t e) {
  if (b == nullptr || e < 0 || e > b->nens) return -1;
  return e == b->nens ? b->qlen : b->ens[e].q_off;
}

vds_status vds_batch_set_tuning(vds_batch b, int32_t impl, int32_t rb, int32_t grid, int32_t use_graph) {
  if (b == nullptr) return VDS_ERR_ARG;
  if (impl != VDS_PAIR_MFMA32 && impl != VDS_PAIR_MFMA && impl != VDS_PAIR_MFMA_F16X2 &&
      impl != VDS_PAIR_MFMA_F16X2_ALL)
    return berr(b, VDS_ERR_ARG, "impl must be VDS_PAIR_MFMA32, VDS_PAIR_MFMA or one of the FP16-split forms");
  if (!(rb == 1 || rb == 2 || (rb == 4 && impl != VDS_PAIR_MFMA32)) || grid < 1 || grid > (1 << 20))
    return berr(b, VDS_ERR_ARG, "rows_per_wave must be 1, 2 or 4 (1 or 2 for VDS_PAIR_MFMA32) and grid >= 1");
  // row tiles of the work list follow rb and the implementation's block height
  const bool items_change = rb != b->rb || (impl == VDS_PAIR_MFMA32) != (b->impl == VDS_PAIR_MFMA32);
  const bool impl_change = impl != b->impl;
  b->impl = impl;
  b->rb = rb;
  b->grid = grid;
  b->use_graph = use_graph ? 1 : 0;
  vds_status st = VDS_OK;
  if (impl_change && b->ws) st = upload_ens(b);
  if (st == VDS_OK && items_change && b->ws) st = upload_items(b);
  return st;
}

vds_status vds_batch_get_tuning(vds_batch b, int32_t *impl, int32_t *rb, int32_t *grid, int32_t *use_graph) {
  if (b == nullptr) return VDS_ERR_ARG;
  if (impl) *impl = b->impl;
  if (rb) *rb = b->rb;
  if (grid) *grid = b->grid;
  if (use_graph) *use_graph = b->use_graph;
  return VDS_OK;
}

vds_status vds_batch_autotune(vds_batch b, const float *q) {
  if (b == nullptr) return VDS_ERR_ARG;
  if (b->ws == nullptr) return berr(b, VDS_ERR_STATE, "no workspace bound");
  if (q == nullptr) return berr(b, VDS_ERR_ARG, "null state");
  vds_status st = bhip(b, hipEventRecord(b->ev_in, b->user), "event");
  if (st == VDS_OK) st = bhip(b, hipStreamWaitEvent(b->priv, b->ev_in, 0), "wait");
  if (st != VDS_OK) return st;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  float best = 1e30f;
  int best_impl = b->impl, best_rb = b->rb, best_grid = b->grid;
  // the launch shape only: the arithmetic (implementation) stays the caller's choice
  for (int impl : {b->impl}) {
    st = vds_batch_set_tuning(b, impl, b->rb, b->grid, b->use_graph);
    if (st != VDS_OK) break;
    pass_a(b, q, b->priv);  // operands in this implementation's format
    for (int rb : {1, 2, 4}) {
      if (rb == 4 && impl == VDS_PAIR_MFMA32) continue;
      for (int per_cu : {2, 4, 8}) {
        st = vds_batch_set_tuning(b, impl, rb, 256 * per_cu, b->use_graph);
        if (st != VDS_OK) break;
        pair_pass(b, b->VB, false, b->priv);  // warm-up
        (void)hipEventRecord(t0, b->priv);
        pair_pass(b, b->VB, false, b->priv);
        (void)hipEventRecord(t1, b->priv);
        st = bhip(b, hipEventSynchronize(t1), "autotune");
        if (st != VDS_OK) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        if (ms < best) {
          best = ms;
          best_impl = impl;
          best_rb = rb;
          best_grid = 256 * per_cu;
        }
      }
      if (st != VDS_OK) break;
    }
    if (st != VDS_OK) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != VDS_OK) return st;
  return vds_batch_set_tuning(b, best_impl, best_rb, best_grid, b->use_graph);
}

vds_status vds_batch_step(vds_batch b, float *q, int32_t nsteps, double *tau_host) {
  if (b == nullptr) return VDS_ERR_ARG;
  if (b->ws == nullptr) return berr(b, VDS_ERR_STATE, "no workspace bound");
  if (q == nullptr || nsteps < 0) return berr(b, VDS_ERR_ARG, "bad arguments");
  vds_status st = bhip(b, hipEventRecord(b->ev_in, b->user), "event");
  if (st == VDS_OK) st = bhip(b, hipStreamWaitEvent(b->priv, b->ev_in, 0), "wait");
  if (st != VDS_OK) return st;
  if (b->use_graph && nsteps > 0) {
    if (b->exec == nullptr || b->graph_q != q || b->graph_impl != b->impl || b->graph_rb != b->rb ||
        b->graph_grid != b->grid) {
      st = capture(b, q);
      if (st != VDS_OK) return st;
    }
    for (int s = 0; s < nsteps && st == VDS_OK; ++s) st = bhip(b, hipGraphLaunch(b->exec, b->priv), "graph launch");
  } else {
    for (int s = 0; s < nsteps; ++s) one_step(b, q, b->priv);
    st = bhip(b, hipGetLastError(), "launch");
  }
  if (st != VDS_OK) return st;
  if (tau_host) {
    launch_batch_stress(view(b), q, b->redp, b->priv);
    launch_batch_stress_sum(b->d_ens, b->nens, b->redp, b->tau, b->priv);
    st = bhip(b, hipMemcpyAsync(tau_host, b->tau, sizeof(double) * 9 * b->nens, hipMemcpyDeviceToHost, b->priv),
              "copy stress");
  }
  if (st == VDS_OK) st = bhip(b, hipEventRecord(b->ev_out, b->priv), "event");
  if (st == VDS_OK) st = bhip(b, hipStreamWaitEvent(b->user, b->ev_out, 0), "wait");
  if (st == VDS_OK && tau_host) st = bhip(b, hipStreamSynchronize(b->priv), "synchronise");
  return st;
}

}  // extern "C"
