// POD offline phase and POD maps (C ABI of include/vds_pod.h).
//
// Gram matrix X^T X by the FP32 MFMA GEMM, symmetric eigensolve in FP64 by
// rocSOLVER (dsyevd), U = X V_R L_R^{-1/2} by the GEMM, then Cholesky-QR
// re-orthonormalisation (the FP32 Gram resolves eigenvalues only down to
// ~1e-7 of the largest, so the trailing columns need it).  Projection and
// reconstruction are skinny products that read U once (HBM bound).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "vds_ctx.h"
#include "vds_linalg.h"
#include "vds_pod.h"

using namespace vds;

namespace {

// q_k = U p_k for the nb bonds k: thread i sums over r in order, reading U
// column by column (coalesced over i; sixteen columns in flight), so U is read
// once.
constexpr int kReconThreads = 256;
constexpr int kReconInFlight = 16;

__global__ __launch_bounds__(kReconThreads) void k_pod_reconstruct(const float *__restrict__ U, int64_t m, int R,
                                                                   int nb, const float *__restrict__ p,
                                                                   float *__restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * kReconThreads + threadIdx.x;
  if (i >= m) return;
  float acc[kMaxNb];
#pragma unroll
  for (int k = 0; k < kMaxNb; ++k) acc[k] = 0.f;
  const float *u = U + i;
  int r = 0;
  for (; r + kReconInFlight <= R; r += kReconInFlight) {
    float uv[kReconInFlight];
#pragma unroll
    for (int j = 0; j < kReconInFlight; ++j) uv[j] = u[(int64_t)(r + j) * m];
#pragma unroll
    for (int k = 0; k < kMaxNb; ++k)
      if (k < nb) {
        const float *pk = p + (int64_t)k * R + r;
#pragma unroll
        for (int j = 0; j < kReconInFlight; ++j) acc[k] = fmaf(uv[j], pk[j], acc[k]);
      }
  }
  for (; r < R; ++r) {
    const float u0 = u[(int64_t)r * m];
#pragma unroll
    for (int k = 0; k < kMaxNb; ++k)
      if (k < nb) acc[k] = fmaf(u0, p[(int64_t)k * R + r], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < kMaxNb; ++k)
    if (k < nb) q[(int64_t)k * m + i] = acc[k];
}

constexpr int kProjThreads = 256;
constexpr int kProjChunks = 32;
constexpr int kProjRows = 8;

// First stage of p_k[r] = U_r . q_k: block (g, c) takes the rows
// r = 8 g .. 8 g + 7 of U against chunk c of the positions; a thread reads
// q_k[i] once for all eight rows (thirteen loads in flight per position), so U
// is read once and q once per eight rows.  Then a fixed-order block reduction
// per (row, bond) into part[c][k][r].
__global__ __launch_bounds__(kProjThreads) void k_pod_project(const float *__restrict__ U, int64_t m, int R, int nb,
                                                              const float *__restrict__ q, float *__restrict__ part) {
  __shared__ float red[kProjRows * kMaxNb][kProjThreads / 64];
  const int r0 = (int)blockIdx.x * kProjRows, c = (int)blockIdx.y;
  const int nr = min(kProjRows, R - r0);
  const int64_t len = (m + kProjChunks - 1) / kProjChunks, i0 = c * len, i1 = min(m, i0 + len);
  float acc[kProjRows][kMaxNb];
#pragma unroll
  for (int j = 0; j < kProjRows; ++j)
#pragma unroll
    for (int k = 0; k < kMaxNb; ++k) acc[j][k] = 0.f;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kProjThreads) {
    float qv[kMaxNb];
#pragma unroll
    for (int k = 0; k < kMaxNb; ++k) qv[k] = k < nb ? q[(int64_t)k * m + i] : 0.f;
#pragma unroll
    for (int j = 0; j < kProjRows; ++j) {
      const float u = j < nr ? U[(int64_t)(r0 + j) * m + i] : 0.f;
#pragma unroll
      for (int k = 0; k < kMaxNb; ++k) acc[j][k] = fmaf(u, qv[k], acc[j][k]);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kProjRows; ++j)
#pragma unroll
    for (int k = 0; k < kMaxNb; ++k) {
      float v = acc[j][k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) red[j * kMaxNb + k][wave] = v;
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kProjRows * kMaxNb) {
    const int j = t / kMaxNb, k = t % kMaxNb;
    if (j < nr && k < nb) {
      float v = 0.f;
      for (int w = 0; w < kProjThreads / 64; ++w) v += red[t][w];
      part[((int64_t)c * nb + k) * R + r0 + j] = v;
    }
  }
}

// Second stage: p[k][r] = sum over the chunks in order.
__global__ void k_pod_project_sum(const float *__restrict__ part, int R, int nb, float *__restrict__ p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nb * R) return;
  float v = 0.f;
  for (int c = 0; c < kProjChunks; ++c) v += part[(int64_t)c * nb * R + e];
  p[e] = v;
}

}  // namespace

namespace vds {
void launch_pod_reconstruct(const float *U, int64_t m, int R, int nb, const float *p, float *q, hipStream_t s) {
  k_pod_reconstruct<<<(unsigned)((m + kReconThreads - 1) / kReconThreads), kReconThreads, 0, s>>>(U, m, R, nb, p, q);
}
}  // namespace vds

namespace {

struct PodLayout {
  size_t gram, gram64, eig, offd, info, Wt, U2, GU, GU64, Linv, work64, part, total;
};

PodLayout pod_layout(int64_t m, int32_t n, int32_t R) {
  PodLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  L.gram = take(sizeof(float) * n * n);
  L.gram64 = take(sizeof(double) * n * n);
  L.eig = take(sizeof(double) * n);
  L.offd = take(sizeof(double) * n);
  L.info = take(sizeof(int) * 4);
  L.Wt = take(sizeof(float) * (size_t)R * n);
  L.U2 = take(sizeof(float) * (size_t)m * R);
  L.GU = take(sizeof(float) * R * R);
  L.GU64 = take(sizeof(double) * R * R);
  L.Linv = take(sizeof(float) * R * R);
  L.work64 = take(sizeof(double) * R * R);
  const int sg = gemm_splits(n, n, m, 1024, true), su = gemm_splits(R, R, m);
  const size_t part = std::max({sizeof(float) * (size_t)sg * n * n, sizeof(float) * (size_t)su * R * R,
                                sizeof(float) * (size_t)m * R});
  L.part = take(part);
  L.total = off;
  return L;
}

// Wt[s][c] = V[c][n-1-s] / sqrt(max(lambda_{n-1-s}, floor)): the R leading
// eigenvectors (eigenvalues ascending in `eig`), scaled.
__global__ void k_scaled_modes(const double *V, const double *eig, int n, int R, double floor_, float *Wt) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)R * n) return;
  const int s = (int)(t / n), c = (int)(t % n);
  const int col = n - 1 - s;
  const double lam = fmax(eig[col], floor_);
  Wt[t] = (float)(V[(int64_t)col * n + c] / sqrt(lam));
}

vds_status gram_into(vds_ctx c, const float *X, int64_t m, int n, float *gram, float *part) {
  GemmShape g;
  g.M = n;
  g.N = n;
  g.K = m;
  g.A = X;
  g.lda = m;
  g.B = X;
  g.ldb = m;
  g.C = gram;
  g.ldc = n;
  g.symmetric = true;
  g.splits = gemm_splits(n, n, m, 1024, true);
  // the symmetric product's own work: n (n + 1) / 2 entries of 2 m FLOP
  timed(c, VDS_TIMER_GEMM, (double)n * (n + 1) * (double)m, [&] { launch_gemm(g, part, c->stream); });
  return hip_check(c, hipGetLastError(), "gram");
}

// dst (m x R col-major) = src (m x R col-major) * B^T where B[j][k] = Bt[j*ldb + k] (R x kdim)
void times_small(vds_ctx c, const float *src, int64_t m, int kdim, const float *Bt, int R, float *dst, float *part) {
  GemmShape g;
  g.M = (int)m;
  g.N = R;
  g.K = kdim;
  g.A = src;
  g.lda = m;
  g.a_mn = true;
  g.B = Bt;
  g.ldb = kdim;
  g.C = dst;
  g.ldc = m;
  g.c_colmajor = true;
  g.splits = 1;
  timed(c, VDS_TIMER_GEMM, 2.0 * m * (double)R * kdim, [&] { launch_gemm(g, part, c->stream); });
}

}  // namespace

extern "C" {

size_t vds_pod_workspace_bytes(int64_t m, int32_t ncols, int32_t R) {
  if (m < 1 || ncols < 1 || R < 1 || R > ncols || R > m) return 0;
  return pod_layout(m, ncols, R).total;
}

vds_status vds_pod_gram(vds_ctx c, const float *X, int64_t m, int32_t n, float *gram, void *ws, size_t bytes) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (!X || !gram || !ws || m < 1 || n < 1) return set_err(c, VDS_ERR_ARG, "bad arguments");
  const PodLayout L = pod_layout(m, n, 1);
  if (bytes < L.total) return set_err(c, VDS_ERR_NOMEM, "POD workspace too small");
  char *w = static_cast<char *>(ws);
  return gram_into(c, X, m, n, gram, reinterpret_cast<float *>(w + L.part));
}

vds_status vds_pod_basis(vds_ctx c, const float *X, int64_t m, int32_t n, int32_t R, float *U, double *eig_host,
                         void *ws, size_t bytes) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (!X || !U || !ws || m < 1 || n < 1 || R < 1 || R > n || R > m)
    return set_err(c, VDS_ERR_ARG, "bad arguments (need 1 <= R <= min(m, ncols))");
  const PodLayout L = pod_layout(m, n, R);
  if (bytes < L.total) return set_err(c, VDS_ERR_NOMEM, "POD workspace too small");
  char *w = static_cast<char *>(ws);
  float *gram = reinterpret_cast<float *>(w + L.gram);
  double *gram64 = reinterpret_cast<double *>(w + L.gram64);
  double *eig = reinterpret_cast<double *>(w + L.eig);
  double *offd = reinterpret_cast<double *>(w + L.offd);
  int *info = reinterpret_cast<int *>(w + L.info);
  float *Wt = reinterpret_cast<float *>(w + L.Wt);
  float *U2 = reinterpret_cast<float *>(w + L.U2);
  float *GU = reinterpret_cast<float *>(w + L.GU);
  double *GU64 = reinterpret_cast<double *>(w + L.GU64);
  float *Linv = reinterpret_cast<float *>(w + L.Linv);
  double *work64 = reinterpret_cast<double *>(w + L.work64);
  float *part = reinterpret_cast<float *>(w + L.part);

  vds_status st = gram_into(c, X, m, n, gram, part);
  if (st != VDS_OK) return st;
  launch_f32_to_f64(gram, gram64, (int64_t)n * n, c->stream);

  rocblas_handle h = static_cast<rocblas_handle>(blas_handle(c));
  if (h == nullptr) return VDS_ERR_HIP;
  const rocblas_status rs =
      rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, gram64, n, eig, offd, info);
  if (rs != rocblas_status_success) return set_err(c, VDS_ERR_HIP, "rocsolver_dsyevd failed");

  std::vector<double> lam(n);
  int hinfo[4] = {0, 0, 0, 0};
  st = hip_check(c, hipMemcpyAsync(lam.data(), eig, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream), "eig");
  if (st == VDS_OK) st = hip_check(c, hipMemcpyAsync(hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c->stream), "info");
  if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  if (st != VDS_OK) return st;
  if (hinfo[0] != 0) return set_err(c, VDS_ERR_HIP, "symmetric eigensolve did not converge");
  if (eig_host)
    for (int i = 0; i < n; ++i) eig_host[i] = lam[n - 1 - i];
  // FP32 Gram resolves eigenvalues to ~1e-7 of the largest; floor the rest
  const double floor_ = std::max(lam[n - 1], 1e-300) * 1e-12;
  k_scaled_modes<<<(unsigned)(((int64_t)R * n + 255) / 256), 256, 0, c->stream>>>(gram64, eig, n, R, floor_, Wt);
  // U2 = X Wt^T  (m x R)
  times_small(c, X, m, n, Wt, R, U2, part);

  // three Cholesky-QR passes: U <- U L^{-T}, L L^T = U^T U (+ shift on the first)
  float *src = U2, *dst = U;
  for (int pass = 0; pass < 3; ++pass) {
    GemmShape g;
    g.M = R;
    g.N = R;
    g.K = m;
    g.A = src;
    g.lda = m;
    g.B = src;
    g.ldb = m;
    g.C = GU;
    g.ldc = R;
    g.splits = gemm_splits(R, R, m);
    timed(c, VDS_TIMER_GEMM, 2.0 * R * (double)R * m, [&] { launch_gemm(g, part, c->stream); });
    launch_f32_to_f64(GU, GU64, (int64_t)R * R, c->stream);
    double shift = 0.0;
    if (pass == 0) {
      // shift ~ 1e-6 of the mean squared column norm
      double tr = 0.0;
      std::vector<float> gh((size_t)R * R);
      st = hip_check(c, hipMemcpyAsync(gh.data(), GU, sizeof(float) * R * R, hipMemcpyDeviceToHost, c->stream), "gu");
      if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
      if (st != VDS_OK) return st;
      for (int i = 0; i < R; ++i) tr += gh[(size_t)i * R + i];
      shift = 1e-6 * tr / R;
    }
    launch_cholesky(GU64, R, shift, info + 1, c->stream);
    launch_tri_inverse(GU64, R, work64, Linv, c->stream);
    // dst = src * Linv^T  (B[j][k] = Linv[j][k])
    times_small(c, src, m, R, Linv, R, dst, part);
    st = hip_check(c, hipMemcpyAsync(hinfo + 1, info + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream), "info");
    if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
    if (st != VDS_OK) return st;
    if (hinfo[1] != 0) return set_err(c, VDS_ERR_ARG, "basis is numerically rank deficient (R exceeds the snapshots' rank)");
    std::swap(src, dst);
  }
  // the last pass wrote into what is now `src`
  if (src != U)
    st = hip_check(c, hipMemcpyAsync(U, src, sizeof(float) * m * R, hipMemcpyDeviceToDevice, c->stream), "copy U");
  if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
  return st;
}

size_t vds_pod_map_workspace_bytes(const vds_problem *prob, int32_t R) {
  if (prob == nullptr || prob->P < 1 || prob->nb < 1 || R < 1) return 0;
  const int64_t m = 3 * prob->P;
  const size_t a = sizeof(float) * (size_t)gemm_splits(prob->nb, R, m, 2048) * prob->nb * R;
  const size_t b = sizeof(float) * (size_t)m * prob->nb;
  const size_t c = sizeof(float) * (size_t)kProjChunks * prob->nb * R;
  return (std::max(std::max(a, b), c) + 255) / 256 * 256;
}

vds_status vds_pod_project(vds_ctx c, const float *U, int32_t R, const float *q, float *p, void *ws, size_t bytes) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (!U || !q || !p || !ws || R < 1) return set_err(c, VDS_ERR_ARG, "bad arguments");
  if (bytes < vds_pod_map_workspace_bytes(&c->prob, R)) return set_err(c, VDS_ERR_NOMEM, "workspace too small");
  const int64_t m = 3 * c->prob.P;
  const int nb = c->prob.nb;
  float *part = static_cast<float *>(ws);
  timed(c, VDS_TIMER_PROJ, 4.0 * m * R, [&] {
    k_pod_project<<<dim3((unsigned)((R + kProjRows - 1) / kProjRows), kProjChunks), kProjThreads, 0, c->stream>>>(
        U, m, R, nb, q, part);
    k_pod_project_sum<<<(nb * R + 255) / 256, 256, 0, c->stream>>>(part, R, nb, p);
  });
  return hip_check(c, hipGetLastError(), "project");
}

vds_status vds_pod_reconstruct(vds_ctx c, const float *U, int32_t R, const float *p, float *q, void *ws,
                               size_t bytes) {
  if (c == nullptr) return VDS_ERR_ARG;
  if (!U || !q || !p || !ws || R < 1) return set_err(c, VDS_ERR_ARG, "bad arguments");
  if (bytes < vds_pod_map_workspace_bytes(&c->prob, R)) return set_err(c, VDS_ERR_NOMEM, "workspace too small");
  const int64_t m = 3 * c->prob.P;
  const int nb = c->prob.nb;
  timed(c, VDS_TIMER_PROJ, 4.0 * m * R, [&] { launch_pod_reconstruct(U, m, R, nb, p, q, c->stream); });
  return hip_check(c, hipGetLastError(), "reconstruct");
}

}  // extern "C"
