// Learned reduced step (C ABI of include/vds_mlp.h): MLP training kernels
// (FP32 MFMA GEMMs, SiLU, MSE gradient, Adam), BF16 MFMA inference, and the
// rollout that checks the network against the particle scheme and falls back.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vds_ctx.h"
#include "vds_linalg.h"
#include "vds_mlp.h"
#include "vds_pod.h"

using namespace vds;

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

thread_local std::string g_mlp_create_error;

struct MlpLayout {
  size_t params, grads, adam_m, adam_v, wbf, wpk, Z1, A1, Z2, A2, Y, dY, dA, dZ, xs, xsc, ys, ysc, xin, tin, part, lossp,
      total;
};

// Resident learned steps (k_learned_steps_reg): one workgroup of 1024 threads
// keeps the BF16 weights on chip for a whole window of steps, layers 1 and 2
// in registers and layer 3 in LDS (gfx950 gives a workgroup 160 KiB).  Layer l
// splits a row over G_l consecutive lanes, each taking CK_l consecutive
// inputs; layer 3 has up to kNout3 * G3 row chunks ("slots"), slot s for
// thread s % 1024.  Shapes that fit: nin <= 8 * 68, width <= 128, nout <= 576.
constexpr int kRegThreads = 1024;
constexpr int kG1 = 8, kCK1 = 68, kG2 = 8, kCK2 = 16, kG3 = 4, kCK3 = 32, kNout3 = 576;
constexpr int kSlots3 = kNout3 * kG3;
constexpr int kS3 = (kSlots3 + kRegThreads - 1) / kRegThreads;
constexpr int64_t kPk1 = (int64_t)kRegThreads * kCK1, kPk2 = (int64_t)kRegThreads * kCK2,
                  kPk3 = (int64_t)kSlots3 * kCK3;  // BF16 elements
bool reg_steps_fit(int nin, int w, int nout) {
  return nin <= kG1 * kCK1 && w <= kRegThreads / kG1 && w <= kG2 * kCK2 && w <= kG3 * kCK3 && nout <= kNout3;
}

int64_t nparams(int nin, int w, int nout) {
  return (int64_t)w * nin + w + (int64_t)w * w + w + (int64_t)nout * w + nout;
}

MlpLayout mlp_layout(int nin, int w, int nout, int B) {
  MlpLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  const int64_t np = nparams(nin, w, nout);
  const int Bp = (B + 15) / 16 * 16;
  L.params = take(sizeof(float) * np);
  L.grads = take(sizeof(float) * np);
  L.adam_m = take(sizeof(float) * np);
  L.adam_v = take(sizeof(float) * np);
  L.wbf = take(sizeof(uint16_t) * np);
  L.wpk = take(sizeof(uint16_t) * (kPk1 + kPk2 + kPk3));
  L.Z1 = take(sizeof(float) * Bp * w);
  L.A1 = take(sizeof(float) * Bp * w);
  L.Z2 = take(sizeof(float) * Bp * w);
  L.A2 = take(sizeof(float) * Bp * w);
  L.Y = take(sizeof(float) * Bp * nout);
  L.dY = take(sizeof(float) * Bp * nout);
  L.dA = take(sizeof(float) * Bp * w);
  L.dZ = take(sizeof(float) * Bp * w);
  L.xs = take(sizeof(float) * nin);
  L.xsc = take(sizeof(float) * nin);
  L.ys = take(sizeof(float) * nout);
  L.ysc = take(sizeof(float) * nout);
  L.xin = take(sizeof(float) * Bp * nin);
  L.tin = take(sizeof(float) * Bp * nout);
  const int64_t g1 = (int64_t)gemm_splits(w, nin, Bp) * w * nin, g3 = (int64_t)gemm_splits(nout, w, Bp) * nout * w;
  const int64_t g0 = (int64_t)Bp * std::max(nout, std::max(w, nin)) * 2;
  L.part = take(sizeof(float) * std::max(std::max(g1, g3), g0));
  L.lossp = take(sizeof(double) * ((int64_t)(Bp * nout + 255) / 256 + 2));
  L.total = off;
  return L;
}

__device__ inline short f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}
__device__ inline float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ inline float silu_grad(float z) {
  const float s = 1.f / (1.f + __expf(-z));
  return s * (1.f + z * (1.f - s));
}

__global__ void k_to_bf16(const float *__restrict__ a, short *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

// Z[i][j] += bias[j]; A = silu(Z) (act) or A = Z.
__global__ void k_bias_act(float *__restrict__ Z, const float *__restrict__ bias, int n, int m, int act,
                           float *__restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * m) return;
  const float z = Z[t] + bias[t % m];
  Z[t] = z;
  if (A) A[t] = act ? silu(z) : z;
}

// dY = 2 (Y - T) / (n m), per-block FP64 partial sums of (Y - T)^2.
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, int n, int m, float *__restrict__ dY,
                      double *__restrict__ lossp) {
  __shared__ double sm[256];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (t < (int64_t)n * m) {
    const float d = Y[t] - T[t];
    dY[t] = 2.f * d / ((float)n * (float)m);
    e2 = (double)d * (double)d;
  }
  sm[threadIdx.x] = e2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = sm[0];
}

__global__ void k_sum_loss(const double *__restrict__ lossp, int nb, double scale, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += lossp[i];
  *out = s * scale;
}

__global__ void k_silu_back(const float *__restrict__ dA, const float *__restrict__ Z, int64_t n,
                            float *__restrict__ dZ) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) dZ[t] = dA[t] * silu_grad(Z[t]);
}

// db[j] = sum_i dZ[i][j], fixed order.
__global__ void k_colsum(const float *__restrict__ dZ, int n, int m, float *__restrict__ db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (double)dZ[(int64_t)i * m + j];
  db[j] = (float)s;
}

__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  th[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// Y[i][j] = act(sum_k X[i][k] W[j][k] + bias[j]) with W in BF16 and X rounded to
// BF16 (FP32 accumulation): one wavefront per 16 x 16 output tile.
__global__ __launch_bounds__(64) void k_dense_bf16(const float *__restrict__ X, int n, int K,
                                                   const short *__restrict__ W, const float *__restrict__ bias,
                                                   int N, int act, float *__restrict__ Y) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int r = lane & 15, g = lane >> 4;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    shortx4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * g + j;
      const int i = i0 + r, c = j0 + r;
      a[j] = (i < n && k < K) ? f2bf(X[(int64_t)i * K + k]) : (short)0;
      b[j] = (c < N && k < K) ? W[(int64_t)c * K + k] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + 4 * g + q, c = j0 + r;
    if (i < n && c < N) {
      const float z = acc[q] + bias[c];
      Y[(int64_t)i * N + c] = act ? silu(z) : z;
    }
  }
}

// x = ((p, log_rate) - shift) / scale
__global__ void k_rollout_input(const float *__restrict__ p, int np_, float log_rate, const float *__restrict__ xs,
                                const float *__restrict__ xsc, float *__restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i > np_) return;
  const float v = i < np_ ? p[i] : log_rate;
  x[i] = (v - xs[i]) / xsc[i];
}

// p += y * scale + shift (or dp = that, when dp != NULL)
__global__ void k_rollout_update(float *__restrict__ p, const float *__restrict__ y, int np_,
                                 const float *__restrict__ ys, const float *__restrict__ ysc, float *__restrict__ dp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np_) return;
  const float d = y[i] * ysc[i] + ys[i];
  if (dp) dp[i] = d;
  else p[i] += d;
}

// ---- fused learned steps: one workgroup runs whole windows of steps ----

constexpr int kFusedThreads = 1024;
constexpr int kFusedMaxLdsFloats = 16384;  // 64 KiB of LDS per workgroup

__device__ inline float bf2f(short b) { return __uint_as_float((unsigned)(unsigned short)b << 16); }
__device__ inline float bf_round(float f) { return bf2f(f2bf(f)); }

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// out[j] = act(sum_k W[j][k] x[k] + bias[j]) for j < N: W in BF16 (row-major,
// N x K), x in LDS already rounded to BF16, FP32 sums (each lane takes
// k = lane, lane + 64, ..., then a butterfly over the wave); wave w of the
// block takes rows w, w + nw, ...  With `round_out` the result is stored
// rounded to BF16 (it is the next layer's input).
__device__ void gemv_bf16(const short *__restrict__ W, int N, int K, const float *x, const float *__restrict__ bias,
                          int act, bool round_out, float *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = kFusedThreads / 64;
  for (int j0 = wave; j0 < N; j0 += 2 * nw) {
    const int j1 = j0 + nw;
    const short *r0 = W + (int64_t)j0 * K;
    const short *r1 = W + (int64_t)(j1 < N ? j1 : j0) * K;
    float s0 = 0.f, s1 = 0.f;
    for (int k = lane; k < K; k += 64) {
      const float xk = x[k];
      s0 = fmaf(bf2f(r0[k]), xk, s0);
      s1 = fmaf(bf2f(r1[k]), xk, s1);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (lane == 0) {
      float z = s0 + bias[j0];
      z = act ? silu(z) : z;
      out[j0] = round_out ? bf_round(z) : z;
      if (j1 < N) {
        z = s1 + bias[j1];
        z = act ? silu(z) : z;
        out[j1] = round_out ? bf_round(z) : z;
      }
    }
  }
}

// nsteps learned steps p += y * ysc + ys with y = network(((p, log_rate) - xs)
// / xsc), the same arithmetic as the BF16 inference path (inputs and hidden
// activations rounded to BF16, BF16 weights, FP32 sums and biases).  With dp
// non-null one increment is written there and p is left unchanged.  One
// workgroup of kFusedThreads; LDS holds x, both hidden layers and p.
__global__ __launch_bounds__(kFusedThreads) void k_rollout_fused(float *__restrict__ p, float *__restrict__ dp,
                                                                int np_, int w, float log_rate, int nsteps,
                                                                const short *__restrict__ W1,
                                                                const float *__restrict__ b1,
                                                                const short *__restrict__ W2,
                                                                const float *__restrict__ b2,
                                                                const short *__restrict__ W3,
                                                                const float *__restrict__ b3,
                                                                const float *__restrict__ xs,
                                                                const float *__restrict__ xsc,
                                                                const float *__restrict__ ys,
                                                                const float *__restrict__ ysc) {
  extern __shared__ float lds[];
  const int nin = np_ + 1;
  float *x = lds, *h1 = x + nin, *h2 = h1 + w, *ps = h2 + w, *y = ps + np_;
  for (int i = threadIdx.x; i < np_; i += kFusedThreads) ps[i] = p[i];
  __syncthreads();
  for (int step = 0; step < nsteps; ++step) {
    for (int i = threadIdx.x; i < nin; i += kFusedThreads) x[i] = bf_round(((i < np_ ? ps[i] : log_rate) - xs[i]) / xsc[i]);
    __syncthreads();
    gemv_bf16(W1, w, nin, x, b1, 1, true, h1);
    __syncthreads();
    gemv_bf16(W2, w, w, h1, b2, 1, true, h2);
    __syncthreads();
    gemv_bf16(W3, np_, w, h2, b3, 0, false, y);
    __syncthreads();
    for (int i = threadIdx.x; i < np_; i += kFusedThreads) {
      const float d = y[i] * ysc[i] + ys[i];
      if (dp != nullptr) dp[i] = d;
      else ps[i] += d;
    }
    __syncthreads();
  }
  if (dp == nullptr)
    for (int i = threadIdx.x; i < np_; i += kFusedThreads) p[i] = ps[i];
}

// Packing of the BF16 weights for k_learned_steps_reg.  Layers 1 and 2:
// thread t's chunk is contiguous, element kk = W_l[row][chunk * CK_l + kk]
// with (row, chunk) = (t / G_l, t % G_l).  Layer 3, as it sits in LDS: eight
// BF16 of slot s, group j (elements 8 j .. 8 j + 7 of its chunk) at uint4
// j * kSlots3 + s, so that neighbouring lanes read neighbouring 16 bytes.
// Zero outside the matrices.  One thread per packed element.
__global__ void k_pack_infer(const float *__restrict__ W1, const float *__restrict__ W2, const float *__restrict__ W3,
                             int nin, int w, int nout, short *__restrict__ pk) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= kPk1 + kPk2 + kPk3) return;
  const float *W;
  int G, CK, N, K;
  int64_t slot, kk;
  if (e < kPk1) {
    W = W1, G = kG1, CK = kCK1, N = w, K = nin, slot = e / kCK1, kk = e % kCK1;
  } else if (e < kPk1 + kPk2) {
    W = W2, G = kG2, CK = kCK2, N = w, K = w, slot = (e - kPk1) / kCK2, kk = (e - kPk1) % kCK2;
  } else {
    const int64_t f = e - kPk1 - kPk2, j = f / (8 * kSlots3);
    W = W3, G = kG3, CK = kCK3, N = nout, K = w, slot = (f / 8) % kSlots3, kk = 8 * j + f % 8;
  }
  const int64_t row = slot / G, k = (slot % G) * CK + kk;
  pk[e] = (row < N && k < K) ? f2bf(W[row * K + k]) : (short)0;
}

// Dot product of CK packed BF16 weights (registers) with CK floats of LDS.
template <int CK>
__device__ inline float dot_bf16(const uint2 (&wr)[CK / 4], const float *x) {
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < CK / 4; ++j) {
    const float4 xv = *reinterpret_cast<const float4 *>(x + 4 * j);
    s = fmaf(__uint_as_float(wr[j].x << 16), xv.x, s);
    s = fmaf(__uint_as_float(wr[j].x & 0xffff0000u), xv.y, s);
    s = fmaf(__uint_as_float(wr[j].y << 16), xv.z, s);
    s = fmaf(__uint_as_float(wr[j].y & 0xffff0000u), xv.w, s);
  }
  return s;
}

template <int G>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// nsteps learned steps with the weights on chip (layout of k_pack_infer), the
// arithmetic of the BF16 inference path: inputs and hidden activations
// rounded to BF16, FP32 products and sums (each lane sums its chunk in order,
// then a fixed butterfly over the row's lanes), FP32 biases.  With dp non-null
// one increment goes to dp and p is unchanged.
__global__ __launch_bounds__(kRegThreads) void k_learned_steps_reg(float *__restrict__ p, float *__restrict__ dp,
                                                                  int np_, int w, float log_rate, int nsteps,
                                                                  const short *__restrict__ pk,
                                                                  const float *__restrict__ b1,
                                                                  const float *__restrict__ b2,
                                                                  const float *__restrict__ b3,
                                                                  const float *__restrict__ xs,
                                                                  const float *__restrict__ xsc,
                                                                  const float *__restrict__ ys,
                                                                  const float *__restrict__ ysc) {
  __shared__ uint4 w3[kCK3 / 8 * kSlots3];
  __shared__ __align__(16) float x[kG1 * kCK1];
  __shared__ __align__(16) float h1[kG2 * kCK2];
  __shared__ __align__(16) float h2[kG3 * kCK3];
  __shared__ float ps[kNout3];
  __shared__ float y[kNout3];
  const int t = threadIdx.x, nin = np_ + 1;
  uint2 w1[kCK1 / 4], w2[kCK2 / 4];
  {
    const uint2 *q1 = reinterpret_cast<const uint2 *>(pk) + (int64_t)t * (kCK1 / 4);
    const uint2 *q2 = reinterpret_cast<const uint2 *>(pk + kPk1) + (int64_t)t * (kCK2 / 4);
#pragma unroll
    for (int j = 0; j < kCK1 / 4; ++j) w1[j] = q1[j];
#pragma unroll
    for (int j = 0; j < kCK2 / 4; ++j) w2[j] = q2[j];
    const uint4 *q3 = reinterpret_cast<const uint4 *>(pk + kPk1 + kPk2);
    for (int i = t; i < kCK3 / 8 * kSlots3; i += kRegThreads) w3[i] = q3[i];
  }
  const int r1 = t / kG1, c1 = t % kG1, c3 = t % kG3;
  for (int i = t; i < np_; i += kRegThreads) ps[i] = p[i];
  // padding of the layer inputs stays zero
  for (int i = t; i < kG1 * kCK1; i += kRegThreads) x[i] = 0.f;
  for (int i = t; i < kG2 * kCK2; i += kRegThreads) h1[i] = 0.f;
  for (int i = t; i < kG3 * kCK3; i += kRegThreads) h2[i] = 0.f;
  __syncthreads();
  for (int step = 0; step < nsteps; ++step) {
    // the packed weights stay packed: without this the BF16-to-FP32 unpacking
    // is hoisted out of the step loop and needs twice the registers
#pragma unroll
    for (int j = 0; j < kCK1 / 4; ++j) asm volatile("" : "+v"(w1[j].x), "+v"(w1[j].y));
#pragma unroll
    for (int j = 0; j < kCK2 / 4; ++j) asm volatile("" : "+v"(w2[j].x), "+v"(w2[j].y));
    for (int i = t; i < nin; i += kRegThreads) x[i] = bf_round(((i < np_ ? ps[i] : log_rate) - xs[i]) / xsc[i]);
    __syncthreads();
    float a = group_sum<kG1>(dot_bf16<kCK1>(w1, x + c1 * kCK1));
    if (c1 == 0 && r1 < w) h1[r1] = bf_round(silu(a + b1[r1]));
    __syncthreads();
    a = group_sum<kG2>(dot_bf16<kCK2>(w2, h1 + c1 * kCK2));
    if (c1 == 0 && r1 < w) h2[r1] = bf_round(silu(a + b2[r1]));
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kS3; ++i) {
      const int slot = t + kRegThreads * i;  // uniform over each group of kG3 lanes
      if (slot < kSlots3) {
        const float *hx = h2 + c3 * kCK3;
        float s3 = 0.f;
#pragma unroll
        for (int j = 0; j < kCK3 / 8; ++j) {
          const uint4 wv = w3[j * kSlots3 + slot];
          const float4 xa = *reinterpret_cast<const float4 *>(hx + 8 * j);
          const float4 xb = *reinterpret_cast<const float4 *>(hx + 8 * j + 4);
          s3 = fmaf(__uint_as_float(wv.x << 16), xa.x, s3);
          s3 = fmaf(__uint_as_float(wv.x & 0xffff0000u), xa.y, s3);
          s3 = fmaf(__uint_as_float(wv.y << 16), xa.z, s3);
          s3 = fmaf(__uint_as_float(wv.y & 0xffff0000u), xa.w, s3);
          s3 = fmaf(__uint_as_float(wv.z << 16), xb.x, s3);
          s3 = fmaf(__uint_as_float(wv.z & 0xffff0000u), xb.y, s3);
          s3 = fmaf(__uint_as_float(wv.w << 16), xb.z, s3);
          s3 = fmaf(__uint_as_float(wv.w & 0xffff0000u), xb.w, s3);
        }
        a = group_sum<kG3>(s3);
        const int row = slot / kG3;
        if (c3 == 0 && row < np_) y[row] = a + b3[row];
      }
    }
    __syncthreads();
    for (int i = t; i < np_; i += kRegThreads) {
      const float d = y[i] * ysc[i] + ys[i];
      if (dp != nullptr) dp[i] = d;
      else ps[i] += d;
    }
    __syncthreads();
  }
  if (dp == nullptr)
    for (int i = t; i < np_; i += kRegThreads) p[i] = ps[i];
}

// SplitMix64 (Steele, Lea and Flood 2014): a counter-based stream of 64-bit
// values; one call per draw.
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
// Standard normal draw number `ctr` of stream `seed` by the Box-Muller
// transform of two SplitMix64 uniforms in (0, 1].
__device__ inline float normal_draw(uint64_t seed, uint64_t ctr) {
  const uint64_t a = splitmix64(seed ^ splitmix64(2 * ctr)), b = splitmix64(seed ^ splitmix64(2 * ctr + 1));
  const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(b >> 11) * 0x1.0p-53;
  return (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

// Minibatch rows i < nb: xin[i] = (X[order[i0 + i]] - xs) / xsc, tin likewise.
// With noise > 0 (learned steps, nin = nout + 1) input c < nout also gets
// noise * (ysc[c] / xsc[c]) * xi, xi standard normal from (seed, draw_base +
// row * nin + c): a perturbation of the state coefficient by `noise` standard
// deviations of its increment, the target unchanged.
__global__ void k_gather_scaled(const float *__restrict__ X, const float *__restrict__ T,
                                const int *__restrict__ order, int i0, int nb, int nin, int nout,
                                const float *__restrict__ xs, const float *__restrict__ xsc,
                                const float *__restrict__ ys, const float *__restrict__ ysc, float *__restrict__ xin,
                                float *__restrict__ tin, float noise, uint64_t seed, uint64_t draw_base) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row_len = nin + nout;
  if (t >= (int64_t)nb * row_len) return;
  const int i = (int)(t / row_len), c = (int)(t % row_len);
  const int64_t src = order ? order[i0 + i] : i0 + i;
  if (c < nin) {
    float x = (X[src * nin + c] - xs[c]) / xsc[c];
    if (noise > 0.f && c < nout)
      x += noise * (ysc[c] / xsc[c]) * normal_draw(seed, draw_base + (uint64_t)i * nin + c);
    xin[(int64_t)i * nin + c] = x;
  } else {
    tin[(int64_t)i * nout + (c - nin)] = (T[src * nout + (c - nin)] - ys[c - nin]) / ysc[c - nin];
  }
}

// Column mean and standard deviation of A[n][m] (FP64 sums); zero spread -> 1.
__global__ void k_col_stats(const float *__restrict__ A, int n, int m, float *__restrict__ mean,
                            float *__restrict__ sd) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  double s = 0.0, s2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = (double)A[(int64_t)i * m + j];
    s += v;
    s2 += v * v;
  }
  const double mu = s / n;
  const double var = fmax(s2 / n - mu * mu, 0.0);
  const double sdv = sqrt(var);
  mean[j] = (float)mu;
  sd[j] = (float)(sdv > 1e-30 * fmax(1.0, fabs(mu)) ? sdv : 1.0);
}

__global__ void k_make_pairs(const float *__restrict__ traj, int nt, int nout, float log_rate,
                             float *__restrict__ X, float *__restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)(nt - 1) * (nout + 1)) return;
  const int i = (int)(t / (nout + 1)), c = (int)(t % (nout + 1));
  if (c < nout) {
    const float a = traj[(int64_t)i * nout + c];
    X[(int64_t)i * (nout + 1) + c] = a;
    T[(int64_t)i * nout + c] = traj[(int64_t)(i + 1) * nout + c] - a;
  } else {
    X[(int64_t)i * (nout + 1) + c] = log_rate;
  }
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct vds_mlp_s {
  int nin, w, nout, B;
  int64_t np;
  hipStream_t s = nullptr;
  MlpLayout L{};
  char *ws = nullptr;
  float *params, *grads, *am, *av, *Z1, *A1, *Z2, *A2, *Y, *dY, *dA, *dZ, *xs, *xsc, *ys, *ysc, *xin, *tin, *part;
  short *wbf, *wpk;
  double *lossp;
  double *loss_out;  // one slot after the per-block partials
  int t = 0;
  bool bf_stale = true;
  float noise = 0.f;          // training input noise (vds_mlp_set_input_noise)
  uint64_t noise_seed = 0, noise_draws = 0;
  std::string err;
  // parameter block views
  float *W1() { return params; }
  float *b1() { return params + (int64_t)w * nin; }
  float *W2() { return b1() + w; }
  float *b2() { return W2() + (int64_t)w * w; }
  float *W3() { return b2() + w; }
  float *b3() { return W3() + (int64_t)nout * w; }
};

namespace {

vds_status merr(vds_mlp m, vds_status st, const std::string &msg) {
  if (m) m->err = msg;
  return st;
}
vds_status mhip(vds_mlp m, hipError_t e, const char *what) {
  if (e == hipSuccess) return VDS_OK;
  return merr(m, VDS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// C = A B^T (row-major), A: n x K, B: N x K, both K-contiguous.
void dense(vds_mlp m, const float *A, int n, int K, const float *B, int N, float *C) {
  GemmShape g;
  g.M = n;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = K;
  g.B = B;
  g.ldb = K;
  g.C = C;
  g.ldc = N;
  launch_gemm(g, m->part, m->s);
}

void forward_fp32(vds_mlp m, const float *X, int n) {
  dense(m, X, n, m->nin, m->W1(), m->w, m->Z1);
  k_bias_act<<<nb256((int64_t)n * m->w), 256, 0, m->s>>>(m->Z1, m->b1(), n, m->w, 1, m->A1);
  dense(m, m->A1, n, m->w, m->W2(), m->w, m->Z2);
  k_bias_act<<<nb256((int64_t)n * m->w), 256, 0, m->s>>>(m->Z2, m->b2(), n, m->w, 1, m->A2);
  dense(m, m->A2, n, m->w, m->W3(), m->nout, m->Y);
  k_bias_act<<<nb256((int64_t)n * m->nout), 256, 0, m->s>>>(m->Y, m->b3(), n, m->nout, 0, nullptr);
}

// dW (N x K) = dZ^T A with dZ: n x N, A: n x K (both row-major)
void weight_grad(vds_mlp m, const float *dZ, int n, int N, const float *A, int K, float *dW) {
  GemmShape g;
  g.M = N;
  g.N = K;
  g.K = n;
  g.A = dZ;
  g.lda = N;
  g.a_mn = true;
  g.B = A;
  g.ldb = K;
  g.b_mn = true;
  g.C = dW;
  g.ldc = K;
  g.splits = gemm_splits(N, K, n, 512);
  launch_gemm(g, m->part, m->s);
}

// dA (n x K) = dZ W with dZ: n x N, W: N x K
void input_grad(vds_mlp m, const float *dZ, int n, int N, const float *W, int K, float *dA) {
  GemmShape g;
  g.M = n;
  g.N = K;
  g.K = N;
  g.A = dZ;
  g.lda = N;
  g.B = W;
  g.ldb = K;
  g.b_mn = true;
  g.C = dA;
  g.ldc = K;
  launch_gemm(g, m->part, m->s);
}

void backward_fp32(vds_mlp m, const float *X, const float *T, int n) {
  const int w = m->w, nin = m->nin, nout = m->nout;
  float *gW1 = m->grads, *gb1 = gW1 + (int64_t)w * nin, *gW2 = gb1 + w, *gb2 = gW2 + (int64_t)w * w,
        *gW3 = gb2 + w, *gb3 = gW3 + (int64_t)nout * w;
  const int64_t ny = (int64_t)n * nout;
  k_mse<<<nb256(ny), 256, 0, m->s>>>(m->Y, T, n, nout, m->dY, m->lossp);
  weight_grad(m, m->dY, n, nout, m->A2, w, gW3);
  k_colsum<<<nb256(nout), 256, 0, m->s>>>(m->dY, n, nout, gb3);
  input_grad(m, m->dY, n, nout, m->W3(), w, m->dA);
  k_silu_back<<<nb256((int64_t)n * w), 256, 0, m->s>>>(m->dA, m->Z2, (int64_t)n * w, m->dZ);
  weight_grad(m, m->dZ, n, w, m->A1, w, gW2);
  k_colsum<<<nb256(w), 256, 0, m->s>>>(m->dZ, n, w, gb2);
  input_grad(m, m->dZ, n, w, m->W2(), w, m->dA);
  k_silu_back<<<nb256((int64_t)n * w), 256, 0, m->s>>>(m->dA, m->Z1, (int64_t)n * w, m->dZ);
  weight_grad(m, m->dZ, n, w, X, nin, gW1);
  k_colsum<<<nb256(w), 256, 0, m->s>>>(m->dZ, n, w, gb1);
}

void refresh_bf16(vds_mlp m) {
  if (!m->bf_stale) return;
  k_to_bf16<<<nb256(m->np), 256, 0, m->s>>>(m->params, m->wbf, m->np);
  if (reg_steps_fit(m->nin, m->w, m->nout))
    k_pack_infer<<<nb256(kPk1 + kPk2 + kPk3), 256, 0, m->s>>>(m->W1(), m->W2(), m->W3(), m->nin, m->w, m->nout,
                                                              m->wpk);
  m->bf_stale = false;
}

// LDS floats of the fused step kernel: x, two hidden layers, p and the output.
int64_t fused_lds_floats(vds_mlp m) { return (int64_t)m->nin + 2 * m->w + 2 * (int64_t)m->nout; }

// nsteps learned steps on p (or one increment into dp): the kernel with the
// weights on chip, or the one streaming them, or the layer-by-layer BF16
// kernels step by step.
void learned_steps(vds_mlp m, float *p, float *dp, float log_rate, int nsteps);

void forward_bf16(vds_mlp m, const float *X, int n, float *Y) {
  refresh_bf16(m);
  const int w = m->w;
  const short *W1 = m->wbf, *W2 = W1 + (int64_t)w * m->nin + w, *W3 = W2 + (int64_t)w * w + w;
  dim3 g1((n + 15) / 16, (w + 15) / 16), g3((n + 15) / 16, (m->nout + 15) / 16);
  k_dense_bf16<<<g1, 64, 0, m->s>>>(X, n, m->nin, W1, m->b1(), w, 1, m->A1);
  k_dense_bf16<<<g1, 64, 0, m->s>>>(m->A1, n, w, W2, m->b2(), w, 1, m->A2);
  k_dense_bf16<<<g3, 64, 0, m->s>>>(m->A2, n, w, W3, m->b3(), m->nout, 0, Y);
}

void learned_steps(vds_mlp m, float *p, float *dp, float log_rate, int nsteps) {
  const int np_ = m->nout;
  refresh_bf16(m);
  if (reg_steps_fit(m->nin, m->w, m->nout)) {
    k_learned_steps_reg<<<1, kRegThreads, 0, m->s>>>(p, dp, np_, m->w, log_rate, dp != nullptr ? 1 : nsteps, m->wpk,
                                                     m->b1(), m->b2(), m->b3(), m->xs, m->xsc, m->ys, m->ysc);
    return;
  }
  if (fused_lds_floats(m) <= kFusedMaxLdsFloats) {
    const int w = m->w;
    const short *W1 = m->wbf, *W2 = W1 + (int64_t)w * m->nin + w, *W3 = W2 + (int64_t)w * w + w;
    const size_t lds = sizeof(float) * (size_t)fused_lds_floats(m);
    k_rollout_fused<<<1, kFusedThreads, lds, m->s>>>(p, dp, np_, w, log_rate, dp != nullptr ? 1 : nsteps, W1, m->b1(),
                                                     W2, m->b2(), W3, m->b3(), m->xs, m->xsc, m->ys, m->ysc);
    return;
  }
  float *xb = m->xin, *yb = m->Y;
  for (int i = 0; i < (dp != nullptr ? 1 : nsteps); ++i) {
    k_rollout_input<<<nb256(np_ + 1), 256, 0, m->s>>>(p, np_, log_rate, m->xs, m->xsc, xb);
    forward_bf16(m, xb, 1, yb);
    k_rollout_update<<<nb256(np_), 256, 0, m->s>>>(dp != nullptr ? nullptr : p, yb, np_, m->ys, m->ysc, dp);
  }
}

}  // namespace

extern "C" {

size_t vds_mlp_workspace_bytes(int32_t nin, int32_t w, int32_t nout, int32_t B) {
  if (nin < 1 || w < 1 || nout < 1 || B < 1 || nin > 65536 || w > 65536 || nout > 65536 || B > (1 << 20)) return 0;
  return mlp_layout(nin, w, nout, B).total;
}

vds_status vds_mlp_create(int32_t nin, int32_t w, int32_t nout, int32_t B, void *stream, vds_mlp *out) {
  if (out == nullptr) {
    g_mlp_create_error = "out is NULL";
    return VDS_ERR_ARG;
  }
  *out = nullptr;
  if (vds_mlp_workspace_bytes(nin, w, nout, B) == 0) {
    g_mlp_create_error = "invalid sizes";
    return VDS_ERR_ARG;
  }
  vds_mlp m = new (std::nothrow) vds_mlp_s();
  if (!m) {
    g_mlp_create_error = "host allocation failed";
    return VDS_ERR_NOMEM;
  }
  m->nin = nin;
  m->w = w;
  m->nout = nout;
  m->B = B;
  m->np = nparams(nin, w, nout);
  m->s = reinterpret_cast<hipStream_t>(stream);
  m->L = mlp_layout(nin, w, nout, B);
  *out = m;
  return VDS_OK;
}

vds_status vds_mlp_bind_workspace(vds_mlp m, void *ws, size_t bytes) {
  if (!m) return VDS_ERR_ARG;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return merr(m, VDS_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < m->L.total) return merr(m, VDS_ERR_NOMEM, "workspace too small");
  m->ws = static_cast<char *>(ws);
  const MlpLayout &L = m->L;
  auto f = [&](size_t o) { return reinterpret_cast<float *>(m->ws + o); };
  m->params = f(L.params);
  m->grads = f(L.grads);
  m->am = f(L.adam_m);
  m->av = f(L.adam_v);
  m->wbf = reinterpret_cast<short *>(m->ws + L.wbf);
  m->wpk = reinterpret_cast<short *>(m->ws + L.wpk);
  m->Z1 = f(L.Z1);
  m->A1 = f(L.A1);
  m->Z2 = f(L.Z2);
  m->A2 = f(L.A2);
  m->Y = f(L.Y);
  m->dY = f(L.dY);
  m->dA = f(L.dA);
  m->dZ = f(L.dZ);
  m->xs = f(L.xs);
  m->xsc = f(L.xsc);
  m->ys = f(L.ys);
  m->ysc = f(L.ysc);
  m->xin = f(L.xin);
  m->tin = f(L.tin);
  m->part = f(L.part);
  m->lossp = reinterpret_cast<double *>(m->ws + L.lossp);
  m->loss_out = m->lossp + ((int64_t)((m->B + 15) / 16 * 16) * m->nout + 255) / 256 + 1;
  // identity scaling until set
  std::vector<float> zx(m->nin, 0.f), ox(m->nin, 1.f), zy(m->nout, 0.f), oy(m->nout, 1.f);
  vds_status st = mhip(m, hipMemcpyAsync(m->xs, zx.data(), 4 * m->nin, hipMemcpyHostToDevice, m->s), "init");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->xsc, ox.data(), 4 * m->nin, hipMemcpyHostToDevice, m->s), "init");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->ys, zy.data(), 4 * m->nout, hipMemcpyHostToDevice, m->s), "init");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->ysc, oy.data(), 4 * m->nout, hipMemcpyHostToDevice, m->s), "init");
  if (st == VDS_OK) st = mhip(m, hipStreamSynchronize(m->s), "synchronise");
  return st;
}

void vds_mlp_destroy(vds_mlp m) { delete m; }
const char *vds_mlp_last_error(vds_mlp m) { return m ? m->err.c_str() : g_mlp_create_error.c_str(); }
int64_t vds_mlp_param_count(vds_mlp m) { return m ? m->np : -1; }

vds_status vds_mlp_set_params(vds_mlp m, const float *p) {
  if (!m || !p) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  vds_status st = mhip(m, hipMemcpyAsync(m->params, p, 4 * m->np, hipMemcpyDeviceToDevice, m->s), "copy");
  if (st == VDS_OK) st = mhip(m, hipMemsetAsync(m->am, 0, 4 * m->np, m->s), "clear");
  if (st == VDS_OK) st = mhip(m, hipMemsetAsync(m->av, 0, 4 * m->np, m->s), "clear");
  m->t = 0;
  m->bf_stale = true;
  return st;
}

vds_status vds_mlp_get_params(vds_mlp m, float *p) {
  if (!m || !p) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  return mhip(m, hipMemcpyAsync(p, m->params, 4 * m->np, hipMemcpyDeviceToDevice, m->s), "copy");
}

vds_status vds_mlp_get_grads(vds_mlp m, float *g) {
  if (!m || !g) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  return mhip(m, hipMemcpyAsync(g, m->grads, 4 * m->np, hipMemcpyDeviceToDevice, m->s), "copy");
}

vds_status vds_mlp_forward(vds_mlp m, const float *X, int32_t n, float *Y, int32_t bf16) {
  if (!m || !X || !Y) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  if (n < 1 || n > m->B) return merr(m, VDS_ERR_ARG, "batch size out of range");
  if (bf16) {
    forward_bf16(m, X, n, Y);
  } else {
    forward_fp32(m, X, n);
    vds_status st = mhip(m, hipMemcpyAsync(Y, m->Y, 4 * (size_t)n * m->nout, hipMemcpyDeviceToDevice, m->s), "copy");
    if (st != VDS_OK) return st;
  }
  return mhip(m, hipGetLastError(), "forward");
}

vds_status vds_mlp_set_input_noise(vds_mlp m, float sigma, uint64_t seed) {
  if (!m) return VDS_ERR_ARG;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return merr(m, VDS_ERR_ARG, "noise must be finite and >= 0");
  if (sigma > 0.f && m->nin != m->nout + 1) return merr(m, VDS_ERR_ARG, "input noise needs nin = nout + 1");
  m->noise = sigma;
  m->noise_seed = seed;
  m->noise_draws = 0;
  return VDS_OK;
}

vds_status vds_mlp_predict_steps(vds_mlp m, float *p, float log_rate, int32_t nsteps) {
  if (!m || !p) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  if (m->nin != m->nout + 1) return merr(m, VDS_ERR_ARG, "learned steps need nin = nout + 1");
  if (nsteps < 0) return merr(m, VDS_ERR_ARG, "nsteps < 0");
  if (nsteps > 0) learned_steps(m, p, nullptr, log_rate, nsteps);
  return mhip(m, hipGetLastError(), "learned steps");
}

vds_status vds_mlp_loss_grad(vds_mlp m, const float *X, const float *T, int32_t n, double *loss) {
  if (!m || !X || !T) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  if (n < 1 || n > m->B) return merr(m, VDS_ERR_ARG, "batch size out of range");
  forward_fp32(m, X, n);
  backward_fp32(m, X, T, n);
  vds_status st = mhip(m, hipGetLastError(), "loss_grad");
  if (st != VDS_OK || loss == nullptr) return st;
  const int nblk = (int)nb256((int64_t)n * m->nout);
  double *dev = m->loss_out;
  k_sum_loss<<<1, 64, 0, m->s>>>(m->lossp, nblk, 1.0 / ((double)n * m->nout), dev);
  st = mhip(m, hipMemcpyAsync(loss, dev, sizeof(double), hipMemcpyDeviceToHost, m->s), "copy loss");
  if (st == VDS_OK) st = mhip(m, hipStreamSynchronize(m->s), "synchronise");
  return st;
}

vds_status vds_mlp_adam_step(vds_mlp m, float lr, float b1, float b2, float eps) {
  if (!m) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  m->t += 1;
  const float c1 = 1.f - std::pow(b1, (float)m->t), c2 = 1.f - std::pow(b2, (float)m->t);
  k_adam<<<nb256(m->np), 256, 0, m->s>>>(m->params, m->grads, m->am, m->av, m->np, lr, b1, b2, eps, c1, c2);
  m->bf_stale = true;
  return mhip(m, hipGetLastError(), "adam");
}

vds_status vds_mlp_train_epoch(vds_mlp m, const float *X, const float *T, int32_t n, int32_t batch, float lr,
                               const int32_t *order, double *loss) {
  if (!m || !X || !T) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  if (batch < 1 || batch > m->B || n < batch) return merr(m, VDS_ERR_ARG, "bad batch size");
  const int nbatch = n / batch;
  double acc = 0.0;
  for (int bi = 0; bi < nbatch; ++bi) {
    k_gather_scaled<<<nb256((int64_t)batch * (m->nin + m->nout)), 256, 0, m->s>>>(
        X, T, order, bi * batch, batch, m->nin, m->nout, m->xs, m->xsc, m->ys, m->ysc, m->xin, m->tin, m->noise,
        m->noise_seed, m->noise_draws);
    m->noise_draws += (uint64_t)batch * m->nin;
    forward_fp32(m, m->xin, batch);
    backward_fp32(m, m->xin, m->tin, batch);
    vds_mlp_adam_step(m, lr, 0.9f, 0.999f, 1e-8f);
    if (loss) {
      const int nblk = (int)nb256((int64_t)batch * m->nout);
      k_sum_loss<<<1, 64, 0, m->s>>>(m->lossp, nblk, 1.0 / ((double)batch * m->nout), m->loss_out);
      double l = 0.0;
      vds_status st = mhip(m, hipMemcpyAsync(&l, m->loss_out, sizeof(double), hipMemcpyDeviceToHost, m->s), "copy");
      if (st == VDS_OK) st = mhip(m, hipStreamSynchronize(m->s), "synchronise");
      if (st != VDS_OK) return st;
      acc += l;
    }
  }
  if (loss) *loss = acc / nbatch;
  return mhip(m, hipStreamSynchronize(m->s), "synchronise");
}

vds_status vds_mlp_fit_scaling(vds_mlp m, const float *X, const float *T, int32_t n) {
  if (!m || !X || !T || n < 1) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  k_col_stats<<<nb256(m->nin), 256, 0, m->s>>>(X, n, m->nin, m->xs, m->xsc);
  k_col_stats<<<nb256(m->nout), 256, 0, m->s>>>(T, n, m->nout, m->ys, m->ysc);
  return mhip(m, hipGetLastError(), "fit scaling");
}

vds_status vds_mlp_make_pairs(vds_mlp m, const float *traj, int32_t nt, float log_rate, float *X, float *T) {
  if (!m || !traj || !X || !T || nt < 2) return VDS_ERR_ARG;
  if (m->nin != m->nout + 1) return merr(m, VDS_ERR_ARG, "pairs need nin = nout + 1");
  k_make_pairs<<<nb256((int64_t)(nt - 1) * (m->nout + 1)), 256, 0, m->s>>>(traj, nt, m->nout, log_rate, X, T);
  return mhip(m, hipGetLastError(), "make pairs");
}

vds_status vds_mlp_set_scaling(vds_mlp m, const float *xs, const float *xsc, const float *ys, const float *ysc) {
  if (!m || !xs || !xsc || !ys || !ysc) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  vds_status st = mhip(m, hipMemcpyAsync(m->xs, xs, 4 * m->nin, hipMemcpyDeviceToDevice, m->s), "copy");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->xsc, xsc, 4 * m->nin, hipMemcpyDeviceToDevice, m->s), "copy");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->ys, ys, 4 * m->nout, hipMemcpyDeviceToDevice, m->s), "copy");
  if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(m->ysc, ysc, 4 * m->nout, hipMemcpyDeviceToDevice, m->s), "copy");
  return st;
}

size_t vds_mlp_rollout_workspace_bytes(const vds_problem *prob, int32_t R) {
  if (!prob || prob->P < 1 || prob->nb < 1 || R < 1) return 0;
  const size_t q = sizeof(float) * 3 * (size_t)prob->P * prob->nb;
  const size_t pr = sizeof(float) * (size_t)prob->nb * R;
  const size_t mapw = vds_pod_map_workspace_bytes(prob, R);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return 2 * up(q) + 4 * up(pr) + up(mapw) + up(sizeof(float) * 16 * (prob->nb * R + 1));
}

vds_status vds_mlp_rollout_run(vds_mlp m, vds_ctx ctx, const float *U, int32_t R, float *p, float log_rate,
                               int32_t nsteps, int32_t K, double resid_tol, double energy_tol, void *ws,
                               size_t bytes, vds_mlp_rollout *stats) {
  if (!m || !ctx || !U || !p || !ws) return VDS_ERR_ARG;
  if (!m->ws) return merr(m, VDS_ERR_STATE, "no workspace bound");
  const vds_problem &pr = ctx->prob;
  const int np_ = pr.nb * R;
  if (m->nin != np_ + 1 || m->nout != np_) return merr(m, VDS_ERR_ARG, "network sizes do not match nb R");
  if (nsteps < 0 || K < 1) return merr(m, VDS_ERR_ARG, "bad step counts");
  if (bytes < vds_mlp_rollout_workspace_bytes(&pr, R)) return merr(m, VDS_ERR_NOMEM, "rollout workspace too small");
  if (ctx->stream != m->s) return merr(m, VDS_ERR_ARG, "context and network must share a stream");
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  char *w = static_cast<char *>(ws);
  const size_t qb = up(sizeof(float) * 3 * (size_t)pr.P * pr.nb), pb = up(sizeof(float) * np_);
  float *qt = reinterpret_cast<float *>(w);
  float *v = reinterpret_cast<float *>(w + qb);
  float *p_acc = reinterpret_cast<float *>(w + 2 * qb);
  float *dp_vds = reinterpret_cast<float *>(w + 2 * qb + pb);
  float *dp_net = reinterpret_cast<float *>(w + 2 * qb + 2 * pb);
  const size_t mapw = vds_pod_map_workspace_bytes(&pr, R);
  void *mws = w + 2 * qb + 4 * pb;

  vds_mlp_rollout S{};
  // energy at the reconstructed state, and the plain scheme's velocity there
  auto observe = [&](const float *pin, vds_diag *d) -> vds_status {
    vds_status st = vds_pod_reconstruct(ctx, U, R, pin, qt, mws, mapw);
    if (st == VDS_OK) st = vds_velocity(ctx, qt, nullptr, v, d);
    return st;
  };
  vds_diag d0{}, d1{};
  vds_status st = observe(p, &d0);
  if (st != VDS_OK) return st;
  const double dt = pr.dt;
  std::vector<float> a((size_t)np_), b((size_t)np_);
  for (int s0 = 0; s0 < nsteps; s0 += K) {
    const int n = std::min(K, nsteps - s0);
    st = mhip(m, hipMemcpyAsync(p_acc, p, 4 * np_, hipMemcpyDeviceToDevice, m->s), "copy");
    if (st != VDS_OK) return st;
    learned_steps(m, p, nullptr, log_rate, n);
    st = observe(p, &d1);
    // a reconstructed FENE bond outside the spring's domain fails the window
    const bool outside = st == VDS_ERR_ARG && pr.potential == VDS_FENE;
    if (outside) st = VDS_OK;
    if (st != VDS_OK) return st;
    double resid = HUGE_VAL, egap = HUGE_VAL;
    if (!outside) {
      // full-step residual at the window's end state
      learned_steps(m, p, dp_net, log_rate, 1);
      st = vds_pod_project(ctx, U, R, v, dp_vds, mws, mapw);
      if (st != VDS_OK) return st;
      st = mhip(m, hipMemcpyAsync(a.data(), dp_net, 4 * np_, hipMemcpyDeviceToHost, m->s), "copy");
      if (st == VDS_OK) st = mhip(m, hipMemcpyAsync(b.data(), dp_vds, 4 * np_, hipMemcpyDeviceToHost, m->s), "copy");
      if (st == VDS_OK) st = mhip(m, hipStreamSynchronize(m->s), "synchronise");
      if (st != VDS_OK) return st;
      double num = 0.0, den = 0.0;
      for (int i = 0; i < np_; ++i) {
        const double ref = dt * (double)b[i];
        num += ((double)a[i] - ref) * ((double)a[i] - ref);
        den += ref * ref;
      }
      resid = std::sqrt(num / std::max(den, 1e-300));
      const double rate0 = d0.work - d0.dissipation, rate1 = d1.work - d1.dissipation;
      const double gap = std::fabs(d1.F - d0.F - 0.5 * dt * n * (rate0 + rate1));
      const double scale =
          0.5 * dt * n * (std::fabs(d0.work) + d0.dissipation + std::fabs(d1.work) + d1.dissipation);
      egap = gap / std::max(scale, 1e-300);
      S.max_resid = std::max(S.max_resid, resid);
      S.max_energy_gap = std::max(S.max_energy_gap, egap);
    }
    S.checks += 1;
    if (outside || !(resid <= resid_tol) || !(egap <= energy_tol)) {
      // redo the window with the plain scheme from its start
      st = vds_pod_reconstruct(ctx, U, R, p_acc, qt, mws, mapw);
      if (st == VDS_OK) st = vds_step(ctx, qt, nullptr, n, nullptr);
      if (st == VDS_OK) st = vds_pod_project(ctx, U, R, qt, p, mws, mapw);
      if (st == VDS_OK) st = observe(p, &d1);
      if (st != VDS_OK) return st;
      S.fallbacks += 1;
    }
    d0 = d1;
    S.steps += n;
  }
  std::memcpy(S.tau, d0.tau, sizeof(S.tau));
  if (stats) *stats = S;
  return VDS_OK;
}

}  // extern "C"
