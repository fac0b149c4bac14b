// Dense linear algebra for the POD offline phase and the reduced operators:
//  * an FP32 MFMA GEMM  C = alpha * sum_b A_b diag(s) B_b^T  (split-K partials,
//    reduced in a fixed order), operands K-contiguous or MN-contiguous;
//  * single-workgroup FP64 kernels for small dense matrices (Cholesky factor
//    and triangular inverse, conversions).
#include "vds_internal.h"
#include "vds_linalg.h"

namespace vds {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // output tile edge per workgroup
constexpr int GK = 32;   // k-depth staged per LDS round
constexpr int GE = GT * GK / 256;  // slab elements per thread and operand

// One workgroup: a 64x64 output tile over the k range of split blockIdx.z.
// Wave w owns the 32x32 quadrant (w / 2, w % 2) as 2x2 blocks of 16x16.
// A_MN: A element (i, k) of batch b at A[b*sA + k*lda + i] (else at i*lda + k).
// B_MN: B element (j, k) at B[b*sB + k*ldb + j] (else at j*ldb + k).
// scale: optional per-k factor (batch stride sS) applied to B.
// The next 64 x 32 slabs of A and B are loaded into registers while the
// matrix cores work on the current ones in LDS; the products are summed in k
// order, 4 at a time.
template <bool A_MN, bool B_MN>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int64_t K, int nbatch, const float *__restrict__ A,
                                              int64_t lda, int64_t sA, const float *__restrict__ B, int64_t ldb,
                                              int64_t sB, const float *__restrict__ scale, int64_t sS,
                                              int64_t k_per_split, int symmetric, float *__restrict__ part) {
  // a symmetric product computes the tiles on and above the diagonal
  if (symmetric && blockIdx.x > blockIdx.y) return;
  __shared__ float sAt[GT][GK + 1];
  __shared__ float sBt[GT][GK + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * GT, j0 = blockIdx.y * GT;
  const int64_t kb = (int64_t)blockIdx.z * k_per_split;
  const int64_t ke = min(K, kb + k_per_split);
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // slab element e of this thread sits at row r0 + dr e, k offset k0 + dk e:
  // rows fastest in the MN layouts, k fastest otherwise, so that a wave's
  // loads are contiguous
  const int ar0 = A_MN ? (tid & 63) : (tid >> 5), ak0 = A_MN ? (tid >> 6) : (tid & 31);
  const int br0 = B_MN ? (tid & 63) : (tid >> 5), bk0 = B_MN ? (tid >> 6) : (tid & 31);
  constexpr int adr = A_MN ? 0 : 8, adk = A_MN ? 4 : 0, bdr = B_MN ? 0 : 8, bdk = B_MN ? 4 : 0;
  // element strides in memory: between a thread's elements, and per slab
  const int64_t a_step = A_MN ? 4 * lda : 8 * lda, a_slab = A_MN ? (int64_t)GK * lda : GK;
  const int64_t b_step = B_MN ? 4 * ldb : 8 * ldb, b_slab = B_MN ? (int64_t)GK * ldb : GK;

  for (int bt = 0; bt < nbatch; ++bt) {
    const float *Sb = scale ? scale + bt * sS : nullptr;
    // element 0 of this thread in the slab at k = kb
    const float *pa = A + bt * sA + (A_MN ? (kb + ak0) * lda + (i0 + ar0) : (int64_t)(i0 + ar0) * lda + kb + ak0);
    const float *pb = B + bt * sB + (B_MN ? (kb + bk0) * ldb + (j0 + br0) : (int64_t)(j0 + br0) * ldb + kb + bk0);
    float ra[GE], rb[GE];
    auto load = [&](int64_t k0) {
      const float *qa = pa, *qb = pb;
#pragma unroll
      for (int e = 0; e < GE; ++e) {
        const bool va = i0 + ar0 + adr * e < M && k0 + ak0 + adk * e < ke;
        ra[e] = va ? *qa : 0.f;
        qa += a_step;
        const int64_t kB = k0 + bk0 + bdk * e;
        const bool vb = j0 + br0 + bdr * e < N && kB < ke;
        rb[e] = vb ? *qb * (Sb ? Sb[kB] : 1.f) : 0.f;
        qb += b_step;
      }
      pa += a_slab;
      pb += b_slab;
    };
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
      for (int e = 0; e < GE; ++e) {
        sAt[ar0 + adr * e][ak0 + adk * e] = ra[e];
        sBt[br0 + bdr * e][bk0 + bdk * e] = rb[e];
      }
      __syncthreads();
      if (k0 + GK < ke) load(k0 + GK);
#pragma unroll
      for (int ks = 0; ks < GK; ks += 4) {
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = sAt[wi + 16 * a + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = sBt[wj + 16 * b + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  // lane holds C[row 4 (lane / 16) + r][col lane % 16] of each 16x16 block
  float *out = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + 16 * a + 4 * (lane >> 4) + r;
        const int j = j0 + wj + 16 * b + (lane & 15);
        if (i < M && j < N) out[(int64_t)i * N + j] = acc[a][b][r];
      }
}

// C = alpha * sum_splits part (+ C if accumulate), fixed summation order.  A
// symmetric product takes the entries of tiles below the diagonal from their
// mirror images.
__global__ __launch_bounds__(256) void k_gemm_reduce(int M, int N, int splits, const float *__restrict__ part, float alpha,
                                                     float *__restrict__ C, int64_t ldc, int c_colmajor, int accumulate,
                                                     int symmetric) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int i = (int)(t / N), j = (int)(t % N);
  const int64_t src = (symmetric && i / GT > j / GT) ? (int64_t)j * N + i : t;
  const double s = ordered_sum<double>(part + src, splits, (int64_t)M * N);
  float *dst = c_colmajor ? &C[(int64_t)j * ldc + i] : &C[(int64_t)i * ldc + j];
  const float v = (float)((double)alpha * s);
  *dst = accumulate ? *dst + v : v;
}

size_t gemm_part_bytes(const GemmShape &g) {
  return sizeof(float) * (size_t)g.splits * g.M * g.N;
}

void launch_gemm(const GemmShape &g, float *part, hipStream_t s) {
  // split ranges start at multiples of 16 (the products are summed in groups
  // of 4 from each split's start)
  const int64_t kps = round_up((g.K + g.splits - 1) / g.splits, 16);
  dim3 grid((unsigned)((g.M + GT - 1) / GT), (unsigned)((g.N + GT - 1) / GT), (unsigned)g.splits);
  if (!g.a_mn && !g.b_mn)
    k_gemm<false, false><<<grid, 256, 0, s>>>(g.M, g.N, g.K, g.nbatch, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.scale, g.sS, kps, g.symmetric ? 1 : 0, part);
  else if (g.a_mn && !g.b_mn)
    k_gemm<true, false><<<grid, 256, 0, s>>>(g.M, g.N, g.K, g.nbatch, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.scale, g.sS, kps, g.symmetric ? 1 : 0, part);
  else if (!g.a_mn && g.b_mn)
    k_gemm<false, true><<<grid, 256, 0, s>>>(g.M, g.N, g.K, g.nbatch, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.scale, g.sS, kps, g.symmetric ? 1 : 0, part);
  else
    k_gemm<true, true><<<grid, 256, 0, s>>>(g.M, g.N, g.K, g.nbatch, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.scale, g.sS, kps, g.symmetric ? 1 : 0, part);
  const int64_t n = (int64_t)g.M * g.N;
  k_gemm_reduce<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g.M, g.N, g.splits, part, g.alpha, g.C, g.ldc,
                                                            g.c_colmajor ? 1 : 0, g.accumulate ? 1 : 0,
                                                            g.symmetric ? 1 : 0);
}

// ---- small dense FP64 kernels (one workgroup) ----

// In place: A (n x n, row-major, FP64, symmetric) -> lower Cholesky factor L
// of A + shift I (upper part zeroed).  info = 0, or k + 1 if the pivot at k
// is not positive.
__global__ __launch_bounds__(256) void k_cholesky(double *A, int n, double shift, int *info) {
  __shared__ double piv;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) A[(int64_t)i * n + i] += shift;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = A[(int64_t)k * n + k];
      if (!(d > 0.0) && bad == 0) bad = k + 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      A[(int64_t)k * n + k] = piv;
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[(int64_t)i * n + k] /= piv;
    __syncthreads();
    // trailing update of the lower triangle, one row per thread stride
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
      const double lik = A[(int64_t)i * n + k];
      for (int j = k + 1; j <= i; ++j) A[(int64_t)i * n + j] -= lik * A[(int64_t)j * n + k];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    if (j > i) A[t] = 0.0;
  }
  if (threadIdx.x == 0) *info = bad;
}

// Linv (n x n, row-major, FP32 out) = L^{-1} for lower-triangular L (FP64),
// one column of the inverse per thread by forward substitution.
__global__ __launch_bounds__(256) void k_tri_inverse(const double *L, int n, double *work, float *Linv) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double *x = work + (int64_t)c * n;  // column c of L^{-1}
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int j = c; j < i; ++j) s -= L[(int64_t)i * n + j] * x[j];
      x[i] = i < c ? 0.0 : s / L[(int64_t)i * n + i];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    Linv[t] = (float)work[(int64_t)j * n + i];  // Linv[i][j] = column j, entry i
  }
}

__global__ void k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

void launch_cholesky(double *A, int n, double shift, int *info, hipStream_t s) {
  k_cholesky<<<1, 256, 0, s>>>(A, n, shift, info);
}
void launch_tri_inverse(const double *L, int n, double *work, float *Linv, hipStream_t s) {
  k_tri_inverse<<<1, 256, 0, s>>>(L, n, work, Linv);
}
void launch_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t s) {
  k_f32_to_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, b, n);
}

}  // namespace vds
