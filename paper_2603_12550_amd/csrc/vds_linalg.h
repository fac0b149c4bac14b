// Dense linear-algebra helpers shared by the POD and reduced-model code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vds {

// C = alpha * sum_{b < nbatch} A_b diag(scale_b) B_b^T (+ C when accumulate), where
// A_b is M x K and B_b is N x K.  Element (i, k) of A_b is A[b*sA + k*lda + i]
// when a_mn, else A[b*sA + i*lda + k]; likewise B with b_mn.  The output is
// row-major (C[i*ldc + j]) or column-major (C[j*ldc + i]).  K is split over
// `splits` workgroup layers whose partial tiles are summed in a fixed order.
struct GemmShape {
  int M = 0, N = 0;
  int64_t K = 0;
  int nbatch = 1;
  const float *A = nullptr;
  int64_t lda = 0, sA = 0;
  bool a_mn = false;
  const float *B = nullptr;
  int64_t ldb = 0, sB = 0;
  bool b_mn = false;
  const float *scale = nullptr;
  int64_t sS = 0;
  float alpha = 1.f;
  float *C = nullptr;
  int64_t ldc = 0;
  bool c_colmajor = false;
  bool accumulate = false;
  int splits = 1;
  // C = A A^T (A and B the same matrix, M = N): only tiles on and above the
  // diagonal are computed, the others are mirrored in the reduction
  bool symmetric = false;
};

size_t gemm_part_bytes(const GemmShape &g);
void launch_gemm(const GemmShape &g, float *part, hipStream_t s);
void launch_cholesky(double *A, int n, double shift, int *info, hipStream_t s);
void launch_tri_inverse(const double *L, int n, double *work, float *Linv, hipStream_t s);
void launch_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t s);

// Split count giving roughly `target` workgroups for an M x N output.
inline int gemm_splits(int M, int N, int64_t K, int target = 1024, bool symmetric = false) {
  const int64_t tm = (M + 63) / 64, tn = (N + 63) / 64;
  // a symmetric product runs only the tiles on and above the diagonal
  const int64_t tiles = symmetric ? tm * (tm + 1) / 2 : tm * tn;
  int64_t s = (target + tiles - 1) / tiles;
  const int64_t kmax = (K + 255) / 256;  // keep >= 256 k per split
  if (s > kmax) s = kmax;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

}  // namespace vds
