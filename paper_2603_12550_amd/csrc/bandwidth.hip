// Median-heuristic bandwidth (eq. model_bandwidth): h = med / sqrt(2 log P),
// med the median of |x_J - x_K| over all P^2 ordered pairs, J = K included.
//
// The P^2 values are P zeros (J = K) and every unordered pair twice, so rank r
// of the full sorted list is zero for r < P and otherwise rank (r - P) / 2 of
// the sorted unordered distances.  That rank is found exactly by a radix
// select on the bit patterns of the FP32 squared distances (non-negative
// floats order like their bits): three passes over all unordered pairs, each
// histogramming the next 12, 10 and 10 bits of the keys that share the prefix
// found so far.  Distances are recomputed every pass (direct differences, as
// cheap as reading them back), counted in per-block LDS histograms, merged
// into 64-bit global counts with integer atomics (exact, order-independent).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "vds_ctx.h"
#include "vds_internal.h"

using namespace vds;

namespace {

constexpr int kTile = 256;
constexpr int kBins = kHistBins;  // first pass: 12 bits; later passes use 1024

// Histograms of targets t = 0, 1 (ntargets of them) over the unordered pairs of
// tile (blockIdx.x, blockIdx.y), row tile <= column tile.  A key counts for
// target t when its top `prefix_bits` bits equal prefix[t]; its bin is
// (key >> shift) & (nbins - 1).
__global__ __launch_bounds__(kTile) void k_dist_hist(const float *__restrict__ xc, int64_t P, int D,
                                                    int prefix_bits, uint32_t prefix0, uint32_t prefix1,
                                                    int ntargets, int shift, int nbins,
                                                    unsigned long long *__restrict__ hist) {
  if (blockIdx.x > blockIdx.y) return;
  __shared__ float xs[kTile][kMaxD];
  __shared__ uint32_t h[2][kBins];
  for (int b = threadIdx.x; b < 2 * kBins; b += kTile) (&h[0][0])[b] = 0u;
  const int64_t K0 = (int64_t)blockIdx.y * kTile;
  const int64_t Kc = K0 + threadIdx.x;
  for (int a = 0; a < kMaxD; ++a) xs[threadIdx.x][a] = (Kc < P && a < D) ? xc[Kc * D + a] : 0.f;
  __syncthreads();
  const int64_t J = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if (J < P) {
    float xj[kMaxD];
#pragma unroll
    for (int a = 0; a < kMaxD; ++a) xj[a] = a < D ? xc[J * D + a] : 0.f;
    const int64_t kend = min((int64_t)kTile, P - K0);
    // only K > J: in the diagonal tile start after J
    const int64_t kbeg = blockIdx.x == blockIdx.y ? (J - K0) + 1 : 0;
    for (int64_t k = kbeg; k < kend; ++k) {
      float d2 = 0.f;
#pragma unroll
      for (int a = 0; a < kMaxD; ++a) {
        const float df = xj[a] - xs[k][a];
        d2 = fmaf(df, df, d2);
      }
      const uint32_t key = __float_as_uint(d2);
      const uint32_t top = prefix_bits == 0 ? 0u : key >> (32 - prefix_bits);
      const uint32_t bin = (key >> shift) & (uint32_t)(nbins - 1);
      if (top == prefix0) atomicAdd(&h[0][bin], 1u);
      if (ntargets > 1 && top == prefix1) atomicAdd(&h[1][bin], 1u);
    }
  }
  __syncthreads();
  for (int t = 0; t < ntargets; ++t)
    for (int b = threadIdx.x; b < nbins; b += kTile)
      if (h[t][b] != 0u) atomicAdd(&hist[t * kBins + b], (unsigned long long)h[t][b]);
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

extern "C" {

vds_status vds_median_bandwidth(vds_ctx c, const float *q, double *med_out, double *h_out) {
  vds_status st = ready(c);
  if (st != VDS_OK) return st;
  if (!q) return set_err(c, VDS_ERR_ARG, "null state");
  const int64_t P = c->prob.P;
  if (P < 2) return set_err(c, VDS_ERR_ARG, "the median rule needs P >= 2");
  const EvalParams &e = c->ep;
  // centred particle-major coordinates (differences are unchanged by centring)
  launch_mean_partials(e, q, nullptr, c->meanp, nullptr, nullptr, c->stream);
  launch_prep(e, q, nullptr, c->meanp, c->nblk, c->xc, c->wv, c->QB, c->KA, c->VA, c->wscale, &c->f16, nullptr,
              c->stream);

  // ranks of the median in the full list of P^2 values
  const unsigned long long n2 = (unsigned long long)P * (unsigned long long)P;
  const unsigned long long r[2] = {n2 % 2 ? (n2 - 1) / 2 : n2 / 2 - 1, n2 % 2 ? (n2 - 1) / 2 : n2 / 2};
  double d[2] = {0.0, 0.0};
  bool need[2];
  unsigned long long rem[2];
  for (int t = 0; t < 2; ++t) {
    need[t] = r[t] >= (unsigned long long)P;
    rem[t] = need[t] ? (r[t] - (unsigned long long)P) / 2 : 0;
  }
  uint32_t prefix[2] = {0u, 0u};
  if ((P + kTile - 1) / kTile > 65535) return set_err(c, VDS_ERR_ARG, "P too large for the median rule");
  const int tiles = (int)((P + kTile - 1) / kTile);
  const dim3 grid((unsigned)tiles, (unsigned)tiles);
  const int shifts[3] = {20, 10, 0}, bits[3] = {12, 10, 10}, pbits[3] = {0, 12, 22};
  std::vector<unsigned long long> hh(2 * kBins);
  if (need[0] || need[1]) {
    for (int pass = 0; pass < 3; ++pass) {
      const int nbins = 1 << bits[pass];
      // the two targets share their prefix unless an earlier pass split them
      const int two = (need[0] && need[1] && prefix[0] != prefix[1]) ? 2 : 1;
      const int t0 = need[0] ? 0 : 1;
      k_zero_u64<<<(2 * kBins + 255) / 256, 256, 0, c->stream>>>(c->hist, 2 * kBins);
      k_dist_hist<<<grid, kTile, 0, c->stream>>>(c->xc, P, e.D, pbits[pass], prefix[t0], prefix[1], two,
                                                  shifts[pass], nbins, c->hist);
      st = hip_check(c, hipMemcpyAsync(hh.data(), c->hist, sizeof(unsigned long long) * 2 * kBins,
                                       hipMemcpyDeviceToHost, c->stream), "copy histogram");
      if (st == VDS_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "synchronise");
      if (st != VDS_OK) return st;
      for (int t = 0; t < 2; ++t) {
        if (!need[t]) continue;
        // histogram slot of target t: slot 0 unless both were counted separately
        const unsigned long long *ht = hh.data() + ((two == 2 && t == 1) ? kBins : 0);
        unsigned long long cum = 0;
        int b = 0;
        for (; b < nbins; ++b) {
          if (rem[t] < cum + ht[b]) break;
          cum += ht[b];
        }
        if (b == nbins) return set_err(c, VDS_ERR_HIP, "median selection lost its rank (non-finite input?)");
        rem[t] -= cum;
        prefix[t] = (prefix[t] << bits[pass]) | (uint32_t)b;
      }
    }
  }
  for (int t = 0; t < 2; ++t) {
    if (!need[t]) continue;
    float d2;
    const uint32_t key = prefix[t];
    std::memcpy(&d2, &key, sizeof(d2));
    d[t] = std::sqrt((double)d2);
  }
  const double med = 0.5 * (d[0] + d[1]);
  if (med_out) *med_out = med;
  if (h_out) *h_out = med / std::sqrt(2.0 * std::log((double)P));
  return VDS_OK;
}

}  // extern "C"
