// Fixed-order reduction of the integrate step's per-block partial sums (host
// library kernels only: the generated amplitude kernels write the partials,
// block_partials in generated_common.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heget {

// Adds the triples of blocks b, b + 256, ..., b + (Q - 1) 256 to the
// compensated sums s, c in block order, their Q loads issued together.
template <int Q>
__device__ __forceinline__ void add_blocks(const double* partials, int64_t b, double s[3], double c[3]) {
  double x[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int k = 0; k < 3; ++k) x[q][k] = partials[3 * (b + q * 256) + k];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double u = s[k] + x[q][k];
      c[k] += (fabs(s[k]) >= fabs(x[q][k])) ? ((s[k] - u) + x[q][k]) : ((x[q][k] - u) + s[k]);
      s[k] = u;
    }
}

// Fixed-order reduction of per-block partial triples with Neumaier
// compensation, by one block of 256 threads: thread t sums blocks t, t + 256,
// ... in order, then a pairwise tree (t with t + 128, then t + 64, ...) combines
// the 256 compensated sums.  Used by the single-request reduction and by the
// serving engine's batched one, so both give the same bits.
__device__ inline void reduce_triples(const double* partials, int64_t nblocks, double* out) {
  __shared__ double sm[3][256];
  __shared__ double cm[3][256];
  const int t = threadIdx.x;
  double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
  int64_t b = t;
  // loads in flight sixteen blocks at a time (a launch of 2^20 events has 16
  // blocks per lane), then four, then one; the additions stay in block order
  for (; b + 15 * 256 < nblocks; b += 16 * 256) add_blocks<16>(partials, b, s, c);
  for (; b + 3 * 256 < nblocks; b += 4 * 256) add_blocks<4>(partials, b, s, c);
  for (; b < nblocks; b += 256) add_blocks<1>(partials, b, s, c);
  for (int k = 0; k < 3; ++k) {
    sm[k][t] = s[k];
    cm[k][t] = c[k];
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double a = sm[k][t], x = sm[k][t + h];
        const double u = a + x;
        cm[k][t] += ((fabs(a) >= fabs(x)) ? ((a - u) + x) : ((x - u) + a)) + cm[k][t + h];
        sm[k][t] = u;
      }
    }
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < 3; ++k) out[k] = sm[k][0] + cm[k][0];
  __syncthreads();
}

}  // namespace heget
