// Adaptive integration of a resonance-tree process: VEGAS grids over the
// uniforms of its phase space (G. P. Lepage, J. Comput. Phys. 27 (1978) 192),
// the part the BASES integrator plays in the paper's runs (Sec. 1 and 6).
// Each pass evaluates n events through the process's amplitude kernel with the
// current grid (the kernel records every event's bin per dimension and its full
// weight), sums w^2 per bin on the device in a fixed order and refines the grid
// in place on the device; the passes run back to back on the stream, and the
// host reads the pass results and the final grid once at the end.  Declarations: include/heget.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "generated_common.hpp"
#include "reduce.hpp"
#include "heget.h"
#include "heget_internal.hpp"

using heget::KernelArgs;
using heget::detail::fail;

namespace {

constexpr int kMaxBins = 32;          // bins per dimension: a bin index fits a byte, a block's
                                      // per-thread histogram rows fit 64 KiB of LDS
constexpr int kMaxDims = 64;          // uniforms per event (a tree of 16 nodes draws at most 47)
constexpr int kPerThread = 16;        // consecutive events per thread of a histogram block
constexpr int64_t kChunk = 256 * kPerThread;   // events per histogram block
constexpr double kAlpha = 1.5;        // compression exponent of the refinement

// Neumaier's compensated addition: (s, c) += x.
__device__ __forceinline__ void csum(double& s, double& c, double x) {
  const double u = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - u) + x) : ((x - u) + s);
  s = u;
}

// Block c: sums of w^2 per (dimension, bin) over events [c kChunk, min(n,
// (c + 1) kChunk)).  Thread t owns the 16 consecutive events from c kChunk + 16 t
// (their w^2 in registers, their bins one 16-byte load per dimension, the next
// dimension's load issued before this one is summed).  Per dimension, thread t
// adds its events in order into its own LDS row; the rows are then added in a
// fixed order (G = 256 / B groups of consecutive rows, one thread per (group,
// bin), then the groups in order by thread b < B), so the result does not
// depend on scheduling.  bins rows have stride `stride` (a multiple of 16, the
// buffer padded to it); out: [chunks][D][B].
__global__ __launch_bounds__(256) void bin_sums_partial(const uint8_t* bins, int64_t stride, const double* w,
                                                         int64_t n, int D, int B, double* out) {
  // rows of 257: the column sums read a bin's 256 entries with a lane per
  // bin, which a stride of 256 doubles would put on one LDS bank
  constexpr int kRow = 257;
  __shared__ double acc[kMaxBins * kRow];
  __shared__ double grp[2][256];
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t e0 = c * kChunk + int64_t(t) * kPerThread;
  const int valid = int(std::max<int64_t>(0, std::min<int64_t>(kPerThread, n - e0)));
  double w2[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const double x = k < valid ? w[e0 + k] : 0.0;
    w2[k] = x * x;
  }
  const int G = 256 / B, rows = (256 + G - 1) / G;
  uint4 next = valid > 0 ? *reinterpret_cast<const uint4*>(bins + e0) : make_uint4(0, 0, 0, 0);
  for (int d = 0; d < D; ++d) {
    const uint4 cur = next;
    if (d + 1 < D && valid > 0) next = *reinterpret_cast<const uint4*>(bins + (d + 1) * stride + e0);
    for (int j = 0; j < B; ++j) acc[j * kRow + t] = 0.0;
    const uint32_t words[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int j = (words[k >> 2] >> (8 * (k & 3))) & 0xff;
      if (k < valid && j < B) acc[j * kRow + t] += w2[k];
    }
    __syncthreads();
    double* g2 = grp[d & 1];   // alternate buffers: the next dimension's groups may be written
                               // while this one's are still being added
    if (t < G * B) {
      const int b = t % B, g = t / B;
      const int r1 = min(256, (g + 1) * rows);
      double s = 0.0, cc = 0.0;
      for (int r = g * rows; r < r1; ++r) csum(s, cc, acc[b * kRow + r]);
      g2[g * B + b] = s + cc;
    }
    __syncthreads();
    if (t < B) {
      double s = 0.0, cc = 0.0;
      for (int g = 0; g < G; ++g) csum(s, cc, g2[g * B + t]);
      out[(c * D + d) * B + t] = s + cc;
    }
  }
}

// Block d: the per-chunk sums of dimension d added over the chunks in a fixed
// order (G groups of consecutive chunks, then the groups in order), then one
// refinement of the dimension's edges e[0..B] in place: smoothing over
// neighbouring bins, compression of the shares x to ((x - 1) / ln x)^alpha (a
// thread per bin), then, by one thread in order, the new edges that give every
// new bin the same share, an old bin's share growing linearly across it.  A
// dimension whose sums are all zero keeps its edges.
__global__ __launch_bounds__(256) void refine_grid(const double* partial, int64_t chunks, int D, int B,
                                                    double* edges) {
  __shared__ double grp[256];
  __shared__ double h[kMaxBins], r[kMaxBins], e[kMaxBins + 1];
  __shared__ double S_sh;
  const int t = threadIdx.x, d = blockIdx.x;
  const int G = 256 / B;
  const int64_t rows = (chunks + G - 1) / G;
  if (t < G * B) {
    const int b = t % B, g = t / B;
    const int64_t c1 = std::min<int64_t>(chunks, (g + 1) * rows);
    double s = 0.0, cc = 0.0;
    int64_t q = g * rows;
    for (; q + 8 <= c1; q += 8) {   // eight loads in flight, added in chunk order
      double x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = partial[((q + k) * D + d) * B + b];
#pragma unroll
      for (int k = 0; k < 8; ++k) csum(s, cc, x[k]);
    }
    for (; q < c1; ++q) csum(s, cc, partial[(q * D + d) * B + b]);
    grp[g * B + b] = s + cc;
  }
  double* ed = edges + d * (B + 1);
  if (t <= B) e[t] = ed[t];
  __syncthreads();
  if (t < B) {
    double s = 0.0, cc = 0.0;
    for (int g = 0; g < G; ++g) csum(s, cc, grp[g * B + t]);
    h[t] = s + cc;
  }
  __syncthreads();
  if (t < B) {   // smoothing
    double sm;
    if (t == 0) sm = (h[0] + h[1]) / 2.0;
    else if (t == B - 1) sm = (h[B - 2] + h[B - 1]) / 2.0;
    else sm = (h[t - 1] + h[t] + h[t + 1]) / 3.0;
    r[t] = sm;
  }
  __syncthreads();
  if (t == 0) {
    double S = 0.0;
    for (int j = 0; j < B; ++j) S += r[j];
    S_sh = S;
  }
  __syncthreads();
  const double S = S_sh;
  if (!(S > 0.0)) return;   // uniform over the block
  if (t < B) {   // compression
    const double x = r[t] / S;
    double v;
    if (x <= 0.0) v = 0.0;
    else if (x >= 1.0) v = 1.0;
    else v = pow((x - 1.0) / log(x), kAlpha);
    r[t] = v;
  }
  __syncthreads();
  if (t == 0) {   // redistribution
    double R = 0.0;
    for (int j = 0; j < B; ++j) R += r[j];
    R /= B;
    double acc = 0.0;
    int j = 0;
    for (int m = 1; m < B; ++m) {
      const double target = m * R;
      while (j < B - 1 && acc + r[j] < target) {
        acc += r[j];
        ++j;
      }
      ed[m] = r[j] > 0.0 ? e[j] + (target - acc) / r[j] * (e[j + 1] - e[j]) : e[j];
    }
    ed[0] = 0.0;
    ed[B] = 1.0;
  }
}

// Fixed-order reduction of the amplitude kernel's per-block partials (one
// block) into the pass's (sum w, sum w^2, accepted).
__global__ __launch_bounds__(256) void reduce_pass(const double* partials, int64_t nblocks, double* out) {
  heget::reduce_triples(partials, nblocks, out);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int32_t heget_process_grid_dims(heget_process_t p) { return p ? p->entry->ps_dims : -1; }

heget_status heget_integrate_adaptive(heget_process_t p, int64_t n, int32_t iterations, int32_t bins,
                                      double sqrt_s, uint64_t seed, heget_result* per_iteration,
                                      heget_result* combined, double* chi2_per_dof, double* grid_out,
                                      void* stream) {
  fail(HEGET_OK, "");   // clears the thread's last error
  if (!p || !combined) return fail(HEGET_E_INVALID, "null argument");
  if (n < 2) return fail(HEGET_E_INVALID, "need n >= 2 events");
  if (iterations < 1) return fail(HEGET_E_INVALID, "need iterations >= 1");
  if (bins < 2 || bins > kMaxBins) return fail(HEGET_E_INVALID, "bins must be 2 .. 32");
  if (!(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0");
  if (!p->entry->generate || p->entry->ps_dims <= 0)
    return fail(HEGET_E_UNSUPPORTED, "adaptive integration needs a process with a resonance tree");
  if (p->entry->ps_dims > kMaxDims) return fail(HEGET_E_UNSUPPORTED, "more than 64 phase-space uniforms");
  const int D = p->entry->ps_dims, B = bins;
  const int64_t nblocks = (n + 255) / 256;
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  if (nblocks > 0x7fffffff) return fail(HEGET_E_INVALID, "n too large for one launch");
  hipStream_t st = static_cast<hipStream_t>(stream);

  // one allocation: grid, weights, kernel partials, pass results, histogram
  // partials, bins (rows padded to a multiple of 16 events, the weights to the
  // same length, for the histogram's 16-byte loads)
  const int64_t stride = (n + 15) / 16 * 16;
  const size_t o_grid = 0;
  const size_t o_w = align256(o_grid + sizeof(double) * D * (B + 1));
  const size_t o_part = align256(o_w + sizeof(double) * stride);
  const size_t o_res = align256(o_part + sizeof(double) * 3 * nblocks);
  const size_t o_hpart = align256(o_res + sizeof(double) * 3 * iterations);
  const size_t o_bins = align256(o_hpart + sizeof(double) * chunks * D * B);
  const size_t total = o_bins + size_t(D) * stride;
  if (p->adapt_cap < total) {
    hipError_t e = hipStreamSynchronize(st);   // a previous call's kernels may still use the old buffer
    if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));
    if (p->d_adapt) (void)hipFree(p->d_adapt);
    p->d_adapt = nullptr;
    p->adapt_cap = 0;
    if (hipMalloc(&p->d_adapt, total) != hipSuccess) {
      p->d_adapt = nullptr;
      return fail(HEGET_E_OOM, "adaptive integration buffers");
    }
    p->adapt_cap = total;
  }
  char* base = static_cast<char*>(p->d_adapt);
  double* d_grid = reinterpret_cast<double*>(base + o_grid);
  double* d_w = reinterpret_cast<double*>(base + o_w);
  double* d_part = reinterpret_cast<double*>(base + o_part);
  double* d_res = reinterpret_cast<double*>(base + o_res);
  double* d_hpart = reinterpret_cast<double*>(base + o_hpart);
  uint8_t* d_bins = reinterpret_cast<uint8_t*>(base + o_bins);

  // the uniform starting grid, e_j = j / B
  std::vector<double> edges(size_t(D) * (B + 1));
  for (int d = 0; d < D; ++d)
    for (int j = 0; j <= B; ++j) edges[size_t(d) * (B + 1) + j] = double(j) / B;
  hipError_t e = hipMemcpyAsync(d_grid, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));

  // the passes, back to back on the stream: evaluate through the grid, reduce,
  // sum w^2 per bin, refine the grid in place for the next pass (a block per dimension)
  for (int it = 0; it < iterations; ++it) {
    KernelArgs a = heget::detail::base_args(p);
    a.n = n;
    a.mom_stride = n;
    a.seed = seed;
    a.counter_offset = uint64_t(it) * uint64_t(n);
    a.sqrt_s = sqrt_s;
    a.weight_factor = heget::detail::weight_factor(p, sqrt_s);
    a.partials = d_part;
    a.grid = d_grid;
    a.grid_bins = B;
    a.grid_bin_stride = stride;
    a.grid_bin_out = d_bins;
    a.w_out = d_w;
    heget_status rc = heget::detail::launch(p, a, st);
    if (rc != HEGET_OK) {
      (void)hipStreamSynchronize(st);   // the grid's host copy must outlive queued work
      return rc;
    }
    hipLaunchKernelGGL(reduce_pass, dim3(1), dim3(256), 0, st, d_part, nblocks, d_res + 3 * it);
    hipLaunchKernelGGL(bin_sums_partial, dim3(unsigned(chunks)), dim3(256), 0, st, d_bins, stride, d_w, n, D, B,
                       d_hpart);
    hipLaunchKernelGGL(refine_grid, dim3(unsigned(D)), dim3(256), 0, st, d_hpart, chunks, D, B, d_grid);
    e = hipGetLastError();
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));
    }
  }
  std::vector<double> res(size_t(3) * iterations);
  e = hipMemcpyAsync(res.data(), d_res, sizeof(double) * res.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(edges.data(), d_grid, sizeof(double) * edges.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));

  std::vector<double> sig(iterations), err(iterations);
  combined->n_generated = combined->n_accepted = 0;
  combined->sum_w = combined->sum_w2 = 0.0;
  for (int it = 0; it < iterations; ++it) {
    heget_result r;
    heget::detail::fill_result(&res[size_t(3) * it], n, &r);
    if (per_iteration) per_iteration[it] = r;
    sig[it] = r.sigma_gev2;
    err[it] = r.err_gev2;
    combined->n_generated += r.n_generated;
    combined->n_accepted += r.n_accepted;
    combined->sum_w += r.sum_w;
    combined->sum_w2 += r.sum_w2;
  }

  // inverse-variance combination; passes with zero variance carry no weight
  // unless every pass has zero variance (then the plain average, error 0)
  double sw = 0.0, swx = 0.0, plain = 0.0;
  for (int it = 0; it < iterations; ++it) {
    plain += sig[it];
    if (err[it] > 0.0) {
      const double wv = 1.0 / (err[it] * err[it]);
      sw += wv;
      swx += wv * sig[it];
    }
  }
  double mean, cerr, chi2 = 0.0;
  if (sw > 0.0) {
    mean = swx / sw;
    cerr = 1.0 / std::sqrt(sw);
    for (int it = 0; it < iterations; ++it)
      if (err[it] > 0.0) chi2 += (sig[it] - mean) * (sig[it] - mean) / (err[it] * err[it]);
    chi2 /= std::max(iterations - 1, 1);
  } else {
    mean = plain / iterations;
    cerr = 0.0;
  }
  const double hbarc2 = 0.3893793721e9;
  combined->sigma_gev2 = mean;
  combined->err_gev2 = cerr;
  combined->sigma_pb = mean * hbarc2;
  combined->err_pb = cerr * hbarc2;
  if (chi2_per_dof) *chi2_per_dof = chi2;
  if (grid_out) std::copy(edges.begin(), edges.end(), grid_out);
  return HEGET_OK;
}

}  // extern "C"
