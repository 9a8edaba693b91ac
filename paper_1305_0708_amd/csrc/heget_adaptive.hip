// Adaptive integration of a resonance-tree process: VEGAS grids over the
// uniforms of its phase space (G. P. Lepage, J. Comput. Phys. 27 (1978) 192),
// the part the BASES integrator plays in the paper's runs (Sec. 1 and 6).
// Each pass evaluates n events through the process's amplitude kernel with the
// current grid (the kernel records every event's bin per dimension and its full
// weight), histograms w^2 per bin on the device in a fixed order, and refines
// the grid on the host (D x B numbers).  Declarations: include/heget.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "generated_common.hpp"
#include "heget.h"
#include "heget_internal.hpp"

using heget::KernelArgs;
using heget::detail::fail;

namespace {

constexpr int kMaxBins = 32;          // bins per dimension: a bin index fits a byte, a block's
                                      // per-thread histogram rows fit 64 KiB of LDS
constexpr int64_t kChunk = 4096;      // events per histogram block
constexpr double kAlpha = 1.5;        // compression exponent of the refinement

// Neumaier's compensated addition: (s, c) += x.
__device__ __forceinline__ void csum(double& s, double& c, double x) {
  const double u = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - u) + x) : ((x - u) + s);
  s = u;
}

// Block (chunk c, dimension d): sums of w^2 per bin over events [c kChunk,
// min(n, (c + 1) kChunk)).  Thread t takes events t, t + 256, ... into its own
// LDS row; thread b < B then sums column b over the rows in order, so the
// result does not depend on scheduling.  out: [chunks][D][B].
__global__ __launch_bounds__(256) void bin_sums_partial(const uint8_t* bins, const double* w, int64_t n, int D,
                                                         int B, double* out) {
  __shared__ double acc[kMaxBins * 256];
  const int t = threadIdx.x;
  const int d = blockIdx.y;
  const int64_t c = blockIdx.x;
  for (int j = 0; j < B; ++j) acc[j * 256 + t] = 0.0;
  const int64_t end = std::min<int64_t>(n, (c + 1) * kChunk);
  const uint8_t* bd = bins + int64_t(d) * n;
  for (int64_t e = c * kChunk + t; e < end; e += 256) {
    const int j = bd[e];
    const double x = w[e];
    if (j < B) acc[j * 256 + t] += x * x;
  }
  __syncthreads();
  if (t < B) {
    double s = 0.0, cc = 0.0;
    for (int r = 0; r < 256; ++r) csum(s, cc, acc[t * 256 + r]);
    out[(c * D + d) * B + t] = s + cc;
  }
}

// Block d: the per-chunk sums of dimension d added over the chunks in order.
__global__ __launch_bounds__(64) void bin_sums_reduce(const double* partial, int64_t chunks, int D, int B,
                                                       double* out) {
  const int t = threadIdx.x, d = blockIdx.x;
  if (t >= B) return;
  double s = 0.0, cc = 0.0;
  for (int64_t c = 0; c < chunks; ++c) csum(s, cc, partial[(c * D + d) * B + t]);
  out[d * B + t] = s + cc;
}

// Fixed-order reduction of the amplitude kernel's per-block partials (one block).
__global__ __launch_bounds__(256) void reduce_pass(const double* partials, int64_t nblocks, double* out) {
  heget::reduce_triples(partials, nblocks, out);
}

// One refinement of every dimension's edges e[d][0..B] from its bin sums
// h[d][0..B-1]: smoothing over neighbouring bins, compression of the shares x
// to ((x - 1) / ln x)^alpha, then new edges that give every new bin the same
// share, an old bin's share growing linearly across it.  A dimension whose
// sums are all zero keeps its edges.
void refine(std::vector<double>& e, const std::vector<double>& h, int D, int B) {
  std::vector<double> sm(B), r(B), nw(B + 1);
  for (int d = 0; d < D; ++d) {
    const double* hd = &h[size_t(d) * B];
    double* ed = &e[size_t(d) * (B + 1)];
    sm[0] = (hd[0] + hd[1]) / 2.0;
    sm[B - 1] = (hd[B - 2] + hd[B - 1]) / 2.0;
    for (int j = 1; j < B - 1; ++j) sm[j] = (hd[j - 1] + hd[j] + hd[j + 1]) / 3.0;
    double S = 0.0;
    for (int j = 0; j < B; ++j) S += sm[j];
    if (!(S > 0.0)) continue;
    for (int j = 0; j < B; ++j) {
      const double x = sm[j] / S;
      if (x <= 0.0) r[j] = 0.0;
      else if (x >= 1.0) r[j] = 1.0;
      else r[j] = std::pow((x - 1.0) / std::log(x), kAlpha);
    }
    double R = 0.0;
    for (int j = 0; j < B; ++j) R += r[j];
    R /= B;
    nw[0] = 0.0;
    double acc = 0.0;
    int j = 0;
    for (int m = 1; m < B; ++m) {
      const double target = m * R;
      while (j < B - 1 && acc + r[j] < target) {
        acc += r[j];
        ++j;
      }
      nw[m] = r[j] > 0.0 ? ed[j] + (target - acc) / r[j] * (ed[j + 1] - ed[j]) : ed[j];
    }
    nw[B] = 1.0;
    std::copy(nw.begin(), nw.end(), ed);
  }
}

// Frees the pass buffers on every exit path (after the stream has drained).
struct DeviceBuffer {
  void* ptr = nullptr;
  hipStream_t stream = nullptr;
  ~DeviceBuffer() {
    if (ptr) {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(ptr);
    }
  }
};

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
  const int D = p->entry->ps_dims, B = bins;
  const int64_t nblocks = (n + 255) / 256;
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  if (nblocks > 0x7fffffff) return fail(HEGET_E_INVALID, "n too large for one launch");
  hipStream_t st = static_cast<hipStream_t>(stream);

  // one allocation: grid, weights, kernel partials, histogram partials and sums, bins
  const size_t o_grid = 0;
  const size_t o_w = align256(o_grid + sizeof(double) * D * (B + 1));
  const size_t o_part = align256(o_w + sizeof(double) * n);
  const size_t o_hpart = align256(o_part + sizeof(double) * (3 * nblocks + 3));
  const size_t o_hist = align256(o_hpart + sizeof(double) * chunks * D * B);
  const size_t o_bins = align256(o_hist + sizeof(double) * D * B);
  const size_t total = o_bins + size_t(D) * n;
  DeviceBuffer buf;
  buf.stream = st;
  if (hipMalloc(&buf.ptr, total) != hipSuccess) {
    buf.ptr = nullptr;
    return fail(HEGET_E_OOM, "adaptive integration buffers");
  }
  char* base = static_cast<char*>(buf.ptr);
  double* d_grid = reinterpret_cast<double*>(base + o_grid);
  double* d_w = reinterpret_cast<double*>(base + o_w);
  double* d_part = reinterpret_cast<double*>(base + o_part);
  double* d_hpart = reinterpret_cast<double*>(base + o_hpart);
  double* d_hist = reinterpret_cast<double*>(base + o_hist);
  uint8_t* d_bins = reinterpret_cast<uint8_t*>(base + o_bins);

  std::vector<double> edges(size_t(D) * (B + 1)), hist(size_t(D) * B);
  for (int d = 0; d < D; ++d)
    for (int j = 0; j <= B; ++j) edges[size_t(d) * (B + 1) + j] = double(j) / B;
  std::vector<double> sig(iterations), err(iterations);
  combined->n_generated = combined->n_accepted = 0;
  combined->sum_w = combined->sum_w2 = 0.0;

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
    a.grid_bin_out = d_bins;
    a.w_out = d_w;
    double h[3] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(d_grid, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));
    heget_status rc = heget::detail::launch(p, a, st);
    if (rc != HEGET_OK) return rc;
    hipLaunchKernelGGL(reduce_pass, dim3(1), dim3(256), 0, st, d_part, nblocks, d_part + 3 * nblocks);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(bin_sums_partial, dim3(unsigned(chunks), unsigned(D)), dim3(256), 0, st, d_bins, d_w, n, D,
                         B, d_hpart);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(bin_sums_reduce, dim3(unsigned(D)), dim3(64), 0, st, d_hpart, chunks, D, B, d_hist);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, d_part + 3 * nblocks, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hist.data(), d_hist, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("adaptive: ") + hipGetErrorString(e));
    heget_result r;
    heget::detail::fill_result(h, n, &r);
    if (per_iteration) per_iteration[it] = r;
    sig[it] = r.sigma_gev2;
    err[it] = r.err_gev2;
    combined->n_generated += r.n_generated;
    combined->n_accepted += r.n_accepted;
    combined->sum_w += r.sum_w;
    combined->sum_w2 += r.sum_w2;
    refine(edges, hist, D, B);
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
