// Common code included by every generated amplitude kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "colour_mfma.hpp"
#include "heget_device.hpp"
#include "kernel_args.hpp"
#include "phase_space.hpp"

namespace heget {

// Compiled kernel of one process IR, looked up by fingerprint at create time.
struct GenEntry {
  uint64_t fingerprint;
  const char* name;
  int n_legs;
  const void* kernel_fp64;    // __global__ void(KernelArgs), T = double
  const void* kernel_mixed;   // T = float, FP64 momenta and denominators
  int colour_mfma;            // 1: the colour form runs on MFMA and needs the tables below
  int nks, nfo;               // its k-steps (ceil(n_flows / 4)) and output tiles (ceil(n_flows / 16))
  const void* batch_fp64;     // the kernels of fused launches (the same kernels: a launch whose
                              // KernelArgs::batch is set walks the batch table)
  const void* batch_mixed;
  const int8_t* hel_canon;    // full helicity product the kernel's loop nest sums, or null
  int n_hel_canon;            // its rows (n_legs entries each)
  int persistent;             // 1: persistent grid with a workspace slot per block (ordering templates)
  int cterm_cap;              // capacity of the kernel's LDS term table (words)
  const void* generate;       // the process's own phase-space kernel (resonance tree), or null (RAMBO)
  int ps_dims;                // uniforms per event of the resonance tree (0: RAMBO)
  int colour_mfma_mixed;      // 1: the FP32 (mixed) kernel's colour form runs on MFMA too
  // split division: the orderings' kernels and the colour-form kernels (null when fused)
  const void* chain_fp64;
  const void* chain_mixed;
  const void* colour_fp64;
  const void* colour_mixed;
};

// The launch arguments of one request's segment in a fused launch.
__device__ __forceinline__ KernelArgs segment_args(const KernelArgs& a, const Segment& g) {
  KernelArgs b = a;
  b.n = g.n;
  b.mom_in = nullptr;
  b.mom_stride = g.n;
  b.seed = g.seed;
  b.counter_offset = 0;
  b.sqrt_s = g.sqrt_s;
  b.me2_out = g.me2_out;
  b.mom_out = nullptr;
  b.weight_factor = g.weight_factor;
  b.partials = g.partials;
  return b;
}
void register_kernel(const GenEntry* e);
struct Registrar {
  explicit Registrar(const GenEntry* e) { register_kernel(e); }
};

template <int NL>
__device__ __forceinline__ void store_momenta(const KernelArgs& a, int64_t i, const mom* p) {
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    double* b = a.mom_out + int64_t(k) * 4 * a.mom_stride + i;
    b[0] = p[k].e;
    b[a.mom_stride] = p[k].x;
    b[2 * a.mom_stride] = p[k].y;
    b[3 * a.mom_stride] = p[k].z;
  }
}

// Per-lane LDS stash of an event value made of words of type T (column
// threadIdx.x of a [words][256] array: consecutive lanes hit consecutive
// banks).  stash_get builds its address from an opaque offset, so a read placed
// inside a loop stays in that loop: the value is not kept in registers across
// the outer loops.  Each lane reads back only what it wrote itself.
template <class T, class V>
__device__ __forceinline__ void stash_put(T (*s)[256], int off, const V& v) {
  static_assert(sizeof(V) % sizeof(T) == 0, "a stashed value is a whole number of words");
  T w[sizeof(V) / sizeof(T)];
  __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
  for (int j = 0; j < int(sizeof(V) / sizeof(T)); ++j) s[off + j][threadIdx.x] = w[j];
}
template <class V, class T>
__device__ __forceinline__ V stash_get(T (*s)[256], int off) {
  const int b = opaque_int(off);
  T w[sizeof(V) / sizeof(T)];
#pragma unroll
  for (int j = 0; j < int(sizeof(V) / sizeof(T)); ++j) w[j] = s[b + j][threadIdx.x];
  V v;
  __builtin_memcpy(&v, w, sizeof(V));
  return v;
}

// A 64-bit value moved by a DPP row shift of N lanes: lane l of each row of 16
// reads lane l - N of its row, or 0 where that lane is outside the row.
template <int N>
__device__ __forceinline__ double row_shr(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), 0x110 + N, 0xF, 0xF, true));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), 0x110 + N, 0xF, 0xF, true));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
// The value of one lane, read by every lane
__device__ __forceinline__ double lane_value(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), lane));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b >> 32)), lane));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
// Sum over the 64 lanes of a wavefront in a fixed order, in registers: an
// inclusive scan inside each row of 16 lanes by DPP row shifts of 1, 2, 4 and 8
// lanes, then the rows' last lanes added in row order.  Every lane of the wave
// must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += row_shr<1>(v);
  v += row_shr<2>(v);
  v += row_shr<4>(v);
  v += row_shr<8>(v);
  return ((lane_value(v, 15) + lane_value(v, 31)) + lane_value(v, 47)) + lane_value(v, 63);
}

// Deterministic per-block partial sums (w, w^2, accepted) for the cross
// section: a fixed-order sum inside each 64-lane wavefront, then the waves in
// order.  Every thread of the block must call it; blk is the block's index
// within its request.
__device__ __forceinline__ void block_partials(const KernelArgs& a, int64_t blk, double wgt, bool acc) {
  const double s = wave_sum(wgt), s2 = wave_sum(wgt * wgt), c = wave_sum(acc ? 1.0 : 0.0);
  __shared__ double red[3][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = s;
    red[1][wave] = s2;
    red[2][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double t = 0.0, t2 = 0.0, tc = 0.0;
    for (int k = 0; k < nw; ++k) {
      t += red[0][k];
      t2 += red[1][k];
      tc += red[2][k];
    }
    a.partials[3 * blk + 0] = t;
    a.partials[3 * blk + 1] = t2;
    a.partials[3 * blk + 2] = tc;
  }
}

}  // namespace heget
