// Colour quadratic form Re(J^dagger C J) on the matrix cores (Sec. 5.4: the
// colour sum of every event is the same dense symmetric form, so a batch of
// events is one dense product).
//
// For one wavefront and one helicity, the 64 events are four column tiles of
// 16 events.  With X the real (or imaginary) parts of the jamps, events x
// flows, the kernel forms Z = C X^T with 16x16x4 MFMAs (rows = flows, columns
// = events) and then sum_f X[e][f] Z[f][e] per event.  The K index of the
// product is arranged so that the B operand a lane supplies at k-step
// 4 fo + r is exactly the X element that multiplies the D element it holds in
// register r of output tile fo: the final dot product is lane-local and only
// the four lane groups are summed with two butterflies.
//
// Lane layouts on gfx950 (checked with an in-bounds probe): for both
// v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32, A[i][k] is in lane i + 16 k
// and B[k][j] in lane j + 16 k.  D[i][j] is in lane j + 16 (i % 4), register
// i / 4 for f64, and in lane j + 16 (i / 4), register i % 4 for f32.
//
// Flow indices are those of the sorted order built by the library (flows
// sorted by their number of flow-map terms, so that the four flows of one
// k-step share one term count): k-step s, lane group g holds sorted flow
// 4 s + g.  Lane group g, register r of output tile fo must then hold the
// flow 16 fo + 4 r + g, so row i of tile fo is sorted flow 16 fo + i (f64)
// or 16 fo + 4 (i % 4) + i / 4 (f32).  The A fragments (colour matrix,
// permuted that way and zero-padded) and the term table are built on the
// host at process creation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "heget_device.hpp"
#include "kernel_args.hpp"

namespace heget {

typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc = mfma_d4;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using acc = mfma_f4;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// LDS home of the term table: one static allocation per kernel, filled once
// per block by colour_stage.  (The colour fragments stream from L2.)
template <class T, int NTERM>
struct ColourLds {
  static __device__ __forceinline__ uint32_t* term() {
    __shared__ uint32_t buf[NTERM];
    return buf;
  }
};

// Copy the term table to LDS; every thread of the block calls it, before its
// first colour form.
template <class T, int NKS, int NFO, int NTERM>
__device__ inline void colour_stage(const KernelArgs& a) {
  uint32_t* tl = ColourLds<T, NTERM>::term();
  for (int i = threadIdx.x; i < a.cterm_words; i += blockDim.x) tl[i] = a.cterm[i];
  __syncthreads();
}

// Returns Re(J^dagger C J) for the calling lane's event, where J_f = sum_o
// coef * A_o over the flow-map terms and A_o = (jl[2o][lane], jl[2o + 1][lane])
// (real and imaginary rows of 256 events) are the ordering amplitudes the
// block staged in LDS.
// Every lane of the wavefront must call it (the MFMAs need the full wave) and
// the wave's own 64 columns of jl must be written before the call.  Output
// tiles are taken in pairs, so that four independent accumulations keep the
// matrix pipeline busy.
template <class T, int NKS, int NFO, int NTERM>
__device__ inline T colour_form_mfma(const T* jl, const int* cstep, const KernelArgs& a) {
  static_assert(NKS >= 1 && NKS <= 4 * NFO, "k-steps must fit the output tiles");
  const uint32_t* terms = ColourLds<T, NTERM>::term();
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, col = lane & 15;
  const int wbase = tid - lane;
  T result = T(0);
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int ev = wbase + 16 * c + col;
    T xr[4 * NFO], xi[4 * NFO];
#pragma unroll
    for (int s = 0; s < 4 * NFO; ++s) {
      xr[s] = T(0);
      xi[s] = T(0);
      if (s < NKS) {
        const int nt = __builtin_amdgcn_readfirstlane(cstep[2 * s]);
        const int off = __builtin_amdgcn_readfirstlane(cstep[2 * s + 1]);
        for (int t = 0; t < nt; ++t) {
          const uint32_t e = terms[4 * (off + t) + g];
          const int o = int(e & 0xffffu);
          const T vr = jl[(2 * o) * 256 + ev], vi = jl[(2 * o + 1) * 256 + ev];
          const T cf = T(int(int16_t(uint16_t(e >> 16))));
          xr[s] += cf * vr;
          xi[s] += cf * vi;
        }
      }
    }
    // The fragments are the same for every chunk and helicity; an opaque base
    // keeps them streaming from L2 instead of being hoisted into registers.
    const int base = opaque_int(0);
    const T* frag = static_cast<const T*>(a.cfrag);
    T part = T(0);
#pragma unroll
    for (int fo = 0; fo < NFO; fo += 2) {
      const bool two = fo + 1 < NFO;
      typename Mfma<T>::acc zr0 = {T(0), T(0), T(0), T(0)}, zi0 = zr0, zr1 = zr0, zi1 = zr0;
#pragma unroll
      for (int s = 0; s < NKS; ++s) {
        const T a0 = frag[base + (fo * NKS + s) * 64 + lane];
        zr0 = Mfma<T>::step(a0, xr[s], zr0);
        zi0 = Mfma<T>::step(a0, xi[s], zi0);
        if (two) {
          const T a1 = frag[base + ((fo + 1) * NKS + s) * 64 + lane];
          zr1 = Mfma<T>::step(a1, xr[s], zr1);
          zi1 = Mfma<T>::step(a1, xi[s], zi1);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) part += zr0[r] * xr[4 * fo + r] + zi0[r] * xi[4 * fo + r];
      if (two) {
#pragma unroll
        for (int r = 0; r < 4; ++r) part += zr1[r] * xr[4 * fo + 4 + r] + zi1[r] * xi[4 * fo + 4 + r];
      }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == c) result = part;
  }
  return result;
}

}  // namespace heget
