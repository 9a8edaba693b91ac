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
// the wave's own 64 columns of jl must be written before the call.  The wave's
// 64 events are four 16-event chunks (the N side of the MFMA), taken CH at a
// time: each colour fragment loaded serves CH chunks, and output tiles are
// taken in pairs, so that 4 CH independent accumulations keep the matrix
// pipeline busy.
template <class T, int NKS, int NFO, int NTERM, int CH = 2>
__device__ inline T colour_form_mfma(const T* jl, const int* cstep, const KernelArgs& a) {
  static_assert(NKS >= 1 && NKS <= 4 * NFO, "k-steps must fit the output tiles");
  static_assert(CH == 1 || CH == 2 || CH == 4, "chunks per pass divide the four chunks of a wave");
  const uint32_t* terms = ColourLds<T, NTERM>::term();
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, col = lane & 15;
  const int wbase = tid - lane;
  T result = T(0);
#pragma unroll 1
  for (int c0 = 0; c0 < 4; c0 += CH) {
    T xr[CH][4 * NFO], xi[CH][4 * NFO];
#pragma unroll
    for (int s = 0; s < 4 * NFO; ++s) {
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        xr[q][s] = T(0);
        xi[q][s] = T(0);
      }
      if (s < NKS) {
        const int nt = __builtin_amdgcn_readfirstlane(cstep[2 * s]);
        const int off = __builtin_amdgcn_readfirstlane(cstep[2 * s + 1]);
        for (int t = 0; t < nt; ++t) {
          const uint32_t e = terms[4 * (off + t) + g];
          const int o = int(e & 0xffffu);
          const T cf = T(int(int16_t(uint16_t(e >> 16))));
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int ev = wbase + 16 * (c0 + q) + col;
            xr[q][s] += cf * jl[(2 * o) * 256 + ev];
            xi[q][s] += cf * jl[(2 * o + 1) * 256 + ev];
          }
        }
      }
    }
    // The fragments are the same for every chunk and helicity; an opaque base
    // keeps them streaming from L2 instead of being hoisted into registers.
    const int base = opaque_int(0);
    const T* frag = static_cast<const T*>(a.cfrag);
    T part[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) part[q] = T(0);
    // C is symmetric: output tile fo takes the k-steps from its own diagonal
    // block on (s >= 4 fo), the later blocks with the factor 2 built into the
    // fragments, so that sum_fo x_fo . z_fo is the whole quadratic form.
#pragma unroll
    for (int fo = 0; fo < NFO; fo += 2) {
      const bool two = fo + 1 < NFO;
      typename Mfma<T>::acc zr0[CH], zi0[CH], zr1[CH], zi1[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        zr0[q] = typename Mfma<T>::acc{T(0), T(0), T(0), T(0)};
        zi0[q] = zr0[q];
        zr1[q] = zr0[q];
        zi1[q] = zr0[q];
      }
#pragma unroll
      for (int s = 4 * fo; s < NKS; ++s) {
        // uniform fragment address (scalar registers) + the lane's offset
        const T a0 = (frag + (base + (fo * NKS + s) * 64))[lane];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          zr0[q] = Mfma<T>::step(a0, xr[q][s], zr0[q]);
          zi0[q] = Mfma<T>::step(a0, xi[q][s], zi0[q]);
        }
        if (two && s >= 4 * (fo + 1)) {
          const T a1 = (frag + (base + ((fo + 1) * NKS + s) * 64))[lane];
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            zr1[q] = Mfma<T>::step(a1, xr[q][s], zr1[q]);
            zi1[q] = Mfma<T>::step(a1, xi[q][s], zi1[q]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < CH; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) part[q] += zr0[q][r] * xr[q][4 * fo + r] + zi0[q][r] * xi[q][4 * fo + r];
        if (two) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            part[q] += zr1[q][r] * xr[q][4 * fo + 4 + r] + zi1[q][r] * xi[q][4 * fo + 4 + r];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      T pq = part[q];
      pq += __shfl_xor(pq, 16, 64);
      pq += __shfl_xor(pq, 32, 64);
      if (g == c0 + q) result = pq;
    }
  }
  return result;
}

// Number of colour fragments of the upper triangle of 16 x 16 blocks: output
// tile fo reads the k-steps 4 fo .. NKS - 1.
constexpr int tri_fragments(int nks, int nfo) {
  int n = 0;
  for (int fo = 0; fo < nfo; ++fo) n += nks > 4 * fo ? nks - 4 * fo : 0;
  return n;
}
constexpr int tri_offset(int nks, int fo) {
  int n = 0;
  for (int f = 0; f < fo; ++f) n += nks > 4 * f ? nks - 4 * f : 0;
  return n;
}

// The colour fragments of the triangle, one value per lane each, held in
// registers for a whole colour-form phase (every helicity and every chunk of
// the wave's events reuses them); loaded once per phase from the table built at
// process creation ([nfo][nks][64], the lower blocks zero and never read).
template <class T, int NKS, int NFO>
struct ResidentFrags {
  static constexpr int kCount = tri_fragments(NKS, NFO);
  T v[kCount];
  __device__ __forceinline__ void load(const void* cfrag) {
    const T* f = static_cast<const T*>(cfrag);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int fo = 0; fo < NFO; ++fo)
#pragma unroll
      for (int s = 4 * fo; s < NKS; ++s) v[tri_offset(NKS, fo) + s - 4 * fo] = f[(fo * NKS + s) * 64 + lane];
  }
};

// The same quadratic form as colour_form_mfma, with the fragments taken from
// registers: per 16-event chunk the B operands of every k-step are gathered
// once, then the output tiles run in pairs (four independent accumulations)
// over the resident fragments.  Every lane of the wavefront must call it.
template <class T, int NKS, int NFO, int NTERM>
__device__ inline T colour_form_resident(const ResidentFrags<T, NKS, NFO>& fr, const T* jl, const int* cstep) {
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
          const T cf = T(int(int16_t(uint16_t(e >> 16))));
          xr[s] += cf * jl[(2 * o) * 256 + ev];
          xi[s] += cf * jl[(2 * o + 1) * 256 + ev];
        }
      }
    }
    T part = T(0);
#pragma unroll
    for (int fo = 0; fo < NFO; fo += 2) {
      const bool two = fo + 1 < NFO;
      typename Mfma<T>::acc zr0{T(0), T(0), T(0), T(0)}, zi0 = zr0, zr1 = zr0, zi1 = zr0;
#pragma unroll
      for (int s = 4 * fo; s < NKS; ++s) {
        const T a0 = fr.v[tri_offset(NKS, fo) + s - 4 * fo];
        zr0 = Mfma<T>::step(a0, xr[s], zr0);
        zi0 = Mfma<T>::step(a0, xi[s], zi0);
        if (two && s >= 4 * (fo + 1)) {
          const T a1 = fr.v[tri_offset(NKS, fo + 1) + s - 4 * (fo + 1)];
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
