// Host stand-in for <hip/hip_runtime.h> used ONLY by the CPU lane emulator
// (tests/emu): it lets the library's own kernel and host sources compile as
// plain C++ for x86-64, where every GPU lane is a fiber, every 64 fibers a
// wavefront and every block a group of fibers run to completion before the
// next block starts.  Wave-level operations (ballot, shuffle, readfirstlane,
// the 16x16x4 MFMAs) and barriers are rendezvous points of the fibers of one
// wave or block; device memory is host memory from malloc, so that
// AddressSanitizer checks every access the kernels make.  Nothing in the
// product loads this file.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
  unsigned x, y, z;
};

typedef double emu_d4 __attribute__((ext_vector_type(4)));
typedef float emu_f4 __attribute__((ext_vector_type(4)));

namespace emu {
extern emu_uint3 thread_idx_of_current();
extern emu_uint3 block_idx, block_dim, grid_dim;
void wave_barrier();
void block_barrier();
bool any(bool v);
double shfl_xor_f64(double v, int mask);
float shfl_xor_f32(float v, int mask);
int shfl_xor_i32(int v, int mask);
int readfirstlane(int v);
int update_dpp(int old, int src, int ctrl);
int readlane(int v, int lane);
emu_d4 mfma_f64(double a, double b, emu_d4 c);
emu_f4 mfma_f32(float a, float b, emu_f4 c);
void run_grid(dim3 grid, dim3 block, void (*entry)(void*), void* ctx);
template <class F>
void launch(dim3 grid, dim3 block, F f) {
  run_grid(grid, block, [](void* c) { (*static_cast<F*>(c))(); }, &f);
}
inline double shfl_xor(double v, int m) { return shfl_xor_f64(v, m); }
inline float shfl_xor(float v, int m) { return shfl_xor_f32(v, m); }
inline int shfl_xor(int v, int m) { return shfl_xor_i32(v, m); }
}  // namespace emu

#define threadIdx (emu::thread_idx_of_current())
#define blockIdx (emu::block_idx)
#define blockDim (emu::block_dim)
#define gridDim (emu::grid_dim)
#define __syncthreads() emu::block_barrier()
#define __any(x) emu::any(x)
#define __shfl_xor(v, m, w) emu::shfl_xor((v), (m))
#define __builtin_amdgcn_readfirstlane(x) emu::readfirstlane(x)
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) emu::update_dpp((old), (src), (ctrl))
#define __builtin_amdgcn_readlane(v, l) emu::readlane((v), (l))
#define __builtin_amdgcn_wave_barrier() emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu::mfma_f64((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu::mfma_f32((a), (b), (c))

inline unsigned __umulhi(unsigned a, unsigned b) { return unsigned((uint64_t(a) * b) >> 32); }
// gfx950 primitives of the device code: three-input bit function by truth
// table (bit S0 * 4 + S1 * 2 + S2 of the table gives the result bit), FP64
// exponent and mantissa, reciprocal and reciprocal square root (exact here; the
// device's estimates are refined by Newton steps in the code that uses them)
inline uint32_t emu_bitop3_b32(uint32_t a, uint32_t b, uint32_t c, unsigned table) {
  uint32_t r = 0;
  for (int i = 0; i < 32; ++i) {
    const unsigned idx = (((a >> i) & 1u) << 2) | (((b >> i) & 1u) << 1) | ((c >> i) & 1u);
    r |= ((table >> idx) & 1u) << i;
  }
  return r;
}
#define __builtin_amdgcn_bitop3_b32(a, b, c, t) emu_bitop3_b32((a), (b), (c), (t))
inline int emu_frexp_exp(double x) {
  int e = 0;
  std::frexp(x, &e);
  return e;
}
inline double emu_frexp_mant(double x) {
  int e = 0;
  return std::frexp(x, &e);
}
#define __builtin_amdgcn_frexp_exp(x) emu_frexp_exp(x)
#define __builtin_amdgcn_frexp_mant(x) emu_frexp_mant(x)
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
// sin(pi x) and cos(pi x): x reduced exactly to [-1, 1] by whole periods first
inline void sincospi(double x, double* s, double* c) {
  const double r = x - 2.0 * std::nearbyint(0.5 * x);
  *s = std::sin(3.14159265358979323846 * r);
  *c = std::cos(3.14159265358979323846 * r);
}
using std::max;
using std::min;

// ---- runtime API subset used by the library's host code ----
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorNotReady = 600,
  hipErrorLaunchFailure = 719
} hipError_t;
typedef struct emu_stream* hipStream_t;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 63 } hipDeviceAttribute_t;
#define hipHostMallocDefault 0u

hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n);
}
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags = 0) {
  return hipHostMalloc(reinterpret_cast<void**>(p), n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
enum hipMemoryType { hipMemoryTypeUnregistered = 0, hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2 };
struct hipPointerAttribute_t {
  hipMemoryType type;
  int device;
  void* devicePointer;
  void* hostPointer;
  int isManaged;
  unsigned allocationFlags;
};
// every pointer is device memory to the emulator (its device memory is host memory)
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetDevice(int* d);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int block, size_t shmem);
hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t shmem, hipStream_t s);
// a __device__ variable is host memory here: its address is the symbol's
#define HIP_SYMBOL(x) (&(x))
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) emu::launch(dim3(g), dim3(b), [=]() { k(__VA_ARGS__); })
