// CPU lane emulator (tests only): runs the library's kernels with one fiber
// per GPU lane, so that AddressSanitizer checks every memory access the
// kernels make and a test can compare their results with the oracle's on the
// CPU.  A launch runs its blocks one after another; the fibers of a block run
// until each reaches a rendezvous (a wave operation, a wave or block barrier)
// and the last fiber to arrive completes it for all.  Lanes run in the order
// EMU_LANE_ORDER sets (0: ascending, 1: descending), so that a kernel whose
// lanes read what other lanes wrote without a barrier in between gives
// different results in the two orders.
//
// Wave operations follow the hardware's lane layouts: __shfl_xor and
// readfirstlane as on any 64-wide wavefront; v_mfma_f64_16x16x4f64 with
// A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k and D[i][j] in lane
// j + 16 (i % 4), register i / 4; v_mfma_f32_16x16x4f32 the same for A and B
// with D[i][j] in lane j + 16 (i / 4), register i % 4 (gfx950).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "kernel_args.hpp"

extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old);
}

// x86-64 System V context switch: saves the callee-saved registers on the
// current stack, stores the stack pointer in *save and resumes the context
// whose stack pointer is next.
extern "C" void emu_ctx_swap(void** save, void* next);
asm(R"(
.text
.globl emu_ctx_swap
.type emu_ctx_swap,@function
emu_ctx_swap:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size emu_ctx_swap, .-emu_ctx_swap
)");

namespace emu {

emu_uint3 block_idx{0, 0, 0}, block_dim{1, 1, 1}, grid_dim{1, 1, 1};

namespace {

constexpr size_t kStack = size_t(8) << 20;   // per fiber (mapped lazily)
constexpr int kWave = 64;

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  unsigned tid = 0;
  bool done = false;
  // waiting for the generation counter *wait_on to move past wait_gen
  const uint64_t* wait_on = nullptr;
  uint64_t wait_gen = 0;
};

enum Kind { K_NONE, K_WAVE_BARRIER, K_ANY, K_SHFL_D, K_SHFL_F, K_SHFL_I, K_RFL, K_DPP, K_RL, K_MFMA_D, K_MFMA_F, K_BLOCK };

struct WaveState {
  int arrived = 0;
  int kind = K_NONE;
  int mask = 0;
  uint64_t gen = 0;
  double in_d[kWave], in_d2[kWave];
  float in_f[kWave], in_f2[kWave];
  int in_i[kWave];
  emu_d4 in_c[kWave];
  emu_f4 in_cf[kWave];
  double out_d[kWave];
  float out_f[kWave];
  int out_i[kWave];
  emu_d4 out_c[kWave];
  emu_f4 out_cf[kWave];
  bool out_b;
};

struct BlockState {
  int arrived = 0;
  uint64_t gen = 0;
};

std::vector<Fiber> g_fib;
std::vector<WaveState> g_wave;
BlockState g_block;
Fiber* g_cur = nullptr;
void* g_sched_sp = nullptr;
const void* g_main_bottom = nullptr;
size_t g_main_size = 0;
void (*g_entry)(void*) = nullptr;
void* g_ctx = nullptr;
int g_order = 0;

void switch_to(void** save, void* next, const void* bottom, size_t size) {
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, bottom, size);
  emu_ctx_swap(save, next);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}

// back to the scheduler (from a fiber)
void yield_to_scheduler() { switch_to(&g_cur->sp, g_sched_sp, g_main_bottom, g_main_size); }

[[noreturn]] void fiber_main() {
  __sanitizer_finish_switch_fiber(nullptr, &g_main_bottom, &g_main_size);
  g_entry(g_ctx);
  g_cur->done = true;
  __sanitizer_start_switch_fiber(nullptr, g_main_bottom, g_main_size);
  void* dead;
  emu_ctx_swap(&dead, g_sched_sp);
  abort();
}

void wait_gen(const uint64_t* counter, uint64_t gen) {
  g_cur->wait_on = counter;
  g_cur->wait_gen = gen;
  while (*counter == gen) yield_to_scheduler();
  g_cur->wait_on = nullptr;
}

[[noreturn]] void die(const char* what) {
  fprintf(stderr, "lane emulator: %s (block %u, thread %u)\n", what, block_idx.x, g_cur ? g_cur->tid : 0u);
  fflush(stderr);
  abort();
}

// One wave-level rendezvous: deposit this lane's operands, and when the last
// lane of the wave arrives, compute every lane's result.
template <class Deposit, class Compute>
WaveState& wave_op(int kind, Deposit dep, Compute comp) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = g_wave[g_cur->tid / kWave];
  if (w.arrived == 0) {
    w.kind = kind;
  } else if (w.kind != kind) {
    die("lanes of one wave reached different wave operations (divergent collective)");
  }
  dep(w, lane);
  if (++w.arrived == kWave) {
    comp(w);
    w.arrived = 0;
    ++w.gen;
  } else {
    wait_gen(&w.gen, w.gen);
  }
  return w;
}

}  // namespace

emu_uint3 thread_idx_of_current() { return emu_uint3{g_cur->tid, 0, 0}; }

void wave_barrier() {
  wave_op(K_WAVE_BARRIER, [](WaveState&, int) {}, [](WaveState&) {});
}

bool any(bool v) {
  WaveState& w = wave_op(K_ANY, [&](WaveState& s, int l) { s.in_i[l] = v ? 1 : 0; },
                         [](WaveState& s) {
                           bool r = false;
                           for (int l = 0; l < kWave; ++l) r = r || s.in_i[l];
                           s.out_b = r;
                         });
  return w.out_b;
}

double shfl_xor_f64(double v, int m) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_SHFL_D, [&](WaveState& s, int l) { s.in_d[l] = v; s.mask = m; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l) s.out_d[l] = s.in_d[(l ^ s.mask) & (kWave - 1)];
                         });
  return w.out_d[lane];
}

float shfl_xor_f32(float v, int m) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_SHFL_F, [&](WaveState& s, int l) { s.in_f[l] = v; s.mask = m; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l) s.out_f[l] = s.in_f[(l ^ s.mask) & (kWave - 1)];
                         });
  return w.out_f[lane];
}

int shfl_xor_i32(int v, int m) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_SHFL_I, [&](WaveState& s, int l) { s.in_i[l] = v; s.mask = m; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l) s.out_i[l] = s.in_i[(l ^ s.mask) & (kWave - 1)];
                         });
  return w.out_i[lane];
}

int readfirstlane(int v) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_RFL, [&](WaveState& s, int l) { s.in_i[l] = v; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l) s.out_i[l] = s.in_i[0];
                         });
  return w.out_i[lane];
}

// DPP move with a row shift right by N = ctrl - 0x110 lanes (the only control
// the device code uses): lane l of each row of 16 reads lane l - N of its row;
// lanes with no source in the row get 0 (bound_ctrl).
int update_dpp(int old, int src, int ctrl) {
  if (ctrl < 0x111 || ctrl > 0x11F) die("unsupported DPP control");
  (void)old;
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_DPP, [&](WaveState& s, int l) { s.in_i[l] = src; s.mask = ctrl - 0x110; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l)
                             s.out_i[l] = (l % 16) >= s.mask ? s.in_i[l - s.mask] : 0;
                         });
  return w.out_i[lane];
}

int readlane(int v, int src_lane) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_RL, [&](WaveState& s, int l) { s.in_i[l] = v; s.mask = src_lane; },
                         [](WaveState& s) {
                           for (int l = 0; l < kWave; ++l) s.out_i[l] = s.in_i[s.mask & (kWave - 1)];
                         });
  return w.out_i[lane];
}

emu_d4 mfma_f64(double a, double b, emu_d4 c) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_MFMA_D, [&](WaveState& s, int l) { s.in_d[l] = a; s.in_d2[l] = b; s.in_c[l] = c; },
                         [](WaveState& s) {
                           for (int i = 0; i < 16; ++i)
                             for (int j = 0; j < 16; ++j) {
                               const int l = j + 16 * (i % 4), r = i / 4;
                               double acc = s.in_c[l][r];
                               for (int k = 0; k < 4; ++k) acc += s.in_d[i + 16 * k] * s.in_d2[j + 16 * k];
                               s.out_c[l][r] = acc;
                             }
                         });
  return w.out_c[lane];
}

emu_f4 mfma_f32(float a, float b, emu_f4 c) {
  const int lane = int(g_cur->tid) % kWave;
  WaveState& w = wave_op(K_MFMA_F, [&](WaveState& s, int l) { s.in_f[l] = a; s.in_f2[l] = b; s.in_cf[l] = c; },
                         [](WaveState& s) {
                           for (int i = 0; i < 16; ++i)
                             for (int j = 0; j < 16; ++j) {
                               const int l = j + 16 * (i / 4), r = i % 4;
                               float acc = s.in_cf[l][r];
                               for (int k = 0; k < 4; ++k) acc += s.in_f[i + 16 * k] * s.in_f2[j + 16 * k];
                               s.out_cf[l][r] = acc;
                             }
                         });
  return w.out_cf[lane];
}

void block_barrier() {
  if (++g_block.arrived == int(g_fib.size())) {
    g_block.arrived = 0;
    ++g_block.gen;
  } else {
    wait_gen(&g_block.gen, g_block.gen);
  }
}

void run_grid(dim3 grid, dim3 block, void (*entry)(void*), void* ctx) {
  const char* ord = getenv("EMU_LANE_ORDER");
  g_order = ord ? atoi(ord) : 0;
  const unsigned nt = block.x * block.y * block.z;
  if (nt % kWave != 0 || block.y != 1 || block.z != 1) die("blocks must be whole wavefronts in x");
  grid_dim = {grid.x, grid.y, grid.z};
  block_dim = {block.x, block.y, block.z};
  g_entry = entry;
  g_ctx = ctx;
  for (unsigned b = 0; b < grid.x; ++b) {
    block_idx = {b, 0, 0};
    g_fib.assign(nt, Fiber());
    g_wave.assign(nt / kWave, WaveState());
    g_block = BlockState();
    for (unsigned t = 0; t < nt; ++t) {
      Fiber& f = g_fib[t];
      f.tid = t;
      f.stack = static_cast<char*>(mmap(nullptr, kStack, PROT_READ | PROT_WRITE,
                                        MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0));
      if (f.stack == MAP_FAILED) die("fiber stack");
      // entered through `ret`: the slot above the saved registers holds the
      // entry point; rsp is 8 mod 16 at entry as after a call
      uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + kStack) & ~uintptr_t(15);
      uintptr_t* sp = reinterpret_cast<uintptr_t*>(top - 8);
      *--sp = reinterpret_cast<uintptr_t>(&fiber_main);
      for (int r = 0; r < 6; ++r) *--sp = 0;
      f.sp = sp;
    }
    for (;;) {
      bool all_done = true, progressed = false;
      for (unsigned k = 0; k < nt; ++k) {
        Fiber& f = g_fib[g_order ? nt - 1 - k : k];
        if (f.done) continue;
        all_done = false;
        if (f.wait_on && *f.wait_on == f.wait_gen) continue;
        g_cur = &f;
        switch_to(&g_sched_sp, f.sp, f.stack, kStack);
        g_cur = nullptr;
        progressed = true;
      }
      if (all_done) break;
      if (!progressed) {
        int waiting = 0;
        for (auto& f : g_fib) waiting += !f.done;
        fprintf(stderr, "lane emulator: deadlock in block %u: %d lanes waiting, block barrier %d arrived\n", b,
                waiting, g_block.arrived);
        for (size_t w = 0; w < g_wave.size(); ++w)
          fprintf(stderr, "  wave %zu: %d lanes at operation %d\n", w, g_wave[w].arrived, g_wave[w].kind);
        abort();
      }
    }
    for (auto& f : g_fib) munmap(f.stack, kStack);
  }
  g_fib.clear();
}

}  // namespace emu

// ---- runtime API ----
static hipError_t g_last = hipSuccess;
hipError_t hipMalloc(void** p, size_t n) {
  *p = malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
  a->type = hipMemoryTypeDevice;
  a->device = 0;
  a->devicePointer = const_cast<void*>(p);
  a->hostPointer = const_cast<void*>(p);
  a->isManaged = 0;
  a->allocationFlags = 0;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetLastError() {
  hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulator error"; }
// a small device, so that persistent grids walk several blocks each
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  const char* s = getenv("EMU_CUS");
  *v = s ? atoi(s) : 2;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t, hipStream_t) {
  using K = void (*)(heget::KernelArgs);
  K k = reinterpret_cast<K>(const_cast<void*>(f));
  heget::KernelArgs a = *static_cast<heget::KernelArgs*>(args[0]);
  emu::launch(grid, block, [k, a]() { k(a); });
  return hipSuccess;
}
