// Declarations shared by the library's translation units (not part of the C ABI).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "generated_common.hpp"
#include "heget.h"

// A created process: its compiled kernel and its resident device tables.
struct heget_process {
  const heget::GenEntry* entry = nullptr;
  heget_precision prec = HEGET_FP64;
  int n_legs = 0;
  int n_hel = 0;
  int hel_nest = 0;          // the table is the kernel's full helicity product (loop nest)
  int cut_enabled = 0;
  double cut_pt = 0, cut_dr = 0;
  int n_a_n_b = 1, symmetry = 1;
  int spin_states = 4;       // polarisation states of the two incoming legs (spin average)
  int hadronic = 0;          // hadronic collision: the partonic flux is in the per-event weight
  double beam_m[2] = {0, 0}; // masses of the incoming legs (flux)
  double* d_cpl = nullptr;
  heget::PropEntry* d_prop = nullptr;
  int8_t* d_hel = nullptr;
  int8_t* d_ord = nullptr;   // ordering table (colour-ordered processes)
  int* d_cstep = nullptr;    // MFMA colour form: k-step table, term table, colour fragments
  uint32_t* d_cterm = nullptr;
  void* d_cfrag = nullptr;
  int cterm_words = 0;
  double* d_part = nullptr;  // integrate partials, grown on demand and reused
  int64_t part_cap = 0;
  double* h_res = nullptr;   // integrate: pinned host copy of the reduced (sum w, sum w^2, accepted)
  void* d_adapt = nullptr;   // adaptive integration buffers, grown on demand and reused
  size_t adapt_cap = 0;
  std::vector<int8_t> hel;   // host copy of the current table
  // persistent kernels (ordering templates): grid cap and one workspace slot per block
  int grid_cap = 0;
  void* d_work = nullptr;
  int64_t work_stride = 0;   // complex values per slot
  int n_orderings = 0;
};

namespace heget {
namespace detail {

// Records msg as the calling thread's last error and returns s.
heget_status fail(heget_status s, const std::string& msg);

// Whether a helicity table is the compiled kernel's full product in canonical order.
bool is_full_product(const GenEntry* e, const int8_t* table, int n_hel, int n_legs);

// Kernel arguments with the process's resident tables filled in.
KernelArgs base_args(heget_process_t p);

// Resident blocks of a kernel on the current device (occupancy x compute units).
int resident_blocks(const void* fn);

// Bytes of one complex value of the process's arithmetic type.
size_t complex_bytes(heget_process_t p);

// Massless n-body phase-space volume at sqrt_s (every RAMBO weight).
double phase_space_volume(double sqrt_s, int n);

// Per-event weight factor of heget_integrate: Phi_n / (2 lambda^(1/2)(s, m_a^2, m_b^2))
// x 1/(spin states of the incoming legs) x 1/(n_a n_b) x 1/S (massless beams: 2 s, 4 states).
double weight_factor(heget_process_t p, double sqrt_s);

// Launches the process's amplitude kernel over a.n events (256 per block; a
// persistent kernel's grid capped at its workspace slots).  HEGET_OK for n = 0.
heget_status launch(heget_process_t p, KernelArgs& a, hipStream_t stream);

// heget_result from the reduced (sum w, sum w^2, accepted) of n generated events.
void fill_result(const double h[3], int64_t n, heget_result* out);

}  // namespace detail
}  // namespace heget
