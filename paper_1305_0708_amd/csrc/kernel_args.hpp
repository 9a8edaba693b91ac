// Arguments shared by every generated amplitude kernel and the library.
#pragma once
#include <stdint.h>

namespace heget {

// Per-particle propagator data, filled by the library from the SM inputs.
struct PropEntry {
  double m, w;            // mass and width
  double pole_r, pole_i;  // pole of the denominator q^2 - pole (m^2 - i m Gamma, or the complex mass)
  double inum_r, inum_i;  // 1 / (mass^2 in the unitary-gauge numerator)
};

struct BatchTable;

struct KernelArgs {
  int64_t n;                 // events in this launch
  const double* mom_in;      // SoA [n_legs][4][n] physical momenta, or null (generate)
  int64_t mom_stride;        // n of the SoA arrays (>= n)
  uint64_t seed;             // Philox key
  uint64_t counter_offset;   // event index of the first event of this launch
  double sqrt_s;
  double* me2_out;           // [n] helicity- and colour-summed |M|^2, or null
  double* mom_out;           // SoA [n_legs][4][mom_stride] or null
  const int8_t* hel;         // [n_hel][n_legs]
  int32_t n_hel;
  int32_t hel_nest;          // 1: the table is the full product; sum it as the kernel's loop nest
  int32_t cut_enabled;
  const double* cpl;         // 4 doubles per coupling: g0 (re, im), g1 (re, im)
  const PropEntry* prop;     // indexed by particle id
  double cut_pt, cut_dr;
  double weight_factor;      // integrate: flux x averages x 1/S, times the RAMBO volume (a resonance
                             // tree's per-event weight multiplies in the kernel); generate: the
                             // RAMBO volume written to psw_out
  double* psw_out;           // generate: per-event phase-space weight [n], or null
  // adaptive integration (resonance-tree processes): the uniforms of the phase
  // space go through a grid of grid_bins bins per dimension ([dims][grid_bins + 1]
  // edges); each event's bin per dimension ([dims][grid_bin_stride], uint8) and
  // its weight [n] are written out for the grid's refinement.  Null grid: plain
  // uniforms.
  const double* grid;
  int32_t grid_bins;
  int64_t grid_bin_stride;
  uint8_t* grid_bin_out;
  double* w_out;
  double* partials;          // integrate: [gridDim.x][3] (sum w, sum w^2, accepted), or null
  const int8_t* ord;         // ordering table [n_orderings][n_legs] of colour-ordered processes
  // MFMA colour form (ordering templates with many flows; see colour_mfma.hpp)
  const int* cstep;          // [nks][2]: terms per flow in k-step s, offset of its term rows
  const uint32_t* cterm;     // [sum nterm][4]: (ordering | coefficient << 16) per lane group
  const void* cfrag;         // [nfo][nks][64] colour-matrix A fragments, double or float
  int32_t cterm_words;       // length of cterm
  const BatchTable* batch;   // fused launches of the serving engine, else null
  void* work;                // persistent kernels: gridDim.x slots of work_stride complex values
  int64_t work_stride;       //   (ordering amplitudes [n_orderings][n_hel][256] per block)
  int64_t block_base;        // split kernels: the launch's block b evaluates events of block block_base + b
};

// One request's share of a fused launch: virtual blocks [block_begin, next
// segment's block_begin) evaluate the request's own blocks block_offset,
// block_offset + 1, ... (256 events each), exactly as a launch of that request
// alone would (same counters, same per-block partial slots).
struct Segment {
  int64_t block_begin;
  int64_t block_offset;
  int64_t n;               // the request's event count
  uint64_t seed;           // the request's Philox key
  double sqrt_s;
  double weight_factor;
  double* me2_out;         // [n] or null
  double* partials;        // [ceil(n / 256)][3]
};

// Final reduction of a request whose last blocks are in this launch.
struct ReduceJob {
  const double* partials;
  int64_t nblocks;
};

constexpr int kMaxSegments = 64;
constexpr int kMaxJobs = 64;

// Device-resident description of one fused launch, uploaded as a whole.
struct BatchTable {
  int64_t total_blocks;
  int32_t n_seg, n_jobs;
  Segment seg[kMaxSegments];   // ordered by block_begin, seg[0].block_begin = 0
  ReduceJob job[kMaxJobs];
  double result[kMaxJobs][3];  // sum w, sum w^2, accepted (written by the reduction)
};

}  // namespace heget
