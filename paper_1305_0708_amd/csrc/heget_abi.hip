// C ABI of libheget: process handles, coupling derivation, kernel launches and
// the deterministic cross-section reduction.  Declarations: include/heget.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "generated_common.hpp"
#include "reduce.hpp"
#include "heget.h"
#include "heget_internal.hpp"

namespace heget {

static std::vector<const GenEntry*>& registry() {
  static std::vector<const GenEntry*> r;
  return r;
}
void register_kernel(const GenEntry* e) { registry().push_back(e); }

}  // namespace heget

using heget::GenEntry;
using heget::KernelArgs;
using heget::PropEntry;

namespace {
thread_local std::string g_err;
}  // namespace

heget_status heget::detail::fail(heget_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

namespace {

using heget::detail::fail;

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(HEGET_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// rows of the jamp matrix: one per flow, or one per ordering for a template
int jamp_rows(const heget_process_ir* ir) { return ir->n_orderings > 0 ? ir->n_orderings : ir->n_flows; }

// FNV-1a over the canonical serialisation of the kernel-relevant IR structure
struct Hasher {
  uint64_t h = 0xCBF29CE484222325ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t k = 0; k < n; ++k) {
      h ^= b[k];
      h *= 0x100000001B3ull;
    }
  }
  void i32(int32_t x) { bytes(&x, 4); }
  void f64(double x) { bytes(&x, 8); }
};

uint64_t fingerprint(const heget_process_ir* ir) {
  Hasher H;
  H.i32(ir->n_legs);
  for (int k = 0; k < ir->n_legs; ++k) {
    const heget_leg& l = ir->legs[k];
    H.i32(l.kind);
    H.i32(l.incoming);
    H.i32(l.flow);
    H.i32(l.particle);
    H.i32(l.colour);
  }
  H.i32(ir->n_couplings);
  for (int k = 0; k < ir->n_couplings; ++k) {
    const heget_coupling& c = ir->couplings[k];
    H.i32(c.kind);
    H.f64(c.charge);
    H.f64(c.t3);
    H.i32(c.particle);
  }
  H.i32(ir->n_calls);
  for (int k = 0; k < ir->n_calls; ++k) {
    const heget_call& c = ir->calls[k];
    H.i32(c.op);
    for (int j = 0; j < 4; ++j) H.i32(c.in[j]);
    H.i32(c.out);
    H.i32(c.coupling);
    H.i32(c.prop);
  }
  H.i32(ir->n_amps);
  H.i32(ir->n_flows);
  for (int f = 0; f < jamp_rows(ir); ++f)
    for (int a = 0; a < ir->n_amps; ++a) {
      H.f64(ir->jamp[(f * ir->n_amps + a) * 2]);
      H.f64(ir->jamp[(f * ir->n_amps + a) * 2 + 1]);
    }
  for (int k = 0; k < ir->n_flows * ir->n_flows; ++k) H.f64(ir->colour_num[k]);
  H.f64(ir->colour_den);
  H.i32(ir->cut_enabled);
  H.i32(ir->n_orderings);
  for (int k = 0; k < ir->n_orderings * ir->n_legs; ++k) H.i32(ir->orderings[k]);
  H.i32(ir->flow_map ? 1 : 0);
  if (ir->flow_map)
    for (int k = 0; k < ir->n_flows * ir->n_orderings; ++k) H.i32(ir->flow_map[k]);
  if (ir->n_ps_nodes > 0) {
    H.i32(ir->n_ps_nodes);
    for (int k = 0; k < ir->n_ps_nodes; ++k) {
      const heget_ps_node& nd = ir->ps_nodes[k];
      H.i32(nd.particle);
      H.i32(nd.mapping);
      H.i32(nd.daughter[0]);
      H.i32(nd.daughter[1]);
    }
    H.f64(ir->ps_window);
  }
  if (ir->ps_hadron_ymax > 0) {
    H.i32(1);
    H.f64(ir->ps_hadron_ymax);
    H.f64(ir->ps_hadron_ptmin);
  }
  if (ir->colour_form != 0 || ir->division != 0) {
    H.i32(ir->colour_form);
    H.i32(ir->division);
  }
  return H.h;
}

// inputs per opcode: 'F', 'V', 'S'; output kind or 'A' for amplitudes
struct OpSig {
  const char* in;
  char out;
};
const OpSig kSig[HEGET_N_OPS] = {
    {"FFV", 'A'}, {"FV", 'F'}, {"FV", 'F'}, {"FF", 'V'},     // iov fvi fvo jio
    {"FFS", 'A'}, {"FS", 'F'}, {"FS", 'F'}, {"FF", 'S'},     // ios fsi fso hio
    {"VVV", 'A'}, {"VV", 'V'},                               // vvv jvv
    {"VVVV", 'A'}, {"VVV", 'V'}, {"VVVV", 'A'}, {"VVV", 'V'},  // gggg jggg wwww jwww
    {"VVS", 'A'}, {"VS", 'V'}, {"VV", 'S'},                  // vvs jvs hvv
    {"VVSS", 'A'}, {"VSS", 'V'}, {"VVS", 'S'},               // vvss jvss hvvs
    {"SSS", 'A'}, {"SS", 'S'}, {"SSSS", 'A'}, {"SSS", 'S'},  // sss hss ssss hsss
    {"VV", 'V'}, {"VV", 'V'},                                // vadd vsub
};

heget_status validate(const heget_process_ir* ir) {
  if (ir->colour_form != 0 && ir->colour_form != 1) return fail(HEGET_E_IR, "unknown colour form");
  if (ir->division != 0 && ir->division != 1) return fail(HEGET_E_IR, "unknown division");
  if (ir->division == 1 && ir->n_orderings == 0) return fail(HEGET_E_IR, "the split division needs orderings");
  if (ir->n_legs < 3 || ir->n_legs > 12 || !ir->legs) return fail(HEGET_E_IR, "n_legs must be 3..12");
  if (!ir->legs[0].incoming || !ir->legs[1].incoming)
    return fail(HEGET_E_IR, "legs 0 and 1 must be the incoming partons");
  for (int k = 2; k < ir->n_legs; ++k)
    if (ir->legs[k].incoming) return fail(HEGET_E_IR, "only legs 0 and 1 may be incoming");
  for (int k = 0; k < ir->n_legs; ++k) {
    const heget_leg& l = ir->legs[k];
    if (l.kind < 0 || l.kind > 2 || l.particle < 0 || l.particle >= HEGET_N_PARTICLES)
      return fail(HEGET_E_IR, "leg " + std::to_string(k) + ": bad kind or particle");
    if (l.particle != HEGET_P_ZERO && ir->n_ps_nodes == 0)
      return fail(HEGET_E_UNSUPPORTED, "RAMBO phase space needs massless legs (give a resonance tree)");
  }
  if (ir->n_couplings < 1 || !ir->couplings) return fail(HEGET_E_IR, "no couplings");
  for (int k = 0; k < ir->n_couplings; ++k)
    if (ir->couplings[k].kind < 0 || ir->couplings[k].kind >= HEGET_N_CPL)
      return fail(HEGET_E_IR, "coupling " + std::to_string(k) + ": bad kind");
  if (ir->n_calls < 1 || !ir->calls) return fail(HEGET_E_IR, "no calls");
  std::vector<char> kind(ir->n_legs + ir->n_calls + 1, 0);
  for (int k = 0; k < ir->n_legs; ++k) kind[k] = "FVS"[ir->legs[k].kind];
  std::vector<char> amp_seen(ir->n_amps > 0 ? ir->n_amps : 1, 0);
  for (int k = 0; k < ir->n_calls; ++k) {
    const heget_call& c = ir->calls[k];
    const std::string at = "call " + std::to_string(k) + ": ";
    if (c.op < 0 || c.op >= HEGET_N_OPS) return fail(HEGET_E_IR, at + "bad opcode");
    const OpSig& sg = kSig[c.op];
    const int nin = int(std::strlen(sg.in));
    for (int j = 0; j < 4; ++j) {
      if (j < nin) {
        const int s = c.in[j];
        if (s < 0 || s >= int(kind.size()) || kind[s] == 0) return fail(HEGET_E_IR, at + "input slot undefined");
        if (kind[s] != sg.in[j]) return fail(HEGET_E_IR, at + "input slot has the wrong kind");
      } else if (c.in[j] != -1) {
        return fail(HEGET_E_IR, at + "unused inputs must be -1");
      }
    }
    const bool linear = c.op == HEGET_OP_VADD || c.op == HEGET_OP_VSUB;
    if (linear ? c.coupling != -1 : (c.coupling < 0 || c.coupling >= ir->n_couplings))
      return fail(HEGET_E_IR, at + "bad coupling index");
    if (c.prop < 0 || c.prop >= HEGET_N_PARTICLES) return fail(HEGET_E_IR, at + "bad propagator particle");
    if (sg.out == 'A') {
      if (c.out < 0 || c.out >= ir->n_amps || amp_seen[c.out]) return fail(HEGET_E_IR, at + "bad amplitude index");
      amp_seen[c.out] = 1;
    } else {
      if (c.out < ir->n_legs || c.out >= int(kind.size()) || kind[c.out] != 0)
        return fail(HEGET_E_IR, at + "output slot reused or out of range");
      kind[c.out] = sg.out;
    }
  }
  for (int a = 0; a < ir->n_amps; ++a)
    if (!amp_seen[a]) return fail(HEGET_E_IR, "amplitude " + std::to_string(a) + " is never produced");
  if (ir->n_flows < 1 || !ir->jamp || !ir->colour_num || !(ir->colour_den > 0))
    return fail(HEGET_E_IR, "jamp / colour matrix missing");
  for (int f = 0; f < ir->n_flows; ++f)
    for (int g = 0; g < ir->n_flows; ++g)
      if (ir->colour_num[f * ir->n_flows + g] != ir->colour_num[g * ir->n_flows + f])
        return fail(HEGET_E_IR, "colour matrix is not symmetric");
  if (ir->n_hel < 1 || !ir->helicities) return fail(HEGET_E_IR, "empty helicity table");
  for (int h = 0; h < ir->n_hel * ir->n_legs; ++h) {
    const int v = ir->helicities[h];
    if (!(v == -1 || v == 0 || v == 1 || v == 4)) return fail(HEGET_E_IR, "helicity values must be -1, 0, 1 or 4");
  }
  if (ir->n_a_n_b < 1 || ir->symmetry < 1) return fail(HEGET_E_IR, "averaging factors must be >= 1");
  if (ir->n_orderings < 0 || (ir->n_orderings > 0 && !ir->orderings))
    return fail(HEGET_E_IR, "ordering table missing");
  if (ir->n_orderings > 127) return fail(HEGET_E_IR, "at most 127 orderings");
  if (ir->flow_map) {
    if (ir->n_orderings == 0) return fail(HEGET_E_IR, "a flow map needs an ordering table");
    for (int f = 0; f < ir->n_flows; ++f) {
      bool any = false;
      for (int o = 0; o < ir->n_orderings; ++o) any |= ir->flow_map[f * ir->n_orderings + o] != 0;
      if (!any) return fail(HEGET_E_IR, "flow map row " + std::to_string(f) + " is all zero");
    }
  } else if (ir->n_orderings > 0 && ir->n_orderings != ir->n_flows) {
    return fail(HEGET_E_IR, "without a flow map the ordering table must have one row per flow");
  }
  for (int o = 0; o < ir->n_orderings; ++o) {
    std::vector<char> seen(ir->n_legs, 0);
    for (int k = 0; k < ir->n_legs; ++k) {
      const int x = ir->orderings[o * ir->n_legs + k];
      if (x < 0 || x >= ir->n_legs || seen[x]) return fail(HEGET_E_IR, "orderings must be permutations of the legs");
      seen[x] = 1;
    }
  }
  if (ir->n_ps_nodes < 0 || ir->n_ps_nodes > 16 || (ir->n_ps_nodes > 0 && !ir->ps_nodes))
    return fail(HEGET_E_IR, "phase-space tree: 0..16 nodes");
  if (ir->n_ps_nodes > 0) {
    if (!(ir->ps_window > 0) || !std::isfinite(ir->ps_window))
      return fail(HEGET_E_IR, "phase-space tree: window must be > 0");
    std::vector<int> leg_seen(ir->n_legs, 0), node_seen(ir->n_ps_nodes, 0);
    for (int k = 0; k < ir->n_ps_nodes; ++k) {
      const heget_ps_node& nd = ir->ps_nodes[k];
      if (k > 0 && (nd.particle < 0 || nd.particle >= HEGET_N_PARTICLES ||
                    (nd.mapping != HEGET_PS_FLAT && nd.mapping != HEGET_PS_BREIT_WIGNER)))
        return fail(HEGET_E_IR, "phase-space node " + std::to_string(k) + ": bad particle or mapping");
      for (int d : nd.daughter) {
        if (d >= 0) {
          if (d < 2 || d >= ir->n_legs) return fail(HEGET_E_IR, "phase-space tree: daughter is not a final leg");
          ++leg_seen[d];
        } else {
          const int j = -1 - d;
          if (j <= k || j >= ir->n_ps_nodes)
            return fail(HEGET_E_IR, "phase-space tree: a daughter node must come after its parent");
          ++node_seen[j];
        }
      }
    }
    for (int L = 2; L < ir->n_legs; ++L)
      if (leg_seen[L] != 1) return fail(HEGET_E_IR, "phase-space tree: every final leg is a daughter exactly once");
    for (int k = 1; k < ir->n_ps_nodes; ++k)
      if (node_seen[k] != 1) return fail(HEGET_E_IR, "phase-space tree: every node but the first is a daughter once");
  }
  if (!(ir->ps_hadron_ymax >= 0) || !std::isfinite(ir->ps_hadron_ymax) || !(ir->ps_hadron_ptmin >= 0))
    return fail(HEGET_E_IR, "hadronic collision: ymax and ptmin must be >= 0");
  if (ir->ps_hadron_ymax > 0) {
    if (ir->n_ps_nodes == 0) return fail(HEGET_E_IR, "hadronic collision: needs a phase-space tree");
    for (int d : ir->ps_nodes[0].daughter)
      if (d >= 0 && ir->legs[d].particle == HEGET_P_ZERO && !(ir->ps_hadron_ptmin > 0))
        return fail(HEGET_E_IR, "hadronic collision: a massless daughter of the collision needs ptmin > 0");
  }
  return HEGET_OK;
}

// ------------------------------------------------------------ SM couplings
using cd = std::complex<double>;

struct Derived {
  double e, sw, cw, gw, gz, gs, mw, ww, v;
  cd muw2, muz2, numw2, numz2, muw, muz;
};

Derived derive(const heget_sm& sm) {
  Derived d;
  const double pi = 3.14159265358979323846;
  d.e = std::sqrt(4.0 * pi * sm.alpha);
  d.sw = std::sqrt(sm.sw2);
  d.cw = std::sqrt(1.0 - sm.sw2);
  d.gw = d.e / d.sw;
  d.gz = d.e / (d.sw * d.cw);
  d.gs = std::sqrt(4.0 * pi * sm.alpha_s);
  if (sm.complex_mass) {
    d.mw = d.cw * sm.mz;   // mu_W^2 = c_W^2 mu_Z^2
    d.ww = d.cw * sm.wz;
  } else {
    d.mw = sm.mw;
    d.ww = sm.ww;
  }
  d.muw2 = cd(d.mw * d.mw, -d.mw * d.ww);
  d.muz2 = cd(sm.mz * sm.mz, -sm.mz * sm.wz);
  d.numw2 = sm.complex_mass ? d.muw2 : cd(d.mw * d.mw, 0.0);
  d.numz2 = sm.complex_mass ? d.muz2 : cd(sm.mz * sm.mz, 0.0);
  d.muw = sm.complex_mass ? std::sqrt(d.muw2) : cd(d.mw, 0.0);
  d.muz = sm.complex_mass ? std::sqrt(d.muz2) : cd(sm.mz, 0.0);
  d.v = 2.0 * d.mw / d.gw;
  return d;
}

void coupling_values(const heget_sm& sm, const heget_coupling& c, double out[4]) {
  const Derived d = derive(sm);
  cd g0 = 0.0, g1 = 0.0;
  switch (c.kind) {
    case HEGET_CPL_GAMMA_FF: g0 = g1 = -d.e * c.charge; break;
    case HEGET_CPL_Z_FF: g0 = -d.gz * (c.t3 - c.charge * sm.sw2); g1 = d.gz * c.charge * sm.sw2; break;
    case HEGET_CPL_W_FF: g0 = -d.gw / std::sqrt(2.0); g1 = 0.0; break;
    case HEGET_CPL_G_QQ: g0 = g1 = d.gs; break;
    case HEGET_CPL_GGG: g0 = d.gs; break;
    case HEGET_CPL_GGGG: g0 = d.gs * d.gs; break;
    case HEGET_CPL_WWZ: g0 = d.gw * d.cw; break;
    case HEGET_CPL_WWA: g0 = d.e; break;
    case HEGET_CPL_WWH: g0 = d.gw * d.muw; break;
    case HEGET_CPL_ZZH: g0 = d.gz * d.muz; break;
    case HEGET_CPL_WWHH: g0 = 0.5 * d.gw * d.gw; break;
    case HEGET_CPL_ZZHH: g0 = 0.5 * d.gz * d.gz; break;
    case HEGET_CPL_HHH: g0 = -3.0 * sm.mh * sm.mh / d.v; break;
    case HEGET_CPL_HHHH: g0 = -3.0 * sm.mh * sm.mh / (d.v * d.v); break;
    case HEGET_CPL_HBB: g0 = g1 = -sm.mb_yuk / d.v; break;
    case HEGET_CPL_WWWW: g0 = -d.gw * d.gw; break;
    case HEGET_CPL_WWZZ: g0 = d.gw * d.gw * d.cw * d.cw; break;
    default: break;
  }
  out[0] = g0.real();
  out[1] = g0.imag();
  out[2] = g1.real();
  out[3] = g1.imag();
}

// The generated kernels take what coupling_values fixes by construction as
// constants (every kind real but W W H and Z Z H; g1 = g0 for the vector
// couplings; g1 = 0 for the W-fermion and the boson vertices): a change here
// that broke it would give wrong amplitudes, so create checks the values.
bool coupling_structure_ok(int kind, const double v[4]) {
  if (kind != HEGET_CPL_WWH && kind != HEGET_CPL_ZZH && (v[1] != 0.0 || v[3] != 0.0)) return false;
  switch (kind) {
    case HEGET_CPL_GAMMA_FF:
    case HEGET_CPL_G_QQ:
    case HEGET_CPL_HBB: return v[2] == v[0] && v[3] == v[1];
    case HEGET_CPL_Z_FF: return true;
    default: return v[2] == 0.0 && v[3] == 0.0;
  }
}

void prop_table(const heget_sm& sm, PropEntry t[HEGET_N_PARTICLES]) {
  const Derived d = derive(sm);
  auto fill = [](PropEntry& e, double m, double w, cd pole, cd num) {
    e.m = m;
    e.w = w;
    e.pole_r = pole.real();
    e.pole_i = pole.imag();
    const cd inv = (std::abs(num) > 0) ? 1.0 / num : cd(0.0, 0.0);
    e.inum_r = inv.real();
    e.inum_i = inv.imag();
  };
  fill(t[HEGET_P_ZERO], 0.0, 0.0, 0.0, 0.0);
  fill(t[HEGET_P_W], d.mw, d.ww, d.muw2, d.numw2);
  fill(t[HEGET_P_Z], sm.mz, sm.wz, d.muz2, d.numz2);
  fill(t[HEGET_P_TOP], sm.mt, sm.wt, cd(sm.mt * sm.mt, -sm.mt * sm.wt), 0.0);
  fill(t[HEGET_P_H], sm.mh, sm.wh, cd(sm.mh * sm.mh, -sm.mh * sm.wh), 0.0);
}

}  // namespace

double heget::detail::phase_space_volume(double sqrt_s, int n) {
  const double pi = 3.14159265358979323846;
  double f1 = 1.0, f2 = 1.0;
  for (int i = 2; i <= n - 1; ++i) f1 *= i;
  for (int i = 2; i <= n - 2; ++i) f2 *= i;
  const double s = sqrt_s * sqrt_s;
  return std::pow(2.0 * pi, 4 - 3 * n) * std::pow(0.5 * pi, n - 1) * std::pow(s, n - 2) / (f1 * f2);
}

double heget::detail::weight_factor(heget_process_t p, double sqrt_s) {
  const double s = sqrt_s * sqrt_s;
  // a resonance tree's weight is per event (multiplied in the kernel)
  const double volume = p->entry->generate ? 1.0 : phase_space_volume(sqrt_s, p->n_legs - 2);
  if (p->hadronic) return 1.0 / double(p->spin_states) / p->n_a_n_b / p->symmetry;   // flux per event
  const double ma = p->beam_m[0], mb = p->beam_m[1];
  const double flux = (ma == 0.0 && mb == 0.0)
                          ? s
                          : std::sqrt(std::max((s - (ma + mb) * (ma + mb)) * (s - (ma - mb) * (ma - mb)), 0.0));
  return volume / (2.0 * flux) / double(p->spin_states) / p->n_a_n_b / p->symmetry;
}

void heget::detail::fill_result(const double h[3], int64_t n, heget_result* out) {
  const double N = double(n);
  out->sum_w = h[0];
  out->sum_w2 = h[1];
  out->n_generated = n;
  out->n_accepted = int64_t(h[2] + 0.5);
  out->sigma_gev2 = h[0] / N;
  const double var = std::max(h[1] / N - out->sigma_gev2 * out->sigma_gev2, 0.0);
  out->err_gev2 = std::sqrt(var / (N - 1.0));
  const double hbarc2 = 0.3893793721e9;
  out->sigma_pb = out->sigma_gev2 * hbarc2;
  out->err_pb = out->err_gev2 * hbarc2;
}

namespace {

// Philox -> RAMBO -> SoA momenta, the generation step of heget_eval alone.
template <int NOUT>
__global__ __launch_bounds__(256) void generate_momenta(KernelArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  heget::mom p[NOUT + 2];
  const double h = 0.5 * a.sqrt_s;
  p[0] = {h, 0.0, 0.0, h};
  p[1] = {h, 0.0, 0.0, -h};
  heget::rambo<NOUT>(a.seed, a.counter_offset + uint64_t(i), a.sqrt_s, p + 2);
  heget::store_momenta<NOUT + 2>(a, i, p);
  if (a.psw_out) a.psw_out[i] = a.weight_factor;   // RAMBO: the constant n-body volume
}

template <int NOUT>
const void* generate_kernel() {
  return reinterpret_cast<const void*>(&generate_momenta<NOUT>);
}

// The Philox step alone: uniforms of events counter_offset .. + n - 1, block j
// of event i giving u[2 j][i] and u[2 j + 1][i] (SoA, coalesced per draw).
__global__ __launch_bounds__(256) void uniforms_kernel(uint64_t seed, uint64_t counter_offset, int64_t n,
                                                       int n_u, double* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t ev = counter_offset + uint64_t(i);
  for (int j = 0; 2 * j < n_u; ++j) {
    uint32_t c[4] = {uint32_t(ev), uint32_t(ev >> 32), uint32_t(j), 0u};
    heget::philox4x32_10(c, uint32_t(seed), uint32_t(seed >> 32));
    out[int64_t(2 * j) * n + i] = heget::unit_open(c[0], c[1]);
    if (2 * j + 1 < n_u) out[int64_t(2 * j + 1) * n + i] = heget::unit_open(c[2], c[3]);
  }
}

// Fixed-order reduction of one request's per-block partials (one block).
__global__ __launch_bounds__(256) void reduce_partials(const double* partials, int64_t nblocks, double* out) {
  heget::reduce_triples(partials, nblocks, out);
}

// Scratch of heget_integrate_noalloc: the per-block partial sums (w, w^2,
// accepted) of one call and its three reduced sums, for callers that cannot
// allocate.  Every GPU the library runs on holds its own copy (6 MiB) until the
// process ends.  Host code must use the address hipGetSymbolAddress returns for
// the current device, never the array's name.
constexpr int64_t kNoAllocMaxBlocks = HEGET_NOALLOC_MAX_EVENTS / 256;
__device__ __align__(256) double scratch[3 * kNoAllocMaxBlocks + 3];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array, looked up once per device.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace


heget_status heget::detail::launch(heget_process_t p, KernelArgs& a, hipStream_t stream) {
  if (a.n == 0) return HEGET_OK;
  const int block = 256;
  int64_t grid = (a.n + block - 1) / block;
  if (grid > 0x7fffffff) return fail(HEGET_E_INVALID, "n too large for one launch");
  const GenEntry* e = p->entry;
  if (e->chain_fp64) {
    // split division: per round of resident blocks (one workspace slot each), the
    // orderings' kernel then the colour-form kernel, in order on the stream
    const bool f64 = p->prec == HEGET_FP64;
    const void* chain = f64 ? e->chain_fp64 : e->chain_mixed;
    const void* colour = f64 ? e->colour_fp64 : e->colour_mixed;
    const int64_t nb = grid;
    for (int64_t base = 0; base < nb; base += p->grid_cap) {
      const int64_t g = std::min<int64_t>(p->grid_cap, nb - base);
      a.block_base = base;
      void* args[] = {&a};
      HIP_TRY(hipLaunchKernel(chain, dim3(unsigned(g)), dim3(block), args, 0, stream));
      HIP_TRY(hipLaunchKernel(colour, dim3(unsigned(g)), dim3(block), args, 0, stream));
    }
    a.block_base = 0;
    return HEGET_OK;
  }
  if (e->persistent) grid = std::min<int64_t>(grid, p->grid_cap);   // one workspace slot per block
  const void* fn = p->prec == HEGET_FP64 ? e->kernel_fp64 : e->kernel_mixed;
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(block), args, 0, stream));
  return HEGET_OK;
}

bool heget::detail::is_full_product(const GenEntry* e, const int8_t* table, int n_hel, int n_legs) {
  return e->hel_canon && e->n_hel_canon == n_hel &&
         std::memcmp(e->hel_canon, table, size_t(n_hel) * n_legs) == 0;
}

KernelArgs heget::detail::base_args(heget_process_t p) {
  KernelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.hel = p->d_hel;
  a.n_hel = p->n_hel;
  a.hel_nest = p->hel_nest;
  a.cut_enabled = p->cut_enabled;
  a.cpl = p->d_cpl;
  a.prop = p->d_prop;
  a.cut_pt = p->cut_pt;
  a.cut_dr = p->cut_dr;
  a.ord = p->d_ord;
  a.cstep = p->d_cstep;
  a.cterm = p->d_cterm;
  a.cfrag = p->d_cfrag;
  a.cterm_words = p->cterm_words;
  a.work = p->d_work;
  a.work_stride = p->work_stride;
  return a;
}

int heget::detail::resident_blocks(const void* fn) {
  int dev = 0, per_cu = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) n_cu = 1;
  return per_cu * n_cu;
}

size_t heget::detail::complex_bytes(heget_process_t p) {
  return p->prec == HEGET_FP64 ? 2 * sizeof(double) : 2 * sizeof(float);
}

namespace {

using heget::detail::base_args;
using heget::detail::launch;

void release(heget_process* p) {
  if (!p) return;
  if (p->d_cpl) (void)hipFree(p->d_cpl);
  if (p->d_prop) (void)hipFree(p->d_prop);
  if (p->d_hel) (void)hipFree(p->d_hel);
  if (p->d_part) (void)hipFree(p->d_part);
  if (p->d_ord) (void)hipFree(p->d_ord);
  if (p->d_cstep) (void)hipFree(p->d_cstep);
  if (p->d_cterm) (void)hipFree(p->d_cterm);
  if (p->d_cfrag) (void)hipFree(p->d_cfrag);
  if (p->d_work) (void)hipFree(p->d_work);
  if (p->d_adapt) (void)hipFree(p->d_adapt);
  if (p->h_res) (void)hipHostFree(p->h_res);
  delete p;
}

// Host tables of the MFMA colour form (layouts in colour_mfma.hpp).  Flows are
// sorted by their number of flow-map terms (stable), so that the four flows of
// one k-step share one term count; a k-step's shorter rows are padded with
// zero-coefficient terms.
struct ColourTables {
  std::vector<int> cstep;        // [nks][2] (terms, offset)
  std::vector<uint32_t> cterm;   // [sum terms][4]
  std::vector<double> cfrag;     // [nfo][nks][64]
};

heget_status colour_tables(const heget_process_ir* ir, const GenEntry* e, heget_precision prec, ColourTables& t) {
  const int nf = ir->n_flows, no = ir->n_orderings;
  if (no <= 0) return fail(HEGET_E_IR, "the MFMA colour form needs an ordering table");
  if (e->nks != (nf + 3) / 4 || e->nfo != (nf + 15) / 16)
    return fail(HEGET_E_IR, "kernel tile counts disagree with n_flows");
  std::vector<std::vector<std::pair<int, int>>> rows(nf);
  for (int f = 0; f < nf; ++f)
    for (int o = 0; o < no; ++o) {
      const int c = ir->flow_map ? ir->flow_map[f * no + o] : (o == f ? 1 : 0);
      if (c != 0) rows[f].push_back({o, c});
    }
  std::vector<int> order(nf);
  for (int f = 0; f < nf; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return rows[a].size() < rows[b].size(); });
  const int nks = e->nks, nfo = e->nfo;
  t.cstep.assign(2 * size_t(nks), 0);
  t.cterm.clear();
  int off = 0;
  for (int s = 0; s < nks; ++s) {
    int nt = 0;
    for (int g = 0; g < 4; ++g)
      if (4 * s + g < nf) nt = std::max(nt, int(rows[order[4 * s + g]].size()));
    t.cstep[2 * s] = nt;
    t.cstep[2 * s + 1] = off;
    for (int k = 0; k < nt; ++k)
      for (int g = 0; g < 4; ++g) {
        uint32_t word = 0;
        if (4 * s + g < nf) {
          const auto& r = rows[order[4 * s + g]];
          if (k < int(r.size())) word = uint32_t(r[k].first) | (uint32_t(uint16_t(int16_t(r[k].second))) << 16);
        }
        t.cterm.push_back(word);
      }
    off += nt;
  }
  auto cs = [&](int a, int b) {
    return (a < nf && b < nf) ? ir->colour_num[order[a] * nf + order[b]] / ir->colour_den : 0.0;
  };
  // row i of output tile fo is the flow whose B operand the lane holding D[i][.] supplied at
  // k-step 4 fo + (register of D[i][.]); the D layouts of the two MFMAs differ (colour_mfma.hpp)
  auto out_flow = [&](int fo, int i) {
    return prec == HEGET_FP64 ? 16 * fo + i : 16 * fo + 4 * (i % 4) + i / 4;
  };
  // C is symmetric: tile fo reads the k-steps of its diagonal 16 x 16 block as
  // they are and those of the later blocks doubled; earlier k-steps are not read
  t.cfrag.assign(size_t(nfo) * nks * 64, 0.0);
  for (int fo = 0; fo < nfo; ++fo)
    for (int s = 4 * fo; s < nks; ++s)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, k = lane >> 4;
        const double f = s >= 4 * (fo + 1) ? 2.0 : 1.0;
        t.cfrag[(size_t(fo) * nks + s) * 64 + lane] = f * cs(out_flow(fo, i), 4 * s + k);
      }
  return HEGET_OK;
}

}  // namespace

extern "C" {

const char* heget_last_error(void) { return g_err.c_str(); }

heget_status heget_process_create(const heget_process_ir* ir, heget_precision prec, heget_process_t* out) {
  g_err.clear();
  if (!ir || !out) return fail(HEGET_E_INVALID, "null argument");
  *out = nullptr;
  if (prec != HEGET_FP64 && prec != HEGET_MIXED) return fail(HEGET_E_INVALID, "unknown precision");
  if (heget_status s = validate(ir)) return s;
  {
    PropEntry prop[HEGET_N_PARTICLES];
    prop_table(ir->sm, prop);
    for (int k = 1; k < ir->n_ps_nodes; ++k) {
      const heget_ps_node& nd = ir->ps_nodes[k];
      if (nd.mapping == HEGET_PS_BREIT_WIGNER && !(prop[nd.particle].m > 0 && prop[nd.particle].w > 0))
        return fail(HEGET_E_IR, "phase-space node " + std::to_string(k) + ": Breit-Wigner needs a mass and a width");
    }
  }
  const uint64_t fp = fingerprint(ir);
  const GenEntry* entry = nullptr;
  for (const GenEntry* e : heget::registry())
    if (e->fingerprint == fp && e->n_legs == ir->n_legs) entry = e;
  if (!entry) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "no kernel compiled for this IR structure (fingerprint 0x%016llx)",
                  (unsigned long long)fp);
    return fail(HEGET_E_UNSUPPORTED, buf);
  }
  // Mixed-precision kernels with the MFMA colour form have made illegal memory
  // accesses on the GPU (an FP32 colour form over FP32 rows, and an FP32 chain
  // feeding an FP64 colour form) with no cause found in their code: refused
  // until one is, so that no caller launches them.
  if (prec == HEGET_MIXED && entry->colour_mfma_mixed)
    return fail(HEGET_E_UNSUPPORTED, "mixed precision is switched off for processes whose colour form runs on "
                "MFMA (an unexplained GPU fault); use FP64, or a basis with the VALU colour form");
  heget_process* p = new heget_process();
  p->entry = entry;
  p->prec = prec;
  p->n_legs = ir->n_legs;
  p->n_hel = ir->n_hel;
  p->cut_enabled = ir->cut_enabled;
  p->cut_pt = ir->cut_pt;
  p->cut_dr = ir->cut_dr;
  p->n_a_n_b = ir->n_a_n_b;
  p->symmetry = ir->symmetry;
  p->hel.assign(ir->helicities, ir->helicities + size_t(ir->n_hel) * ir->n_legs);
  p->hel_nest = heget::detail::is_full_product(entry, ir->helicities, ir->n_hel, ir->n_legs) ? 1 : 0;
  std::vector<double> cpl(size_t(ir->n_couplings) * 4);
  for (int k = 0; k < ir->n_couplings; ++k) {
    coupling_values(ir->sm, ir->couplings[k], &cpl[4 * k]);
    if (!coupling_structure_ok(ir->couplings[k].kind, &cpl[4 * k])) {
      release(p);
      return fail(HEGET_E_UNSUPPORTED, "coupling " + std::to_string(k) + " breaks the structure the kernels assume");
    }
  }
  PropEntry prop[HEGET_N_PARTICLES];
  prop_table(ir->sm, prop);
  p->hadronic = ir->ps_hadron_ymax > 0 ? 1 : 0;
  p->spin_states = 1;
  for (int k = 0; k < 2; ++k) {
    const heget_leg& l = ir->legs[k];
    const bool massive = l.particle != HEGET_P_ZERO;
    p->beam_m[k] = massive ? prop[l.particle].m : 0.0;
    p->spin_states *= l.kind == 2 ? 1 : (l.kind == 1 && massive ? 3 : 2);   // S; massive V; F or massless V
  }
  if (hipMalloc(&p->d_cpl, cpl.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->d_prop, sizeof(prop)) != hipSuccess || hipMalloc(&p->d_hel, p->hel.size()) != hipSuccess) {
    release(p);
    return fail(HEGET_E_OOM, "device allocation of process tables failed");
  }
  if (hipMemcpy(p->d_cpl, cpl.data(), cpl.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_prop, prop, sizeof(prop), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_hel, p->hel.data(), p->hel.size(), hipMemcpyHostToDevice) != hipSuccess) {
    release(p);
    return fail(HEGET_E_HIP, "upload of process tables failed");
  }
  if (ir->n_orderings > 0) {
    const size_t nb = size_t(ir->n_orderings) * ir->n_legs;
    if (hipMalloc(&p->d_ord, nb) != hipSuccess) {
      release(p);
      return fail(HEGET_E_OOM, "device allocation of the ordering table failed");
    }
    if (hipMemcpy(p->d_ord, ir->orderings, nb, hipMemcpyHostToDevice) != hipSuccess) {
      release(p);
      return fail(HEGET_E_HIP, "upload of the ordering table failed");
    }
  }
  if (entry->persistent) {
    // ordering amplitudes of every resident block's 256 events, all orderings and helicities
    p->n_orderings = ir->n_orderings;
    p->grid_cap = heget::detail::resident_blocks(prec == HEGET_FP64 ? entry->kernel_fp64 : entry->kernel_mixed);
    if (entry->chain_fp64) {
      // split: both kernels of a round must fit the workspace's slots
      const bool f64 = prec == HEGET_FP64;
      p->grid_cap = std::min(heget::detail::resident_blocks(f64 ? entry->chain_fp64 : entry->chain_mixed),
                             heget::detail::resident_blocks(f64 ? entry->colour_fp64 : entry->colour_mixed));
    }
    p->work_stride = int64_t(ir->n_orderings) * ir->n_hel * 256;
    const size_t wb = size_t(p->grid_cap) * size_t(p->work_stride) * heget::detail::complex_bytes(p);
    if (hipMalloc(&p->d_work, wb) != hipSuccess) {
      release(p);
      return fail(HEGET_E_OOM, "device allocation of the workspace failed (" + std::to_string(wb >> 20) + " MiB)");
    }
  }
  if (entry->colour_mfma) {
    ColourTables t;
    if (heget_status st = colour_tables(ir, entry, prec, t)) {
      release(p);
      return st;
    }
    if (int(t.cterm.size()) > entry->cterm_cap) {
      release(p);
      return fail(HEGET_E_IR, "colour term table larger than the kernel's");
    }
    p->cterm_words = int(t.cterm.size());
    std::vector<float> f32(t.cfrag.begin(), t.cfrag.end());
    const void* frag = prec == HEGET_FP64 ? static_cast<const void*>(t.cfrag.data()) : f32.data();
    const size_t fb = t.cfrag.size() * (prec == HEGET_FP64 ? sizeof(double) : sizeof(float));
    if (hipMalloc(&p->d_cstep, t.cstep.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_cterm, std::max<size_t>(t.cterm.size(), 4) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&p->d_cfrag, fb) != hipSuccess) {
      release(p);
      return fail(HEGET_E_OOM, "device allocation of the colour tables failed");
    }
    if (hipMemcpy(p->d_cstep, t.cstep.data(), t.cstep.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_cterm, t.cterm.data(), t.cterm.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_cfrag, frag, fb, hipMemcpyHostToDevice) != hipSuccess) {
      release(p);
      return fail(HEGET_E_HIP, "upload of the colour tables failed");
    }
  }
  {
    // set-up of heget_integrate_noalloc's scratch on this device
    double* sp = nullptr;
    if (hipError_t e = scratch_address(&sp)) {
      release(p);
      return fail(HEGET_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
    }
  }
  *out = p;
  return HEGET_OK;
}

heget_status heget_process_destroy(heget_process_t p) {
  g_err.clear();
  if (!p) return fail(HEGET_E_INVALID, "null handle");
  (void)hipDeviceSynchronize();
  release(p);
  return HEGET_OK;
}

int32_t heget_process_n_helicities(heget_process_t p) { return p ? p->n_hel : -1; }

heget_status heget_eval(heget_process_t p, int64_t n, const double* momenta_in, uint64_t seed,
                        uint64_t counter_offset, double sqrt_s, double* me2_out, double* momenta_out,
                        void* stream) {
  g_err.clear();
  if (!p) return fail(HEGET_E_INVALID, "null handle");
  if (n < 0) return fail(HEGET_E_INVALID, "n < 0");
  if (!momenta_in && !(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0 when generating momenta");
  KernelArgs a = base_args(p);
  a.n = n;
  a.mom_in = momenta_in;
  a.mom_stride = n;
  a.seed = seed;
  a.counter_offset = counter_offset;
  a.sqrt_s = sqrt_s;
  a.me2_out = me2_out;
  a.mom_out = momenta_out;
  return launch(p, a, static_cast<hipStream_t>(stream));
}

heget_status heget_generate(heget_process_t p, int64_t n, uint64_t seed, uint64_t counter_offset, double sqrt_s,
                            double* momenta_out, double* weights_out, void* stream) {
  g_err.clear();
  if (!p) return fail(HEGET_E_INVALID, "null handle");
  if (n < 0) return fail(HEGET_E_INVALID, "n < 0");
  if (!(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0");
  if (n > 0 && !momenta_out) return fail(HEGET_E_INVALID, "null momenta_out");
  const void* fn = p->entry->generate;   // the process's resonance tree, else RAMBO by final-state count
  if (!fn) switch (p->n_legs - 2) {
    case 2: fn = generate_kernel<2>(); break;
    case 3: fn = generate_kernel<3>(); break;
    case 4: fn = generate_kernel<4>(); break;
    case 5: fn = generate_kernel<5>(); break;
    case 6: fn = generate_kernel<6>(); break;
    case 7: fn = generate_kernel<7>(); break;
    case 8: fn = generate_kernel<8>(); break;
    case 9: fn = generate_kernel<9>(); break;
    case 10: fn = generate_kernel<10>(); break;
    default: return fail(HEGET_E_UNSUPPORTED, "generation supports 2..10 final-state legs");
  }
  if (n == 0) return HEGET_OK;
  const int64_t grid = (n + 255) / 256;
  if (grid > 0x7fffffff) return fail(HEGET_E_INVALID, "n too large for one launch");
  KernelArgs a = base_args(p);
  a.n = n;
  a.mom_stride = n;
  a.seed = seed;
  a.counter_offset = counter_offset;
  a.sqrt_s = sqrt_s;
  a.mom_out = momenta_out;
  a.psw_out = weights_out;
  a.weight_factor = heget::detail::phase_space_volume(sqrt_s, p->n_legs - 2);
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(256), args, 0, static_cast<hipStream_t>(stream)));
  return HEGET_OK;
}

heget_status heget_uniforms(uint64_t seed, uint64_t counter_offset, int64_t n, int32_t n_u, double* u_out,
                            void* stream) {
  g_err.clear();
  if (n < 0 || n_u < 1 || n_u > 64) return fail(HEGET_E_INVALID, "need n >= 0 and 1 <= n_u <= 64");
  if (n == 0) return HEGET_OK;
  if (!u_out) return fail(HEGET_E_INVALID, "null u_out");
  const int64_t grid = (n + 255) / 256;
  if (grid > 0x7fffffff) return fail(HEGET_E_INVALID, "n too large for one launch");
  hipLaunchKernelGGL(uniforms_kernel, dim3(unsigned(grid)), dim3(256), 0, static_cast<hipStream_t>(stream), seed,
                     counter_offset, n, int(n_u), u_out);
  HIP_TRY(hipGetLastError());
  return HEGET_OK;
}

namespace {
// Wait for the stream: poll it for up to 200 us before a blocking wait.  An
// integrate step's result is usually that close, and waking from a blocking
// wait takes longer than the poll.
hipError_t wait_stream(hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t q;
  while ((q = hipStreamQuery(st)) == hipErrorNotReady)
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200)) return hipStreamSynchronize(st);
  return q;
}
}  // namespace

namespace {
// One integrate step enqueued on st: the amplitude kernel writes per-block
// partial sums into the handle's buffer (grown, after a wait for st, when a
// larger n arrives) and the fixed-order reduction writes its three sums to
// `sums` (device memory or pinned host memory).  Does not wait for st.
heget_status enqueue_integrate(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, double* sums,
                               hipStream_t st) {
  const int64_t nblocks = (n + 255) / 256;
  if (p->part_cap < nblocks * 3 + 3) {
    HIP_TRY(hipStreamSynchronize(st));
    if (p->d_part) (void)hipFree(p->d_part);
    p->d_part = nullptr;
    p->part_cap = 0;
    if (hipMalloc(&p->d_part, size_t(nblocks * 3 + 3) * sizeof(double)) != hipSuccess)
      return fail(HEGET_E_OOM, "partials allocation failed");
    p->part_cap = nblocks * 3 + 3;
  }
  KernelArgs a = base_args(p);
  a.n = n;
  a.mom_stride = n;
  a.seed = seed;
  a.sqrt_s = sqrt_s;
  a.weight_factor = heget::detail::weight_factor(p, sqrt_s);
  a.partials = p->d_part;
  heget_status rc = launch(p, a, st);
  if (rc != HEGET_OK) return rc;
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, st, p->d_part, nblocks, sums);
  HIP_TRY(hipGetLastError());
  return HEGET_OK;
}

heget_status check_integrate_args(heget_process_t p, int64_t n, double sqrt_s, const void* out) {
  if (!p || !out) return fail(HEGET_E_INVALID, "null argument");
  if (n < 2) return fail(HEGET_E_INVALID, "need n >= 2 events");
  if (!(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0");
  return HEGET_OK;
}
}  // namespace

heget_status heget_integrate(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, heget_result* out,
                             void* stream) {
  g_err.clear();
  heget_status rc = check_integrate_args(p, n, sqrt_s, out);
  if (rc != HEGET_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!p->h_res && hipHostMalloc(reinterpret_cast<void**>(&p->h_res), 3 * sizeof(double), hipHostMallocDefault) !=
                       hipSuccess) {
    p->h_res = nullptr;
    return fail(HEGET_E_OOM, "pinned result allocation failed");
  }
  // the reduction writes its three sums straight into the pinned result
  // buffer (host memory the device can write): no separate copy back
  rc = enqueue_integrate(p, n, sqrt_s, seed, p->h_res, st);
  if (rc != HEGET_OK) return rc;
  const hipError_t e = wait_stream(st);
  if (e != hipSuccess) return fail(HEGET_E_HIP, std::string("integrate: ") + hipGetErrorString(e));
  heget::detail::fill_result(p->h_res, n, out);
  return HEGET_OK;
}

heget_status heget_integrate_async(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, double* sums_out,
                                   void* stream) {
  g_err.clear();
  const heget_status rc = check_integrate_args(p, n, sqrt_s, sums_out);
  if (rc != HEGET_OK) return rc;
  // the reduction writes sums_out from the device: refuse pageable host memory
  // (unregistered with HIP) before anything is launched
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, sums_out) != hipSuccess || attr.type == hipMemoryTypeUnregistered) {
    (void)hipGetLastError();
    return fail(HEGET_E_INVALID, "sums_out must be device memory or pinned host memory");
  }
  return enqueue_integrate(p, n, sqrt_s, seed, sums_out, static_cast<hipStream_t>(stream));
}

heget_status heget_result_from_sums(const double* sums, int64_t n, heget_result* out) {
  g_err.clear();
  if (!sums || !out) return fail(HEGET_E_INVALID, "null argument");
  if (n < 2) return fail(HEGET_E_INVALID, "need n >= 2 events");
  heget::detail::fill_result(sums, n, out);
  return HEGET_OK;
}

heget_status heget_integrate_noalloc(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, heget_result* out,
                                     void* stream) {
  g_err.clear();
  if (!p || !out) return fail(HEGET_E_INVALID, "null argument");
  if (n < 2) return fail(HEGET_E_INVALID, "need n >= 2 events");
  if (n > HEGET_NOALLOC_MAX_EVENTS)
    return fail(HEGET_E_INVALID, "n = " + std::to_string(n) + " exceeds the no-allocation limit of " +
                                     std::to_string(int64_t(HEGET_NOALLOC_MAX_EVENTS)) + " events");
  if (!(sqrt_s > 0)) return fail(HEGET_E_INVALID, "sqrt_s must be > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* d_part = nullptr;
  HIP_TRY(scratch_address(&d_part));
  const int64_t nblocks = (n + 255) / 256;
  // every block writes its own partial triple and the reduction its three sums:
  // nothing in the scratch has to start at zero
  KernelArgs a = base_args(p);
  a.n = n;
  a.mom_stride = n;
  a.seed = seed;
  a.sqrt_s = sqrt_s;
  a.weight_factor = heget::detail::weight_factor(p, sqrt_s);
  a.partials = d_part;
  heget_status rc = launch(p, a, st);
  double h[3] = {0.0, 0.0, 0.0};
  if (rc == HEGET_OK) {
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, st, d_part, nblocks, d_part + 3 * nblocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, d_part + 3 * nblocks, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(HEGET_E_HIP, std::string("integrate_noalloc: ") + hipGetErrorString(e));
  }
  if (rc != HEGET_OK) return rc;
  heget::detail::fill_result(h, n, out);
  return HEGET_OK;
}

heget_status heget_filter_helicities(heget_process_t p, int64_t n_probe, uint64_t seed, double sqrt_s,
                                     double rel_threshold, int32_t* n_kept) {
  g_err.clear();
  if (!p || !n_kept) return fail(HEGET_E_INVALID, "null argument");
  if (n_probe < 1 || !(sqrt_s > 0) || !(rel_threshold >= 0)) return fail(HEGET_E_INVALID, "bad probe arguments");
  const int nh = p->n_hel, nl = p->n_legs;
  double* d_me2 = nullptr;
  if (hipMalloc(&d_me2, size_t(nh) * n_probe * sizeof(double)) != hipSuccess)
    return fail(HEGET_E_OOM, "probe allocation failed");
  heget_status rc = HEGET_OK;
  for (int h = 0; h < nh && rc == HEGET_OK; ++h) {
    KernelArgs a = base_args(p);
    a.hel = p->d_hel + size_t(h) * nl;
    a.n_hel = 1;
    a.hel_nest = 0;
    a.n = n_probe;
    a.mom_stride = n_probe;
    a.seed = seed;
    a.sqrt_s = sqrt_s;
    a.me2_out = d_me2 + size_t(h) * n_probe;
    rc = launch(p, a, nullptr);
  }
  std::vector<double> me(size_t(nh) * n_probe);
  if (rc == HEGET_OK && (hipMemcpy(me.data(), d_me2, me.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
    rc = fail(HEGET_E_HIP, "probe copy failed");
  (void)hipFree(d_me2);
  if (rc != HEGET_OK) return rc;
  std::vector<int8_t> kept;
  int nk = 0;
  for (int h = 0; h < nh; ++h) {
    bool keep = false;
    for (int64_t e = 0; e < n_probe && !keep; ++e) {
      double mx = 0.0;
      for (int g = 0; g < nh; ++g) mx = std::max(mx, me[size_t(g) * n_probe + e]);
      keep = me[size_t(h) * n_probe + e] > rel_threshold * mx;
    }
    if (keep) {
      kept.insert(kept.end(), p->hel.begin() + size_t(h) * nl, p->hel.begin() + size_t(h + 1) * nl);
      ++nk;
    }
  }
  if (nk == 0) return fail(HEGET_E_INVALID, "every helicity vanished on the probe events");
  if (hipMemcpy(p->d_hel, kept.data(), kept.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(HEGET_E_HIP, "helicity table upload failed");
  p->hel = kept;
  p->n_hel = nk;
  p->hel_nest = heget::detail::is_full_product(p->entry, kept.data(), nk, nl) ? 1 : 0;
  *n_kept = nk;
  return HEGET_OK;
}

}  // extern "C"
