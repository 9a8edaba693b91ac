// Oracle: C entry points.  Test infrastructure only.
#include <cstring>
#include <vector>

#include "oracle.h"
#include "procs.hpp"

#ifdef _OPENMP
#include <omp.h>
#endif

using namespace orc;

namespace {
int gluon_count(int proc) {
  switch (proc) {
    case OR_GG_GG: return 4;
    case OR_GG_GGG: return 5;
    case OR_GG_4G: return 6;
    case OR_GG_5G: return 7;
    default: return 0;
  }
}
// 1 + the number of gluons of a u ubar -> t tbar + gluons process, else 0
int uu_tt_count(int proc) {
  switch (proc) {
    case OR_UU_TT_DIAG: return 1;
    case OR_UU_TTG: return 2;
    case OR_UU_TTGG: return 3;
    case OR_UU_TTGGG: return 4;
    default: return 0;
  }
}
void load(const double* mom, int nl, Vec4* p) {
  for (int k = 0; k < nl; ++k)
    for (int m = 0; m < 4; ++m) p[k][m] = mom[4 * k + m];
}
}  // namespace

extern "C" int or_nlegs(int proc) {
  if (int n = gluon_count(proc)) return n;
  if (int k = uu_tt_count(proc)) return 3 + k;
  const ProcDef* P = find_proc(proc);
  return P ? P->nlegs : -1;
}

extern "C" int or_eval(int proc, const or_params* prm, int64_t n_events, const double* mom, double* me2,
                       int n_threads) {
  const SM sm(*prm);
  if (int k = uu_tt_count(proc)) {
    const int ngl = k - 1;
    uu_tt_gluons_me2(ngl, sm, nullptr);   // builds the diagrams and the colour matrix once
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_events; ++i) {
      Vec4 p[8];
      load(mom + i * (4 + ngl) * 4, 4 + ngl, p);
      me2[i] = double(uu_tt_gluons_me2(ngl, sm, p));
    }
    return 0;
  }
  const int ng = gluon_count(proc);
  const ProcDef* P = ng ? nullptr : find_proc(proc);
  if (!ng && !P) return -1;
  const int nl = ng ? ng : P->nlegs;
  if (ng) gluon_colour_matrix(ng);
  const std::vector<std::vector<cd>>* C = P ? &colour_assignments(proc, *P) : nullptr;
  const auto hels = P ? helicity_table(*P) : std::vector<std::vector<int>>{};
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_events; ++i) {
    Vec4 p[16];
    load(mom + i * nl * 4, nl, p);
    if (ng) {
      me2[i] = gluon_me2(ng, sm, p);
    } else {
      real s = 0.0;
      for (const auto& h : hels) s += me2_one_helicity(*P, *C, sm, p, h.data());
      me2[i] = double(s);
    }
  }
  return 0;
}

extern "C" int or_condition(int proc, const or_params* prm, int64_t n_events, const double* mom, double* kappa,
                            int n_threads) {
  const SM sm(*prm);
  const ProcDef* P = find_proc(proc);
  if (!P) return -1;
  const auto& C = colour_assignments(proc, *P);
  const auto hels = helicity_table(*P);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_events; ++i) {
    Vec4 p[16];
    load(mom + i * P->nlegs * 4, P->nlegs, p);
    real a2 = 0.0, b2 = 0.0;
    for (const auto& h : hels) condition_one_helicity(*P, C, sm, p, h.data(), a2, b2);
    kappa[i] = double(std::sqrt(b2 / a2));
  }
  return 0;
}

extern "C" int or_amp_colour(int proc, const or_params* prm, const double* mom, const int* hel, const int* col,
                             double* out) {
  const ProcDef* P = find_proc(proc);
  if (!P) return -1;
  const SM sm(*prm);
  Vec4 p[16];
  load(mom, P->nlegs, p);
  std::vector<cd> M(P->ndiag), c(P->ndiag);
  P->amp(sm, p, hel, M.data());
  P->colf(col, c.data());
  cd s = 0;
  for (int d = 0; d < P->ndiag; ++d) s += c[d] * M[d];
  out[0] = s.real();
  out[1] = s.imag();
  return 0;
}

extern "C" int or_helicities(int proc, int* table) {
  const ProcDef* P = find_proc(proc);
  if (!P) return -1;
  const auto hels = helicity_table(*P);
  if (table)
    for (size_t k = 0; k < hels.size(); ++k)
      for (int l = 0; l < P->nlegs; ++l) table[k * P->nlegs + l] = hels[k][l];
  return int(hels.size());
}

extern "C" int or_me2_per_helicity(int proc, const or_params* prm, const double* mom, double* out) {
  const ProcDef* P = find_proc(proc);
  if (!P) return -1;
  const SM sm(*prm);
  Vec4 p[16];
  load(mom, P->nlegs, p);
  const auto& C = colour_assignments(proc, *P);
  const auto hels = helicity_table(*P);
  for (size_t k = 0; k < hels.size(); ++k) out[k] = me2_one_helicity(*P, C, sm, p, hels[k].data());
  return int(hels.size());
}

extern "C" int or_me2_hel(int proc, const or_params* prm, const double* mom, const int* hel, double* out) {
  const ProcDef* P = find_proc(proc);
  if (!P) return -1;
  const SM sm(*prm);
  Vec4 p[16];
  load(mom, P->nlegs, p);
  out[0] = me2_one_helicity(*P, colour_assignments(proc, *P), sm, p, hel);
  return 0;
}

extern "C" int or_gluon_partial(int n, const or_params* prm, const double* mom, const int* hel, const int* order,
                                double* out) {
  if (n < 4 || n > 7) return -1;
  const SM sm(*prm);
  Vec4 p[16];
  load(mom, n, p);
  const cd a = gluon_partial(n, sm, p, hel, order);
  out[0] = a.real();
  out[1] = a.imag();
  return 0;
}

extern "C" int or_uu_tt_gluons_diagrams(int ng) { return ng < 0 || ng > 3 ? -1 : uu_tt_gluons_diagrams(ng); }

extern "C" int or_gluon_colour_matrix(int n, double* C) {
  if (n < 3 || n > 6) return -1;
  const std::vector<real>& M = gluon_colour_matrix(n);
  std::copy(M.begin(), M.end(), C);
  return int(M.size());
}

extern "C" int or_gluon_colour_matrix_fierz(int n, double* C) {
  if (n < 3 || n > 8) return -1;
  const std::vector<real> M = fierz_colour_matrix(n);
  std::copy(M.begin(), M.end(), C);
  return 0;
}

extern "C" int or_trace_me2(int proc, const or_params* prm, const double* mom, double* out) {
  const SM sm(*prm);
  Vec4 p[4];
  load(mom, 4, p);
  out[0] = trace_me2(proc, sm, p);
  return out[0] < 0 ? -1 : 0;
}

extern "C" int or_decay_width(int which, const or_params* prm, double* out) {
  const SM sm(*prm);
  out[0] = double(decay_width(sm, which));
  return out[0] < 0 ? -1 : 0;
}

extern "C" double or_selfcheck_spinors(const double* pin, double m) {
  // Dirac equation, completeness and helicity eigenvalue checks for one momentum
  Vec4 p = {pin[0], pin[1], pin[2], pin[3]};
  const Mat4 ps = slash(p);
  const Mat4 mm = mscale(m, ident4());
  real worst = 0.0;
  const real scale = p[0] + 1;
  Mat4 su = zero4(), sv = zero4();
  for (int lam : {-1, 1}) {
    const Spinor u = u_spinor(p, m, lam), v = v_spinor(p, m, lam);
    const Spinor du = mv(madd(ps, mscale(-1.0, mm)), u);   // (pslash - m) u = 0
    const Spinor dv = mv(madd(ps, mm), v);                  // (pslash + m) v = 0
    for (int i = 0; i < 4; ++i) worst = std::max(worst, std::max(std::abs(du[i]), std::abs(dv[i])) / scale);
    const Spinor ub = dbar(u), vb = dbar(v);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        su.m[i][j] += u[i] * ub[j];
        sv.m[i][j] += v[i] * vb[j];
      }
  }
  const Mat4 eu = madd(su, mscale(-1.0, madd(ps, mm)));   // sum u ubar - (pslash + m)
  const Mat4 ev = madd(sv, mscale(-1.0, madd(ps, mscale(-1.0, mm))));
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) worst = std::max(worst, std::max(std::abs(eu.m[i][j]), std::abs(ev.m[i][j])) / scale);
  return worst;
}
