// Oracle: process descriptors shared by the oracle's translation units.
// Test infrastructure only.
#pragma once
#include <vector>

#include "dirac.hpp"
#include "sm.hpp"

namespace orc {

struct ProcDef {
  int nlegs;
  std::vector<std::vector<int>> helvals;  // allowed helicities per leg
  int ndiag;
  std::vector<int> coldim;                // 1, 3 or 8 per leg
  void (*amp)(const SM&, const Vec4*, const int*, cd*);   // colour-stripped M_d
  void (*colf)(const int*, cd*);                          // colour factor c_d
};

const ProcDef* find_proc(int id);
const std::vector<cd>& colour_matrix(int id, const ProcDef& P);
std::vector<std::vector<int>> helicity_table(const ProcDef& P);
const std::vector<std::vector<cd>>& colour_assignments(int id, const ProcDef& P);
real me2_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm, const Vec4* p,
                        const int* h);
real trace_me2(int id, const SM& sm, const Vec4* p);
real decay_width(const SM& sm, int which);
void condition_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm,
                            const Vec4* p, const int* h, real& a2, real& b2);

// n-gluon Berends-Giele
real gluon_me2(int n, const SM& sm, const Vec4* p);
cd gluon_partial(int n, const SM& sm, const Vec4* p, const int* hel, const int* order);
const std::vector<real>& gluon_colour_matrix(int n);
std::vector<real> fierz_colour_matrix(int n);

// u ubar -> t tbar + n gluons by Feynman diagrams (quark_lines.cpp)
real uu_tt_gluons_me2(int ng, const SM& sm, const Vec4* p);
int uu_tt_gluons_diagrams(int ng);

}  // namespace orc
