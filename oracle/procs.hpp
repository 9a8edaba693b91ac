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
double me2_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm, const Vec4* p,
                        const int* h);
double trace_me2(int id, const SM& sm, const Vec4* p);
void condition_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm,
                            const Vec4* p, const int* h, double& a2, double& b2);

// n-gluon Berends-Giele
double gluon_me2(int n, const SM& sm, const Vec4* p);
cd gluon_partial(int n, const SM& sm, const Vec4* p, const int* hel, const int* order);
const std::vector<double>& gluon_colour_matrix(int n);
std::vector<double> fierz_colour_matrix(int n);

}  // namespace orc
