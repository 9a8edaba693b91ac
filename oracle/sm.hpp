// Oracle: Standard Model couplings in the oracle's own conventions, and SU(3)
// colour generators.  Test infrastructure only.
//
// Conventions (textbook, unitary gauge):
//   L_f  = -e Q fbar A f - g_Z fbar Zslash (T3 P_L - Q s_W^2) f
//          - (g_W / sqrt2) (ubar Wslash+ P_L d + h.c.)
//   L_h  = g_W m_W H W+.W- + (g_Z m_Z / 2) H Z.Z + (g_W^2/4) H^2 W+.W-
//          + (g_Z^2/8) H^2 Z.Z - lambda v H^3 - (lambda / 4) H^4 - (m_b / v) H bbar b
//   QCD  : Peskin-Schroeder sign conventions, D = d - i g_s A^a T^a.
// (The paper's HELAS couplings differ from these by field-sign conventions that
//  cancel in |M|^2.)  Feynman rule = i x coefficient x identical-field factor.
#pragma once
#include <cmath>
#include <complex>

#include "dirac.hpp"
#include "oracle.h"

namespace orc {

struct SM {
  real e, sw2, sw, cw, gw, gz, gs;
  real mz, wz, mw, ww, mt, wt, mh, wh, mb_yuk, v;
  cd muw2, muz2;        // complex masses squared (propagator poles)
  cd numw2, numz2;      // masses squared in the unitary-gauge numerator
  cd g_wwh, g_zzh;      // Feynman rule / i for W+W-H and ZZH (metric tensor stripped)
  real g_wwhh, g_zzhh, g_hhh, g_hhhh, y_b;
  int gauge_leg;
  explicit SM(const or_params& p) {
    e = std::sqrt(4.0 * PI * p.alpha);
    sw2 = p.sw2;
    sw = std::sqrt(sw2);
    cw = std::sqrt(1.0 - sw2);
    gw = e / sw;
    gz = e / (sw * cw);
    gs = std::sqrt(4.0 * PI * p.alpha_s);
    mz = p.mz;
    wz = p.wz;
    if (p.cms) {
      // mu_W^2 = c_W^2 mu_Z^2  =>  m_W = c_W m_Z, Gamma_W = c_W Gamma_Z
      mw = cw * mz;
      ww = cw * wz;
    } else {
      mw = p.mw;
      ww = p.ww;
    }
    mt = p.mt;
    wt = p.wt;
    mh = p.mh;
    wh = p.wh;
    mb_yuk = p.mb_yuk;
    muw2 = cd(mw * mw, -mw * ww);
    muz2 = cd(mz * mz, -mz * wz);
    numw2 = p.cms ? muw2 : cd(mw * mw, 0.0);
    numz2 = p.cms ? muz2 : cd(mz * mz, 0.0);
    const cd muw = p.cms ? std::sqrt(muw2) : cd(mw, 0.0);
    const cd muz = p.cms ? std::sqrt(muz2) : cd(mz, 0.0);
    v = 2.0 * mw / gw;
    g_wwh = gw * muw;              // from g_W m_W H W+.W-
    g_zzh = gz * muz;              // 2 x (g_Z m_Z / 2)
    g_wwhh = 0.5 * gw * gw;        // 2 x g_W^2/4
    g_zzhh = 0.5 * gz * gz;        // 2 x 2 x g_Z^2/8
    g_hhh = -3.0 * mh * mh / v;    // -3! lambda v with m_H^2 = 2 lambda v^2
    g_hhhh = -3.0 * mh * mh / (v * v);   // -4! lambda / 4 from the (lambda / 4) H^4 term
    y_b = mb_yuk / v;
    gauge_leg = p.gauge_leg;
  }
  // fermion couplings to neutral bosons: coefficient of fbar gamma^mu P_{L,R} f V_mu
  real gl_z(real t3, real q) const { return -gz * (t3 - q * sw2); }
  real gr_z(real q) const { return gz * q * sw2; }
  real g_a(real q) const { return -e * q; }
  real g_w() const { return -gw / std::sqrt(real(2)); }
};

// SU(3) generators T^a = lambda^a / 2 and structure constants
// f^{abc} = -2 i Tr([T^a, T^b] T^c).
struct Colour {
  cd T[8][3][3];
  real f[8][8][8];
  Colour() {
    for (auto& a : T)
      for (auto& r : a)
        for (auto& x : r) x = 0.0;
    const real h = 0.5;
    T[0][0][1] = h; T[0][1][0] = h;
    T[1][0][1] = -h * I1; T[1][1][0] = h * I1;
    T[2][0][0] = h; T[2][1][1] = -h;
    T[3][0][2] = h; T[3][2][0] = h;
    T[4][0][2] = -h * I1; T[4][2][0] = h * I1;
    T[5][1][2] = h; T[5][2][1] = h;
    T[6][1][2] = -h * I1; T[6][2][1] = h * I1;
    const real r3 = 1 / std::sqrt(real(3));
    T[7][0][0] = h * r3; T[7][1][1] = h * r3; T[7][2][2] = -2.0 * h * r3;
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int c = 0; c < 8; ++c) {
          cd tr = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int k = 0; k < 3; ++k)
                tr += (T[a][i][j] * T[b][j][k] - T[b][i][j] * T[a][j][k]) * T[c][k][i];
          f[a][b][c] = std::real(real(-2) * I1 * tr);
        }
  }
};
const Colour& colour();

}  // namespace orc
