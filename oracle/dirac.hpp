// Oracle (test infrastructure only): plain FP64 Dirac/Lorentz algebra.
//
// Nothing here is used by the product library; only tests, the smoke check and
// the CPU-baseline leg of the benchmark may load the oracle.
//
// Everything is written out with explicit 4x4 matrices in the Dirac-Pauli
// representation (deliberately not the chiral basis the product uses), so that
// a mistake in the product's spinor or vertex algebra cannot be mirrored here.
// Metric (+,-,-,-).  All momenta are physical (positive energy) unless stated.
#pragma once
#include <array>
#include <cmath>
#include <complex>
#include <vector>

// The arithmetic type: double, or (for the extended-precision reference build
// of the same sources) long double, chosen with -DORC_REAL=...
#ifndef ORC_REAL
#define ORC_REAL double
#endif

namespace orc {

using real = ORC_REAL;
using cd = std::complex<real>;
static const cd I1(0.0, 1.0);
static const real PI = 3.14159265358979323846264338327950288L;

using Vec4 = std::array<real, 4>;   // real contravariant four-vector (E, px, py, pz)
using CVec4 = std::array<cd, 4>;      // complex contravariant four-vector
using Spinor = std::array<cd, 4>;     // Dirac spinor (column) or adjoint spinor (row)

struct Mat4 {
  cd m[4][4];
};

inline real metric(int mu) { return mu == 0 ? 1.0 : -1.0; }

inline Vec4 add(const Vec4& a, const Vec4& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2], a[3] + b[3]}; }
inline Vec4 sub(const Vec4& a, const Vec4& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2], a[3] - b[3]}; }
inline Vec4 neg(const Vec4& a) { return {-a[0], -a[1], -a[2], -a[3]}; }
inline real dot(const Vec4& a, const Vec4& b) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
inline cd dot(const CVec4& a, const CVec4& b) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
inline cd dot(const CVec4& a, const Vec4& b) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
inline CVec4 cvec(const Vec4& a) { return {a[0], a[1], a[2], a[3]}; }
inline CVec4 cadd(const CVec4& a, const CVec4& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2], a[3] + b[3]}; }
inline CVec4 cscale(cd s, const CVec4& a) { return {s * a[0], s * a[1], s * a[2], s * a[3]}; }
inline CVec4 conjv(const CVec4& a) { return {std::conj(a[0]), std::conj(a[1]), std::conj(a[2]), std::conj(a[3])}; }

// ---------------------------------------------------------------- matrices
inline Mat4 zero4() {
  Mat4 r;
  for (auto& row : r.m)
    for (auto& x : row) x = 0.0;
  return r;
}
inline Mat4 ident4() {
  Mat4 r = zero4();
  for (int i = 0; i < 4; ++i) r.m[i][i] = 1.0;
  return r;
}
inline Mat4 mul(const Mat4& a, const Mat4& b) {
  Mat4 r = zero4();
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) r.m[i][j] += a.m[i][k] * b.m[k][j];
  return r;
}
inline Mat4 madd(const Mat4& a, const Mat4& b) {
  Mat4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.m[i][j] = a.m[i][j] + b.m[i][j];
  return r;
}
inline Mat4 mscale(cd s, const Mat4& a) {
  Mat4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.m[i][j] = s * a.m[i][j];
  return r;
}
inline Spinor mv(const Mat4& a, const Spinor& s) {
  Spinor r{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r[i] += a.m[i][j] * s[j];
  return r;
}
// row spinor times matrix
inline Spinor vm(const Spinor& r, const Mat4& a) {
  Spinor o{};
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) o[j] += r[i] * a.m[i][j];
  return o;
}
inline cd sandwich(const Spinor& row, const Spinor& col) {
  cd s = 0.0;
  for (int i = 0; i < 4; ++i) s += row[i] * col[i];
  return s;
}
inline cd trace(const Mat4& a) { return a.m[0][0] + a.m[1][1] + a.m[2][2] + a.m[3][3]; }

// Dirac-Pauli representation: gamma^0 = diag(1,1,-1,-1),
// gamma^k = [[0, sigma^k], [-sigma^k, 0]], gamma5 = i g0 g1 g2 g3.
struct Gammas {
  Mat4 g[4];
  Mat4 g5, pl, pr, one;
  Gammas() {
    const cd s[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}},
                           {{0.0, -I1}, {I1, 0.0}},
                           {{1.0, 0.0}, {0.0, -1.0}}};
    g[0] = zero4();
    g[0].m[0][0] = g[0].m[1][1] = 1.0;
    g[0].m[2][2] = g[0].m[3][3] = -1.0;
    for (int k = 0; k < 3; ++k) {
      g[k + 1] = zero4();
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          g[k + 1].m[a][b + 2] = s[k][a][b];
          g[k + 1].m[a + 2][b] = -s[k][a][b];
        }
    }
    g5 = mscale(I1, mul(mul(g[0], g[1]), mul(g[2], g[3])));
    one = ident4();
    pl = mscale(0.5, madd(one, mscale(-1.0, g5)));
    pr = mscale(0.5, madd(one, g5));
  }
};
const Gammas& gam();

// a-slash = gamma^mu a_mu (lower index: a_0 = a^0, a_k = -a^k)
inline Mat4 slash(const CVec4& a) {
  const Gammas& G = gam();
  Mat4 r = zero4();
  for (int mu = 0; mu < 4; ++mu) r = madd(r, mscale(a[mu] * metric(mu), G.g[mu]));
  return r;
}
inline Mat4 slash(const Vec4& a) { return slash(cvec(a)); }

// Dirac adjoint of a column spinor: psi^dagger gamma^0 (as a row)
inline Spinor dbar(const Spinor& s) {
  Spinor c{};
  for (int i = 0; i < 4; ++i) c[i] = std::conj(s[i]);
  return vm(c, gam().g[0]);
}

// ------------------------------------------------------- external states
// Two-component helicity eigenstates along direction (theta, phi):
// (sigma . n) chi_lam = lam chi_lam, lam = +1 / -1.
inline std::array<cd, 2> chi(const Vec4& p, int lam) {
  real pp = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  real th = std::atan2(std::sqrt(p[1] * p[1] + p[2] * p[2]), p[3]);
  real ph = std::atan2(p[2], p[1]);
  (void)pp;
  real c = std::cos(0.5 * th), s = std::sin(0.5 * th);
  if (lam > 0) return {cd(c, 0.0), std::exp(I1 * ph) * s};
  return {-std::exp(-I1 * ph) * s, cd(c, 0.0)};
}

// Fermion spinor u(p, lam) in the Dirac-Pauli representation:
// u = ( sqrt(E+m) chi ; lam sqrt(E-m) chi ), since sigma.p chi = lam |p| chi.
inline Spinor u_spinor(const Vec4& p, real m, int lam) {
  real pp = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  real E = std::sqrt(pp * pp + m * m);
  auto x = chi(p, lam);
  real a = std::sqrt(E + m), b = lam * std::sqrt(std::max(E - m, real(0)));
  return {a * x[0], a * x[1], b * x[0], b * x[1]};
}
// Antifermion spinor by charge conjugation: v(p, lam) = i gamma^2 u(p, lam)^*
inline Spinor v_spinor(const Vec4& p, real m, int lam) {
  Spinor u = u_spinor(p, m, lam);
  Spinor uc{};
  for (int i = 0; i < 4; ++i) uc[i] = std::conj(u[i]);
  return mv(mscale(I1, gam().g[2]), uc);
}

// Polarisation vector epsilon^mu(k, lam): transverse lam = +-1 are
// (1/sqrt2)(-lam e1 - i e2) with e1 = (0, cos th cos ph, cos th sin ph, -sin th),
// e2 = (0, -sin ph, cos ph, 0); lam = 0 is longitudinal (|k|, E khat)/m.
// lam = 4 is the gauge-check vector k^mu / k^0; lam = 10 + alpha is the
// contravariant unit vector along axis alpha (for covariant polarisation sums).
inline CVec4 eps_vec(const Vec4& k, real m, int lam) {
  if (lam == 4) return {1.0, k[1] / k[0], k[2] / k[0], k[3] / k[0]};
  if (lam >= 10 && lam < 14) {
    CVec4 e{};
    e[lam - 10] = 1.0;
    return e;
  }
  real kt = std::sqrt(k[1] * k[1] + k[2] * k[2]);
  real kk = std::sqrt(kt * kt + k[3] * k[3]);
  real th = std::atan2(kt, k[3]), ph = std::atan2(k[2], k[1]);
  if (lam == 0) {
    real E = std::sqrt(kk * kk + m * m);
    return {kk / m, E / m * std::sin(th) * std::cos(ph), E / m * std::sin(th) * std::sin(ph), E / m * std::cos(th)};
  }
  Vec4 e1 = {0.0, std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th)};
  Vec4 e2 = {0.0, -std::sin(ph), std::cos(ph), 0.0};
  const real r = 1 / std::sqrt(real(2));
  CVec4 e;
  for (int mu = 0; mu < 4; ++mu) e[mu] = r * (-real(lam) * e1[mu] - I1 * e2[mu]);
  return e;
}

// ----------------------------------------------------------- propagators
// Each returns the Feynman-rule factor including its explicit i.
// Fermion: i (pslash + m) / (p^2 - m^2 + i m Gamma), p along the fermion arrow.
inline Mat4 fermion_prop(const Vec4& p, real m, real w) {
  cd den = dot(p, p) - m * m + I1 * m * w;
  return mscale(I1 / den, madd(slash(p), mscale(m, ident4())));
}
// Massive vector, unitary gauge: -i (g^{mu nu} - q^mu q^nu / num2) / (q^2 - pole2)
// with pole2 = m^2 - i m Gamma; num2 = m^2 (fixed width) or pole2 (complex mass).
// Returned as a contravariant tensor T^{mu nu}; contract with lower-index vectors.
struct Tens {
  cd t[4][4];
};
inline Tens vector_prop(const Vec4& q, cd num2, cd pole2) {
  Tens r;
  cd den = dot(q, q) - pole2;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      cd g = (a == b) ? cd(metric(a), 0.0) : cd(0.0, 0.0);
      r.t[a][b] = -I1 * (g - q[a] * q[b] / num2) / den;
    }
  return r;
}
// Massless vector, Feynman gauge: -i g^{mu nu} / q^2
inline Tens massless_prop(const Vec4& q) {
  Tens r;
  real den = dot(q, q);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) r.t[a][b] = (a == b) ? -I1 * metric(a) / den : cd(0.0, 0.0);
  return r;
}
// T^{mu nu} x_nu with the metric applied to the contracted index
inline CVec4 contract(const Tens& T, const CVec4& x) {
  CVec4 r{};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) r[a] += T.t[a][b] * metric(b) * x[b];
  return r;
}
// Scalar: i / (q^2 - m^2 + i m Gamma)
inline cd scalar_prop(const Vec4& q, real m, real w) { return I1 / (dot(q, q) - m * m + I1 * m * w); }

// Spinor current  row gamma^mu Gamma col  as a contravariant vector
inline CVec4 current(const Spinor& row, const Mat4& chiral, const Spinor& col) {
  const Gammas& G = gam();
  CVec4 j;
  Spinor c = mv(chiral, col);
  for (int mu = 0; mu < 4; ++mu) j[mu] = sandwich(row, mv(G.g[mu], c));
  return j;
}

}  // namespace orc
