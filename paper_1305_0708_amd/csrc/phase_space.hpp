// Counter-based uniforms, RAMBO momenta and the gluon generation cut (device).
//
// Philox4x32-10 follows its published definition (Salmon et al., SC'11): ten
// rounds of two 32x32->64-bit products with the Weyl key schedule; each product
// is one 64-bit multiply and each round's two three-way xors one gfx950
// three-input bit instruction each.  Counter
// layout per event i: (i_lo, i_hi, block j, 0), key (seed_lo, seed_hi); each
// block gives two uniforms u = (floor(x / 2^12) + 1/2) 2^-52 from the 64-bit
// words x = w0 2^32 + w1 and x = w2 2^32 + w3 (exact in FP64, strictly inside
// (0,1)).  RAMBO (Kleiss, Stirling, Ellis 1986) draws per particle
// (cos theta, phi, u3, u4) and maps to massless momenta at sqrt_s; its weight is
// the closed-form n-body volume of the paper's invariant phase space (Sec. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "heget_device.hpp"

namespace heget {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product gives both words in one instruction
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0], p1 = uint64_t(0xCD9E8D57u) * c[2];
    // a ^ b ^ c in one instruction (truth table 0x96)
    c[0] = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c[1], k0, 0x96);
    c[1] = uint32_t(p1);
    c[2] = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c[3], k1, 0x96);
    c[3] = uint32_t(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double unit_open(uint32_t hi, uint32_t lo) {
  // the top 52 bits of x as the mantissa of a double in [1, 2): 1 + floor(x / 2^12) 2^-52;
  // adding 2^-53 - 1 is exact and gives (floor(x / 2^12) + 1/2) 2^-52
  const uint64_t x = (uint64_t(hi) << 32) | uint64_t(lo);
  return __builtin_bit_cast(double, (x >> 12) | 0x3FF0000000000000ull) + (0x1.0p-53 - 1.0);
}

// Natural logarithm of a positive normal x (the RAMBO energies' -log(u u')):
// x = 2^k m with m in [1/sqrt2, sqrt2), log x = k ln2 + 2 atanh f with
// f = (m - 1) / (m + 1), |f| <= 0.1716, the range reduction of Cody and Waite
// (Software Manual for the Elementary Functions, 1980); 2 atanh f = 2f (1 + s/3 +
// s^2/5 + ... + s^9/19), s = f^2, whose first omitted term is below 2.5e-17 of
// the sum.  The quotient f takes the hardware reciprocal estimate, two Newton
// steps and one correction of the quotient.  A few units in the last place.
__device__ __forceinline__ double log_positive(double x) {
  int k = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);   // [0.5, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    k -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  double f = num * r;
  f = fma(r, fma(-den, f, num), f);
  const double s = f * f;
  double q = 1.0 / 19.0;
  q = fma(q, s, 1.0 / 17.0);
  q = fma(q, s, 1.0 / 15.0);
  q = fma(q, s, 1.0 / 13.0);
  q = fma(q, s, 1.0 / 11.0);
  q = fma(q, s, 1.0 / 9.0);
  q = fma(q, s, 1.0 / 7.0);
  q = fma(q, s, 1.0 / 5.0);
  q = fma(q, s, 1.0 / 3.0);
  const double t = 2.0 * f;
  const double lm = fma(t * s, q, t);
  const double kd = double(k);
  return fma(kd, 0x1.62e42fefa39efp-1, fma(kd, 0x1.abc9e3b39803fp-56, lm));
}

// RAMBO for NOUT massless particles; writes the physical momenta p[0..NOUT-1]
template <int NOUT>
__device__ __forceinline__ void rambo(uint64_t seed, uint64_t event, double sqrt_s, mom* p) {
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0, Q3 = 0.0;
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    double u[4];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      uint32_t c[4] = {uint32_t(event), uint32_t(event >> 32), uint32_t(2 * k + b), 0u};
      philox4x32_10(c, k0, k1);
      u[2 * b] = unit_open(c[0], c[1]);
      u[2 * b + 1] = unit_open(c[2], c[3]);
    }
    const double ct = 2.0 * u[0] - 1.0;
    const double st = sqrt_pos(1.0 - ct * ct);
    double sf, cf;
    // the azimuth 2 pi u: sincospi reduces its argument exactly
    sincospi(2.0 * u[1], &sf, &cf);
    const double e = -log_positive(u[2] * u[3]);
    p[k] = {e, e * st * cf, e * st * sf, e * ct};
    Q0 += p[k].e;
    Q1 += p[k].x;
    Q2 += p[k].y;
    Q3 += p[k].z;
  }
  const double M = sqrt_pos(Q0 * Q0 - Q1 * Q1 - Q2 * Q2 - Q3 * Q3);
  const double iM = recip(M);
  const double b1 = -Q1 * iM, b2 = -Q2 * iM, b3 = -Q3 * iM;
  const double g = Q0 * iM;
  const double a = recip(1.0 + g);
  const double x = sqrt_s * iM;
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    const double bq = b1 * p[k].x + b2 * p[k].y + b3 * p[k].z;
    const double q0 = p[k].e;
    p[k] = {x * (g * q0 + bq), x * (p[k].x + b1 * q0 + a * bq * b1), x * (p[k].y + b2 * q0 + a * bq * b2),
            x * (p[k].z + b3 * q0 + a * bq * b3)};
  }
}

// ---------------------------------------------------------------- resonance tree
// The paper's Appendix A phase space at a fixed collision energy: nested
// two-body decays, dPhi_n = dPhi_2(collision) prod_k ds_k / (2 pi) dPhi_2(R_k),
// the invariant mass of a resonance Breit-Wigner mapped (s = m^2 + m Gamma
// tan theta, theta uniform over |s - m^2| / (m Gamma) < min(window, m / Gamma)
// within the kinematic range) or flat over its kinematic range.  The process's
// tree is compiled into a generated device function built from these pieces.

// The first N uniforms of an event (two per Philox counter block, blocks 0, 1, ...).
template <int N>
__device__ __forceinline__ void ps_uniforms(uint64_t seed, uint64_t event, double* u) {
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
#pragma unroll
  for (int j = 0; 2 * j < N; ++j) {
    uint32_t c[4] = {uint32_t(event), uint32_t(event >> 32), uint32_t(j), 0u};
    philox4x32_10(c, k0, k1);
    u[2 * j] = unit_open(c[0], c[1]);
    if (2 * j + 1 < N) u[2 * j + 1] = unit_open(c[2], c[3]);
  }
}

// Adaptive integration: the event's N uniforms through the grid of KernelArgs
// (bins of [e_j, e_(j+1)] per dimension, u -> e_j + (u B - j)(e_(j+1) - e_j));
// returns the Jacobian prod B (e_(j+1) - e_j) and records the bins of event i.
// Every edge is loaded before the first bin is stored: the byte stores may
// alias the grid as far as the compiler knows, and would otherwise serialise
// the loads behind them.
template <int N, class A>
__device__ __forceinline__ double grid_map(const A& a, int64_t i, double* u) {
#pragma clang fp contract(off)
  const int B = a.grid_bins;
  int j[N];
  double lo[N], hi[N];
#pragma unroll
  for (int d = 0; d < N; ++d) {
    j[d] = min(int(u[d] * B), B - 1);
    lo[d] = a.grid[d * (B + 1) + j[d]];
    hi[d] = a.grid[d * (B + 1) + j[d] + 1];
  }
  double jac = 1.0;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    u[d] = lo[d] + (u[d] * B - j[d]) * (hi[d] - lo[d]);
    jac *= B * (hi[d] - lo[d]);
  }
  if (a.grid_bin_out) {
#pragma unroll
    for (int d = 0; d < N; ++d) a.grid_bin_out[d * a.grid_bin_stride + i] = uint8_t(j[d]);
  }
  return jac;
}

// The tree's arithmetic is not contracted into fused multiply-adds: each
// product and sum rounds on its own, as in a plain IEEE evaluation, so that
// masses near a threshold (where lambda cancels) come out with the same bits.

// Invariant mass s of a resonance within [lo, hi]; returns its ds / (2 pi)
// weight, 0 (and s = max(lo, 0)) when the window leaves no room.
__device__ __forceinline__ double ps_mass(double u, double lo, double hi, double m, double g, bool bw,
                                          double window, double& s) {
#pragma clang fp contract(off)
  const double inv2pi = 0.15915494309189533577;
  if (bw) {
    const double w = fmin(window, m / g);
    lo = fmax(lo, m * m - w * m * g);
    hi = fmin(hi, m * m + w * m * g);
  }
  if (!(hi > lo)) {
    s = fmax(lo, 0.0);
    return 0.0;
  }
  if (bw) {
    const double mg = m * g;
    const double t_lo = atan((lo - m * m) / mg), t_hi = atan((hi - m * m) / mg);
    s = m * m + mg * tan(t_lo + u * (t_hi - t_lo));
    return (t_hi - t_lo) * ((s - m * m) * (s - m * m) + mg * mg) / mg * inv2pi;
  }
  s = lo + u * (hi - lo);
  return (hi - lo) * inv2pi;
}

// q, given in the rest frame of P (mass M), in the frame where P is given
__device__ __forceinline__ mom ps_boost(const mom& P, double M, const mom& q) {
#pragma clang fp contract(off)
  const double pq = P.x * q.x + P.y * q.y + P.z * q.z;
  const double e = (P.e * q.e + pq) / M;
  const double f = (q.e + e) / (P.e + M);
  return {e, q.x + f * P.x, q.y + f * P.y, q.z + f * P.z};
}

// Two-body decay of P (mass M) into masses m0, m1, isotropic in P's rest frame
// (cos theta = 2 uc - 1, phi = 2 pi uphi); returns dPhi_2 = lambda^(1/2) / (8 pi M^2).
// P at rest (the collision) is not boosted.
__device__ __forceinline__ double ps_decay(double uc, double uphi, const mom& P, double M, double m0, double m1,
                                           bool at_rest, mom& q0, mom& q1) {
#pragma clang fp contract(off)
  const double pi = 3.14159265358979323846;
  const double lam = fmax((M * M - (m0 + m1) * (m0 + m1)) * (M * M - (m0 - m1) * (m0 - m1)), 0.0);
  const double rl = sqrt(lam);
  const double pst = rl / (2.0 * M);
  const double ct = 2.0 * uc - 1.0;
  const double st = sqrt(1.0 - ct * ct);
  double sf, cf;
  sincospi(2.0 * uphi, &sf, &cf);
  const double nx = st * cf, ny = st * sf;
  const double e0 = (M * M + m0 * m0 - m1 * m1) / (2.0 * M), e1 = (M * M + m1 * m1 - m0 * m0) / (2.0 * M);
  const mom a = {e0, pst * nx, pst * ny, pst * ct}, b = {e1, -pst * nx, -pst * ny, -pst * ct};
  q0 = at_rest ? a : ps_boost(P, M, a);
  q1 = at_rest ? b : ps_boost(P, M, b);
  return rl / (8.0 * pi * M * M);
}

// A parton collision at a hadron collider of energy sqrt_S (the paper's
// Appendix A with parton densities set to 1): daughter 0 (mass m0) and
// daughter 1 (mass m1) get rapidities flat in [-y_max, y_max] (u[0], u[3]);
// daughter 0 gets ln(m0^2 + pT^2) flat from pT = pt_min to the kinematic
// limit lambda^(1/2)(S, m0^2, m1^2) / (2 sqrt_S) (u[1]) and a flat azimuth
// (u[2]); daughter 1 balances pT.  x_a, x_b = sum (E +- p_z) / sqrt_S give the
// incoming partons along +-z.  Returns dSigma_2 / (2 s_hat) with
// dSigma_2 = (2 pi / S) dy_1 dy_0 dpT^2 / (4 pi)^2 dphi / (2 pi), or 0 unless
// x_a, x_b < 1.
__device__ __forceinline__ double ps_hadronic(const double* u, double sqrt_S, double m0, double m1, double y_max,
                                              double pt_min, mom& q0, mom& q1, mom& pa, mom& pb) {
#pragma clang fp contract(off)
  const double pi = 3.14159265358979323846;
  const double S = sqrt_S * sqrt_S;
  const double y0 = -y_max + 2.0 * y_max * u[0];
  const double y1 = -y_max + 2.0 * y_max * u[3];
  const double lam = fmax((S - (m0 + m1) * (m0 + m1)) * (S - (m0 - m1) * (m0 - m1)), 0.0);
  const double pt2max = lam / (4.0 * S);
  const double llo = log(m0 * m0 + pt_min * pt_min), lhi = log(m0 * m0 + pt2max);
  const double L = llo + u[1] * (lhi - llo);
  const double mt0sq = exp(L);
  const double pt = sqrt(fmax(mt0sq - m0 * m0, 0.0));
  double sf, cf;
  sincospi(2.0 * u[2], &sf, &cf);
  const double px = pt * cf, py = pt * sf;
  const double mt0 = sqrt(mt0sq), mt1 = sqrt(m1 * m1 + pt * pt);
  const double e0 = mt0 * cosh(y0), z0 = mt0 * sinh(y0);
  const double e1 = mt1 * cosh(y1), z1 = mt1 * sinh(y1);
  const double xa = (e0 + z0 + e1 + z1) / sqrt_S, xb = (e0 - z0 + e1 - z1) / sqrt_S;
  q0 = {e0, px, py, z0};
  q1 = {e1, -px, -py, z1};
  const double h = 0.5 * sqrt_S;
  pa = {xa * h, 0.0, 0.0, xa * h};
  pb = {xb * h, 0.0, 0.0, -xb * h};
  if (!(lhi > llo && xa < 1.0 && xb < 1.0)) return 0.0;
  const double sh = xa * xb * S;
  const double w = (2.0 * pi / S) * (2.0 * y_max) * (2.0 * y_max) * mt0sq * (lhi - llo) / (16.0 * pi * pi);
  return w / (2.0 * sh);
}

// every final particle has pT > pt_min and every final pair Delta R > dr_min
template <int NOUT>
__device__ __forceinline__ bool pass_pt_dr(const mom* p, double pt_min, double dr_min) {
  double eta[NOUT], phi[NOUT];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    const double pt = sqrt_pos(p[k].x * p[k].x + p[k].y * p[k].y);
    const double pp = sqrt_pos(pt * pt + p[k].z * p[k].z);
    ok = ok && (pt > pt_min);
    eta[k] = 0.5 * log((pp + p[k].z) / (pp - p[k].z));
    phi[k] = atan2(p[k].y, p[k].x);
  }
  const double pi = 3.14159265358979323846;
#pragma unroll
  for (int k = 0; k < NOUT; ++k)
#pragma unroll
    for (int l = k + 1; l < NOUT; ++l) {
      double dphi = fabs(phi[k] - phi[l]);
      if (dphi > pi) dphi = 2.0 * pi - dphi;
      const double deta = eta[k] - eta[l];
      ok = ok && (sqrt(deta * deta + dphi * dphi) > dr_min);
    }
  return ok;
}

}  // namespace heget
