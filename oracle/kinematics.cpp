// Oracle: counter-based random numbers, RAMBO phase space and the gluon cut.
// Test infrastructure only; shares no code with the product path.
#include <cmath>
#include <cstdint>

#include "dirac.hpp"
#include "oracle.h"

namespace {

const double kPi = 3.14159265358979323846;

// One Philox round: two 32x32 -> 64 bit products, words permuted and keyed.
void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = uint64_t(0xD2511F53u) * uint64_t(c[0]);
  const uint64_t p1 = uint64_t(0xCD9E8D57u) * uint64_t(c[2]);
  const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
  const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

// (floor(x / 2^12) + 1/2) 2^-52: every value is exact in FP64 and lies in
// [2^-53, 1 - 2^-53], so the interval is open at both ends.
double u52(uint32_t hi, uint32_t lo) {
  uint64_t x = (uint64_t(hi) << 32) | uint64_t(lo);
  return (double(x >> 12) + 0.5) * std::ldexp(1.0, -52);
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

}  // namespace

extern "C" void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

extern "C" void or_uniforms(uint64_t seed, uint64_t event, int n_u, double* u) {
  const uint32_t key[2] = {uint32_t(seed), uint32_t(seed >> 32)};
  for (int j = 0; 2 * j < n_u; ++j) {
    const uint32_t ctr[4] = {uint32_t(event), uint32_t(event >> 32), uint32_t(j), 0u};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    u[2 * j] = u52(w[0], w[1]);
    if (2 * j + 1 < n_u) u[2 * j + 1] = u52(w[2], w[3]);
  }
}

extern "C" void or_uniforms_bulk(uint64_t seed, uint64_t counter_offset, int64_t n_events, int n_u, double* u) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_events; ++i) or_uniforms(seed, counter_offset + uint64_t(i), n_u, u + i * n_u);
}

extern "C" double or_phase_space_volume(double sqrt_s, int n) {
  const double s = sqrt_s * sqrt_s;
  return std::pow(2.0 * kPi, 4 - 3 * n) * std::pow(0.5 * kPi, n - 1) * std::pow(s, n - 2) /
         (factorial(n - 1) * factorial(n - 2));
}

extern "C" double or_rambo(double sqrt_s, int n, const double* u, double* p) {
  // isotropic massless momenta with exponential energies
  double Q[4] = {0, 0, 0, 0};
  for (int k = 0; k < n; ++k) {
    const double c = 2.0 * u[4 * k] - 1.0;
    const double s = std::sqrt(1.0 - c * c);
    const double f = 2.0 * kPi * u[4 * k + 1];
    const double q0 = -std::log(u[4 * k + 2] * u[4 * k + 3]);
    double* q = p + 4 * k;
    q[0] = q0;
    q[1] = q0 * s * std::cos(f);
    q[2] = q0 * s * std::sin(f);
    q[3] = q0 * c;
    for (int m = 0; m < 4; ++m) Q[m] += q[m];
  }
  // conformal transformation to the centre-of-mass frame at sqrt_s
  const double M = std::sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  const double g = Q[0] / M;
  const double a = 1.0 / (1.0 + g);
  const double x = sqrt_s / M;
  for (int k = 0; k < n; ++k) {
    double* q = p + 4 * k;
    const double bq = b[0] * q[1] + b[1] * q[2] + b[2] * q[3];
    const double q0 = q[0];
    const double e = x * (g * q0 + bq);
    const double v1 = x * (q[1] + b[0] * q0 + a * bq * b[0]);
    const double v2 = x * (q[2] + b[1] * q0 + a * bq * b[1]);
    const double v3 = x * (q[3] + b[2] * q0 + a * bq * b[2]);
    q[0] = e;
    q[1] = v1;
    q[2] = v2;
    q[3] = v3;
  }
  return or_phase_space_volume(sqrt_s, n);
}

extern "C" void or_generate(uint64_t seed, uint64_t counter_offset, int64_t n_events, int n_out,
                            double sqrt_s, double* mom) {
  const int nl = n_out + 2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_events; ++i) {
    double u[4 * 16];
    or_uniforms(seed, counter_offset + uint64_t(i), 4 * n_out, u);
    double* ev = mom + i * nl * 4;
    const double h = 0.5 * sqrt_s;
    ev[0] = h; ev[1] = 0; ev[2] = 0; ev[3] = h;
    ev[4] = h; ev[5] = 0; ev[6] = 0; ev[7] = -h;
    or_rambo(sqrt_s, n_out, u, ev + 8);
  }
}

extern "C" void or_cut_gluons(int64_t n_events, int n_legs, const double* mom, double pt_min,
                              double dr_min, int32_t* pass) {
  for (int64_t i = 0; i < n_events; ++i) {
    const double* ev = mom + i * n_legs * 4;
    int ok = 1;
    double eta[16], phi[16];
    for (int k = 2; k < n_legs; ++k) {
      const double* q = ev + 4 * k;
      const double pt = std::sqrt(q[1] * q[1] + q[2] * q[2]);
      const double pp = std::sqrt(pt * pt + q[3] * q[3]);
      if (!(pt > pt_min)) ok = 0;
      eta[k] = 0.5 * std::log((pp + q[3]) / (pp - q[3]));
      phi[k] = std::atan2(q[2], q[1]);
    }
    for (int k = 2; k < n_legs; ++k)
      for (int l = k + 1; l < n_legs; ++l) {
        double dphi = std::fabs(phi[k] - phi[l]);
        if (dphi > kPi) dphi = 2.0 * kPi - dphi;
        const double deta = eta[k] - eta[l];
        if (!(std::sqrt(deta * deta + dphi * dphi) > dr_min)) ok = 0;
      }
    pass[i] = ok;
  }
}

extern "C" int or_weights(double phase_space_weight, double factor, int64_t n_events, const double* me2,
                          const int32_t* pass, double* w) {
  for (int64_t i = 0; i < n_events; ++i)
    w[i] = (pass && !pass[i]) ? 0.0 : phase_space_weight * factor * me2[i];
  return 0;
}
