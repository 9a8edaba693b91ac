// CPU check of the generation step's own arithmetic (tests only): the device
// header compiled for x86-64 against the host stand-in of the HIP runtime.
//
//   device_math_check philox KAT_FILE   -> the device Philox4x32-10 on every
//                                          known-answer row; prints mismatches
//   device_math_check log N SEED        -> log_positive against long double log
//                                          on N inputs distributed as RAMBO's
//                                          u u' (and single u, and x near 1);
//                                          prints the largest error in units in
//                                          the last place of the exact result
//   device_math_check roots N SEED      -> sqrt_pos, recip and quot against long
//                                          double on N inputs over 2^-60 .. 2^60
//   device_math_check unit N SEED       -> unit_open against its definition
//                                          (floor(x / 2^12) + 1/2) 2^-52, bit for
//                                          bit, on N random words and edge words
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

#include "phase_space.hpp"

static int philox(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return 2;
  char line[512];
  int rows = 0, bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    unsigned v[10];
    if (std::sscanf(line, "%x %x %x %x %x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7],
                    &v[8], &v[9]) != 10)
      continue;
    uint32_t c[4] = {v[0], v[1], v[2], v[3]};
    heget::philox4x32_10(c, v[4], v[5]);
    ++rows;
    if (c[0] != v[6] || c[1] != v[7] || c[2] != v[8] || c[3] != v[9]) {
      ++bad;
      std::printf("mismatch row %d: %08x %08x %08x %08x\n", rows, c[0], c[1], c[2], c[3]);
    }
  }
  std::fclose(f);
  std::printf("rows %d mismatches %d\n", rows, bad);
  return bad ? 1 : 0;
}

static int logcheck(long n, uint64_t seed) {
  std::mt19937_64 g(seed);
  double worst = 0.0, at = 0.0;
  for (long i = 0; i < n; ++i) {
    const uint64_t a = g(), b = g();
    const double u1 = (double(a >> 12) + 0.5) * 0x1.0p-52, u2 = (double(b >> 12) + 0.5) * 0x1.0p-52;
    double x = (i % 4 == 0) ? u1 : u1 * u2;
    if (i % 1000 == 0) x = 1.0 - double((a >> 40) + 1) * 0x1.0p-53;
    const long double ref = logl((long double)x);
    const double r = double(ref);
    const double ulp = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    const double e = double(fabsl((long double)heget::log_positive(x) - ref) / ulp);
    if (e > worst) {
      worst = e;
      at = x;
    }
  }
  std::printf("inputs %ld max_ulp %.4f at %.17g\n", n, worst, at);
  return 0;
}

static double ulps(double got, long double ref) {
  const double r = double(ref);
  const double ulp = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
  return double(fabsl((long double)got - ref) / ulp);
}

static int roots(long n, uint64_t seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> ex(-60.0, 60.0), mant(1.0, 2.0);
  double ws = 0, wr = 0, wq = 0;
  for (long i = 0; i < n; ++i) {
    const double x = std::ldexp(mant(g), int(ex(g))), y = std::ldexp(mant(g), int(ex(g)));
    ws = std::fmax(ws, ulps(heget::sqrt_pos(x), sqrtl((long double)x)));
    wr = std::fmax(wr, ulps(heget::recip(x), 1.0L / (long double)x));
    wq = std::fmax(wq, ulps(heget::quot(y, x), (long double)y / (long double)x));
  }
  std::printf("inputs %ld sqrt_ulp %.4f recip_ulp %.4f quot_ulp %.4f sqrt0 %g sqrtneg %g\n", n, ws, wr, wq,
              heget::sqrt_pos(0.0), heget::sqrt_pos(-1e-300));
  return 0;
}

static int unit(long n, uint64_t seed) {
  std::mt19937_64 g(seed);
  const uint32_t edge[] = {0u, 1u, 0xFFFu, 0x1000u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFF000u, 0xFFFFFFFFu};
  long bad = 0, count = 0;
  auto one = [&](uint32_t hi, uint32_t lo) {
    const uint64_t x = (uint64_t(hi) << 32) | lo;
    const double want = (double(x >> 12) + 0.5) * 0x1.0p-52;
    ++count;
    if (heget::unit_open(hi, lo) != want) ++bad;
  };
  for (uint32_t a : edge)
    for (uint32_t b : edge) one(a, b);
  for (long i = 0; i < n; ++i) {
    const uint64_t v = g();
    one(uint32_t(v >> 32), uint32_t(v));
  }
  std::printf("words %ld mismatches %ld\n", count, bad);
  return bad ? 1 : 0;
}

int main(int argc, char** argv) {
  if (argc >= 3 && !std::strcmp(argv[1], "philox")) return philox(argv[2]);
  if (argc >= 4 && !std::strcmp(argv[1], "log")) return logcheck(std::atol(argv[2]), std::strtoull(argv[3], 0, 0));
  if (argc >= 4 && !std::strcmp(argv[1], "roots")) return roots(std::atol(argv[2]), std::strtoull(argv[3], 0, 0));
  if (argc >= 4 && !std::strcmp(argv[1], "unit")) return unit(std::atol(argv[2]), std::strtoull(argv[3], 0, 0));
  return 2;
}
