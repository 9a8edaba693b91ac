// Oracle: n-gluon tree amplitudes by the colour-ordered Berends-Giele
// recursion, and the trace-basis colour matrix by brute force over SU(3).
// Test infrastructure only; shares no code with the product path.
//
// Colour decomposition (generators normalised Tr(T^a T^b) = delta/2):
//   M = sum_{sigma in S_{n-1}} Tr(T^a0 T^a_sigma1 ... T^a_sigma(n-1)) A(0, sigma).
// Colour-ordered rules, obtained from the Peskin-Schroeder vertices with
// f^abc = -2i Tr([T^a,T^b] T^c) and one Fierz factor 1/2 per internal line
// (the 1/N pieces cancel for pure-gluon trees):
//   3-vertex, cyclic legs (1,2,3):  -2 i g V(1,2,3),
//     V = g^{mu1 mu2}(k1-k2)^mu3 + g^{mu2 mu3}(k2-k3)^mu1 + g^{mu3 mu1}(k3-k1)^mu2
//   4-vertex, cyclic legs (1,2,3,4): 2 i g^2 [2 g13 g24 - g12 g34 - g14 g23]
//   propagator: (1/2) (-i g_{mu nu} / P^2).
// All momenta are taken incoming; legs 0 and 1 are incoming gluons, the others
// outgoing (incoming momentum -p, polarisation conjugated).
#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>

#include "procs.hpp"

namespace orc {
namespace {

struct Cur {
  CVec4 J;
  Vec4 P;
};

CVec4 v3(const Cur& A, const Cur& B) {
  const Vec4 PC = neg(add(A.P, B.P));
  const cd ab = dot(A.J, B.J);
  const cd a = dot(A.J, sub(B.P, PC));
  const cd b = dot(B.J, sub(PC, A.P));
  CVec4 r;
  for (int m = 0; m < 4; ++m) r[m] = ab * (A.P[m] - B.P[m]) + B.J[m] * a + A.J[m] * b;
  return r;
}
CVec4 v4(const Cur& A, const Cur& B, const Cur& C) {
  const cd ac = dot(A.J, C.J), ab = dot(A.J, B.J), bc = dot(B.J, C.J);
  CVec4 r;
  for (int m = 0; m < 4; ++m) r[m] = real(2) * ac * B.J[m] - ab * C.J[m] - bc * A.J[m];
  return r;
}

struct BG {
  const SM& sm;
  std::vector<Cur> ext;
  std::unordered_map<uint64_t, Cur> memo;
  BG(const SM& s, int n, const Vec4* p, const int* hel) : sm(s), ext(n) {
    for (int i = 0; i < n; ++i) {
      const int h = (sm.gauge_leg == i) ? 4 : hel[i];
      if (i < 2) {
        ext[i] = {eps_vec(p[i], 0.0, h), p[i]};
      } else {
        ext[i] = {conjv(eps_vec(p[i], 0.0, h)), neg(p[i])};
      }
    }
  }
  static uint64_t key(const int* legs, int len) {
    uint64_t k = 0;
    for (int i = 0; i < len; ++i) k = k * 16 + uint64_t(legs[i] + 1);
    return k;
  }
  // vertex sum (no propagator) for the ordered legs, off-shell leg last
  CVec4 vertex_sum(const int* legs, int len) {
    const cd c3 = real(-2) * I1 * sm.gs;
    const cd c4 = real(2) * I1 * sm.gs * sm.gs;
    CVec4 K{};
    for (int m = 1; m < len; ++m) {
      const Cur& A = current(legs, m);
      const Cur& B = current(legs + m, len - m);
      K = cadd(K, cscale(c3, v3(A, B)));
    }
    for (int m = 1; m < len; ++m)
      for (int l = m + 1; l < len; ++l) {
        const Cur& A = current(legs, m);
        const Cur& B = current(legs + m, l - m);
        const Cur& C = current(legs + l, len - l);
        K = cadd(K, cscale(c4, v4(A, B, C)));
      }
    return K;
  }
  const Cur& current(const int* legs, int len) {
    if (len == 1) return ext[legs[0]];
    const uint64_t k = key(legs, len);
    auto it = memo.find(k);
    if (it != memo.end()) return it->second;
    Vec4 P = {0, 0, 0, 0};
    for (int i = 0; i < len; ++i) P = add(P, ext[legs[i]].P);
    const CVec4 K = vertex_sum(legs, len);
    const cd prop = real(0.5) * (-I1) / dot(P, P);
    Cur c{cscale(prop, K), P};
    return memo.emplace(k, c).first->second;
  }
  // A(order[0], order[1], ...) with order[0] the root leg
  cd partial(const int* order, int n) {
    const CVec4 K = vertex_sum(order + 1, n - 1);
    return dot(ext[order[0]].J, K) / I1;
  }
};

std::vector<std::vector<int>> orderings(int n) {
  std::vector<int> s;
  for (int i = 1; i < n; ++i) s.push_back(i);
  std::vector<std::vector<int>> out;
  do {
    std::vector<int> o = {0};
    o.insert(o.end(), s.begin(), s.end());
    out.push_back(o);
  } while (std::next_permutation(s.begin(), s.end()));
  return out;
}

}  // namespace

cd gluon_partial(int n, const SM& sm, const Vec4* p, const int* hel, const int* order) {
  BG bg(sm, n, p, hel);
  return bg.partial(order, n);
}

// The same matrix by Fierz expansion, for more gluons than the brute-force sum
// reaches: conj Tr(T^{a_s0} ... ) = Tr(... T^{a_s0}) (hermitian generators),
// and each gluon's pair of generators, one in each trace, is replaced by
//   T^a_{ij} T^a_{kl} = (1/2) [delta_il delta_jk - (1/N) delta_ij delta_kl].
// Each of the 2^n choices of terms joins the 2n fundamental indices into
// closed loops, worth N per loop.
std::vector<real> fierz_colour_matrix(int n) {
  const auto ords = orderings(n);
  const int no = int(ords.size());
  const real N = 3.0;
  std::vector<real> C(size_t(no) * no, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int x = 0; x < no; ++x) {
    int pos1[8], pos2[8], par[16];
    for (int p = 0; p < n; ++p) pos1[ords[x][n - 1 - p]] = p;   // reversed: the conjugated trace
    for (int y = 0; y < no; ++y) {
      for (int q = 0; q < n; ++q) pos2[ords[y][q]] = q;
      real sum = 0.0;
      for (int choice = 0; choice < (1 << n); ++choice) {
        // nodes 0..n-1: indices I_p of trace 1 (T at p runs I_p -> I_(p+1)); n..2n-1: J_q of trace 2
        for (int k = 0; k < 2 * n; ++k) par[k] = k;
        auto find = [&](int a) {
          while (par[a] != a) a = par[a] = par[par[a]];
          return a;
        };
        auto join = [&](int a, int b) { par[find(a)] = find(b); };
        int k1 = 0;
        for (int g = 0; g < n; ++g) {
          const int p = pos1[g], q = pos2[g];
          const int ip = p, ip1 = (p + 1) % n, jq = n + q, jq1 = n + (q + 1) % n;
          if ((choice >> g) & 1) {   // -(1/N) delta(I_p, I_p+1) delta(J_q, J_q+1)
            join(ip, ip1);
            join(jq, jq1);
            ++k1;
          } else {                   // delta(I_p, J_q+1) delta(I_p+1, J_q)
            join(ip, jq1);
            join(ip1, jq);
          }
        }
        int loops = 0;
        for (int k = 0; k < 2 * n; ++k) loops += find(k) == k;
        sum += std::pow(N, loops) * std::pow(-1.0 / N, k1);
      }
      C[size_t(x) * no + y] = sum / real(1 << n);
    }
  }
  return C;
}

const std::vector<real>& gluon_colour_matrix(int n) {
  static std::map<int, std::vector<real>> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(n);
  if (it != cache.end()) return it->second;
  if (n > 6) return cache[n] = fierz_colour_matrix(n);   // 8^n explicit colours: brute force up to 6
  const auto ords = orderings(n);
  const int no = int(ords.size());
  const Colour& CL = colour();
  int ncfg = 1;
  for (int i = 0; i < n; ++i) ncfg *= 8;
  std::vector<real> C(no * no, 0.0);
#pragma omp parallel
  {
    std::vector<cd> loc(no * no, 0.0);
    std::vector<cd> tr(no);
#pragma omp for schedule(dynamic, 64)
    for (int cfg = 0; cfg < ncfg; ++cfg) {
      int a[8];
      int r = cfg;
      for (int i = n - 1; i >= 0; --i) {
        a[i] = r % 8;
        r /= 8;
      }
      bool any = false;
      for (int o = 0; o < no; ++o) {
        // Tr(T^{a_ord0} T^{a_ord1} ...)
        cd M[3][3];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) M[i][j] = CL.T[a[ords[o][0]]][i][j];
        for (int k = 1; k < n; ++k) {
          const auto& Tk = CL.T[a[ords[o][k]]];
          cd R[3][3];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              R[i][j] = M[i][0] * Tk[0][j] + M[i][1] * Tk[1][j] + M[i][2] * Tk[2][j];
            }
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = R[i][j];
        }
        tr[o] = M[0][0] + M[1][1] + M[2][2];
        if (std::abs(tr[o]) > 0.0) any = true;
      }
      if (!any) continue;
      for (int x = 0; x < no; ++x)
        for (int y = 0; y < no; ++y) loc[x * no + y] += tr[x] * std::conj(tr[y]);
    }
#pragma omp critical
    for (int i = 0; i < no * no; ++i) C[i] += std::real(loc[i]);
  }
  return cache[n] = C;
}

real gluon_me2(int n, const SM& sm, const Vec4* p) {
  const auto ords = orderings(n);
  const int no = int(ords.size());
  const std::vector<real>& C = gluon_colour_matrix(n);
  std::vector<cd> A(no);
  real tot = 0.0;
  int hel[8];
  for (int hc = 0; hc < (1 << n); ++hc) {
    for (int i = 0; i < n; ++i) hel[i] = ((hc >> (n - 1 - i)) & 1) ? 1 : -1;
    BG bg(sm, n, p, hel);
    for (int o = 0; o < no; ++o) A[o] = bg.partial(ords[o].data(), n);
    cd s = 0;
    for (int x = 0; x < no; ++x) {
      cd row = 0;
      for (int y = 0; y < no; ++y) row += C[x * no + y] * A[y];
      s += std::conj(A[x]) * row;
    }
    tot += std::real(s);
  }
  return tot;
}

}  // namespace orc
