// Oracle: u ubar -> t tbar + n gluons (n <= 3) as the sum of every tree-level
// Feynman diagram, with explicit Dirac matrices and the colour summed by brute
// force over explicit SU(3) indices.  Test infrastructure only; shares no
// code with the product path.
//
// Legs: 0 u (incoming), 1 ubar (incoming), 2 t (outgoing), 3 tbar (outgoing),
// 4 .. 3+n gluons (outgoing).  Feynman rules (Peskin-Schroeder, Feynman gauge,
// the colour generators T^a and f^abc of sm.hpp):
//   quark-gluon vertex      i g_s gamma^mu T^a_ij
//   triple-gluon vertex     g_s f^abc [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
//                           (momenta k, p, q of legs a, b, c, all flowing in)
//   four-gluon vertex       -i g_s^2 [f^abe f^cde (g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho})
//                                    + f^ace f^bde (g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho})
//                                    + f^ade f^bce (g^{mu nu} g^{rho sigma} - g^{mu rho} g^{nu sigma})]
//                           (the paper's Sec. 4.2 splits it into the same three colour structures)
//   quark propagator        i (k-slash + m) / (k^2 - m^2 + i m Gamma), k along the fermion arrow
//   gluon propagator        -i g_{mu nu} delta^ab / k^2
// External states: u(p0) and vbar(p1) for the incoming quark and antiquark,
// ubar(p2) and v(p3) for the outgoing top and antitop, epsilon^*(k) for an
// outgoing gluon.
//
// Every diagram is enumerated once by the vertex that the ubar line (leg 1)
// enters: vbar(p1) [i g gamma^mu T^a] U(S1) G_mu^a(S2), where U(S1) is a
// sub-diagram ending in an off-shell u quark (the u line from leg 0 with the
// gluon sub-diagrams attached along it) and G(S2) a sub-diagram ending in an
// off-shell gluon that carries the whole t line.  A sub-diagram is stored once
// and shared by every diagram that contains it; its Lorentz value (a spinor or
// a gluon current, propagator included) and its colour tensor (one free
// fundamental or adjoint index) are evaluated separately, so that each diagram
// is c_d(colours) x M_d(helicities) and
//   F = sum_hel sum_{d,d'} conj(M_d) C_dd' M_d',  C_dd' = sum_colours conj(c_d) c_d'.
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "procs.hpp"

namespace orc {
namespace {

int lowest_leg(uint32_t s) { return __builtin_ctz(s); }

enum Kind { K_U, K_TB, K_T2, K_G };   // u-line column from leg 0, t-line column from leg 3,
                                      // t-line row from leg 2, gluon current
enum Vtx { V_EXT, V_QG, V_GGG, V_GGGG, V_TT };

struct Node {
  Kind kind;
  uint32_t legs;   // bitmask of the external legs in the sub-diagram
  Vtx vtx;
  int term;        // four-gluon vertex: colour structure 0, 1, 2
  int ch[3];       // children (V_QG: quark, gluon; V_GGG: a, b; V_GGGG: a, b, c; V_TT: tbar side, t side)
};

struct Diagrams {
  int ng = 0, nl = 0;
  std::vector<Node> nodes;
  std::vector<std::pair<int, int>> diag;   // (U node, G node)
  std::map<std::pair<int, uint32_t>, std::vector<int>> memo;

  uint32_t gluon_legs() const { return ((1u << nl) - 1) & ~0xFu; }
  static int lowest(uint32_t s) { return __builtin_ctz(s); }
  // subsets that can end in an off-shell gluon: no u line, the t line whole or absent
  bool g_ok(uint32_t s) const {
    if (!s || (s & 3u)) return false;
    if (bool(s & 4u) != bool(s & 8u)) return false;
    if (__builtin_popcount(s) == 1) return (s & gluon_legs()) != 0;
    return true;
  }
  int add(const Node& n) {
    nodes.push_back(n);
    return int(nodes.size()) - 1;
  }
  const std::vector<int>& get(Kind k, uint32_t s) {
    auto key = std::make_pair(int(k), s);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    std::vector<int> out;
    if (k == K_G) {
      if (__builtin_popcount(s) == 1) {
        out.push_back(add({K_G, s, V_EXT, 0, {-1, -1, -1}}));
      } else {
        const uint32_t low = 1u << lowest(s);
        // proper subsets a of s containing the lowest leg: the pair {a, s \ a}
        for (uint32_t a = (s - 1) & s; a; a = (a - 1) & s) {
          if (!(a & low)) continue;
          const uint32_t b = s & ~a;
          if (g_ok(a) && g_ok(b)) {
            const std::vector<int> A = get(K_G, a), B = get(K_G, b);
            for (int x : A)
              for (int y : B) out.push_back(add({K_G, s, V_GGG, 0, {x, y, -1}}));
          }
          // triples {a, b, c}: b holds the lowest leg of s \ a
          const uint32_t r = s & ~a;
          if (__builtin_popcount(r) < 2) continue;
          const uint32_t lowr = 1u << lowest(r);
          for (uint32_t bb = (r - 1) & r; bb; bb = (bb - 1) & r) {
            if (!(bb & lowr)) continue;
            const uint32_t c = r & ~bb;
            if (!(g_ok(a) && g_ok(bb) && g_ok(c))) continue;
            const std::vector<int> A = get(K_G, a), B = get(K_G, bb), C = get(K_G, c);
            for (int x : A)
              for (int y : B)
                for (int z : C)
                  for (int t = 0; t < 3; ++t) out.push_back(add({K_G, s, V_GGGG, t, {x, y, z}}));
          }
        }
        // the t line closed into the gluon: tbar side a (with leg 3), t side s \ a (with leg 2)
        if ((s & 4u) && (s & 8u)) {
          for (uint32_t a = (s - 1) & s; a; a = (a - 1) & s) {
            if (!(a & 8u) || (a & 4u)) continue;
            const std::vector<int> A = get(K_TB, a), B = get(K_T2, s & ~a);
            for (int x : A)
              for (int y : B) out.push_back(add({K_G, s, V_TT, 0, {x, y, -1}}));
          }
        }
      }
    } else {
      const uint32_t own = k == K_U ? 1u : k == K_TB ? 8u : 4u;
      if (s == own) {
        out.push_back(add({k, s, V_EXT, 0, {-1, -1, -1}}));
      } else {
        // the vertex next to the off-shell end: quark sub-diagram q (with the own leg), gluon s \ q
        for (uint32_t q = (s - 1) & s; q; q = (q - 1) & s) {
          if (!(q & own)) continue;
          const uint32_t g = s & ~q;
          if (!g_ok(g)) continue;
          const std::vector<int> Q = get(k, q), G = get(K_G, g);
          for (int x : Q)
            for (int y : G) out.push_back(add({k, s, V_QG, 0, {x, y, -1}}));
        }
      }
    }
    return memo[key] = out;
  }
  explicit Diagrams(int n) : ng(n), nl(4 + n) {
    const uint32_t all = (1u << nl) - 1;
    const uint32_t rest = all & ~2u;   // every leg but the ubar
    for (uint32_t s1 = rest; s1; s1 = (s1 - 1) & rest) {
      if (!(s1 & 1u)) continue;
      const uint32_t s2 = rest & ~s1;
      if (!g_ok(s2)) continue;
      const std::vector<int> U = get(K_U, s1), G = get(K_G, s2);
      for (int u : U)
        for (int g : G) diag.push_back({u, g});
    }
  }
};

const Diagrams& diagrams(int ng) {
  static std::map<int, Diagrams> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(ng);
  if (it == cache.end()) it = cache.emplace(ng, Diagrams(ng)).first;
  return it->second;
}

// ------------------------------------------------------------------ colour
// The colour tensor of a node for one explicit colour assignment: 3 (quark
// lines) or 8 (gluons) complex components of its free index.
struct ColVec {
  cd v[8];
};

void node_colours(const Diagrams& D, const int* col, std::vector<ColVec>& out) {
  const Colour& CL = colour();
  out.resize(D.nodes.size());
  for (size_t i = 0; i < D.nodes.size(); ++i) {
    const Node& n = D.nodes[i];
    ColVec r;
    for (auto& x : r.v) x = 0.0;
    if (n.vtx == V_EXT) {
      const int leg = lowest_leg(n.legs);
      r.v[col[leg]] = 1.0;
    } else if (n.vtx == V_QG) {
      const ColVec& q = out[n.ch[0]];
      const ColVec& g = out[n.ch[1]];
      for (int a = 0; a < 8; ++a) {
        if (g.v[a] == cd(0.0)) continue;
        for (int x = 0; x < 3; ++x)
          for (int y = 0; y < 3; ++y) {
            // column lines: out_x = T^a_xy q_y; the row line from the top: out_y = q_x T^a_xy
            if (n.kind == K_T2)
              r.v[y] += q.v[x] * CL.T[a][x][y] * g.v[a];
            else
              r.v[x] += CL.T[a][x][y] * q.v[y] * g.v[a];
          }
      }
    } else if (n.vtx == V_GGG) {
      const ColVec& A = out[n.ch[0]];
      const ColVec& B = out[n.ch[1]];
      for (int a = 0; a < 8; ++a) {
        if (A.v[a] == cd(0.0)) continue;
        for (int b = 0; b < 8; ++b) {
          if (B.v[b] == cd(0.0)) continue;
          for (int c = 0; c < 8; ++c) r.v[c] += CL.f[a][b][c] * A.v[a] * B.v[b];
        }
      }
    } else if (n.vtx == V_GGGG) {
      const ColVec& A = out[n.ch[0]];
      const ColVec& B = out[n.ch[1]];
      const ColVec& C = out[n.ch[2]];
      for (int a = 0; a < 8; ++a) {
        if (A.v[a] == cd(0.0)) continue;
        for (int b = 0; b < 8; ++b) {
          if (B.v[b] == cd(0.0)) continue;
          for (int c = 0; c < 8; ++c) {
            if (C.v[c] == cd(0.0)) continue;
            const cd w = A.v[a] * B.v[b] * C.v[c];
            for (int d = 0; d < 8; ++d) {
              real s = 0.0;
              for (int e = 0; e < 8; ++e) {
                if (n.term == 0)
                  s += CL.f[a][b][e] * CL.f[c][d][e];
                else if (n.term == 1)
                  s += CL.f[a][c][e] * CL.f[b][d][e];
                else
                  s += CL.f[a][d][e] * CL.f[b][c][e];
              }
              r.v[d] += s * w;
            }
          }
        }
      }
    } else {   // V_TT: out_a = t2_x T^a_xy tb_y
      const ColVec& tb = out[n.ch[0]];
      const ColVec& t2 = out[n.ch[1]];
      for (int a = 0; a < 8; ++a)
        for (int x = 0; x < 3; ++x)
          for (int y = 0; y < 3; ++y) r.v[a] += t2.v[x] * CL.T[a][x][y] * tb.v[y];
    }
    out[i] = r;
  }
}

// c_d: the ubar line's vertex, T^a_{i1 j} U_j G_a
void diagram_colours(const Diagrams& D, const int* col, const std::vector<ColVec>& nc, cd* c) {
  const Colour& CL = colour();
  for (size_t d = 0; d < D.diag.size(); ++d) {
    const ColVec& U = nc[D.diag[d].first];
    const ColVec& G = nc[D.diag[d].second];
    cd s = 0.0;
    for (int a = 0; a < 8; ++a)
      for (int j = 0; j < 3; ++j) s += CL.T[a][col[1]][j] * U.v[j] * G.v[a];
    c[d] = s;
  }
}

const std::vector<cd>& diagram_colour_matrix(int ng) {
  static std::map<int, std::vector<cd>> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(ng);
  if (it != cache.end()) return it->second;
  const Diagrams& D = diagrams(ng);
  const int nd = int(D.diag.size()), nl = D.nl;
  int ncfg = 81;
  for (int g = 0; g < ng; ++g) ncfg *= 8;
  std::vector<cd> C(size_t(nd) * nd, 0.0);
#pragma omp parallel
  {
    std::vector<cd> loc(size_t(nd) * nd, 0.0), c(nd);
    std::vector<ColVec> nc;
    int col[8];
#pragma omp for schedule(dynamic, 16)
    for (int cfg = 0; cfg < ncfg; ++cfg) {
      int r = cfg;
      for (int k = nl - 1; k >= 0; --k) {
        const int dim = k < 4 ? 3 : 8;
        col[k] = r % dim;
        r /= dim;
      }
      node_colours(D, col, nc);
      diagram_colours(D, col, nc, c.data());
      bool any = false;
      for (const cd& x : c) any = any || x != cd(0.0);
      if (!any) continue;
      for (int x = 0; x < nd; ++x) {
        if (c[x] == cd(0.0)) continue;
        const cd cx = std::conj(c[x]);
        for (int y = 0; y < nd; ++y) loc[size_t(x) * nd + y] += cx * c[y];
      }
    }
#pragma omp critical
    for (size_t i = 0; i < loc.size(); ++i) C[i] += loc[i];
  }
  return cache[ng] = C;
}

// ------------------------------------------------------------------ Lorentz
struct LVal {
  Spinor s;     // quark lines (column or row)
  CVec4 v;      // gluon currents, contravariant, propagator included
};

Mat4 quark_prop(const Vec4& k, real m, real w) {
  // i (k-slash + m) / (k^2 - m^2 + i m Gamma)
  const cd den = cd(dot(k, k) - m * m, m * w);
  return mscale(I1 / den, madd(slash(k), mscale(m, ident4())));
}

void amplitudes(const Diagrams& D, const SM& sm, const Vec4* p, const int* hel, std::vector<cd>& M) {
  const Gammas& G = gam();
  const int nl = D.nl;
  // momentum flowing into the diagram from each leg
  Vec4 q[8];
  for (int k = 0; k < nl; ++k) q[k] = k < 2 ? p[k] : neg(p[k]);
  auto mom = [&](uint32_t s) {
    Vec4 r = {0, 0, 0, 0};
    for (int k = 0; k < nl; ++k)
      if (s & (1u << k)) r = add(r, q[k]);
    return r;
  };
  std::vector<LVal> val(D.nodes.size());
  const cd ig = I1 * sm.gs;
  for (size_t i = 0; i < D.nodes.size(); ++i) {
    const Node& n = D.nodes[i];
    LVal r{};
    const Vec4 P = mom(n.legs);
    if (n.vtx == V_EXT) {
      const int leg = lowest_leg(n.legs);
      if (n.kind == K_U) r.s = u_spinor(p[0], 0.0, hel[0]);
      else if (n.kind == K_TB) r.s = v_spinor(p[3], sm.mt, hel[3]);
      else if (n.kind == K_T2) r.s = dbar(u_spinor(p[2], sm.mt, hel[2]));
      else r.v = conjv(eps_vec(p[leg], 0.0, sm.gauge_leg == leg ? 4 : hel[leg]));
    } else if (n.vtx == V_QG) {
      const Mat4 vg = mscale(ig, slash(val[n.ch[1]].v));
      const Spinor& c = val[n.ch[0]].s;
      if (n.kind == K_U) r.s = mv(quark_prop(P, 0.0, 0.0), mv(vg, c));
      else if (n.kind == K_TB) r.s = mv(quark_prop(P, sm.mt, sm.wt), mv(vg, c));
      else r.s = vm(vm(c, vg), quark_prop(neg(P), sm.mt, sm.wt));
    } else {
      CVec4 V{};
      if (n.vtx == V_GGG) {
        const CVec4& A = val[n.ch[0]].v;
        const CVec4& B = val[n.ch[1]].v;
        const Vec4 k = mom(D.nodes[n.ch[0]].legs), pp = mom(D.nodes[n.ch[1]].legs);
        const Vec4 qq = neg(add(k, pp));
        const cd ab = dot(A, B), bq = dot(A, sub(pp, qq)), aq = dot(B, sub(qq, k));
        const Vec4 kp = sub(k, pp);
        for (int m = 0; m < 4; ++m) V[m] = sm.gs * (ab * kp[m] + bq * B[m] + aq * A[m]);
      } else if (n.vtx == V_GGGG) {
        const CVec4& A = val[n.ch[0]].v;
        const CVec4& B = val[n.ch[1]].v;
        const CVec4& C = val[n.ch[2]].v;
        const cd ab = dot(A, B), ac = dot(A, C), bc = dot(B, C);
        const cd f = -I1 * sm.gs * sm.gs;
        for (int m = 0; m < 4; ++m) {
          cd t;
          if (n.term == 0) t = ac * B[m] - bc * A[m];
          else if (n.term == 1) t = ab * C[m] - bc * A[m];
          else t = ab * C[m] - ac * B[m];
          V[m] = f * t;
        }
      } else {   // V_TT: i g (t2 gamma^sigma tb)
        const Spinor& tb = val[n.ch[0]].s;
        const Spinor& t2 = val[n.ch[1]].s;
        for (int m = 0; m < 4; ++m) V[m] = ig * sandwich(t2, mv(G.g[m], tb));
      }
      r.v = cscale(-I1 / dot(P, P), V);
    }
    val[i] = r;
  }
  const Spinor vb = dbar(v_spinor(p[1], 0.0, hel[1]));
  M.resize(D.diag.size());
  for (size_t d = 0; d < D.diag.size(); ++d) {
    const Spinor& u = val[D.diag[d].first].s;
    const CVec4& g = val[D.diag[d].second].v;
    M[d] = sandwich(vb, mv(mscale(ig, slash(g)), u)) / I1;
  }
}

}  // namespace

int uu_tt_gluons_diagrams(int ng) { return int(diagrams(ng).diag.size()); }

// p == nullptr: build the diagrams and the colour matrix only (before a parallel loop)
real uu_tt_gluons_me2(int ng, const SM& sm, const Vec4* p) {
  const Diagrams& D = diagrams(ng);
  const std::vector<cd>& C = diagram_colour_matrix(ng);
  if (!p) return 0.0;
  const int nd = int(D.diag.size()), nl = D.nl;
  std::vector<cd> M;
  int hel[8];
  real tot = 0.0;
  for (int hc = 0; hc < (1 << nl); ++hc) {
    for (int k = 0; k < nl; ++k) hel[k] = ((hc >> (nl - 1 - k)) & 1) ? 1 : -1;
    amplitudes(D, sm, p, hel, M);
    cd s = 0.0;
    for (int x = 0; x < nd; ++x) {
      cd row = 0.0;
      for (int y = 0; y < nd; ++y) row += C[size_t(x) * nd + y] * M[y];
      s += std::conj(M[x]) * row;
    }
    tot += std::real(s);
  }
  return tot;
}

}  // namespace orc
