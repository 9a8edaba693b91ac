// Oracle: Feynman-diagram sums for the processes with quarks and leptons,
// written from the Lagrangians of the paper's Sec. 4.2 with explicit Dirac
// matrices; colour sums by brute force over explicit SU(3) indices.
// Test infrastructure only; shares no code with the product path.
//
// Every diagram is assembled as i*M_d = (product of Feynman-rule factors,
// each carrying its own i) and returned as M_d = (i*M_d)/i.  Relative signs of
// diagrams that pair external fermions differently are the signs of the
// corresponding permutations (Wick's theorem).
#include "procs.hpp"

#include <functional>
#include <map>
#include <mutex>

namespace orc {

const Gammas& gam() {
  static const Gammas G;
  return G;
}
const Colour& colour() {
  static const Colour C;
  return C;
}

namespace {

// external states --------------------------------------------------------
Spinor u_in(const Vec4& p, real m, int h) { return u_spinor(p, m, h); }           // incoming fermion
Spinor vbar_in(const Vec4& p, real m, int h) { return dbar(v_spinor(p, m, h)); }  // incoming antifermion
Spinor ubar_out(const Vec4& p, real m, int h) { return dbar(u_spinor(p, m, h)); } // outgoing fermion
Spinor v_out(const Vec4& p, real m, int h) { return v_spinor(p, m, h); }          // outgoing antifermion
CVec4 eps_in(const SM& sm, int leg, const Vec4& k, real m, int h) {
  return eps_vec(k, m, sm.gauge_leg == leg ? 4 : h);
}
CVec4 eps_out(const SM& sm, int leg, const Vec4& k, real m, int h) {
  return conjv(eps_vec(k, m, sm.gauge_leg == leg ? 4 : h));
}
Mat4 chiral(cd gl, cd gr) { return madd(mscale(gl, gam().pl), mscale(gr, gam().pr)); }

// ------------------------------------------------------------------ C0
// e-(p0) e+(p1) -> mu-(p2) mu+(p3): s-channel photon and Z.
void amp_ee_mumu(const SM& sm, const Vec4* p, const int* h, cd* M) {
  const Spinor u0 = u_in(p[0], 0, h[0]);
  const Spinor vb1 = vbar_in(p[1], 0, h[1]);
  const Spinor ub2 = ubar_out(p[2], 0, h[2]);
  const Spinor v3 = v_out(p[3], 0, h[3]);
  const Vec4 q = add(p[0], p[1]);
  const real Ql = -1.0, T3 = -0.5;
  // photon
  {
    const Mat4 c = chiral(sm.g_a(Ql), sm.g_a(Ql));
    const CVec4 je = cscale(I1, current(vb1, c, u0));
    const CVec4 jm = cscale(I1, current(ub2, c, v3));
    M[0] = dot(je, contract(massless_prop(q), jm)) / I1;
  }
  // Z
  {
    const Mat4 c = chiral(sm.gl_z(T3, Ql), sm.gr_z(Ql));
    const CVec4 je = cscale(I1, current(vb1, c, u0));
    const CVec4 jm = cscale(I1, current(ub2, c, v3));
    M[1] = dot(je, contract(vector_prop(q, sm.numz2, sm.muz2), jm)) / I1;
  }
}
void col_trivial2(const int*, cd* c) { c[0] = c[1] = 1.0; }

// --------------------------------------------------- gluon-pair -> top pair
// Production pieces X_d acting between the top and antitop ends of the heavy
// fermion line, for incoming gluons (k1, e1), (k2, e2); pt is the momentum
// along the fermion arrow at the top end.  Colour stripped:
//   T: gluon 1 next to the top   (T^a T^b)_{ij}
//   U: gluon 2 next to the top   (T^b T^a)_{ij}
//   S: s-channel gluon           f^{abc} T^c_{ij}
void ttbar_production(const SM& sm, const Vec4& k1, const CVec4& e1, const Vec4& k2, const CVec4& e2,
                      const Vec4& pt, Mat4 X[3]) {
  const cd igs = I1 * sm.gs;
  const Mat4 v1 = mscale(igs, slash(e1));
  const Mat4 v2 = mscale(igs, slash(e2));
  X[0] = mul(mul(v1, fermion_prop(sub(pt, k1), sm.mt, sm.wt)), v2);
  X[1] = mul(mul(v2, fermion_prop(sub(pt, k2), sm.mt, sm.wt)), v1);
  // triple-gluon vertex g f^{abc}[g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
  // with legs (k1,a,mu), (k2,b,nu), (-(k1+k2),c,rho), all momenta incoming
  const Vec4 k3 = neg(add(k1, k2));
  const cd e12 = dot(e1, e2);
  const cd e1p = dot(e1, sub(k2, k3));   // (p - q).e1
  const cd e2p = dot(e2, sub(k3, k1));   // (q - k).e2
  CVec4 G;
  for (int r = 0; r < 4; ++r) G[r] = sm.gs * (e12 * (k1[r] - k2[r]) + e2[r] * e1p + e1[r] * e2p);
  const CVec4 A = contract(massless_prop(add(k1, k2)), G);   // propagator -i g/q^2
  X[2] = mscale(igs, slash(A));
}
void col_ttbar(const int* col, int a, int b, int i, int j, cd* c) {
  const Colour& C = colour();
  (void)col;
  cd t = 0, u = 0, s = 0;
  for (int k = 0; k < 3; ++k) {
    t += C.T[a][i][k] * C.T[b][k][j];
    u += C.T[b][i][k] * C.T[a][k][j];
  }
  for (int e = 0; e < 8; ++e) s += C.f[a][b][e] * C.T[e][i][j];
  c[0] = t;
  c[1] = u;
  c[2] = s;
}

// ------------------------------------------------------------------ C1
// g(p0) g(p1) -> t tbar -> b(p2) e+(p3) nu_e(p4) bbar(p5) mu-(p6) nu_mu~(p7)
void amp_gg_tt_6f(const SM& sm, const Vec4* p, const int* h, cd* M) {
  const CVec4 e1 = eps_in(sm, 0, p[0], 0, h[0]);
  const CVec4 e2 = eps_in(sm, 1, p[1], 0, h[1]);
  const Spinor ub = ubar_out(p[2], 0, h[2]);
  const Spinor vep = v_out(p[3], 0, h[3]);
  const Spinor ubnu = ubar_out(p[4], 0, h[4]);
  const Spinor vbb = v_out(p[5], 0, h[5]);
  const Spinor ubmu = ubar_out(p[6], 0, h[6]);
  const Spinor vnub = v_out(p[7], 0, h[7]);
  const cd igw = I1 * sm.g_w();
  const Mat4 PL = gam().pl;
  // W+ -> e+ nu_e and W- -> mu- nu_mu~ with their propagators
  const CVec4 Wp = contract(vector_prop(add(p[3], p[4]), sm.numw2, sm.muw2), cscale(igw, current(ubnu, PL, vep)));
  const CVec4 Wm = contract(vector_prop(add(p[6], p[7]), sm.numw2, sm.muw2), cscale(igw, current(ubmu, PL, vnub)));
  const Vec4 pt = add(add(p[2], p[3]), p[4]);
  const Vec4 ptb = add(add(p[5], p[6]), p[7]);
  // b <- t (W+ emission) ... tbar -> bbar (W- emission)
  const Spinor left = vm(vm(ub, mul(mscale(igw, slash(Wp)), PL)), fermion_prop(pt, sm.mt, sm.wt));
  const Spinor right = mv(fermion_prop(neg(ptb), sm.mt, sm.wt), mv(mul(mscale(igw, slash(Wm)), PL), vbb));
  Mat4 X[3];
  ttbar_production(sm, p[0], e1, p[1], e2, pt, X);
  for (int d = 0; d < 3; ++d) M[d] = sandwich(left, mv(X[d], right)) / I1;
}
void col_gg_tt_6f(const int* col, cd* c) { col_ttbar(col, col[0], col[1], col[2], col[5], c); }

// g(p0) g(p1) -> t(p2) tbar(p3), stable tops
void amp_gg_tt(const SM& sm, const Vec4* p, const int* h, cd* M) {
  const CVec4 e1 = eps_in(sm, 0, p[0], 0, h[0]);
  const CVec4 e2 = eps_in(sm, 1, p[1], 0, h[1]);
  const Spinor left = ubar_out(p[2], sm.mt, h[2]);
  const Spinor right = v_out(p[3], sm.mt, h[3]);
  Mat4 X[3];
  ttbar_production(sm, p[0], e1, p[1], e2, p[2], X);
  for (int d = 0; d < 3; ++d) M[d] = sandwich(left, mv(X[d], right)) / I1;
}
void col_gg_tt(const int* col, cd* c) { col_ttbar(col, col[0], col[1], col[2], col[3], c); }

// u(p0) ubar(p1) -> t(p2) tbar(p3) via an s-channel gluon
void amp_uu_tt(const SM& sm, const Vec4* p, const int* h, cd* M) {
  const Spinor u0 = u_in(p[0], 0, h[0]);
  const Spinor vb1 = vbar_in(p[1], 0, h[1]);
  const Spinor ub2 = ubar_out(p[2], sm.mt, h[2]);
  const Spinor v3 = v_out(p[3], sm.mt, h[3]);
  const cd igs = I1 * sm.gs;
  const Mat4 one = ident4();
  const CVec4 jq = cscale(igs, current(vb1, one, u0));
  const CVec4 jt = cscale(igs, current(ub2, one, v3));
  M[0] = dot(jq, contract(massless_prop(add(p[0], p[1])), jt)) / I1;
}
void col_uu_tt(const int* col, cd* c) {
  const Colour& C = colour();
  cd s = 0;
  for (int a = 0; a < 8; ++a) s += C.T[a][col[1]][col[0]] * C.T[a][col[2]][col[3]];
  c[0] = s;
}

// ---------------------------------------------------- V V -> H H blocks
struct Boson {
  cd num2, pole2;  // unitary-gauge numerator mass^2 and pole
  cd g_vvh;        // Feynman rule / i of V V H
  real g_vvhh;   // Feynman rule / i of V V H H
};
Boson boson_w(const SM& sm) { return {sm.numw2, sm.muw2, sm.g_wwh, sm.g_wwhh}; }
Boson boson_z(const SM& sm) { return {sm.numz2, sm.muz2, sm.g_zzh, sm.g_zzhh}; }

// i*(amplitude pieces) of V(E1,q1) V(E2,q2) -> H(h1) H(h2): contact, s-channel
// Higgs, t- and u-channel vector exchange.  E1, E2 are contravariant
// polarisations (or propagated currents), q1, q2 incoming, h1, h2 outgoing.
void vv_hh(const SM& sm, const Boson& B, const CVec4& E1, const Vec4& q1, const CVec4& E2, const Vec4& q2,
           const Vec4& h1, const Vec4& h2, cd out[4]) {
  const cd e12 = dot(E1, E2);
  out[0] = I1 * B.g_vvhh * e12;
  out[1] = (I1 * B.g_vvh * e12) * scalar_prop(add(q1, q2), sm.mh, sm.wh) * (I1 * sm.g_hhh);
  const cd ig2 = (I1 * B.g_vvh) * (I1 * B.g_vvh);
  out[2] = ig2 * dot(E1, contract(vector_prop(sub(q1, h1), B.num2, B.pole2), E2));
  out[3] = ig2 * dot(E1, contract(vector_prop(sub(q1, h2), B.num2, B.pole2), E2));
}

// i*(amplitude pieces) of V(E1,q1) V(E2,q2) -> H(h[0]) H(h[1]) H(h[2]): every
// tree of the VVH, VVHH, HHH and HHHH vertices, 25 in all.  The vector line runs
// from E1 to E2; along it sit one, two or three attachments, each a VVH vertex
// carrying one Higgs or an off-shell H* that splits into the rest, or a VVHH
// vertex carrying two.  The vector line's momentum after an attachment is q1
// minus the Higgs momenta attached so far.
void vv_hhh(const SM& sm, const Boson& B, const CVec4& E1, const Vec4& q1, const CVec4& E2, const Vec4& q2,
            const Vec4* h, cd* out) {
  const cd g3 = I1 * B.g_vvh, g4 = I1 * B.g_vvhh, s3 = I1 * sm.g_hhh, s4 = I1 * sm.g_hhhh;
  auto sp = [&](const Vec4& q) { return scalar_prop(q, sm.mh, sm.wh); };
  auto vp = [&](const Vec4& q) { return vector_prop(q, B.num2, B.pole2); };
  auto line1 = [&](const Vec4& k) { return dot(E1, contract(vp(k), E2)); };   // E1 . D(k) . E2
  const int split[3][3] = {{0, 1, 2}, {1, 0, 2}, {2, 0, 1}};                  // Higgs i alone, pair (j, k)
  const cd e12 = dot(E1, E2);
  const Vec4 Q = add(q1, q2);
  int d = 0;
  // one attachment: VVH with H* -> H H H (the quartic vertex, or H* -> H H* -> H H H),
  // or VVHH with one Higgs and an H* -> H H
  out[d++] = g3 * e12 * sp(Q) * s4;
  for (const auto& ijk : split) {
    const Vec4 hjk = add(h[ijk[1]], h[ijk[2]]);
    out[d++] = g3 * e12 * sp(Q) * s3 * sp(hjk) * s3;
    out[d++] = g4 * e12 * sp(hjk) * s3;
  }
  // two attachments
  for (const auto& ijk : split) {
    const int i = ijk[0], j = ijk[1], k = ijk[2];
    const Vec4 hjk = add(h[j], h[k]);
    out[d++] = g3 * g3 * line1(sub(q1, h[i])) * sp(hjk) * s3;   // VVH(i), VVH(H* -> j k)
    out[d++] = g3 * g3 * line1(sub(q1, hjk)) * sp(hjk) * s3;    // VVH(H* -> j k), VVH(i)
    out[d++] = g3 * g4 * line1(sub(q1, h[i]));                  // VVH(i), VVHH(j, k)
    out[d++] = g4 * g3 * line1(sub(q1, hjk));                   // VVHH(j, k), VVH(i)
  }
  // three VVH attachments, in each order along the line
  const int order[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (const auto& o : order) {
    const Vec4 k1 = sub(q1, h[o[0]]), k2 = sub(k1, h[o[1]]);
    out[d++] = g3 * g3 * g3 * dot(E1, contract(vp(k1), contract(vp(k2), E2)));
  }
}

// ------------------------------------------------------------------ C3
// q(p0) q'(p1) -> q(p2) q'(p3) H H, H -> b(p4) bbar(p5), b(p6) bbar(p7)
// Quark-line "classes": which outgoing quark each incoming quark turns into,
// the exchanged boson and the Fermi sign of that pairing.
struct QuarkLine {
  int in, out;
  cd gl, gr;
};
struct FusionClass {
  QuarkLine l1, l2;
  int boson;  // 0 = W, 1 = Z
  real sign;
};
const real Qu = real(2) / 3, Qd = real(-1) / 3;

void amp_qq_qqhh_4b(const SM& sm, const std::vector<FusionClass>& classes, const Vec4* p, const int* h,
                    cd* M) {
  Spinor uin[2], ubout[2];
  uin[0] = u_in(p[0], 0, h[0]);
  uin[1] = u_in(p[1], 0, h[1]);
  ubout[0] = ubar_out(p[2], 0, h[2]);
  ubout[1] = ubar_out(p[3], 0, h[3]);
  const Spinor ub4 = ubar_out(p[4], 0, h[4]), v5 = v_out(p[5], 0, h[5]);
  const Spinor ub6 = ubar_out(p[6], 0, h[6]), v7 = v_out(p[7], 0, h[7]);
  // Higgs decays for the two b pairings (Yukawa vertex -i y_b, Higgs propagator)
  const cd iy = -I1 * sm.y_b;
  struct Pair {
    Vec4 h1, h2;
    cd d;
    real sign;
  } pairs[2];
  pairs[0].h1 = add(p[4], p[5]);
  pairs[0].h2 = add(p[6], p[7]);
  pairs[0].d = iy * sandwich(ub4, v5) * scalar_prop(pairs[0].h1, sm.mh, sm.wh) * iy * sandwich(ub6, v7) *
               scalar_prop(pairs[0].h2, sm.mh, sm.wh);
  pairs[0].sign = 1.0;
  pairs[1].h1 = add(p[4], p[7]);
  pairs[1].h2 = add(p[6], p[5]);
  pairs[1].d = iy * sandwich(ub4, v7) * scalar_prop(pairs[1].h1, sm.mh, sm.wh) * iy * sandwich(ub6, v5) *
               scalar_prop(pairs[1].h2, sm.mh, sm.wh);
  pairs[1].sign = -1.0;
  int d = 0;
  for (const FusionClass& fc : classes) {
    const Boson B = fc.boson == 0 ? boson_w(sm) : boson_z(sm);
    const QuarkLine* ls[2] = {&fc.l1, &fc.l2};
    CVec4 E[2];
    Vec4 q[2];
    for (int k = 0; k < 2; ++k) {
      const QuarkLine& L = *ls[k];
      q[k] = sub(p[L.in], p[L.out]);
      const CVec4 J = cscale(I1, current(ubout[L.out - 2], chiral(L.gl, L.gr), uin[L.in]));
      E[k] = contract(vector_prop(q[k], B.num2, B.pole2), J);
    }
    for (const Pair& pr : pairs) {
      cd part[4];
      vv_hh(sm, B, E[0], q[0], E[1], q[1], pr.h1, pr.h2, part);
      for (int j = 0; j < 4; ++j) M[d++] = fc.sign * pr.sign * part[j] * pr.d / I1;
    }
  }
}
std::vector<FusionClass> classes_ud(const SM& sm) {
  const cd gw = sm.g_w();
  return {
      {{0, 2, sm.gl_z(0.5, Qu), sm.gr_z(Qu)}, {1, 3, sm.gl_z(-0.5, Qd), sm.gr_z(Qd)}, 1, 1.0},  // ZZ
      {{0, 3, gw, 0.0}, {1, 2, gw, 0.0}, 0, -1.0},                                            // WW
  };
}
std::vector<FusionClass> classes_uu(const SM& sm) {
  return {
      {{0, 2, sm.gl_z(0.5, Qu), sm.gr_z(Qu)}, {1, 3, sm.gl_z(0.5, Qu), sm.gr_z(Qu)}, 1, 1.0},
      {{0, 3, sm.gl_z(0.5, Qu), sm.gr_z(Qu)}, {1, 2, sm.gl_z(0.5, Qu), sm.gr_z(Qu)}, 1, -1.0},
  };
}
void amp_ud_udhh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_qq_qqhh_4b(sm, classes_ud(sm), p, h, M); }
void amp_uu_uuhh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_qq_qqhh_4b(sm, classes_uu(sm), p, h, M); }
// colour: class 0 connects (0->2, 1->3), class 1 (0->3, 1->2); b pairing A
// (4,5)(6,7), pairing B (4,7)(6,5).
void col_qq_qqhh(const int* c, cd* out) {
  const real cls[2] = {real(c[2] == c[0] && c[3] == c[1]), real(c[3] == c[0] && c[2] == c[1])};
  const real prs[2] = {real(c[4] == c[5] && c[6] == c[7]), real(c[4] == c[7] && c[6] == c[5])};
  int d = 0;
  for (int k = 0; k < 2; ++k)
    for (int r = 0; r < 2; ++r)
      for (int j = 0; j < 4; ++j) out[d++] = cls[k] * prs[r];
}

// W-(p0) W+(p1) -> W-(p2) W+(p3) with on-shell external W's: the quartic
// contact, photon and Z exchange in the s and t channels through the W W V
// vertex, and Higgs exchange in the s and t channels (7 diagrams).  Feynman
// rules with every momentum incoming (an outgoing W- is an incoming W+ of
// momentum -p and polarisation eps*, and the reverse):
//   W+_mu(k1) W-_nu(k2) V_la(k3):  i g_V [g_mu nu (k1 - k2)_la + g_nu la (k2 - k3)_mu
//                                          + g_la mu (k3 - k1)_nu],  g_gamma = e, g_Z = g_W c_W;
//   W+_mu W+_nu W-_la W-_rho:      i g_W^2 [2 g_mu nu g_la rho - g_mu la g_nu rho - g_mu rho g_nu la];
//   W+_mu W-_nu H:                 i g_WWH g_mu nu.
// (eps_P, k_P) W+ and (eps_M, k_M) W- meet a vector boson of incoming momentum
// kV = -(k_P + k_M): the vertex contracted with both polarisations.
CVec4 wwv_current(const CVec4& eP, const Vec4& kP, const CVec4& eM, const Vec4& kM) {
  const Vec4 kV = neg(add(kP, kM));
  const cd pm = dot(eP, eM);
  const cd a = dot(eP, sub(kM, kV)), b = dot(eM, sub(kV, kP));
  const Vec4 d = sub(kP, kM);
  CVec4 r;
  for (int m = 0; m < 4; ++m) r[m] = pm * d[m] + a * eM[m] + b * eP[m];
  return r;
}
void amp_ww_ww(const SM& sm, const Vec4* p, const int* h, cd* M) {
  struct Ext {
    CVec4 e;
    Vec4 k;
  };
  const Ext A = {eps_in(sm, 1, p[1], sm.mw, h[1]), p[1]};            // W+ in
  const Ext B = {eps_out(sm, 2, p[2], sm.mw, h[2]), neg(p[2])};      // W- out = W+ in
  const Ext C = {eps_in(sm, 0, p[0], sm.mw, h[0]), p[0]};            // W- in
  const Ext D = {eps_out(sm, 3, p[3], sm.mw, h[3]), neg(p[3])};      // W+ out = W- in
  const cd gw2 = sm.gw * sm.gw, ga = sm.e, gzv = sm.gw * sm.cw, gh = sm.g_wwh;
  int d = 0;
  // contact
  M[d++] = (I1 * gw2 * (real(2) * dot(A.e, B.e) * dot(C.e, D.e) - dot(A.e, C.e) * dot(B.e, D.e) -
                        dot(A.e, D.e) * dot(B.e, C.e))) / I1;
  // s channel: (A, C) | (B, D); t channel: (A, D) | (B, C)
  const Ext* ch[2][4] = {{&A, &C, &B, &D}, {&A, &D, &B, &C}};
  for (const auto& c : ch) {
    const Ext &P1 = *c[0], &M1 = *c[1], &P2 = *c[2], &M2 = *c[3];
    const Vec4 q = add(P1.k, M1.k);
    const CVec4 G1 = wwv_current(P1.e, P1.k, M1.e, M1.k);
    const CVec4 G2 = wwv_current(P2.e, P2.k, M2.e, M2.k);
    M[d++] = ((I1 * ga) * (I1 * ga) * dot(G1, contract(massless_prop(q), G2))) / I1;
    M[d++] = ((I1 * gzv) * (I1 * gzv) * dot(G1, contract(vector_prop(q, sm.numz2, sm.muz2), G2))) / I1;
    M[d++] = ((I1 * gh) * (I1 * gh) * dot(P1.e, M1.e) * scalar_prop(q, sm.mh, sm.wh) * dot(P2.e, M2.e)) / I1;
  }
}
void col_trivial7(const int*, cd* c) {
  for (int j = 0; j < 7; ++j) c[j] = 1.0;
}

// u(p0) d(p1) -> u(p2) d(p3) H(p4) H(p5) H(p6) by Z Z and W W fusion: 2 x 25
// diagrams, the W W class with the Fermi sign of its quark pairing.
void amp_ud_udhhh(const SM& sm, const Vec4* p, const int* h, cd* M) {
  const Spinor uin[2] = {u_in(p[0], 0, h[0]), u_in(p[1], 0, h[1])};
  const Spinor ubout[2] = {ubar_out(p[2], 0, h[2]), ubar_out(p[3], 0, h[3])};
  int d = 0;
  for (const FusionClass& fc : classes_ud(sm)) {
    const Boson B = fc.boson == 0 ? boson_w(sm) : boson_z(sm);
    const QuarkLine* ls[2] = {&fc.l1, &fc.l2};
    CVec4 E[2];
    Vec4 q[2];
    for (int k = 0; k < 2; ++k) {
      const QuarkLine& L = *ls[k];
      q[k] = sub(p[L.in], p[L.out]);
      const CVec4 J = cscale(I1, current(ubout[L.out - 2], chiral(L.gl, L.gr), uin[L.in]));
      E[k] = contract(vector_prop(q[k], B.num2, B.pole2), J);
    }
    cd part[25];
    vv_hhh(sm, B, E[0], q[0], E[1], q[1], p + 4, part);
    for (int j = 0; j < 25; ++j) M[d++] = fc.sign * part[j] / I1;
  }
}
// colour: class 0 connects (0->2, 1->3), class 1 (0->3, 1->2)
void col_qq_qqhhh(const int* c, cd* out) {
  const real cls[2] = {real(c[2] == c[0] && c[3] == c[1]), real(c[3] == c[0] && c[2] == c[1])};
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 25; ++j) out[25 * k + j] = cls[k];
}

// V(p0) V(p1) -> H(p2) H(p3) H(p4) with on-shell external vectors
void amp_vv_hhh(const SM& sm, const Boson& B, real mv, const Vec4* p, const int* h, cd* M) {
  const CVec4 E1 = eps_in(sm, 0, p[0], mv, h[0]);
  const CVec4 E2 = eps_in(sm, 1, p[1], mv, h[1]);
  cd part[25];
  vv_hhh(sm, B, E1, p[0], E2, p[1], p + 2, part);
  for (int j = 0; j < 25; ++j) M[j] = part[j] / I1;
}
void amp_ww_hhh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_vv_hhh(sm, boson_w(sm), sm.mw, p, h, M); }
void amp_zz_hhh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_vv_hhh(sm, boson_z(sm), sm.mz, p, h, M); }
void col_trivial25(const int*, cd* c) {
  for (int j = 0; j < 25; ++j) c[j] = 1.0;
}

// V(p0) V(p1) -> H(p2) H(p3) with on-shell external vectors
void amp_vv_hh(const SM& sm, const Boson& B, real mv, const Vec4* p, const int* h, cd* M) {
  const CVec4 E1 = eps_in(sm, 0, p[0], mv, h[0]);
  const CVec4 E2 = eps_in(sm, 1, p[1], mv, h[1]);
  cd part[4];
  vv_hh(sm, B, E1, p[0], E2, p[1], p[2], p[3], part);
  for (int j = 0; j < 4; ++j) M[j] = part[j] / I1;
}
void amp_ww_hh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_vv_hh(sm, boson_w(sm), sm.mw, p, h, M); }
void amp_zz_hh(const SM& sm, const Vec4* p, const int* h, cd* M) { amp_vv_hh(sm, boson_z(sm), sm.mz, p, h, M); }
void col_trivial4(const int*, cd* c) { c[0] = c[1] = c[2] = c[3] = 1.0; }

const std::vector<int> F = {-1, 1}, V0 = {-1, 1}, VM = {-1, 0, 1}, S = {0};

}  // namespace

const ProcDef* find_proc(int id) {
  static std::map<int, ProcDef> table;
  static std::once_flag once;
  std::call_once(once, [] {
    table[OR_EE_MUMU] = {4, {F, F, F, F}, 2, {1, 1, 1, 1}, amp_ee_mumu, col_trivial2};
    table[OR_GG_TT_6F] = {8, {V0, V0, F, F, F, F, F, F}, 3, {8, 8, 3, 1, 1, 3, 1, 1}, amp_gg_tt_6f, col_gg_tt_6f};
    table[OR_UD_UDHH_4B] = {8, {F, F, F, F, F, F, F, F}, 16, {3, 3, 3, 3, 3, 3, 3, 3}, amp_ud_udhh, col_qq_qqhh};
    table[OR_UU_UUHH_4B] = {8, {F, F, F, F, F, F, F, F}, 16, {3, 3, 3, 3, 3, 3, 3, 3}, amp_uu_uuhh, col_qq_qqhh};
    table[OR_UU_TT] = {4, {F, F, F, F}, 1, {3, 3, 3, 3}, amp_uu_tt, col_uu_tt};
    table[OR_GG_TT] = {4, {V0, V0, F, F}, 3, {8, 8, 3, 3}, amp_gg_tt, col_gg_tt};
    table[OR_WW_HH] = {4, {VM, VM, S, S}, 4, {1, 1, 1, 1}, amp_ww_hh, col_trivial4};
    table[OR_ZZ_HH] = {4, {VM, VM, S, S}, 4, {1, 1, 1, 1}, amp_zz_hh, col_trivial4};
    table[OR_UD_UDHHH] = {7, {F, F, F, F, S, S, S}, 50, {3, 3, 3, 3, 1, 1, 1}, amp_ud_udhhh, col_qq_qqhhh};
    table[OR_WW_HHH] = {5, {VM, VM, S, S, S}, 25, {1, 1, 1, 1, 1}, amp_ww_hhh, col_trivial25};
    table[OR_ZZ_HHH] = {5, {VM, VM, S, S, S}, 25, {1, 1, 1, 1, 1}, amp_zz_hhh, col_trivial25};
    table[OR_WW_WW] = {4, {VM, VM, VM, VM}, 7, {1, 1, 1, 1}, amp_ww_ww, col_trivial7};
  });
  auto it = table.find(id);
  return it == table.end() ? nullptr : &it->second;
}

// C_dd' = sum over all explicit colour assignments of conj(c_d) c_d'
const std::vector<cd>& colour_matrix(int id, const ProcDef& P) {
  static std::map<int, std::vector<cd>> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(id);
  if (it != cache.end()) return it->second;
  const int nd = P.ndiag;
  std::vector<cd> C(nd * nd, 0.0);
  std::vector<int> col(P.nlegs, 0);
  std::vector<cd> c(nd);
  while (true) {
    P.colf(col.data(), c.data());
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < nd; ++b) C[a * nd + b] += std::conj(c[a]) * c[b];
    int k = P.nlegs - 1;
    while (k >= 0 && col[k] + 1 >= P.coldim[k]) col[k--] = 0;
    if (k < 0) break;
    ++col[k];
  }
  return cache[id] = C;
}

std::vector<std::vector<int>> helicity_table(const ProcDef& P) {
  std::vector<std::vector<int>> out;
  std::vector<int> idx(P.nlegs, 0);
  while (true) {
    std::vector<int> h(P.nlegs);
    for (int k = 0; k < P.nlegs; ++k) h[k] = P.helvals[k][idx[k]];
    out.push_back(h);
    int k = P.nlegs - 1;
    while (k >= 0 && idx[k] + 1 >= int(P.helvals[k].size())) idx[k--] = 0;
    if (k < 0) break;
    ++idx[k];
  }
  return out;
}

// Colour-factor vectors c_d of every explicit colour assignment with at least
// one non-zero factor (assignments with all factors zero contribute nothing).
const std::vector<std::vector<cd>>& colour_assignments(int id, const ProcDef& P) {
  static std::map<int, std::vector<std::vector<cd>>> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(id);
  if (it != cache.end()) return it->second;
  std::vector<std::vector<cd>> out;
  std::vector<int> col(P.nlegs, 0);
  std::vector<cd> c(P.ndiag);
  while (true) {
    P.colf(col.data(), c.data());
    bool any = false;
    for (const cd& x : c) any = any || std::abs(x) > 0.0;
    if (any) out.push_back(c);
    int k = P.nlegs - 1;
    while (k >= 0 && col[k] + 1 >= P.coldim[k]) col[k--] = 0;
    if (k < 0) break;
    ++col[k];
  }
  return cache[id] = out;
}

// sum over explicit colours of |sum_d c_d M_d|^2 for one helicity combination
real me2_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm, const Vec4* p,
                        const int* h) {
  const int nd = P.ndiag;
  std::vector<cd> M(nd);
  P.amp(sm, p, h, M.data());
  real s = 0.0;
  for (const auto& c : cols) {
    cd a = 0;
    for (int d = 0; d < nd; ++d) a += c[d] * M[d];
    s += std::norm(a);
  }
  return s;
}

// Conditioning of the diagram sum for one helicity: accumulates
// sum_col |sum_d c_d M_d|^2 into a2 and sum_col (sum_d |c_d M_d|)^2 into b2.
void condition_one_helicity(const ProcDef& P, const std::vector<std::vector<cd>>& cols, const SM& sm,
                            const Vec4* p, const int* h, real& a2, real& b2) {
  const int nd = P.ndiag;
  std::vector<cd> M(nd);
  P.amp(sm, p, h, M.data());
  for (const auto& c : cols) {
    cd a = 0;
    real b = 0;
    for (int d = 0; d < nd; ++d) {
      a += c[d] * M[d];
      b += std::abs(c[d] * M[d]);
    }
    a2 += std::norm(a);
    b2 += b * b;
  }
}

// ------------------------------------------------ trace-based 2 -> 2 pins
// Spin sums from the completeness relations sum u ubar = pslash + m,
// sum v vbar = pslash - m and the physical gluon polarisation sum
// -g + (k r + r k)/(k.r) with reference vector r = the other gluon.
namespace {
Mat4 bar(const Mat4& A) {
  // gamma^0 A^dagger gamma^0
  Mat4 d;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) d.m[i][j] = std::conj(A.m[j][i]);
  return mul(mul(gam().g[0], d), gam().g[0]);
}
Mat4 pm(const Vec4& p, real m) { return madd(slash(p), mscale(m, ident4())); }
}  // namespace

real trace_me2(int id, const SM& sm, const Vec4* p) {
  const Gammas& G = gam();
  if (id == OR_UU_TT) {
    const real s = dot(add(p[0], p[1]), add(p[0], p[1]));
    cd tot = 0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        const cd t1 = trace(mul(mul(G.g[mu], slash(p[0])), mul(G.g[nu], slash(p[1]))));
        const cd t2 = trace(mul(mul(G.g[mu], pm(p[3], -sm.mt)), mul(G.g[nu], pm(p[2], sm.mt))));
        tot += metric(mu) * metric(nu) * t1 * t2;
      }
    const real g4 = std::pow(sm.gs, 4);
    return 2.0 * g4 / (s * s) * std::real(tot);   // colour: Tr(T^a T^b) Tr(T^a T^b) = 2
  }
  if (id == OR_GG_TT) {
    // X_d with open gluon indices: replace e1 -> unit vector along mu (lower index)
    Mat4 X[4][4][3];
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        CVec4 e1{}, e2{};
        e1[mu] = metric(mu);  // contravariant components of the basis covector
        e2[nu] = metric(nu);
        ttbar_production(sm, p[0], e1, p[1], e2, p[2], X[mu][nu]);
      }
    auto proj = [](const Vec4& k, const Vec4& r, int a, int b) {
      // lower-index projector P_ab = -g_ab + (k_a r_b + r_a k_b)/(k.r)
      const real ka = metric(a) * k[a], kb = metric(b) * k[b];
      const real ra = metric(a) * r[a], rb = metric(b) * r[b];
      return -(a == b ? metric(a) : 0.0) + (ka * rb + ra * kb) / dot(k, r);
    };
    const ProcDef& P = *find_proc(OR_GG_TT);
    const std::vector<cd>& C = colour_matrix(OR_GG_TT, P);
    const Mat4 At = pm(p[3], -sm.mt), Bt = pm(p[2], sm.mt);
    cd tot = 0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu)
        for (int mp = 0; mp < 4; ++mp)
          for (int np = 0; np < 4; ++np) {
            const real w = proj(p[0], p[1], mu, mp) * proj(p[1], p[0], nu, np);
            if (w == 0.0) continue;
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) {
                // sum_col (c_a X_a)(c_b X_b)^bar -> conj-weighted C
                const cd c = C[b * 3 + a];
                tot += w * c * trace(mul(mul(X[mu][nu][a], At), mul(bar(X[mp][np][b]), Bt)));
              }
          }
    return std::real(tot);
  }
  return -1.0;
}

// Two-body decay widths at tree level from the oracle's own W-fermion vertex
// (coefficient -i g_w gamma^mu P_L, g_w = SM::g_w()), helicity spinors and
// massive polarisation vectors, summed over every spin state, averaged over
// the decaying particle's, and integrated over the (isotropic) two-body phase
// space: Gamma = |p| / (8 pi M^2) * (1 / N_spin) * sum |M|^2.
//   which 0: W+ -> e+ nu_e  (massless leptons), W at rest with mass m_W;
//   which 1: t -> b W+      (massless b), top at rest with mass m_t.
real decay_width(const SM& sm, int which) {
  const Mat4 PL = gam().pl;
  const real st = real(0.6), ct = real(0.8);   // any decay axis: the spin sum is isotropic
  if (which == 0) {
    const real m = sm.mw, e = m / 2;
    const Vec4 pe = {e, e * st, 0, e * ct}, pn = {e, -e * st, 0, -e * ct};
    const Vec4 kw = {m, 0, 0, 0};
    real sum = 0;
    for (int lw : {-1, 0, 1}) {
      const CVec4 ew = eps_vec(kw, m, lw);
      for (int hn : {-1, 1})
        for (int he : {-1, 1}) {
          const CVec4 j = current(dbar(u_spinor(pn, 0, hn)), PL, v_spinor(pe, 0, he));
          const cd M = sm.g_w() * dot(j, ew);
          sum += std::norm(M);
        }
    }
    return (e / (8 * PI * m * m)) * sum / 3;
  }
  if (which == 1) {
    const real mt = sm.mt, mw = sm.mw;
    const real p = (mt * mt - mw * mw) / (2 * mt);
    const Vec4 pb = {p, p * st, 0, p * ct};
    const Vec4 kw = {std::sqrt(p * p + mw * mw), -p * st, 0, -p * ct};
    const Vec4 kt = {mt, 0, 0, 0};
    real sum = 0;
    for (int ht : {-1, 1})
      for (int hb : {-1, 1})
        for (int lw : {-1, 0, 1}) {
          const CVec4 ew = conjv(eps_vec(kw, mw, lw));
          const CVec4 j = current(dbar(u_spinor(pb, 0, hb)), PL, u_spinor(kt, mt, ht));
          sum += std::norm(sm.g_w() * dot(j, ew));
        }
    return (p / (8 * PI * mt * mt)) * sum / 2;
  }
  return -1;
}

}  // namespace orc
