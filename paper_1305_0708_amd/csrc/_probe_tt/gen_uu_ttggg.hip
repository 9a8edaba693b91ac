// Generated from the process IR 'uu_ttggg' (fingerprint 0x8e3e43d03eccb7b8); do not edit.
#include "../generated_common.hpp"

namespace heget {
namespace {

// phase space: the collision and its resonances decay in two bodies (tree of 4 nodes);
// fills p[0 .. n_legs-1] and returns the event's weight dPhi_n
__device__ __forceinline__ double ps_tree_uu_ttggg(const KernelArgs& a, uint64_t event, int64_t i, mom* p) {
#pragma clang fp contract(off)   // each product and sum rounds on its own (plain IEEE)
  double u[11];
  ps_uniforms<11>(a.seed, event, u);
  const double h = 0.5 * a.sqrt_s;
  p[0] = {h, 0.0, 0.0, h};
  p[1] = {h, 0.0, 0.0, -h};
  // adaptive integration: the uniforms through the grid, its Jacobian in the weight
  double w = a.grid ? grid_map<11>(a, i, u) : 1.0;
  const double M0 = a.sqrt_s;
  const mom P0 = {a.sqrt_s, 0.0, 0.0, 0.0};
  double s1;
  w *= ps_mass(u[0], (a.prop[3].m) * (a.prop[3].m), (M0 - a.prop[3].m) * (M0 - a.prop[3].m), a.prop[0].m, a.prop[0].w, false, 20.0, s1);
  const double M1 = sqrt(s1);
  mom P1;
  w *= ps_decay(u[1], u[2], P0, M0, a.prop[3].m, M1, true, p[2], P1);
  double s2;
  w *= ps_mass(u[3], 0.0, (M1 - a.prop[3].m) * (M1 - a.prop[3].m), a.prop[0].m, a.prop[0].w, false, 20.0, s2);
  const double M2 = sqrt(s2);
  mom P2;
  w *= ps_decay(u[4], u[5], P1, M1, a.prop[3].m, M2, false, p[3], P2);
  double s3;
  w *= ps_mass(u[6], 0.0, M2 * M2, a.prop[0].m, a.prop[0].w, false, 20.0, s3);
  const double M3 = sqrt(s3);
  mom P3;
  w *= ps_decay(u[7], u[8], P2, M2, 0.0, M3, false, p[4], P3);
  w *= ps_decay(u[9], u[10], P3, M3, 0.0, 0.0, false, p[5], p[6]);
  return w;
}

// the event's physical momenta, one column per lane, read by every part
__shared__ mom pm_uu_ttggg[7][256];

// part 0: amplitudes 0 .. 39 (101 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part0(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5_6 = (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs4_5_6 = tv<T>(qs4_5_6);
  const cx<T> d4_5_6_0 = cvt<T>(inv_denominator(qs4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w9 = jvvxxx<T, false>(w4, Qs4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w10 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w11 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w12 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const wf<T> w14 = jvvxxx<T, false>(w13, Qs4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const wf<T> w16 = jvvxxx<T, false>(w15, Qs4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs2_3_4_5_6 = (-pr2) + (-pr3) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_4_5_6 = tv<T>(qs2_3_4_5_6);
  const cx<T> d2_3_4_5_6_0 = cvt<T>(inv_denominator(qs2_3_4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w17 = jvvxxx<T, false>(w7, Qs2_3, w9, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w18 = jvvxxx<T, false>(w7, Qs2_3, w10, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w19 = jvvxxx<T, false>(w7, Qs2_3, w11, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w20 = jvvxxx<T, false>(w7, Qs2_3, w12, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w21 = jvvxxx<T, false>(w7, Qs2_3, w14, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w22 = jvvxxx<T, false>(w7, Qs2_3, w16, Qs4_5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w23 = jgggxx<T, false>(w7, w4, w8, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w24 = jgggxx<T, false>(w8, w7, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w25 = jgggxx<T, false>(w4, w8, w7, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w26 = jgggxx<T, false>(w7, w13, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w27 = jgggxx<T, false>(w6, w7, w13, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w28 = jgggxx<T, false>(w13, w6, w7, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w29 = jgggxx<T, false>(w7, w15, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w30 = jgggxx<T, false>(w5, w7, w15, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w31 = jgggxx<T, false>(w15, w5, w7, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const wf<T> w37 = jvvxxx<T, false>(w32, Qs2_3_4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w38 = jvvxxx<T, false>(w34, Qs2_3_4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w39 = jvvxxx<T, false>(w36, Qs2_3_4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w40 = jgggxx<T, false>(w32, w5, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w41 = jgggxx<T, false>(w6, w32, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w42 = jgggxx<T, false>(w5, w6, w32, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w43 = jgggxx<T, false>(w34, w5, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w44 = jgggxx<T, false>(w6, w34, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w45 = jgggxx<T, false>(w5, w6, w34, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w46 = jgggxx<T, false>(w36, w5, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w47 = jgggxx<T, false>(w6, w36, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w48 = jgggxx<T, false>(w5, w6, w36, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const wf<T> w54 = jvvxxx<T, false>(w49, Qs2_3_5, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w55 = jvvxxx<T, false>(w51, Qs2_3_5, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w56 = jvvxxx<T, false>(w53, Qs2_3_5, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w57 = jgggxx<T, false>(w49, w4, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w58 = jgggxx<T, false>(w6, w49, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w59 = jgggxx<T, false>(w4, w6, w49, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w60 = jgggxx<T, false>(w51, w4, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w61 = jgggxx<T, false>(w6, w51, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w62 = jgggxx<T, false>(w4, w6, w51, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w63 = jgggxx<T, false>(w53, w4, w6, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w64 = jgggxx<T, false>(w6, w53, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w65 = jgggxx<T, false>(w4, w6, w53, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const wf<T> w71 = jvvxxx<T, false>(w66, Qs2_3_6, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const cx<T> amp0 = iovxxx<T>(w0, w1, w17, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp0);
  J[7] = J[7] + (T(-0.5) * amp0);
  J[9] = J[9] + (T(-0.5) * amp0);
  J[11] = J[11] + (T(0.5) * amp0);
  J[19] = J[19] + (T(-0.5) * amp0);
  J[23] = J[23] + (T(0.5) * amp0);
  J[35] = J[35] + (T(0.5) * amp0);
  J[47] = J[47] + (T(-0.5) * amp0);
  const cx<T> amp1 = iovxxx<T>(w0, w1, w18, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp1);
  J[8] = J[8] + (T(0.5) * amp1);
  J[10] = J[10] + (T(0.5) * amp1);
  J[11] = J[11] + (T(-0.5) * amp1);
  J[19] = J[19] + (T(0.5) * amp1);
  J[31] = J[31] + (T(-0.5) * amp1);
  J[43] = J[43] + (T(-0.5) * amp1);
  J[47] = J[47] + (T(0.5) * amp1);
  const cx<T> amp2 = iovxxx<T>(w0, w1, w19, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp2);
  J[8] = J[8] + (T(-0.5) * amp2);
  J[9] = J[9] + (T(0.5) * amp2);
  J[10] = J[10] + (T(-0.5) * amp2);
  J[23] = J[23] + (T(-0.5) * amp2);
  J[31] = J[31] + (T(0.5) * amp2);
  J[35] = J[35] + (T(-0.5) * amp2);
  J[43] = J[43] + (T(0.5) * amp2);
  const cx<T> amp3 = iovxxx<T>(w0, w1, w20, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp3);
  J[7] = J[7] + (T(-0.5) * amp3);
  J[9] = J[9] + (T(-0.5) * amp3);
  J[11] = J[11] + (T(0.5) * amp3);
  J[19] = J[19] + (T(-0.5) * amp3);
  J[23] = J[23] + (T(0.5) * amp3);
  J[35] = J[35] + (T(0.5) * amp3);
  J[47] = J[47] + (T(-0.5) * amp3);
  const cx<T> amp4 = iovxxx<T>(w0, w1, w21, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp4);
  J[8] = J[8] + (T(-0.5) * amp4);
  J[10] = J[10] + (T(-0.5) * amp4);
  J[11] = J[11] + (T(0.5) * amp4);
  J[19] = J[19] + (T(-0.5) * amp4);
  J[31] = J[31] + (T(0.5) * amp4);
  J[43] = J[43] + (T(0.5) * amp4);
  J[47] = J[47] + (T(-0.5) * amp4);
  const cx<T> amp5 = iovxxx<T>(w0, w1, w22, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp5);
  J[8] = J[8] + (T(-0.5) * amp5);
  J[9] = J[9] + (T(0.5) * amp5);
  J[10] = J[10] + (T(-0.5) * amp5);
  J[23] = J[23] + (T(-0.5) * amp5);
  J[31] = J[31] + (T(0.5) * amp5);
  J[35] = J[35] + (T(-0.5) * amp5);
  J[43] = J[43] + (T(0.5) * amp5);
  const cx<T> amp6 = iovxxx<T>(w0, w1, w23, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp6);
  J[7] = J[7] + (T(0.5) * amp6);
  J[14] = J[14] + (T(0.5) * amp6);
  J[15] = J[15] + (T(-0.5) * amp6);
  J[33] = J[33] + (T(0.5) * amp6);
  J[35] = J[35] + (T(-0.5) * amp6);
  J[45] = J[45] + (T(-0.5) * amp6);
  J[47] = J[47] + (T(0.5) * amp6);
  const cx<T> amp7 = iovxxx<T>(w0, w1, w24, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp7);
  J[11] = J[11] + (T(-0.5) * amp7);
  J[14] = J[14] + (T(-0.5) * amp7);
  J[15] = J[15] + (T(0.5) * amp7);
  J[19] = J[19] + (T(0.5) * amp7);
  J[23] = J[23] + (T(-0.5) * amp7);
  J[33] = J[33] + (T(-0.5) * amp7);
  J[45] = J[45] + (T(0.5) * amp7);
  const cx<T> amp8 = iovxxx<T>(w0, w1, w25, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp8);
  J[7] = J[7] + (T(-0.5) * amp8);
  J[9] = J[9] + (T(-0.5) * amp8);
  J[11] = J[11] + (T(0.5) * amp8);
  J[19] = J[19] + (T(-0.5) * amp8);
  J[23] = J[23] + (T(0.5) * amp8);
  J[35] = J[35] + (T(0.5) * amp8);
  J[47] = J[47] + (T(-0.5) * amp8);
  const cx<T> amp9 = iovxxx<T>(w0, w1, w26, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp9);
  J[8] = J[8] + (T(0.5) * amp9);
  J[17] = J[17] + (T(0.5) * amp9);
  J[29] = J[29] + (T(-0.5) * amp9);
  J[38] = J[38] + (T(0.5) * amp9);
  J[39] = J[39] + (T(-0.5) * amp9);
  J[43] = J[43] + (T(-0.5) * amp9);
  J[47] = J[47] + (T(0.5) * amp9);
  const cx<T> amp10 = iovxxx<T>(w0, w1, w27, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp10);
  J[11] = J[11] + (T(-0.5) * amp10);
  J[17] = J[17] + (T(-0.5) * amp10);
  J[19] = J[19] + (T(0.5) * amp10);
  J[29] = J[29] + (T(0.5) * amp10);
  J[31] = J[31] + (T(-0.5) * amp10);
  J[38] = J[38] + (T(-0.5) * amp10);
  J[39] = J[39] + (T(0.5) * amp10);
  const cx<T> amp11 = iovxxx<T>(w0, w1, w28, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp11);
  J[8] = J[8] + (T(-0.5) * amp11);
  J[10] = J[10] + (T(-0.5) * amp11);
  J[11] = J[11] + (T(0.5) * amp11);
  J[19] = J[19] + (T(-0.5) * amp11);
  J[31] = J[31] + (T(0.5) * amp11);
  J[43] = J[43] + (T(0.5) * amp11);
  J[47] = J[47] + (T(-0.5) * amp11);
  const cx<T> amp12 = iovxxx<T>(w0, w1, w29, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp12);
  J[10] = J[10] + (T(0.5) * amp12);
  J[21] = J[21] + (T(0.5) * amp12);
  J[26] = J[26] + (T(0.5) * amp12);
  J[27] = J[27] + (T(-0.5) * amp12);
  J[31] = J[31] + (T(-0.5) * amp12);
  J[35] = J[35] + (T(0.5) * amp12);
  J[41] = J[41] + (T(-0.5) * amp12);
  const cx<T> amp13 = iovxxx<T>(w0, w1, w30, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp13);
  J[9] = J[9] + (T(-0.5) * amp13);
  J[21] = J[21] + (T(-0.5) * amp13);
  J[23] = J[23] + (T(0.5) * amp13);
  J[26] = J[26] + (T(-0.5) * amp13);
  J[27] = J[27] + (T(0.5) * amp13);
  J[41] = J[41] + (T(0.5) * amp13);
  J[43] = J[43] + (T(-0.5) * amp13);
  const cx<T> amp14 = iovxxx<T>(w0, w1, w31, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp14);
  J[8] = J[8] + (T(-0.5) * amp14);
  J[9] = J[9] + (T(0.5) * amp14);
  J[10] = J[10] + (T(-0.5) * amp14);
  J[23] = J[23] + (T(-0.5) * amp14);
  J[31] = J[31] + (T(0.5) * amp14);
  J[35] = J[35] + (T(-0.5) * amp14);
  J[43] = J[43] + (T(0.5) * amp14);
  const cx<T> amp15 = iovxxx<T>(w0, w1, w37, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp15);
  J[7] = J[7] + (T(-0.5) * amp15);
  J[14] = J[14] + (T(-0.5) * amp15);
  J[15] = J[15] + (T(0.5) * amp15);
  J[33] = J[33] + (T(-0.5) * amp15);
  J[35] = J[35] + (T(0.5) * amp15);
  J[45] = J[45] + (T(0.5) * amp15);
  J[47] = J[47] + (T(-0.5) * amp15);
  const cx<T> amp16 = iovxxx<T>(w0, w1, w38, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp16);
  J[7] = J[7] + (T(0.5) * amp16);
  J[33] = J[33] + (T(0.5) * amp16);
  J[45] = J[45] + (T(-0.5) * amp16);
  const cx<T> amp17 = iovxxx<T>(w0, w1, w39, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp17);
  J[15] = J[15] + (T(0.5) * amp17);
  J[35] = J[35] + (T(0.5) * amp17);
  J[47] = J[47] + (T(-0.5) * amp17);
  const cx<T> amp18 = iovxxx<T>(w0, w1, w40, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp18);
  J[14] = J[14] + (T(0.5) * amp18);
  J[26] = J[26] + (T(0.5) * amp18);
  J[29] = J[29] + (T(-0.5) * amp18);
  J[38] = J[38] + (T(0.5) * amp18);
  J[41] = J[41] + (T(-0.5) * amp18);
  J[45] = J[45] + (T(-0.5) * amp18);
  J[47] = J[47] + (T(0.5) * amp18);
  const cx<T> amp19 = iovxxx<T>(w0, w1, w41, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp19);
  J[15] = J[15] + (T(-0.5) * amp19);
  J[26] = J[26] + (T(-0.5) * amp19);
  J[29] = J[29] + (T(0.5) * amp19);
  J[33] = J[33] + (T(0.5) * amp19);
  J[35] = J[35] + (T(-0.5) * amp19);
  J[38] = J[38] + (T(-0.5) * amp19);
  J[41] = J[41] + (T(0.5) * amp19);
  const cx<T> amp20 = iovxxx<T>(w0, w1, w42, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp20);
  J[7] = J[7] + (T(-0.5) * amp20);
  J[14] = J[14] + (T(-0.5) * amp20);
  J[15] = J[15] + (T(0.5) * amp20);
  J[33] = J[33] + (T(-0.5) * amp20);
  J[35] = J[35] + (T(0.5) * amp20);
  J[45] = J[45] + (T(0.5) * amp20);
  J[47] = J[47] + (T(-0.5) * amp20);
  const cx<T> amp21 = iovxxx<T>(w0, w1, w43, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp21);
  J[26] = J[26] + (T(-0.5) * amp21);
  J[38] = J[38] + (T(-0.5) * amp21);
  J[45] = J[45] + (T(0.5) * amp21);
  const cx<T> amp22 = iovxxx<T>(w0, w1, w44, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp22);
  J[26] = J[26] + (T(0.5) * amp22);
  J[33] = J[33] + (T(-0.5) * amp22);
  J[38] = J[38] + (T(0.5) * amp22);
  const cx<T> amp23 = iovxxx<T>(w0, w1, w45, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp23);
  J[7] = J[7] + (T(0.5) * amp23);
  J[33] = J[33] + (T(0.5) * amp23);
  J[45] = J[45] + (T(-0.5) * amp23);
  const cx<T> amp24 = iovxxx<T>(w0, w1, w46, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp24);
  J[29] = J[29] + (T(-0.5) * amp24);
  J[41] = J[41] + (T(-0.5) * amp24);
  J[47] = J[47] + (T(0.5) * amp24);
  const cx<T> amp25 = iovxxx<T>(w0, w1, w47, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp25);
  J[29] = J[29] + (T(0.5) * amp25);
  J[35] = J[35] + (T(-0.5) * amp25);
  J[41] = J[41] + (T(0.5) * amp25);
  const cx<T> amp26 = iovxxx<T>(w0, w1, w48, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp26);
  J[15] = J[15] + (T(0.5) * amp26);
  J[35] = J[35] + (T(0.5) * amp26);
  J[47] = J[47] + (T(-0.5) * amp26);
  const cx<T> amp27 = iovxxx<T>(w0, w1, w54, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp27);
  J[9] = J[9] + (T(-0.5) * amp27);
  J[21] = J[21] + (T(-0.5) * amp27);
  J[23] = J[23] + (T(0.5) * amp27);
  J[26] = J[26] + (T(-0.5) * amp27);
  J[27] = J[27] + (T(0.5) * amp27);
  J[41] = J[41] + (T(0.5) * amp27);
  J[43] = J[43] + (T(-0.5) * amp27);
  const cx<T> amp28 = iovxxx<T>(w0, w1, w55, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp28);
  J[9] = J[9] + (T(0.5) * amp28);
  J[21] = J[21] + (T(0.5) * amp28);
  J[41] = J[41] + (T(-0.5) * amp28);
  const cx<T> amp29 = iovxxx<T>(w0, w1, w56, g0_0, g0_1);
  J[23] = J[23] + (T(0.5) * amp29);
  J[26] = J[26] + (T(-0.5) * amp29);
  J[27] = J[27] + (T(0.5) * amp29);
  J[43] = J[43] + (T(-0.5) * amp29);
  const cx<T> amp30 = iovxxx<T>(w0, w1, w57, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp30);
  J[14] = J[14] + (T(0.5) * amp30);
  J[17] = J[17] + (T(-0.5) * amp30);
  J[26] = J[26] + (T(0.5) * amp30);
  J[39] = J[39] + (T(0.5) * amp30);
  J[41] = J[41] + (T(-0.5) * amp30);
  J[43] = J[43] + (T(0.5) * amp30);
  J[45] = J[45] + (T(-0.5) * amp30);
  const cx<T> amp31 = iovxxx<T>(w0, w1, w58, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp31);
  J[14] = J[14] + (T(-0.5) * amp31);
  J[17] = J[17] + (T(0.5) * amp31);
  J[21] = J[21] + (T(0.5) * amp31);
  J[23] = J[23] + (T(-0.5) * amp31);
  J[27] = J[27] + (T(-0.5) * amp31);
  J[39] = J[39] + (T(-0.5) * amp31);
  J[45] = J[45] + (T(0.5) * amp31);
  const cx<T> amp32 = iovxxx<T>(w0, w1, w59, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp32);
  J[9] = J[9] + (T(-0.5) * amp32);
  J[21] = J[21] + (T(-0.5) * amp32);
  J[23] = J[23] + (T(0.5) * amp32);
  J[26] = J[26] + (T(-0.5) * amp32);
  J[27] = J[27] + (T(0.5) * amp32);
  J[41] = J[41] + (T(0.5) * amp32);
  J[43] = J[43] + (T(-0.5) * amp32);
  const cx<T> amp33 = iovxxx<T>(w0, w1, w60, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp33);
  J[14] = J[14] + (T(-0.5) * amp33);
  J[39] = J[39] + (T(-0.5) * amp33);
  J[41] = J[41] + (T(0.5) * amp33);
  const cx<T> amp34 = iovxxx<T>(w0, w1, w61, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp34);
  J[14] = J[14] + (T(0.5) * amp34);
  J[21] = J[21] + (T(-0.5) * amp34);
  J[39] = J[39] + (T(0.5) * amp34);
  const cx<T> amp35 = iovxxx<T>(w0, w1, w62, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp35);
  J[9] = J[9] + (T(0.5) * amp35);
  J[21] = J[21] + (T(0.5) * amp35);
  J[41] = J[41] + (T(-0.5) * amp35);
  const cx<T> amp36 = iovxxx<T>(w0, w1, w63, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp36);
  J[26] = J[26] + (T(0.5) * amp36);
  J[43] = J[43] + (T(0.5) * amp36);
  J[45] = J[45] + (T(-0.5) * amp36);
  const cx<T> amp37 = iovxxx<T>(w0, w1, w64, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp37);
  J[23] = J[23] + (T(-0.5) * amp37);
  J[27] = J[27] + (T(-0.5) * amp37);
  J[45] = J[45] + (T(0.5) * amp37);
  const cx<T> amp38 = iovxxx<T>(w0, w1, w65, g0_0, g0_1);
  J[23] = J[23] + (T(0.5) * amp38);
  J[26] = J[26] + (T(-0.5) * amp38);
  J[27] = J[27] + (T(0.5) * amp38);
  J[43] = J[43] + (T(-0.5) * amp38);
  const cx<T> amp39 = iovxxx<T>(w0, w1, w71, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp39);
  J[11] = J[11] + (T(-0.5) * amp39);
  J[17] = J[17] + (T(-0.5) * amp39);
  J[19] = J[19] + (T(0.5) * amp39);
  J[29] = J[29] + (T(0.5) * amp39);
  J[31] = J[31] + (T(-0.5) * amp39);
  J[38] = J[38] + (T(-0.5) * amp39);
  J[39] = J[39] + (T(0.5) * amp39);
}

// part 1: amplitudes 40 .. 79 (134 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part1(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_4_5_6 = (-pr2) + (-pr3) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_4_5_6 = tv<T>(qs2_3_4_5_6);
  const cx<T> d2_3_4_5_6_0 = cvt<T>(inv_denominator(qs2_3_4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w72 = jvvxxx<T, false>(w68, Qs2_3_6, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w73 = jvvxxx<T, false>(w70, Qs2_3_6, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w74 = jgggxx<T, false>(w66, w4, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w75 = jgggxx<T, false>(w5, w66, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w76 = jgggxx<T, false>(w4, w5, w66, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w77 = jgggxx<T, false>(w68, w4, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w78 = jgggxx<T, false>(w5, w68, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w79 = jgggxx<T, false>(w4, w5, w68, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w80 = jgggxx<T, false>(w70, w4, w5, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w81 = jgggxx<T, false>(w5, w70, w4, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w82 = jgggxx<T, false>(w4, w5, w70, g2_0.r, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
  const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w83 = jvvxxx<T, false>(w7, Qs2_3, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w84 = jgggxx<T, false>(w7, w4, w5, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w85 = jgggxx<T, false>(w5, w7, w4, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w86 = jgggxx<T, false>(w4, w5, w7, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w87 = jvvxxx<T, false>(w32, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w88 = jvvxxx<T, false>(w34, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w89 = jvvxxx<T, false>(w36, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w90 = jvvxxx<T, false>(w49, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w91 = jvvxxx<T, false>(w51, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w92 = jvvxxx<T, false>(w53, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
  const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
  const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w93 = fvoxxx<T>(w2, w13, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w94 = fvoxxx<T>(w33, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w95 = fvoxxx<T>(w50, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w96 = jioxxx<T, false>(w3, w93, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w97 = jioxxx<T, false>(w3, w94, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w98 = jioxxx<T, false>(w3, w95, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w99 = jioxxx<T, false>(w35, w50, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w100 = jioxxx<T, false>(w52, w33, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs3_4_5 = (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs3_4_5 = tv<T>(qs3_4_5);
  const cx<T> d3_4_5_3 = cvt<T>(inv_denominator(qs3_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w101 = fvixxx<T>(w3, w13, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w102 = fvixxx<T>(w35, w5, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w103 = fvixxx<T>(w52, w4, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w104 = jioxxx<T, false>(w101, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w105 = jioxxx<T, false>(w102, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w106 = jioxxx<T, false>(w103, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w107 = jvvxxx<T, false>(w83, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w108 = jvvxxx<T, false>(w84, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w109 = jvvxxx<T, false>(w85, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w110 = jvvxxx<T, false>(w86, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w111 = jvvxxx<T, false>(w87, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w112 = jvvxxx<T, false>(w88, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w113 = jvvxxx<T, false>(w89, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w114 = jvvxxx<T, false>(w90, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w115 = jvvxxx<T, false>(w91, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w116 = jvvxxx<T, false>(w92, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w117 = jvvxxx<T, false>(w96, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w118 = jvvxxx<T, false>(w97, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w119 = jvvxxx<T, false>(w98, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w120 = jvvxxx<T, false>(w99, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w121 = jvvxxx<T, false>(w100, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w122 = jvvxxx<T, false>(w104, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w123 = jvvxxx<T, false>(w105, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w124 = jvvxxx<T, false>(w106, Qs2_3_4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_4_6 = (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs2_3_4_6 = tv<T>(qs2_3_4_6);
  const cx<T> d2_3_4_6_0 = cvt<T>(inv_denominator(qs2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w125 = jvvxxx<T, false>(w7, Qs2_3, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w126 = jgggxx<T, false>(w7, w4, w6, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w127 = jgggxx<T, false>(w6, w7, w4, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w128 = jgggxx<T, false>(w4, w6, w7, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w129 = jvvxxx<T, false>(w32, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w130 = jvvxxx<T, false>(w34, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w131 = jvvxxx<T, false>(w36, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w132 = jvvxxx<T, false>(w66, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w133 = jvvxxx<T, false>(w68, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w134 = jvvxxx<T, false>(w70, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_4_6 = (-pr2) + (-pr4) + (-pr6);
  const vec<T> Qs2_4_6 = tv<T>(qs2_4_6);
  const cx<T> d2_4_6_3 = cvt<T>(inv_denominator(qs2_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w135 = fvoxxx<T>(w2, w15, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w138 = jioxxx<T, false>(w3, w135, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w149 = jvvxxx<T, false>(w125, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w150 = jvvxxx<T, false>(w126, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w151 = jvvxxx<T, false>(w127, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w152 = jvvxxx<T, false>(w128, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w153 = jvvxxx<T, false>(w129, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w154 = jvvxxx<T, false>(w130, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w155 = jvvxxx<T, false>(w131, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w156 = jvvxxx<T, false>(w132, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w157 = jvvxxx<T, false>(w133, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w158 = jvvxxx<T, false>(w134, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w159 = jvvxxx<T, false>(w138, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const cx<T> amp40 = iovxxx<T>(w0, w1, w72, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp40);
  J[11] = J[11] + (T(0.5) * amp40);
  J[17] = J[17] + (T(0.5) * amp40);
  J[29] = J[29] + (T(-0.5) * amp40);
  const cx<T> amp41 = iovxxx<T>(w0, w1, w73, g0_0, g0_1);
  J[19] = J[19] + (T(0.5) * amp41);
  J[31] = J[31] + (T(-0.5) * amp41);
  J[38] = J[38] + (T(-0.5) * amp41);
  J[39] = J[39] + (T(0.5) * amp41);
  const cx<T> amp42 = iovxxx<T>(w0, w1, w74, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp42);
  J[15] = J[15] + (T(0.5) * amp42);
  J[21] = J[21] + (T(-0.5) * amp42);
  J[27] = J[27] + (T(0.5) * amp42);
  J[29] = J[29] + (T(-0.5) * amp42);
  J[31] = J[31] + (T(0.5) * amp42);
  J[33] = J[33] + (T(-0.5) * amp42);
  J[38] = J[38] + (T(0.5) * amp42);
  const cx<T> amp43 = iovxxx<T>(w0, w1, w75, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp43);
  J[15] = J[15] + (T(-0.5) * amp43);
  J[17] = J[17] + (T(0.5) * amp43);
  J[19] = J[19] + (T(-0.5) * amp43);
  J[21] = J[21] + (T(0.5) * amp43);
  J[27] = J[27] + (T(-0.5) * amp43);
  J[33] = J[33] + (T(0.5) * amp43);
  J[39] = J[39] + (T(-0.5) * amp43);
  const cx<T> amp44 = iovxxx<T>(w0, w1, w76, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp44);
  J[11] = J[11] + (T(-0.5) * amp44);
  J[17] = J[17] + (T(-0.5) * amp44);
  J[19] = J[19] + (T(0.5) * amp44);
  J[29] = J[29] + (T(0.5) * amp44);
  J[31] = J[31] + (T(-0.5) * amp44);
  J[38] = J[38] + (T(-0.5) * amp44);
  J[39] = J[39] + (T(0.5) * amp44);
  const cx<T> amp45 = iovxxx<T>(w0, w1, w77, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp45);
  J[15] = J[15] + (T(-0.5) * amp45);
  J[27] = J[27] + (T(-0.5) * amp45);
  J[29] = J[29] + (T(0.5) * amp45);
  const cx<T> amp46 = iovxxx<T>(w0, w1, w78, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp46);
  J[15] = J[15] + (T(0.5) * amp46);
  J[17] = J[17] + (T(-0.5) * amp46);
  J[27] = J[27] + (T(0.5) * amp46);
  const cx<T> amp47 = iovxxx<T>(w0, w1, w79, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp47);
  J[11] = J[11] + (T(0.5) * amp47);
  J[17] = J[17] + (T(0.5) * amp47);
  J[29] = J[29] + (T(-0.5) * amp47);
  const cx<T> amp48 = iovxxx<T>(w0, w1, w80, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp48);
  J[31] = J[31] + (T(0.5) * amp48);
  J[33] = J[33] + (T(-0.5) * amp48);
  J[38] = J[38] + (T(0.5) * amp48);
  const cx<T> amp49 = iovxxx<T>(w0, w1, w81, g0_0, g0_1);
  J[19] = J[19] + (T(-0.5) * amp49);
  J[21] = J[21] + (T(0.5) * amp49);
  J[33] = J[33] + (T(0.5) * amp49);
  J[39] = J[39] + (T(-0.5) * amp49);
  const cx<T> amp50 = iovxxx<T>(w0, w1, w82, g0_0, g0_1);
  J[19] = J[19] + (T(0.5) * amp50);
  J[31] = J[31] + (T(-0.5) * amp50);
  J[38] = J[38] + (T(-0.5) * amp50);
  J[39] = J[39] + (T(0.5) * amp50);
  const cx<T> amp51 = iovxxx<T>(w0, w1, w107, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp51);
  J[8] = J[8] + (T(-0.5) * amp51);
  J[17] = J[17] + (T(-0.5) * amp51);
  J[29] = J[29] + (T(0.5) * amp51);
  J[38] = J[38] + (T(-0.5) * amp51);
  J[39] = J[39] + (T(0.5) * amp51);
  J[43] = J[43] + (T(0.5) * amp51);
  J[47] = J[47] + (T(-0.5) * amp51);
  const cx<T> amp52 = iovxxx<T>(w0, w1, w108, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp52);
  J[14] = J[14] + (T(0.5) * amp52);
  J[26] = J[26] + (T(0.5) * amp52);
  J[29] = J[29] + (T(-0.5) * amp52);
  J[38] = J[38] + (T(0.5) * amp52);
  J[41] = J[41] + (T(-0.5) * amp52);
  J[45] = J[45] + (T(-0.5) * amp52);
  J[47] = J[47] + (T(0.5) * amp52);
  const cx<T> amp53 = iovxxx<T>(w0, w1, w109, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp53);
  J[14] = J[14] + (T(-0.5) * amp53);
  J[17] = J[17] + (T(0.5) * amp53);
  J[26] = J[26] + (T(-0.5) * amp53);
  J[39] = J[39] + (T(-0.5) * amp53);
  J[41] = J[41] + (T(0.5) * amp53);
  J[43] = J[43] + (T(-0.5) * amp53);
  J[45] = J[45] + (T(0.5) * amp53);
  const cx<T> amp54 = iovxxx<T>(w0, w1, w110, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp54);
  J[8] = J[8] + (T(-0.5) * amp54);
  J[17] = J[17] + (T(-0.5) * amp54);
  J[29] = J[29] + (T(0.5) * amp54);
  J[38] = J[38] + (T(-0.5) * amp54);
  J[39] = J[39] + (T(0.5) * amp54);
  J[43] = J[43] + (T(0.5) * amp54);
  J[47] = J[47] + (T(-0.5) * amp54);
  const cx<T> amp55 = iovxxx<T>(w0, w1, w111, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp55);
  J[14] = J[14] + (T(-0.5) * amp55);
  J[26] = J[26] + (T(-0.5) * amp55);
  J[29] = J[29] + (T(0.5) * amp55);
  J[38] = J[38] + (T(-0.5) * amp55);
  J[41] = J[41] + (T(0.5) * amp55);
  J[45] = J[45] + (T(0.5) * amp55);
  J[47] = J[47] + (T(-0.5) * amp55);
  const cx<T> amp56 = iovxxx<T>(w0, w1, w112, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp56);
  J[26] = J[26] + (T(0.5) * amp56);
  J[38] = J[38] + (T(0.5) * amp56);
  J[45] = J[45] + (T(-0.5) * amp56);
  const cx<T> amp57 = iovxxx<T>(w0, w1, w113, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp57);
  J[29] = J[29] + (T(0.5) * amp57);
  J[41] = J[41] + (T(0.5) * amp57);
  J[47] = J[47] + (T(-0.5) * amp57);
  const cx<T> amp58 = iovxxx<T>(w0, w1, w114, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp58);
  J[14] = J[14] + (T(-0.5) * amp58);
  J[17] = J[17] + (T(0.5) * amp58);
  J[26] = J[26] + (T(-0.5) * amp58);
  J[39] = J[39] + (T(-0.5) * amp58);
  J[41] = J[41] + (T(0.5) * amp58);
  J[43] = J[43] + (T(-0.5) * amp58);
  J[45] = J[45] + (T(0.5) * amp58);
  const cx<T> amp59 = iovxxx<T>(w0, w1, w115, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp59);
  J[14] = J[14] + (T(0.5) * amp59);
  J[39] = J[39] + (T(0.5) * amp59);
  J[41] = J[41] + (T(-0.5) * amp59);
  const cx<T> amp60 = iovxxx<T>(w0, w1, w116, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp60);
  J[26] = J[26] + (T(-0.5) * amp60);
  J[43] = J[43] + (T(-0.5) * amp60);
  J[45] = J[45] + (T(0.5) * amp60);
  const cx<T> amp61 = iovxxx<T>(w0, w1, w117, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp61);
  J[8] = J[8] + (T(0.5) * amp61);
  J[38] = J[38] + (T(0.5) * amp61);
  J[39] = J[39] + (T(-0.5) * amp61);
  const cx<T> amp62 = iovxxx<T>(w0, w1, w118, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp62);
  J[38] = J[38] + (T(-0.5) * amp62);
  const cx<T> amp63 = iovxxx<T>(w0, w1, w119, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp63);
  J[39] = J[39] + (T(-0.5) * amp63);
  const cx<T> amp64 = iovxxx<T>(w0, w1, w120, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp64);
  J[41] = J[41] + (T(-0.5) * amp64);
  const cx<T> amp65 = iovxxx<T>(w0, w1, w121, g0_0, g0_1);
  J[26] = J[26] + (T(0.5) * amp65);
  J[45] = J[45] + (T(-0.5) * amp65);
  const cx<T> amp66 = iovxxx<T>(w0, w1, w122, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp66);
  J[29] = J[29] + (T(0.5) * amp66);
  J[43] = J[43] + (T(0.5) * amp66);
  J[47] = J[47] + (T(-0.5) * amp66);
  const cx<T> amp67 = iovxxx<T>(w0, w1, w123, g0_0, g0_1);
  J[29] = J[29] + (T(0.5) * amp67);
  J[47] = J[47] + (T(-0.5) * amp67);
  const cx<T> amp68 = iovxxx<T>(w0, w1, w124, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp68);
  J[43] = J[43] + (T(-0.5) * amp68);
  const cx<T> amp69 = iovxxx<T>(w0, w1, w149, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp69);
  J[10] = J[10] + (T(-0.5) * amp69);
  J[21] = J[21] + (T(-0.5) * amp69);
  J[26] = J[26] + (T(-0.5) * amp69);
  J[27] = J[27] + (T(0.5) * amp69);
  J[31] = J[31] + (T(0.5) * amp69);
  J[35] = J[35] + (T(-0.5) * amp69);
  J[41] = J[41] + (T(0.5) * amp69);
  const cx<T> amp70 = iovxxx<T>(w0, w1, w150, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp70);
  J[15] = J[15] + (T(0.5) * amp70);
  J[26] = J[26] + (T(0.5) * amp70);
  J[29] = J[29] + (T(-0.5) * amp70);
  J[33] = J[33] + (T(-0.5) * amp70);
  J[35] = J[35] + (T(0.5) * amp70);
  J[38] = J[38] + (T(0.5) * amp70);
  J[41] = J[41] + (T(-0.5) * amp70);
  const cx<T> amp71 = iovxxx<T>(w0, w1, w151, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp71);
  J[15] = J[15] + (T(-0.5) * amp71);
  J[21] = J[21] + (T(0.5) * amp71);
  J[27] = J[27] + (T(-0.5) * amp71);
  J[29] = J[29] + (T(0.5) * amp71);
  J[31] = J[31] + (T(-0.5) * amp71);
  J[33] = J[33] + (T(0.5) * amp71);
  J[38] = J[38] + (T(-0.5) * amp71);
  const cx<T> amp72 = iovxxx<T>(w0, w1, w152, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp72);
  J[10] = J[10] + (T(-0.5) * amp72);
  J[21] = J[21] + (T(-0.5) * amp72);
  J[26] = J[26] + (T(-0.5) * amp72);
  J[27] = J[27] + (T(0.5) * amp72);
  J[31] = J[31] + (T(0.5) * amp72);
  J[35] = J[35] + (T(-0.5) * amp72);
  J[41] = J[41] + (T(0.5) * amp72);
  const cx<T> amp73 = iovxxx<T>(w0, w1, w153, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp73);
  J[15] = J[15] + (T(-0.5) * amp73);
  J[26] = J[26] + (T(-0.5) * amp73);
  J[29] = J[29] + (T(0.5) * amp73);
  J[33] = J[33] + (T(0.5) * amp73);
  J[35] = J[35] + (T(-0.5) * amp73);
  J[38] = J[38] + (T(-0.5) * amp73);
  J[41] = J[41] + (T(0.5) * amp73);
  const cx<T> amp74 = iovxxx<T>(w0, w1, w154, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp74);
  J[26] = J[26] + (T(0.5) * amp74);
  J[33] = J[33] + (T(-0.5) * amp74);
  J[38] = J[38] + (T(0.5) * amp74);
  const cx<T> amp75 = iovxxx<T>(w0, w1, w155, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp75);
  J[29] = J[29] + (T(0.5) * amp75);
  J[35] = J[35] + (T(-0.5) * amp75);
  J[41] = J[41] + (T(0.5) * amp75);
  const cx<T> amp76 = iovxxx<T>(w0, w1, w156, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp76);
  J[15] = J[15] + (T(-0.5) * amp76);
  J[21] = J[21] + (T(0.5) * amp76);
  J[27] = J[27] + (T(-0.5) * amp76);
  J[29] = J[29] + (T(0.5) * amp76);
  J[31] = J[31] + (T(-0.5) * amp76);
  J[33] = J[33] + (T(0.5) * amp76);
  J[38] = J[38] + (T(-0.5) * amp76);
  const cx<T> amp77 = iovxxx<T>(w0, w1, w157, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp77);
  J[15] = J[15] + (T(0.5) * amp77);
  J[27] = J[27] + (T(0.5) * amp77);
  J[29] = J[29] + (T(-0.5) * amp77);
  const cx<T> amp78 = iovxxx<T>(w0, w1, w158, g0_0, g0_1);
  J[21] = J[21] + (T(0.5) * amp78);
  J[31] = J[31] + (T(-0.5) * amp78);
  J[33] = J[33] + (T(0.5) * amp78);
  J[38] = J[38] + (T(-0.5) * amp78);
  const cx<T> amp79 = iovxxx<T>(w0, w1, w159, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp79);
  J[10] = J[10] + (T(0.5) * amp79);
  J[26] = J[26] + (T(0.5) * amp79);
  J[27] = J[27] + (T(-0.5) * amp79);
}

// part 2: amplitudes 80 .. 119 (157 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part2(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5_6 = (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs4_5_6 = tv<T>(qs4_5_6);
  const cx<T> d4_5_6_0 = cvt<T>(inv_denominator(qs4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w9 = jvvxxx<T, false>(w4, Qs4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w10 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w11 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w12 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const wf<T> w14 = jvvxxx<T, false>(w13, Qs4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const wf<T> w16 = jvvxxx<T, false>(w15, Qs4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
  const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
  const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w93 = fvoxxx<T>(w2, w13, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w94 = fvoxxx<T>(w33, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w95 = fvoxxx<T>(w50, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const mom qs2_4_6 = (-pr2) + (-pr4) + (-pr6);
  const vec<T> Qs2_4_6 = tv<T>(qs2_4_6);
  const cx<T> d2_4_6_3 = cvt<T>(inv_denominator(qs2_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w135 = fvoxxx<T>(w2, w15, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w136 = fvoxxx<T>(w33, w6, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w137 = fvoxxx<T>(w67, w4, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const mom qs2_3_4_6 = (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs2_3_4_6 = tv<T>(qs2_3_4_6);
  const cx<T> d2_3_4_6_0 = cvt<T>(inv_denominator(qs2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w139 = jioxxx<T, false>(w3, w136, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w140 = jioxxx<T, false>(w3, w137, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w141 = jioxxx<T, false>(w35, w67, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w142 = jioxxx<T, false>(w69, w33, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs3_4_6 = (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs3_4_6 = tv<T>(qs3_4_6);
  const cx<T> d3_4_6_3 = cvt<T>(inv_denominator(qs3_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w143 = fvixxx<T>(w3, w15, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w144 = fvixxx<T>(w35, w6, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w145 = fvixxx<T>(w69, w4, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w146 = jioxxx<T, false>(w143, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w147 = jioxxx<T, false>(w144, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w148 = jioxxx<T, false>(w145, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_3_4_5_6 = (-pr2) + (-pr3) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_4_5_6 = tv<T>(qs2_3_4_5_6);
  const cx<T> d2_3_4_5_6_0 = cvt<T>(inv_denominator(qs2_3_4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w160 = jvvxxx<T, false>(w139, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w161 = jvvxxx<T, false>(w140, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w162 = jvvxxx<T, false>(w141, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w163 = jvvxxx<T, false>(w142, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w164 = jvvxxx<T, false>(w146, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w165 = jvvxxx<T, false>(w147, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w166 = jvvxxx<T, false>(w148, Qs2_3_4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_3_5_6 = (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_5_6 = tv<T>(qs2_3_5_6);
  const cx<T> d2_3_5_6_0 = cvt<T>(inv_denominator(qs2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w167 = jvvxxx<T, false>(w7, Qs2_3, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w168 = jgggxx<T, false>(w7, w5, w6, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w169 = jgggxx<T, false>(w6, w7, w5, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w170 = jgggxx<T, false>(w5, w6, w7, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w171 = jvvxxx<T, false>(w49, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w172 = jvvxxx<T, false>(w51, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w173 = jvvxxx<T, false>(w53, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w174 = jvvxxx<T, false>(w66, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w175 = jvvxxx<T, false>(w68, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w176 = jvvxxx<T, false>(w70, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs2_5_6 = (-pr2) + (-pr5) + (-pr6);
  const vec<T> Qs2_5_6 = tv<T>(qs2_5_6);
  const cx<T> d2_5_6_3 = cvt<T>(inv_denominator(qs2_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w177 = fvoxxx<T>(w2, w8, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w178 = fvoxxx<T>(w50, w6, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w179 = fvoxxx<T>(w67, w5, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w180 = jioxxx<T, false>(w3, w177, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w181 = jioxxx<T, false>(w3, w178, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w182 = jioxxx<T, false>(w3, w179, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w183 = jioxxx<T, false>(w52, w67, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w184 = jioxxx<T, false>(w69, w50, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs3_5_6 = (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs3_5_6 = tv<T>(qs3_5_6);
  const cx<T> d3_5_6_3 = cvt<T>(inv_denominator(qs3_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w185 = fvixxx<T>(w3, w8, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w186 = fvixxx<T>(w52, w6, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w187 = fvixxx<T>(w69, w5, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w188 = jioxxx<T, false>(w185, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w189 = jioxxx<T, false>(w186, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w190 = jioxxx<T, false>(w187, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w191 = jvvxxx<T, false>(w167, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w192 = jvvxxx<T, false>(w168, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w193 = jvvxxx<T, false>(w169, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w194 = jvvxxx<T, false>(w170, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w195 = jvvxxx<T, false>(w171, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w196 = jvvxxx<T, false>(w172, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w197 = jvvxxx<T, false>(w173, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w198 = jvvxxx<T, false>(w174, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w199 = jvvxxx<T, false>(w175, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w200 = jvvxxx<T, false>(w176, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w201 = jvvxxx<T, false>(w180, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w202 = jvvxxx<T, false>(w181, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w203 = jvvxxx<T, false>(w182, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w204 = jvvxxx<T, false>(w183, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w205 = jvvxxx<T, false>(w184, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w206 = jvvxxx<T, false>(w188, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w207 = jvvxxx<T, false>(w189, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w208 = jvvxxx<T, false>(w190, Qs2_3_5_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs2_4_5_6 = (-pr2) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_4_5_6 = tv<T>(qs2_4_5_6);
  const cx<T> d2_4_5_6_3 = cvt<T>(inv_denominator(qs2_4_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w209 = fvoxxx<T>(w2, w9, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w210 = fvoxxx<T>(w2, w10, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w211 = fvoxxx<T>(w2, w11, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w212 = fvoxxx<T>(w2, w12, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w213 = fvoxxx<T>(w2, w14, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w214 = fvoxxx<T>(w2, w16, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w215 = fvoxxx<T>(w33, w8, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w216 = fvoxxx<T>(w50, w15, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w217 = fvoxxx<T>(w67, w13, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w218 = fvoxxx<T>(w93, w6, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w219 = fvoxxx<T>(w94, w6, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w220 = fvoxxx<T>(w95, w6, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w221 = fvoxxx<T>(w135, w5, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w222 = fvoxxx<T>(w136, w5, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w223 = fvoxxx<T>(w137, w5, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w227 = jioxxx<T, false>(w3, w209, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w228 = jioxxx<T, false>(w3, w210, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w229 = jioxxx<T, false>(w3, w211, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w230 = jioxxx<T, false>(w3, w212, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w231 = jioxxx<T, false>(w3, w213, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w232 = jioxxx<T, false>(w3, w214, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w233 = jioxxx<T, false>(w3, w215, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w234 = jioxxx<T, false>(w3, w216, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w235 = jioxxx<T, false>(w3, w217, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w236 = jioxxx<T, false>(w3, w218, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w237 = jioxxx<T, false>(w3, w219, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w238 = jioxxx<T, false>(w3, w220, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w239 = jioxxx<T, false>(w3, w221, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w240 = jioxxx<T, false>(w3, w222, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w241 = jioxxx<T, false>(w3, w223, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const cx<T> amp80 = iovxxx<T>(w0, w1, w160, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp80);
  J[26] = J[26] + (T(-0.5) * amp80);
  const cx<T> amp81 = iovxxx<T>(w0, w1, w161, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp81);
  J[27] = J[27] + (T(-0.5) * amp81);
  const cx<T> amp82 = iovxxx<T>(w0, w1, w162, g0_0, g0_1);
  J[15] = J[15] + (T(0.5) * amp82);
  J[29] = J[29] + (T(-0.5) * amp82);
  const cx<T> amp83 = iovxxx<T>(w0, w1, w163, g0_0, g0_1);
  J[33] = J[33] + (T(-0.5) * amp83);
  J[38] = J[38] + (T(0.5) * amp83);
  const cx<T> amp84 = iovxxx<T>(w0, w1, w164, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp84);
  J[31] = J[31] + (T(0.5) * amp84);
  J[35] = J[35] + (T(-0.5) * amp84);
  J[41] = J[41] + (T(0.5) * amp84);
  const cx<T> amp85 = iovxxx<T>(w0, w1, w165, g0_0, g0_1);
  J[35] = J[35] + (T(-0.5) * amp85);
  J[41] = J[41] + (T(0.5) * amp85);
  const cx<T> amp86 = iovxxx<T>(w0, w1, w166, g0_0, g0_1);
  J[21] = J[21] + (T(0.5) * amp86);
  J[31] = J[31] + (T(-0.5) * amp86);
  const cx<T> amp87 = iovxxx<T>(w0, w1, w191, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp87);
  J[11] = J[11] + (T(-0.5) * amp87);
  J[14] = J[14] + (T(-0.5) * amp87);
  J[15] = J[15] + (T(0.5) * amp87);
  J[19] = J[19] + (T(0.5) * amp87);
  J[23] = J[23] + (T(-0.5) * amp87);
  J[33] = J[33] + (T(-0.5) * amp87);
  J[45] = J[45] + (T(0.5) * amp87);
  const cx<T> amp88 = iovxxx<T>(w0, w1, w192, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp88);
  J[14] = J[14] + (T(0.5) * amp88);
  J[17] = J[17] + (T(-0.5) * amp88);
  J[21] = J[21] + (T(-0.5) * amp88);
  J[23] = J[23] + (T(0.5) * amp88);
  J[27] = J[27] + (T(0.5) * amp88);
  J[39] = J[39] + (T(0.5) * amp88);
  J[45] = J[45] + (T(-0.5) * amp88);
  const cx<T> amp89 = iovxxx<T>(w0, w1, w193, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp89);
  J[15] = J[15] + (T(-0.5) * amp89);
  J[17] = J[17] + (T(0.5) * amp89);
  J[19] = J[19] + (T(-0.5) * amp89);
  J[21] = J[21] + (T(0.5) * amp89);
  J[27] = J[27] + (T(-0.5) * amp89);
  J[33] = J[33] + (T(0.5) * amp89);
  J[39] = J[39] + (T(-0.5) * amp89);
  const cx<T> amp90 = iovxxx<T>(w0, w1, w194, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp90);
  J[11] = J[11] + (T(-0.5) * amp90);
  J[14] = J[14] + (T(-0.5) * amp90);
  J[15] = J[15] + (T(0.5) * amp90);
  J[19] = J[19] + (T(0.5) * amp90);
  J[23] = J[23] + (T(-0.5) * amp90);
  J[33] = J[33] + (T(-0.5) * amp90);
  J[45] = J[45] + (T(0.5) * amp90);
  const cx<T> amp91 = iovxxx<T>(w0, w1, w195, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp91);
  J[14] = J[14] + (T(-0.5) * amp91);
  J[17] = J[17] + (T(0.5) * amp91);
  J[21] = J[21] + (T(0.5) * amp91);
  J[23] = J[23] + (T(-0.5) * amp91);
  J[27] = J[27] + (T(-0.5) * amp91);
  J[39] = J[39] + (T(-0.5) * amp91);
  J[45] = J[45] + (T(0.5) * amp91);
  const cx<T> amp92 = iovxxx<T>(w0, w1, w196, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp92);
  J[14] = J[14] + (T(0.5) * amp92);
  J[21] = J[21] + (T(-0.5) * amp92);
  J[39] = J[39] + (T(0.5) * amp92);
  const cx<T> amp93 = iovxxx<T>(w0, w1, w197, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp93);
  J[23] = J[23] + (T(-0.5) * amp93);
  J[27] = J[27] + (T(-0.5) * amp93);
  J[45] = J[45] + (T(0.5) * amp93);
  const cx<T> amp94 = iovxxx<T>(w0, w1, w198, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp94);
  J[15] = J[15] + (T(-0.5) * amp94);
  J[17] = J[17] + (T(0.5) * amp94);
  J[19] = J[19] + (T(-0.5) * amp94);
  J[21] = J[21] + (T(0.5) * amp94);
  J[27] = J[27] + (T(-0.5) * amp94);
  J[33] = J[33] + (T(0.5) * amp94);
  J[39] = J[39] + (T(-0.5) * amp94);
  const cx<T> amp95 = iovxxx<T>(w0, w1, w199, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp95);
  J[15] = J[15] + (T(0.5) * amp95);
  J[17] = J[17] + (T(-0.5) * amp95);
  J[27] = J[27] + (T(0.5) * amp95);
  const cx<T> amp96 = iovxxx<T>(w0, w1, w200, g0_0, g0_1);
  J[19] = J[19] + (T(-0.5) * amp96);
  J[21] = J[21] + (T(0.5) * amp96);
  J[33] = J[33] + (T(0.5) * amp96);
  J[39] = J[39] + (T(-0.5) * amp96);
  const cx<T> amp97 = iovxxx<T>(w0, w1, w201, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp97);
  J[11] = J[11] + (T(0.5) * amp97);
  J[14] = J[14] + (T(0.5) * amp97);
  J[15] = J[15] + (T(-0.5) * amp97);
  const cx<T> amp98 = iovxxx<T>(w0, w1, w202, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp98);
  J[14] = J[14] + (T(-0.5) * amp98);
  const cx<T> amp99 = iovxxx<T>(w0, w1, w203, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp99);
  J[15] = J[15] + (T(-0.5) * amp99);
  const cx<T> amp100 = iovxxx<T>(w0, w1, w204, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp100);
  J[27] = J[27] + (T(0.5) * amp100);
  const cx<T> amp101 = iovxxx<T>(w0, w1, w205, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp101);
  J[39] = J[39] + (T(0.5) * amp101);
  const cx<T> amp102 = iovxxx<T>(w0, w1, w206, g0_0, g0_1);
  J[19] = J[19] + (T(0.5) * amp102);
  J[23] = J[23] + (T(-0.5) * amp102);
  J[33] = J[33] + (T(-0.5) * amp102);
  J[45] = J[45] + (T(0.5) * amp102);
  const cx<T> amp103 = iovxxx<T>(w0, w1, w207, g0_0, g0_1);
  J[23] = J[23] + (T(-0.5) * amp103);
  J[45] = J[45] + (T(0.5) * amp103);
  const cx<T> amp104 = iovxxx<T>(w0, w1, w208, g0_0, g0_1);
  J[19] = J[19] + (T(-0.5) * amp104);
  J[33] = J[33] + (T(0.5) * amp104);
  const cx<T> amp105 = iovxxx<T>(w0, w1, w227, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp105);
  J[1] = J[1] + (T(-0.16666666666666666) * amp105);
  J[3] = J[3] + (T(-0.16666666666666666) * amp105);
  J[5] = J[5] + (T(0.16666666666666666) * amp105);
  J[6] = J[6] + (T(-0.5) * amp105);
  J[7] = J[7] + (T(0.5) * amp105);
  J[9] = J[9] + (T(0.5) * amp105);
  J[11] = J[11] + (T(-0.5) * amp105);
  const cx<T> amp106 = iovxxx<T>(w0, w1, w228, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp106);
  J[2] = J[2] + (T(0.16666666666666666) * amp106);
  J[4] = J[4] + (T(0.16666666666666666) * amp106);
  J[5] = J[5] + (T(-0.16666666666666666) * amp106);
  J[6] = J[6] + (T(0.5) * amp106);
  J[8] = J[8] + (T(-0.5) * amp106);
  J[10] = J[10] + (T(-0.5) * amp106);
  J[11] = J[11] + (T(0.5) * amp106);
  const cx<T> amp107 = iovxxx<T>(w0, w1, w229, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp107);
  J[2] = J[2] + (T(-0.16666666666666666) * amp107);
  J[3] = J[3] + (T(0.16666666666666666) * amp107);
  J[4] = J[4] + (T(-0.16666666666666666) * amp107);
  J[7] = J[7] + (T(-0.5) * amp107);
  J[8] = J[8] + (T(0.5) * amp107);
  J[9] = J[9] + (T(-0.5) * amp107);
  J[10] = J[10] + (T(0.5) * amp107);
  const cx<T> amp108 = iovxxx<T>(w0, w1, w230, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp108);
  J[1] = J[1] + (T(-0.16666666666666666) * amp108);
  J[3] = J[3] + (T(-0.16666666666666666) * amp108);
  J[5] = J[5] + (T(0.16666666666666666) * amp108);
  J[6] = J[6] + (T(-0.5) * amp108);
  J[7] = J[7] + (T(0.5) * amp108);
  J[9] = J[9] + (T(0.5) * amp108);
  J[11] = J[11] + (T(-0.5) * amp108);
  const cx<T> amp109 = iovxxx<T>(w0, w1, w231, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp109);
  J[2] = J[2] + (T(-0.16666666666666666) * amp109);
  J[4] = J[4] + (T(-0.16666666666666666) * amp109);
  J[5] = J[5] + (T(0.16666666666666666) * amp109);
  J[6] = J[6] + (T(-0.5) * amp109);
  J[8] = J[8] + (T(0.5) * amp109);
  J[10] = J[10] + (T(0.5) * amp109);
  J[11] = J[11] + (T(-0.5) * amp109);
  const cx<T> amp110 = iovxxx<T>(w0, w1, w232, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp110);
  J[2] = J[2] + (T(-0.16666666666666666) * amp110);
  J[3] = J[3] + (T(0.16666666666666666) * amp110);
  J[4] = J[4] + (T(-0.16666666666666666) * amp110);
  J[7] = J[7] + (T(-0.5) * amp110);
  J[8] = J[8] + (T(0.5) * amp110);
  J[9] = J[9] + (T(-0.5) * amp110);
  J[10] = J[10] + (T(0.5) * amp110);
  const cx<T> amp111 = iovxxx<T>(w0, w1, w233, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp111);
  J[1] = J[1] + (T(0.16666666666666666) * amp111);
  J[6] = J[6] + (T(0.5) * amp111);
  J[7] = J[7] + (T(-0.5) * amp111);
  const cx<T> amp112 = iovxxx<T>(w0, w1, w234, g0_0, g0_1);
  J[2] = J[2] + (T(-0.16666666666666666) * amp112);
  J[3] = J[3] + (T(0.16666666666666666) * amp112);
  J[8] = J[8] + (T(0.5) * amp112);
  J[9] = J[9] + (T(-0.5) * amp112);
  const cx<T> amp113 = iovxxx<T>(w0, w1, w235, g0_0, g0_1);
  J[4] = J[4] + (T(-0.16666666666666666) * amp113);
  J[5] = J[5] + (T(0.16666666666666666) * amp113);
  J[10] = J[10] + (T(0.5) * amp113);
  J[11] = J[11] + (T(-0.5) * amp113);
  const cx<T> amp114 = iovxxx<T>(w0, w1, w236, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp114);
  J[2] = J[2] + (T(0.16666666666666666) * amp114);
  J[6] = J[6] + (T(0.5) * amp114);
  J[8] = J[8] + (T(-0.5) * amp114);
  const cx<T> amp115 = iovxxx<T>(w0, w1, w237, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp115);
  J[6] = J[6] + (T(-0.5) * amp115);
  const cx<T> amp116 = iovxxx<T>(w0, w1, w238, g0_0, g0_1);
  J[2] = J[2] + (T(0.16666666666666666) * amp116);
  J[8] = J[8] + (T(-0.5) * amp116);
  const cx<T> amp117 = iovxxx<T>(w0, w1, w239, g0_0, g0_1);
  J[1] = J[1] + (T(-0.16666666666666666) * amp117);
  J[4] = J[4] + (T(0.16666666666666666) * amp117);
  J[7] = J[7] + (T(0.5) * amp117);
  J[10] = J[10] + (T(-0.5) * amp117);
  const cx<T> amp118 = iovxxx<T>(w0, w1, w240, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp118);
  J[7] = J[7] + (T(-0.5) * amp118);
  const cx<T> amp119 = iovxxx<T>(w0, w1, w241, g0_0, g0_1);
  J[4] = J[4] + (T(0.16666666666666666) * amp119);
  J[10] = J[10] + (T(-0.5) * amp119);
}

// part 3: amplitudes 120 .. 159 (136 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part3(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5_6 = (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs4_5_6 = tv<T>(qs4_5_6);
  const cx<T> d4_5_6_0 = cvt<T>(inv_denominator(qs4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w9 = jvvxxx<T, false>(w4, Qs4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w10 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w11 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w12 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const wf<T> w14 = jvvxxx<T, false>(w13, Qs4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const wf<T> w16 = jvvxxx<T, false>(w15, Qs4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
  const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
  const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w93 = fvoxxx<T>(w2, w13, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w94 = fvoxxx<T>(w33, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w95 = fvoxxx<T>(w50, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const mom qs3_4_5 = (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs3_4_5 = tv<T>(qs3_4_5);
  const cx<T> d3_4_5_3 = cvt<T>(inv_denominator(qs3_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w101 = fvixxx<T>(w3, w13, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w102 = fvixxx<T>(w35, w5, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w103 = fvixxx<T>(w52, w4, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const mom qs2_4_6 = (-pr2) + (-pr4) + (-pr6);
  const vec<T> Qs2_4_6 = tv<T>(qs2_4_6);
  const cx<T> d2_4_6_3 = cvt<T>(inv_denominator(qs2_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w135 = fvoxxx<T>(w2, w15, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w136 = fvoxxx<T>(w33, w6, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w137 = fvoxxx<T>(w67, w4, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const mom qs3_4_6 = (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs3_4_6 = tv<T>(qs3_4_6);
  const cx<T> d3_4_6_3 = cvt<T>(inv_denominator(qs3_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w143 = fvixxx<T>(w3, w15, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w144 = fvixxx<T>(w35, w6, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w145 = fvixxx<T>(w69, w4, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const mom qs2_3_5_6 = (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_5_6 = tv<T>(qs2_3_5_6);
  const cx<T> d2_3_5_6_0 = cvt<T>(inv_denominator(qs2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w167 = jvvxxx<T, false>(w7, Qs2_3, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs2_5_6 = (-pr2) + (-pr5) + (-pr6);
  const vec<T> Qs2_5_6 = tv<T>(qs2_5_6);
  const cx<T> d2_5_6_3 = cvt<T>(inv_denominator(qs2_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w177 = fvoxxx<T>(w2, w8, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w178 = fvoxxx<T>(w50, w6, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w179 = fvoxxx<T>(w67, w5, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const mom qs3_5_6 = (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs3_5_6 = tv<T>(qs3_5_6);
  const cx<T> d3_5_6_3 = cvt<T>(inv_denominator(qs3_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w185 = fvixxx<T>(w3, w8, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w186 = fvixxx<T>(w52, w6, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w187 = fvixxx<T>(w69, w5, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const mom qs2_4_5_6 = (-pr2) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_4_5_6 = tv<T>(qs2_4_5_6);
  const cx<T> d2_4_5_6_3 = cvt<T>(inv_denominator(qs2_4_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w224 = fvoxxx<T>(w177, w4, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w225 = fvoxxx<T>(w178, w4, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const wf<T> w226 = fvoxxx<T>(w179, w4, g0_0, g0_1, Qs2_4_5_6, T(pe3.m), d2_4_5_6_3);
  const mom qs2_3_4_5_6 = (-pr2) + (-pr3) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_4_5_6 = tv<T>(qs2_3_4_5_6);
  const cx<T> d2_3_4_5_6_0 = cvt<T>(inv_denominator(qs2_3_4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w242 = jioxxx<T, false>(w3, w224, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w243 = jioxxx<T, false>(w3, w225, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w244 = jioxxx<T, false>(w3, w226, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w245 = jioxxx<T, false>(w35, w177, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w246 = jioxxx<T, false>(w35, w178, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w247 = jioxxx<T, false>(w35, w179, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w248 = jioxxx<T, false>(w52, w135, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w249 = jioxxx<T, false>(w52, w136, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w250 = jioxxx<T, false>(w52, w137, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w251 = jioxxx<T, false>(w69, w93, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w252 = jioxxx<T, false>(w69, w94, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w253 = jioxxx<T, false>(w69, w95, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w254 = jioxxx<T, false>(w101, w67, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w255 = jioxxx<T, false>(w102, w67, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w256 = jioxxx<T, false>(w103, w67, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w257 = jioxxx<T, false>(w143, w50, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w258 = jioxxx<T, false>(w144, w50, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w259 = jioxxx<T, false>(w145, w50, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w260 = jioxxx<T, false>(w185, w33, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w261 = jioxxx<T, false>(w186, w33, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w262 = jioxxx<T, false>(w187, w33, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const mom qs3_4_5_6 = (-pr3) + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs3_4_5_6 = tv<T>(qs3_4_5_6);
  const cx<T> d3_4_5_6_3 = cvt<T>(inv_denominator(qs3_4_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w263 = fvixxx<T>(w3, w9, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w264 = fvixxx<T>(w3, w10, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w265 = fvixxx<T>(w3, w11, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w266 = fvixxx<T>(w3, w12, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w267 = fvixxx<T>(w3, w14, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w268 = fvixxx<T>(w3, w16, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w269 = fvixxx<T>(w35, w8, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w270 = fvixxx<T>(w52, w15, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w271 = fvixxx<T>(w69, w13, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w272 = fvixxx<T>(w101, w6, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w273 = fvixxx<T>(w102, w6, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w274 = fvixxx<T>(w103, w6, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w275 = fvixxx<T>(w143, w5, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w276 = fvixxx<T>(w144, w5, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w277 = fvixxx<T>(w145, w5, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w278 = fvixxx<T>(w185, w4, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w279 = fvixxx<T>(w186, w4, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w280 = fvixxx<T>(w187, w4, g0_0, g0_1, Qs3_4_5_6, T(pe3.m), d3_4_5_6_3);
  const wf<T> w281 = jioxxx<T, false>(w263, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w282 = jioxxx<T, false>(w264, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w283 = jioxxx<T, false>(w265, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w284 = jioxxx<T, false>(w266, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w285 = jioxxx<T, false>(w267, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w286 = jioxxx<T, false>(w268, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w287 = jioxxx<T, false>(w269, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w288 = jioxxx<T, false>(w270, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w289 = jioxxx<T, false>(w271, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w290 = jioxxx<T, false>(w272, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w291 = jioxxx<T, false>(w273, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w292 = jioxxx<T, false>(w274, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w293 = jioxxx<T, false>(w275, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w294 = jioxxx<T, false>(w276, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w295 = jioxxx<T, false>(w277, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w296 = jioxxx<T, false>(w278, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w297 = jioxxx<T, false>(w279, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const wf<T> w298 = jioxxx<T, false>(w280, w2, g0_0, g0_1, Qs2_3_4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_6_0);
  const cx<T> amp120 = iovxxx<T>(w0, w1, w242, g0_0, g0_1);
  J[3] = J[3] + (T(-0.16666666666666666) * amp120);
  J[5] = J[5] + (T(0.16666666666666666) * amp120);
  J[9] = J[9] + (T(0.5) * amp120);
  J[11] = J[11] + (T(-0.5) * amp120);
  const cx<T> amp121 = iovxxx<T>(w0, w1, w243, g0_0, g0_1);
  J[3] = J[3] + (T(0.16666666666666666) * amp121);
  J[9] = J[9] + (T(-0.5) * amp121);
  const cx<T> amp122 = iovxxx<T>(w0, w1, w244, g0_0, g0_1);
  J[5] = J[5] + (T(0.16666666666666666) * amp122);
  J[11] = J[11] + (T(-0.5) * amp122);
  const cx<T> amp123 = iovxxx<T>(w0, w1, w245, g0_0, g0_1);
  J[3] = J[3] + (T(-0.16666666666666666) * amp123);
  J[5] = J[5] + (T(0.16666666666666666) * amp123);
  J[14] = J[14] + (T(0.5) * amp123);
  J[15] = J[15] + (T(-0.5) * amp123);
  const cx<T> amp124 = iovxxx<T>(w0, w1, w246, g0_0, g0_1);
  J[3] = J[3] + (T(0.16666666666666666) * amp124);
  J[14] = J[14] + (T(-0.5) * amp124);
  const cx<T> amp125 = iovxxx<T>(w0, w1, w247, g0_0, g0_1);
  J[5] = J[5] + (T(0.16666666666666666) * amp125);
  J[15] = J[15] + (T(-0.5) * amp125);
  const cx<T> amp126 = iovxxx<T>(w0, w1, w248, g0_0, g0_1);
  J[1] = J[1] + (T(-0.16666666666666666) * amp126);
  J[4] = J[4] + (T(0.16666666666666666) * amp126);
  J[26] = J[26] + (T(0.5) * amp126);
  J[27] = J[27] + (T(-0.5) * amp126);
  const cx<T> amp127 = iovxxx<T>(w0, w1, w249, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp127);
  J[26] = J[26] + (T(-0.5) * amp127);
  const cx<T> amp128 = iovxxx<T>(w0, w1, w250, g0_0, g0_1);
  J[4] = J[4] + (T(0.16666666666666666) * amp128);
  J[27] = J[27] + (T(-0.5) * amp128);
  const cx<T> amp129 = iovxxx<T>(w0, w1, w251, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp129);
  J[2] = J[2] + (T(0.16666666666666666) * amp129);
  J[38] = J[38] + (T(0.5) * amp129);
  J[39] = J[39] + (T(-0.5) * amp129);
  const cx<T> amp130 = iovxxx<T>(w0, w1, w252, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp130);
  J[38] = J[38] + (T(-0.5) * amp130);
  const cx<T> amp131 = iovxxx<T>(w0, w1, w253, g0_0, g0_1);
  J[2] = J[2] + (T(0.16666666666666666) * amp131);
  J[39] = J[39] + (T(-0.5) * amp131);
  const cx<T> amp132 = iovxxx<T>(w0, w1, w254, g0_0, g0_1);
  J[4] = J[4] + (T(-0.16666666666666666) * amp132);
  J[5] = J[5] + (T(0.16666666666666666) * amp132);
  J[17] = J[17] + (T(0.5) * amp132);
  J[29] = J[29] + (T(-0.5) * amp132);
  const cx<T> amp133 = iovxxx<T>(w0, w1, w255, g0_0, g0_1);
  J[5] = J[5] + (T(0.16666666666666666) * amp133);
  J[29] = J[29] + (T(-0.5) * amp133);
  const cx<T> amp134 = iovxxx<T>(w0, w1, w256, g0_0, g0_1);
  J[4] = J[4] + (T(0.16666666666666666) * amp134);
  J[17] = J[17] + (T(-0.5) * amp134);
  const cx<T> amp135 = iovxxx<T>(w0, w1, w257, g0_0, g0_1);
  J[2] = J[2] + (T(-0.16666666666666666) * amp135);
  J[3] = J[3] + (T(0.16666666666666666) * amp135);
  J[21] = J[21] + (T(0.5) * amp135);
  J[41] = J[41] + (T(-0.5) * amp135);
  const cx<T> amp136 = iovxxx<T>(w0, w1, w258, g0_0, g0_1);
  J[3] = J[3] + (T(0.16666666666666666) * amp136);
  J[41] = J[41] + (T(-0.5) * amp136);
  const cx<T> amp137 = iovxxx<T>(w0, w1, w259, g0_0, g0_1);
  J[2] = J[2] + (T(0.16666666666666666) * amp137);
  J[21] = J[21] + (T(-0.5) * amp137);
  const cx<T> amp138 = iovxxx<T>(w0, w1, w260, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp138);
  J[1] = J[1] + (T(0.16666666666666666) * amp138);
  J[33] = J[33] + (T(0.5) * amp138);
  J[45] = J[45] + (T(-0.5) * amp138);
  const cx<T> amp139 = iovxxx<T>(w0, w1, w261, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp139);
  J[45] = J[45] + (T(-0.5) * amp139);
  const cx<T> amp140 = iovxxx<T>(w0, w1, w262, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp140);
  J[33] = J[33] + (T(-0.5) * amp140);
  const cx<T> amp141 = iovxxx<T>(w0, w1, w281, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp141);
  J[1] = J[1] + (T(-0.16666666666666666) * amp141);
  J[3] = J[3] + (T(-0.16666666666666666) * amp141);
  J[5] = J[5] + (T(0.16666666666666666) * amp141);
  J[19] = J[19] + (T(-0.5) * amp141);
  J[23] = J[23] + (T(0.5) * amp141);
  J[35] = J[35] + (T(0.5) * amp141);
  J[47] = J[47] + (T(-0.5) * amp141);
  const cx<T> amp142 = iovxxx<T>(w0, w1, w282, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp142);
  J[2] = J[2] + (T(0.16666666666666666) * amp142);
  J[4] = J[4] + (T(0.16666666666666666) * amp142);
  J[5] = J[5] + (T(-0.16666666666666666) * amp142);
  J[19] = J[19] + (T(0.5) * amp142);
  J[31] = J[31] + (T(-0.5) * amp142);
  J[43] = J[43] + (T(-0.5) * amp142);
  J[47] = J[47] + (T(0.5) * amp142);
  const cx<T> amp143 = iovxxx<T>(w0, w1, w283, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp143);
  J[2] = J[2] + (T(-0.16666666666666666) * amp143);
  J[3] = J[3] + (T(0.16666666666666666) * amp143);
  J[4] = J[4] + (T(-0.16666666666666666) * amp143);
  J[23] = J[23] + (T(-0.5) * amp143);
  J[31] = J[31] + (T(0.5) * amp143);
  J[35] = J[35] + (T(-0.5) * amp143);
  J[43] = J[43] + (T(0.5) * amp143);
  const cx<T> amp144 = iovxxx<T>(w0, w1, w284, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp144);
  J[1] = J[1] + (T(-0.16666666666666666) * amp144);
  J[3] = J[3] + (T(-0.16666666666666666) * amp144);
  J[5] = J[5] + (T(0.16666666666666666) * amp144);
  J[19] = J[19] + (T(-0.5) * amp144);
  J[23] = J[23] + (T(0.5) * amp144);
  J[35] = J[35] + (T(0.5) * amp144);
  J[47] = J[47] + (T(-0.5) * amp144);
  const cx<T> amp145 = iovxxx<T>(w0, w1, w285, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp145);
  J[2] = J[2] + (T(-0.16666666666666666) * amp145);
  J[4] = J[4] + (T(-0.16666666666666666) * amp145);
  J[5] = J[5] + (T(0.16666666666666666) * amp145);
  J[19] = J[19] + (T(-0.5) * amp145);
  J[31] = J[31] + (T(0.5) * amp145);
  J[43] = J[43] + (T(0.5) * amp145);
  J[47] = J[47] + (T(-0.5) * amp145);
  const cx<T> amp146 = iovxxx<T>(w0, w1, w286, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp146);
  J[2] = J[2] + (T(-0.16666666666666666) * amp146);
  J[3] = J[3] + (T(0.16666666666666666) * amp146);
  J[4] = J[4] + (T(-0.16666666666666666) * amp146);
  J[23] = J[23] + (T(-0.5) * amp146);
  J[31] = J[31] + (T(0.5) * amp146);
  J[35] = J[35] + (T(-0.5) * amp146);
  J[43] = J[43] + (T(0.5) * amp146);
  const cx<T> amp147 = iovxxx<T>(w0, w1, w287, g0_0, g0_1);
  J[3] = J[3] + (T(-0.16666666666666666) * amp147);
  J[5] = J[5] + (T(0.16666666666666666) * amp147);
  J[35] = J[35] + (T(0.5) * amp147);
  J[47] = J[47] + (T(-0.5) * amp147);
  const cx<T> amp148 = iovxxx<T>(w0, w1, w288, g0_0, g0_1);
  J[1] = J[1] + (T(-0.16666666666666666) * amp148);
  J[4] = J[4] + (T(0.16666666666666666) * amp148);
  J[23] = J[23] + (T(0.5) * amp148);
  J[43] = J[43] + (T(-0.5) * amp148);
  const cx<T> amp149 = iovxxx<T>(w0, w1, w289, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp149);
  J[2] = J[2] + (T(0.16666666666666666) * amp149);
  J[19] = J[19] + (T(0.5) * amp149);
  J[31] = J[31] + (T(-0.5) * amp149);
  const cx<T> amp150 = iovxxx<T>(w0, w1, w290, g0_0, g0_1);
  J[4] = J[4] + (T(-0.16666666666666666) * amp150);
  J[5] = J[5] + (T(0.16666666666666666) * amp150);
  J[43] = J[43] + (T(0.5) * amp150);
  J[47] = J[47] + (T(-0.5) * amp150);
  const cx<T> amp151 = iovxxx<T>(w0, w1, w291, g0_0, g0_1);
  J[5] = J[5] + (T(0.16666666666666666) * amp151);
  J[47] = J[47] + (T(-0.5) * amp151);
  const cx<T> amp152 = iovxxx<T>(w0, w1, w292, g0_0, g0_1);
  J[4] = J[4] + (T(0.16666666666666666) * amp152);
  J[43] = J[43] + (T(-0.5) * amp152);
  const cx<T> amp153 = iovxxx<T>(w0, w1, w293, g0_0, g0_1);
  J[2] = J[2] + (T(-0.16666666666666666) * amp153);
  J[3] = J[3] + (T(0.16666666666666666) * amp153);
  J[31] = J[31] + (T(0.5) * amp153);
  J[35] = J[35] + (T(-0.5) * amp153);
  const cx<T> amp154 = iovxxx<T>(w0, w1, w294, g0_0, g0_1);
  J[3] = J[3] + (T(0.16666666666666666) * amp154);
  J[35] = J[35] + (T(-0.5) * amp154);
  const cx<T> amp155 = iovxxx<T>(w0, w1, w295, g0_0, g0_1);
  J[2] = J[2] + (T(0.16666666666666666) * amp155);
  J[31] = J[31] + (T(-0.5) * amp155);
  const cx<T> amp156 = iovxxx<T>(w0, w1, w296, g0_0, g0_1);
  J[0] = J[0] + (T(-0.16666666666666666) * amp156);
  J[1] = J[1] + (T(0.16666666666666666) * amp156);
  J[19] = J[19] + (T(0.5) * amp156);
  J[23] = J[23] + (T(-0.5) * amp156);
  const cx<T> amp157 = iovxxx<T>(w0, w1, w297, g0_0, g0_1);
  J[1] = J[1] + (T(0.16666666666666666) * amp157);
  J[23] = J[23] + (T(-0.5) * amp157);
  const cx<T> amp158 = iovxxx<T>(w0, w1, w298, g0_0, g0_1);
  J[0] = J[0] + (T(0.16666666666666666) * amp158);
  J[19] = J[19] + (T(-0.5) * amp158);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const cx<T> amp159 = iovxxx<T>(w299, w1, w167, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp159);
  J[11] = J[11] + (T(0.5) * amp159);
  J[33] = J[33] + (T(0.5) * amp159);
  J[45] = J[45] + (T(-0.5) * amp159);
}

// part 4: amplitudes 160 .. 199 (114 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part4(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
  const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w83 = jvvxxx<T, false>(w7, Qs2_3, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w84 = jgggxx<T, false>(w7, w4, w5, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w85 = jgggxx<T, false>(w5, w7, w4, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w86 = jgggxx<T, false>(w4, w5, w7, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w87 = jvvxxx<T, false>(w32, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs2_3_4_6 = (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs2_3_4_6 = tv<T>(qs2_3_4_6);
  const cx<T> d2_3_4_6_0 = cvt<T>(inv_denominator(qs2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w125 = jvvxxx<T, false>(w7, Qs2_3, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w126 = jgggxx<T, false>(w7, w4, w6, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w127 = jgggxx<T, false>(w6, w7, w4, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w128 = jgggxx<T, false>(w4, w6, w7, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w129 = jvvxxx<T, false>(w32, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w130 = jvvxxx<T, false>(w34, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w131 = jvvxxx<T, false>(w36, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w132 = jvvxxx<T, false>(w66, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w133 = jvvxxx<T, false>(w68, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w134 = jvvxxx<T, false>(w70, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_4_6 = (-pr2) + (-pr4) + (-pr6);
  const vec<T> Qs2_4_6 = tv<T>(qs2_4_6);
  const cx<T> d2_4_6_3 = cvt<T>(inv_denominator(qs2_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w135 = fvoxxx<T>(w2, w15, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w136 = fvoxxx<T>(w33, w6, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w137 = fvoxxx<T>(w67, w4, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w138 = jioxxx<T, false>(w3, w135, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w139 = jioxxx<T, false>(w3, w136, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w140 = jioxxx<T, false>(w3, w137, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w141 = jioxxx<T, false>(w35, w67, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w142 = jioxxx<T, false>(w69, w33, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs3_4_6 = (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs3_4_6 = tv<T>(qs3_4_6);
  const cx<T> d3_4_6_3 = cvt<T>(inv_denominator(qs3_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w143 = fvixxx<T>(w3, w15, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w144 = fvixxx<T>(w35, w6, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w145 = fvixxx<T>(w69, w4, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w146 = jioxxx<T, false>(w143, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w147 = jioxxx<T, false>(w144, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w148 = jioxxx<T, false>(w145, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_3_5_6 = (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_5_6 = tv<T>(qs2_3_5_6);
  const cx<T> d2_3_5_6_0 = cvt<T>(inv_denominator(qs2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w168 = jgggxx<T, false>(w7, w5, w6, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w169 = jgggxx<T, false>(w6, w7, w5, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w170 = jgggxx<T, false>(w5, w6, w7, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w171 = jvvxxx<T, false>(w49, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w172 = jvvxxx<T, false>(w51, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w173 = jvvxxx<T, false>(w53, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w174 = jvvxxx<T, false>(w66, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w175 = jvvxxx<T, false>(w68, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w176 = jvvxxx<T, false>(w70, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs2_5_6 = (-pr2) + (-pr5) + (-pr6);
  const vec<T> Qs2_5_6 = tv<T>(qs2_5_6);
  const cx<T> d2_5_6_3 = cvt<T>(inv_denominator(qs2_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w177 = fvoxxx<T>(w2, w8, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w178 = fvoxxx<T>(w50, w6, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w179 = fvoxxx<T>(w67, w5, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w180 = jioxxx<T, false>(w3, w177, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w181 = jioxxx<T, false>(w3, w178, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w182 = jioxxx<T, false>(w3, w179, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w183 = jioxxx<T, false>(w52, w67, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w184 = jioxxx<T, false>(w69, w50, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs3_5_6 = (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs3_5_6 = tv<T>(qs3_5_6);
  const cx<T> d3_5_6_3 = cvt<T>(inv_denominator(qs3_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w185 = fvixxx<T>(w3, w8, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w186 = fvixxx<T>(w52, w6, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w187 = fvixxx<T>(w69, w5, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w188 = jioxxx<T, false>(w185, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w189 = jioxxx<T, false>(w186, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w190 = jioxxx<T, false>(w187, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const cx<T> amp160 = iovxxx<T>(w299, w1, w168, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp160);
  J[27] = J[27] + (T(-0.5) * amp160);
  J[39] = J[39] + (T(-0.5) * amp160);
  J[45] = J[45] + (T(0.5) * amp160);
  const cx<T> amp161 = iovxxx<T>(w299, w1, w169, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp161);
  J[27] = J[27] + (T(0.5) * amp161);
  J[33] = J[33] + (T(-0.5) * amp161);
  J[39] = J[39] + (T(0.5) * amp161);
  const cx<T> amp162 = iovxxx<T>(w299, w1, w170, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp162);
  J[11] = J[11] + (T(0.5) * amp162);
  J[33] = J[33] + (T(0.5) * amp162);
  J[45] = J[45] + (T(-0.5) * amp162);
  const cx<T> amp163 = iovxxx<T>(w299, w1, w171, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp163);
  J[27] = J[27] + (T(0.5) * amp163);
  J[39] = J[39] + (T(0.5) * amp163);
  J[45] = J[45] + (T(-0.5) * amp163);
  const cx<T> amp164 = iovxxx<T>(w299, w1, w172, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp164);
  J[39] = J[39] + (T(-0.5) * amp164);
  const cx<T> amp165 = iovxxx<T>(w299, w1, w173, g0_0, g0_1);
  J[27] = J[27] + (T(0.5) * amp165);
  J[45] = J[45] + (T(-0.5) * amp165);
  const cx<T> amp166 = iovxxx<T>(w299, w1, w174, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp166);
  J[27] = J[27] + (T(0.5) * amp166);
  J[33] = J[33] + (T(-0.5) * amp166);
  J[39] = J[39] + (T(0.5) * amp166);
  const cx<T> amp167 = iovxxx<T>(w299, w1, w175, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp167);
  J[27] = J[27] + (T(-0.5) * amp167);
  const cx<T> amp168 = iovxxx<T>(w299, w1, w176, g0_0, g0_1);
  J[33] = J[33] + (T(-0.5) * amp168);
  J[39] = J[39] + (T(0.5) * amp168);
  const cx<T> amp169 = iovxxx<T>(w299, w1, w180, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp169);
  J[11] = J[11] + (T(-0.5) * amp169);
  J[12] = J[12] + (T(-0.16666666666666666) * amp169);
  J[13] = J[13] + (T(0.16666666666666666) * amp169);
  const cx<T> amp170 = iovxxx<T>(w299, w1, w181, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp170);
  J[12] = J[12] + (T(0.16666666666666666) * amp170);
  const cx<T> amp171 = iovxxx<T>(w299, w1, w182, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp171);
  J[13] = J[13] + (T(0.16666666666666666) * amp171);
  const cx<T> amp172 = iovxxx<T>(w299, w1, w183, g0_0, g0_1);
  J[13] = J[13] + (T(0.16666666666666666) * amp172);
  J[27] = J[27] + (T(-0.5) * amp172);
  const cx<T> amp173 = iovxxx<T>(w299, w1, w184, g0_0, g0_1);
  J[12] = J[12] + (T(0.16666666666666666) * amp173);
  J[39] = J[39] + (T(-0.5) * amp173);
  const cx<T> amp174 = iovxxx<T>(w299, w1, w188, g0_0, g0_1);
  J[12] = J[12] + (T(-0.16666666666666666) * amp174);
  J[13] = J[13] + (T(0.16666666666666666) * amp174);
  J[33] = J[33] + (T(0.5) * amp174);
  J[45] = J[45] + (T(-0.5) * amp174);
  const cx<T> amp175 = iovxxx<T>(w299, w1, w189, g0_0, g0_1);
  J[13] = J[13] + (T(0.16666666666666666) * amp175);
  J[45] = J[45] + (T(-0.5) * amp175);
  const cx<T> amp176 = iovxxx<T>(w299, w1, w190, g0_0, g0_1);
  J[12] = J[12] + (T(0.16666666666666666) * amp176);
  J[33] = J[33] + (T(-0.5) * amp176);
  const mom qs0_5 = pr0 + (-pr5);
  const vec<T> Qs0_5 = tv<T>(qs0_5);
  const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w300 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
  const cx<T> amp177 = iovxxx<T>(w300, w1, w125, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp177);
  J[10] = J[10] + (T(0.5) * amp177);
  J[21] = J[21] + (T(0.5) * amp177);
  J[41] = J[41] + (T(-0.5) * amp177);
  const cx<T> amp178 = iovxxx<T>(w300, w1, w126, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp178);
  J[15] = J[15] + (T(-0.5) * amp178);
  J[38] = J[38] + (T(-0.5) * amp178);
  J[41] = J[41] + (T(0.5) * amp178);
  const cx<T> amp179 = iovxxx<T>(w300, w1, w127, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp179);
  J[15] = J[15] + (T(0.5) * amp179);
  J[21] = J[21] + (T(-0.5) * amp179);
  J[38] = J[38] + (T(0.5) * amp179);
  const cx<T> amp180 = iovxxx<T>(w300, w1, w128, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp180);
  J[10] = J[10] + (T(0.5) * amp180);
  J[21] = J[21] + (T(0.5) * amp180);
  J[41] = J[41] + (T(-0.5) * amp180);
  const cx<T> amp181 = iovxxx<T>(w300, w1, w129, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp181);
  J[15] = J[15] + (T(0.5) * amp181);
  J[38] = J[38] + (T(0.5) * amp181);
  J[41] = J[41] + (T(-0.5) * amp181);
  const cx<T> amp182 = iovxxx<T>(w300, w1, w130, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp182);
  J[38] = J[38] + (T(-0.5) * amp182);
  const cx<T> amp183 = iovxxx<T>(w300, w1, w131, g0_0, g0_1);
  J[15] = J[15] + (T(0.5) * amp183);
  J[41] = J[41] + (T(-0.5) * amp183);
  const cx<T> amp184 = iovxxx<T>(w300, w1, w132, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp184);
  J[15] = J[15] + (T(0.5) * amp184);
  J[21] = J[21] + (T(-0.5) * amp184);
  J[38] = J[38] + (T(0.5) * amp184);
  const cx<T> amp185 = iovxxx<T>(w300, w1, w133, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp185);
  J[15] = J[15] + (T(-0.5) * amp185);
  const cx<T> amp186 = iovxxx<T>(w300, w1, w134, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp186);
  J[38] = J[38] + (T(0.5) * amp186);
  const cx<T> amp187 = iovxxx<T>(w300, w1, w138, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp187);
  J[10] = J[10] + (T(-0.5) * amp187);
  J[24] = J[24] + (T(-0.16666666666666666) * amp187);
  J[25] = J[25] + (T(0.16666666666666666) * amp187);
  const cx<T> amp188 = iovxxx<T>(w300, w1, w139, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp188);
  J[24] = J[24] + (T(0.16666666666666666) * amp188);
  const cx<T> amp189 = iovxxx<T>(w300, w1, w140, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp189);
  J[25] = J[25] + (T(0.16666666666666666) * amp189);
  const cx<T> amp190 = iovxxx<T>(w300, w1, w141, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp190);
  J[25] = J[25] + (T(0.16666666666666666) * amp190);
  const cx<T> amp191 = iovxxx<T>(w300, w1, w142, g0_0, g0_1);
  J[24] = J[24] + (T(0.16666666666666666) * amp191);
  J[38] = J[38] + (T(-0.5) * amp191);
  const cx<T> amp192 = iovxxx<T>(w300, w1, w146, g0_0, g0_1);
  J[21] = J[21] + (T(0.5) * amp192);
  J[24] = J[24] + (T(-0.16666666666666666) * amp192);
  J[25] = J[25] + (T(0.16666666666666666) * amp192);
  J[41] = J[41] + (T(-0.5) * amp192);
  const cx<T> amp193 = iovxxx<T>(w300, w1, w147, g0_0, g0_1);
  J[25] = J[25] + (T(0.16666666666666666) * amp193);
  J[41] = J[41] + (T(-0.5) * amp193);
  const cx<T> amp194 = iovxxx<T>(w300, w1, w148, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp194);
  J[24] = J[24] + (T(0.16666666666666666) * amp194);
  const mom qs0_6 = pr0 + (-pr6);
  const vec<T> Qs0_6 = tv<T>(qs0_6);
  const cx<T> d0_6_0 = cvt<T>(inv_denominator(qs0_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w301 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_6, T(pe0.m), d0_6_0);
  const cx<T> amp195 = iovxxx<T>(w301, w1, w83, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp195);
  J[8] = J[8] + (T(0.5) * amp195);
  J[17] = J[17] + (T(0.5) * amp195);
  J[29] = J[29] + (T(-0.5) * amp195);
  const cx<T> amp196 = iovxxx<T>(w301, w1, w84, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp196);
  J[14] = J[14] + (T(-0.5) * amp196);
  J[26] = J[26] + (T(-0.5) * amp196);
  J[29] = J[29] + (T(0.5) * amp196);
  const cx<T> amp197 = iovxxx<T>(w301, w1, w85, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp197);
  J[14] = J[14] + (T(0.5) * amp197);
  J[17] = J[17] + (T(-0.5) * amp197);
  J[26] = J[26] + (T(0.5) * amp197);
  const cx<T> amp198 = iovxxx<T>(w301, w1, w86, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp198);
  J[8] = J[8] + (T(0.5) * amp198);
  J[17] = J[17] + (T(0.5) * amp198);
  J[29] = J[29] + (T(-0.5) * amp198);
  const cx<T> amp199 = iovxxx<T>(w301, w1, w87, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp199);
  J[14] = J[14] + (T(0.5) * amp199);
  J[26] = J[26] + (T(0.5) * amp199);
  J[29] = J[29] + (T(-0.5) * amp199);
}

// part 5: amplitudes 200 .. 239 (95 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part5(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5_6 = (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs4_5_6 = tv<T>(qs4_5_6);
  const cx<T> d4_5_6_0 = cvt<T>(inv_denominator(qs4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w9 = jvvxxx<T, false>(w4, Qs4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w10 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w11 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w12 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const wf<T> w14 = jvvxxx<T, false>(w13, Qs4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const wf<T> w16 = jvvxxx<T, false>(w15, Qs4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
  const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w88 = jvvxxx<T, false>(w34, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w89 = jvvxxx<T, false>(w36, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w90 = jvvxxx<T, false>(w49, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w91 = jvvxxx<T, false>(w51, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w92 = jvvxxx<T, false>(w53, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
  const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
  const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w93 = fvoxxx<T>(w2, w13, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w94 = fvoxxx<T>(w33, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w95 = fvoxxx<T>(w50, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w96 = jioxxx<T, false>(w3, w93, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w97 = jioxxx<T, false>(w3, w94, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w98 = jioxxx<T, false>(w3, w95, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w99 = jioxxx<T, false>(w35, w50, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w100 = jioxxx<T, false>(w52, w33, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs3_4_5 = (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs3_4_5 = tv<T>(qs3_4_5);
  const cx<T> d3_4_5_3 = cvt<T>(inv_denominator(qs3_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w101 = fvixxx<T>(w3, w13, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w102 = fvixxx<T>(w35, w5, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w103 = fvixxx<T>(w52, w4, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w104 = jioxxx<T, false>(w101, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w105 = jioxxx<T, false>(w102, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w106 = jioxxx<T, false>(w103, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const mom qs0_5 = pr0 + (-pr5);
  const vec<T> Qs0_5 = tv<T>(qs0_5);
  const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w300 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
  const mom qs0_6 = pr0 + (-pr6);
  const vec<T> Qs0_6 = tv<T>(qs0_6);
  const cx<T> d0_6_0 = cvt<T>(inv_denominator(qs0_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w301 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_6, T(pe0.m), d0_6_0);
  const cx<T> amp200 = iovxxx<T>(w301, w1, w88, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp200);
  J[26] = J[26] + (T(-0.5) * amp200);
  const cx<T> amp201 = iovxxx<T>(w301, w1, w89, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp201);
  J[29] = J[29] + (T(-0.5) * amp201);
  const cx<T> amp202 = iovxxx<T>(w301, w1, w90, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp202);
  J[14] = J[14] + (T(0.5) * amp202);
  J[17] = J[17] + (T(-0.5) * amp202);
  J[26] = J[26] + (T(0.5) * amp202);
  const cx<T> amp203 = iovxxx<T>(w301, w1, w91, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp203);
  J[14] = J[14] + (T(-0.5) * amp203);
  const cx<T> amp204 = iovxxx<T>(w301, w1, w92, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp204);
  J[26] = J[26] + (T(0.5) * amp204);
  const cx<T> amp205 = iovxxx<T>(w301, w1, w96, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp205);
  J[8] = J[8] + (T(-0.5) * amp205);
  J[36] = J[36] + (T(-0.16666666666666666) * amp205);
  J[37] = J[37] + (T(0.16666666666666666) * amp205);
  const cx<T> amp206 = iovxxx<T>(w301, w1, w97, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp206);
  J[36] = J[36] + (T(0.16666666666666666) * amp206);
  const cx<T> amp207 = iovxxx<T>(w301, w1, w98, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp207);
  J[37] = J[37] + (T(0.16666666666666666) * amp207);
  const cx<T> amp208 = iovxxx<T>(w301, w1, w99, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp208);
  J[37] = J[37] + (T(0.16666666666666666) * amp208);
  const cx<T> amp209 = iovxxx<T>(w301, w1, w100, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp209);
  J[36] = J[36] + (T(0.16666666666666666) * amp209);
  const cx<T> amp210 = iovxxx<T>(w301, w1, w104, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp210);
  J[29] = J[29] + (T(-0.5) * amp210);
  J[36] = J[36] + (T(-0.16666666666666666) * amp210);
  J[37] = J[37] + (T(0.16666666666666666) * amp210);
  const cx<T> amp211 = iovxxx<T>(w301, w1, w105, g0_0, g0_1);
  J[29] = J[29] + (T(-0.5) * amp211);
  J[37] = J[37] + (T(0.16666666666666666) * amp211);
  const cx<T> amp212 = iovxxx<T>(w301, w1, w106, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp212);
  J[36] = J[36] + (T(0.16666666666666666) * amp212);
  const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w302 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
  const cx<T> amp213 = iovxxx<T>(w302, w1, w9, g0_0, g0_1);
  J[18] = J[18] + (T(0.16666666666666666) * amp213);
  J[19] = J[19] + (T(-0.5) * amp213);
  J[22] = J[22] + (T(-0.16666666666666666) * amp213);
  J[23] = J[23] + (T(0.5) * amp213);
  J[34] = J[34] + (T(-0.16666666666666666) * amp213);
  J[35] = J[35] + (T(0.5) * amp213);
  J[46] = J[46] + (T(0.16666666666666666) * amp213);
  J[47] = J[47] + (T(-0.5) * amp213);
  const cx<T> amp214 = iovxxx<T>(w302, w1, w10, g0_0, g0_1);
  J[18] = J[18] + (T(-0.16666666666666666) * amp214);
  J[19] = J[19] + (T(0.5) * amp214);
  J[30] = J[30] + (T(0.16666666666666666) * amp214);
  J[31] = J[31] + (T(-0.5) * amp214);
  J[42] = J[42] + (T(0.16666666666666666) * amp214);
  J[43] = J[43] + (T(-0.5) * amp214);
  J[46] = J[46] + (T(-0.16666666666666666) * amp214);
  J[47] = J[47] + (T(0.5) * amp214);
  const cx<T> amp215 = iovxxx<T>(w302, w1, w11, g0_0, g0_1);
  J[22] = J[22] + (T(0.16666666666666666) * amp215);
  J[23] = J[23] + (T(-0.5) * amp215);
  J[30] = J[30] + (T(-0.16666666666666666) * amp215);
  J[31] = J[31] + (T(0.5) * amp215);
  J[34] = J[34] + (T(0.16666666666666666) * amp215);
  J[35] = J[35] + (T(-0.5) * amp215);
  J[42] = J[42] + (T(-0.16666666666666666) * amp215);
  J[43] = J[43] + (T(0.5) * amp215);
  const cx<T> amp216 = iovxxx<T>(w302, w1, w12, g0_0, g0_1);
  J[18] = J[18] + (T(0.16666666666666666) * amp216);
  J[19] = J[19] + (T(-0.5) * amp216);
  J[22] = J[22] + (T(-0.16666666666666666) * amp216);
  J[23] = J[23] + (T(0.5) * amp216);
  J[34] = J[34] + (T(-0.16666666666666666) * amp216);
  J[35] = J[35] + (T(0.5) * amp216);
  J[46] = J[46] + (T(0.16666666666666666) * amp216);
  J[47] = J[47] + (T(-0.5) * amp216);
  const cx<T> amp217 = iovxxx<T>(w302, w1, w14, g0_0, g0_1);
  J[18] = J[18] + (T(0.16666666666666666) * amp217);
  J[19] = J[19] + (T(-0.5) * amp217);
  J[30] = J[30] + (T(-0.16666666666666666) * amp217);
  J[31] = J[31] + (T(0.5) * amp217);
  J[42] = J[42] + (T(-0.16666666666666666) * amp217);
  J[43] = J[43] + (T(0.5) * amp217);
  J[46] = J[46] + (T(0.16666666666666666) * amp217);
  J[47] = J[47] + (T(-0.5) * amp217);
  const cx<T> amp218 = iovxxx<T>(w302, w1, w16, g0_0, g0_1);
  J[22] = J[22] + (T(0.16666666666666666) * amp218);
  J[23] = J[23] + (T(-0.5) * amp218);
  J[30] = J[30] + (T(-0.16666666666666666) * amp218);
  J[31] = J[31] + (T(0.5) * amp218);
  J[34] = J[34] + (T(0.16666666666666666) * amp218);
  J[35] = J[35] + (T(-0.5) * amp218);
  J[42] = J[42] + (T(-0.16666666666666666) * amp218);
  J[43] = J[43] + (T(0.5) * amp218);
  const mom qs0_4_5 = pr0 + (-pr4) + (-pr5);
  const vec<T> Qs0_4_5 = tv<T>(qs0_4_5);
  const cx<T> d0_4_5_0 = cvt<T>(inv_denominator(qs0_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w303 = fvixxx<T>(w0, w13, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w304 = fvixxx<T>(w299, w5, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w305 = fvixxx<T>(w300, w4, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const cx<T> amp219 = iovxxx<T>(w303, w1, w66, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp219);
  J[11] = J[11] + (T(0.5) * amp219);
  J[38] = J[38] + (T(0.5) * amp219);
  J[39] = J[39] + (T(-0.5) * amp219);
  const cx<T> amp220 = iovxxx<T>(w303, w1, w68, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp220);
  J[11] = J[11] + (T(-0.5) * amp220);
  J[16] = J[16] + (T(-0.16666666666666666) * amp220);
  J[28] = J[28] + (T(0.16666666666666666) * amp220);
  const cx<T> amp221 = iovxxx<T>(w303, w1, w70, g0_0, g0_1);
  J[16] = J[16] + (T(-0.16666666666666666) * amp221);
  J[28] = J[28] + (T(0.16666666666666666) * amp221);
  J[38] = J[38] + (T(0.5) * amp221);
  J[39] = J[39] + (T(-0.5) * amp221);
  const cx<T> amp222 = iovxxx<T>(w304, w1, w66, g0_0, g0_1);
  J[11] = J[11] + (T(0.5) * amp222);
  J[39] = J[39] + (T(-0.5) * amp222);
  const cx<T> amp223 = iovxxx<T>(w304, w1, w68, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp223);
  J[28] = J[28] + (T(0.16666666666666666) * amp223);
  const cx<T> amp224 = iovxxx<T>(w304, w1, w70, g0_0, g0_1);
  J[28] = J[28] + (T(0.16666666666666666) * amp224);
  J[39] = J[39] + (T(-0.5) * amp224);
  const cx<T> amp225 = iovxxx<T>(w305, w1, w66, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp225);
  J[38] = J[38] + (T(-0.5) * amp225);
  const cx<T> amp226 = iovxxx<T>(w305, w1, w68, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp226);
  J[16] = J[16] + (T(0.16666666666666666) * amp226);
  const cx<T> amp227 = iovxxx<T>(w305, w1, w70, g0_0, g0_1);
  J[16] = J[16] + (T(0.16666666666666666) * amp227);
  J[38] = J[38] + (T(-0.5) * amp227);
  const mom qs0_4_6 = pr0 + (-pr4) + (-pr6);
  const vec<T> Qs0_4_6 = tv<T>(qs0_4_6);
  const cx<T> d0_4_6_0 = cvt<T>(inv_denominator(qs0_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w306 = fvixxx<T>(w0, w15, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w307 = fvixxx<T>(w299, w6, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w308 = fvixxx<T>(w301, w4, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const cx<T> amp228 = iovxxx<T>(w306, w1, w49, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp228);
  J[9] = J[9] + (T(0.5) * amp228);
  J[26] = J[26] + (T(0.5) * amp228);
  J[27] = J[27] + (T(-0.5) * amp228);
  const cx<T> amp229 = iovxxx<T>(w306, w1, w51, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp229);
  J[9] = J[9] + (T(-0.5) * amp229);
  J[20] = J[20] + (T(-0.16666666666666666) * amp229);
  J[40] = J[40] + (T(0.16666666666666666) * amp229);
  const cx<T> amp230 = iovxxx<T>(w306, w1, w53, g0_0, g0_1);
  J[20] = J[20] + (T(-0.16666666666666666) * amp230);
  J[26] = J[26] + (T(0.5) * amp230);
  J[27] = J[27] + (T(-0.5) * amp230);
  J[40] = J[40] + (T(0.16666666666666666) * amp230);
  const cx<T> amp231 = iovxxx<T>(w307, w1, w49, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp231);
  J[27] = J[27] + (T(-0.5) * amp231);
  const cx<T> amp232 = iovxxx<T>(w307, w1, w51, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp232);
  J[40] = J[40] + (T(0.16666666666666666) * amp232);
  const cx<T> amp233 = iovxxx<T>(w307, w1, w53, g0_0, g0_1);
  J[27] = J[27] + (T(-0.5) * amp233);
  J[40] = J[40] + (T(0.16666666666666666) * amp233);
  const cx<T> amp234 = iovxxx<T>(w308, w1, w49, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp234);
  J[26] = J[26] + (T(-0.5) * amp234);
  const cx<T> amp235 = iovxxx<T>(w308, w1, w51, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp235);
  J[20] = J[20] + (T(0.16666666666666666) * amp235);
  const cx<T> amp236 = iovxxx<T>(w308, w1, w53, g0_0, g0_1);
  J[20] = J[20] + (T(0.16666666666666666) * amp236);
  J[26] = J[26] + (T(-0.5) * amp236);
  const mom qs0_5_6 = pr0 + (-pr5) + (-pr6);
  const vec<T> Qs0_5_6 = tv<T>(qs0_5_6);
  const cx<T> d0_5_6_0 = cvt<T>(inv_denominator(qs0_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w309 = fvixxx<T>(w0, w8, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const cx<T> amp237 = iovxxx<T>(w309, w1, w32, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp237);
  J[7] = J[7] + (T(0.5) * amp237);
  J[14] = J[14] + (T(0.5) * amp237);
  J[15] = J[15] + (T(-0.5) * amp237);
  const cx<T> amp238 = iovxxx<T>(w309, w1, w34, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp238);
  J[7] = J[7] + (T(-0.5) * amp238);
  J[32] = J[32] + (T(-0.16666666666666666) * amp238);
  J[44] = J[44] + (T(0.16666666666666666) * amp238);
  const cx<T> amp239 = iovxxx<T>(w309, w1, w36, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp239);
  J[15] = J[15] + (T(-0.5) * amp239);
  J[32] = J[32] + (T(-0.16666666666666666) * amp239);
  J[44] = J[44] + (T(0.16666666666666666) * amp239);
}

// part 6: amplitudes 240 .. 279 (113 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part6(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_5_6 = (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs4_5_6 = tv<T>(qs4_5_6);
  const cx<T> d4_5_6_0 = cvt<T>(inv_denominator(qs4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w9 = jvvxxx<T, false>(w4, Qs4, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w10 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w11 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const wf<T> w12 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs4_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const wf<T> w14 = jvvxxx<T, false>(w13, Qs4_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const wf<T> w16 = jvvxxx<T, false>(w15, Qs4_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
  const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w83 = jvvxxx<T, false>(w7, Qs2_3, w13, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const mom qs0_5 = pr0 + (-pr5);
  const vec<T> Qs0_5 = tv<T>(qs0_5);
  const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w300 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
  const mom qs0_6 = pr0 + (-pr6);
  const vec<T> Qs0_6 = tv<T>(qs0_6);
  const cx<T> d0_6_0 = cvt<T>(inv_denominator(qs0_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w301 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_6, T(pe0.m), d0_6_0);
  const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w302 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
  const mom qs0_4_5 = pr0 + (-pr4) + (-pr5);
  const vec<T> Qs0_4_5 = tv<T>(qs0_4_5);
  const cx<T> d0_4_5_0 = cvt<T>(inv_denominator(qs0_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w303 = fvixxx<T>(w0, w13, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w304 = fvixxx<T>(w299, w5, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w305 = fvixxx<T>(w300, w4, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const mom qs0_4_6 = pr0 + (-pr4) + (-pr6);
  const vec<T> Qs0_4_6 = tv<T>(qs0_4_6);
  const cx<T> d0_4_6_0 = cvt<T>(inv_denominator(qs0_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w306 = fvixxx<T>(w0, w15, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w307 = fvixxx<T>(w299, w6, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w308 = fvixxx<T>(w301, w4, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const mom qs0_5_6 = pr0 + (-pr5) + (-pr6);
  const vec<T> Qs0_5_6 = tv<T>(qs0_5_6);
  const cx<T> d0_5_6_0 = cvt<T>(inv_denominator(qs0_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w309 = fvixxx<T>(w0, w8, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const wf<T> w310 = fvixxx<T>(w300, w6, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const wf<T> w311 = fvixxx<T>(w301, w5, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const cx<T> amp240 = iovxxx<T>(w310, w1, w32, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp240);
  J[15] = J[15] + (T(-0.5) * amp240);
  const cx<T> amp241 = iovxxx<T>(w310, w1, w34, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp241);
  J[44] = J[44] + (T(0.16666666666666666) * amp241);
  const cx<T> amp242 = iovxxx<T>(w310, w1, w36, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp242);
  J[44] = J[44] + (T(0.16666666666666666) * amp242);
  const cx<T> amp243 = iovxxx<T>(w311, w1, w32, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp243);
  J[14] = J[14] + (T(-0.5) * amp243);
  const cx<T> amp244 = iovxxx<T>(w311, w1, w34, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp244);
  J[32] = J[32] + (T(0.16666666666666666) * amp244);
  const cx<T> amp245 = iovxxx<T>(w311, w1, w36, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp245);
  J[32] = J[32] + (T(0.16666666666666666) * amp245);
  const mom qs0_2_3_4 = pr0 + (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs0_2_3_4 = tv<T>(qs0_2_3_4);
  const cx<T> d0_2_3_4_0 = cvt<T>(inv_denominator(qs0_2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w312 = fvixxx<T>(w0, w32, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w313 = fvixxx<T>(w0, w34, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w314 = fvixxx<T>(w0, w36, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w315 = fvixxx<T>(w299, w7, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w316 = fvixxx<T>(w302, w4, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const cx<T> amp246 = iovxxx<T>(w312, w1, w8, g0_0, g0_1);
  J[33] = J[33] + (T(-0.5) * amp246);
  J[35] = J[35] + (T(0.5) * amp246);
  J[45] = J[45] + (T(0.5) * amp246);
  J[47] = J[47] + (T(-0.5) * amp246);
  const cx<T> amp247 = iovxxx<T>(w313, w1, w8, g0_0, g0_1);
  J[32] = J[32] + (T(-0.16666666666666666) * amp247);
  J[33] = J[33] + (T(0.5) * amp247);
  J[44] = J[44] + (T(0.16666666666666666) * amp247);
  J[45] = J[45] + (T(-0.5) * amp247);
  const cx<T> amp248 = iovxxx<T>(w314, w1, w8, g0_0, g0_1);
  J[32] = J[32] + (T(-0.16666666666666666) * amp248);
  J[35] = J[35] + (T(0.5) * amp248);
  J[44] = J[44] + (T(0.16666666666666666) * amp248);
  J[47] = J[47] + (T(-0.5) * amp248);
  const cx<T> amp249 = iovxxx<T>(w315, w1, w8, g0_0, g0_1);
  J[33] = J[33] + (T(0.5) * amp249);
  J[34] = J[34] + (T(-0.16666666666666666) * amp249);
  J[45] = J[45] + (T(-0.5) * amp249);
  J[46] = J[46] + (T(0.16666666666666666) * amp249);
  const cx<T> amp250 = iovxxx<T>(w316, w1, w8, g0_0, g0_1);
  J[34] = J[34] + (T(-0.16666666666666666) * amp250);
  J[35] = J[35] + (T(0.5) * amp250);
  J[46] = J[46] + (T(0.16666666666666666) * amp250);
  J[47] = J[47] + (T(-0.5) * amp250);
  const mom qs0_2_3_5 = pr0 + (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs0_2_3_5 = tv<T>(qs0_2_3_5);
  const cx<T> d0_2_3_5_0 = cvt<T>(inv_denominator(qs0_2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w317 = fvixxx<T>(w0, w49, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w318 = fvixxx<T>(w0, w51, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w319 = fvixxx<T>(w0, w53, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w320 = fvixxx<T>(w300, w7, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w321 = fvixxx<T>(w302, w5, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const cx<T> amp251 = iovxxx<T>(w317, w1, w15, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp251);
  J[23] = J[23] + (T(0.5) * amp251);
  J[41] = J[41] + (T(0.5) * amp251);
  J[43] = J[43] + (T(-0.5) * amp251);
  const cx<T> amp252 = iovxxx<T>(w318, w1, w15, g0_0, g0_1);
  J[20] = J[20] + (T(-0.16666666666666666) * amp252);
  J[21] = J[21] + (T(0.5) * amp252);
  J[40] = J[40] + (T(0.16666666666666666) * amp252);
  J[41] = J[41] + (T(-0.5) * amp252);
  const cx<T> amp253 = iovxxx<T>(w319, w1, w15, g0_0, g0_1);
  J[20] = J[20] + (T(-0.16666666666666666) * amp253);
  J[23] = J[23] + (T(0.5) * amp253);
  J[40] = J[40] + (T(0.16666666666666666) * amp253);
  J[43] = J[43] + (T(-0.5) * amp253);
  const cx<T> amp254 = iovxxx<T>(w320, w1, w15, g0_0, g0_1);
  J[21] = J[21] + (T(0.5) * amp254);
  J[22] = J[22] + (T(-0.16666666666666666) * amp254);
  J[41] = J[41] + (T(-0.5) * amp254);
  J[42] = J[42] + (T(0.16666666666666666) * amp254);
  const cx<T> amp255 = iovxxx<T>(w321, w1, w15, g0_0, g0_1);
  J[22] = J[22] + (T(-0.16666666666666666) * amp255);
  J[23] = J[23] + (T(0.5) * amp255);
  J[42] = J[42] + (T(0.16666666666666666) * amp255);
  J[43] = J[43] + (T(-0.5) * amp255);
  const mom qs0_2_3_6 = pr0 + (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs0_2_3_6 = tv<T>(qs0_2_3_6);
  const cx<T> d0_2_3_6_0 = cvt<T>(inv_denominator(qs0_2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w322 = fvixxx<T>(w0, w66, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w323 = fvixxx<T>(w0, w68, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w324 = fvixxx<T>(w0, w70, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w325 = fvixxx<T>(w301, w7, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w326 = fvixxx<T>(w302, w6, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const cx<T> amp256 = iovxxx<T>(w322, w1, w13, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp256);
  J[19] = J[19] + (T(0.5) * amp256);
  J[29] = J[29] + (T(0.5) * amp256);
  J[31] = J[31] + (T(-0.5) * amp256);
  const cx<T> amp257 = iovxxx<T>(w323, w1, w13, g0_0, g0_1);
  J[16] = J[16] + (T(-0.16666666666666666) * amp257);
  J[17] = J[17] + (T(0.5) * amp257);
  J[28] = J[28] + (T(0.16666666666666666) * amp257);
  J[29] = J[29] + (T(-0.5) * amp257);
  const cx<T> amp258 = iovxxx<T>(w324, w1, w13, g0_0, g0_1);
  J[16] = J[16] + (T(-0.16666666666666666) * amp258);
  J[19] = J[19] + (T(0.5) * amp258);
  J[28] = J[28] + (T(0.16666666666666666) * amp258);
  J[31] = J[31] + (T(-0.5) * amp258);
  const cx<T> amp259 = iovxxx<T>(w325, w1, w13, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp259);
  J[18] = J[18] + (T(-0.16666666666666666) * amp259);
  J[29] = J[29] + (T(-0.5) * amp259);
  J[30] = J[30] + (T(0.16666666666666666) * amp259);
  const cx<T> amp260 = iovxxx<T>(w326, w1, w13, g0_0, g0_1);
  J[18] = J[18] + (T(-0.16666666666666666) * amp260);
  J[19] = J[19] + (T(0.5) * amp260);
  J[30] = J[30] + (T(0.16666666666666666) * amp260);
  J[31] = J[31] + (T(-0.5) * amp260);
  const mom qs0_4_5_6 = pr0 + (-pr4) + (-pr5) + (-pr6);
  const vec<T> Qs0_4_5_6 = tv<T>(qs0_4_5_6);
  const cx<T> d0_4_5_6_0 = cvt<T>(inv_denominator(qs0_4_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w327 = fvixxx<T>(w0, w9, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w328 = fvixxx<T>(w0, w10, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w329 = fvixxx<T>(w0, w11, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w330 = fvixxx<T>(w0, w12, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w331 = fvixxx<T>(w0, w14, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w332 = fvixxx<T>(w0, w16, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w333 = fvixxx<T>(w299, w8, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w334 = fvixxx<T>(w300, w15, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w335 = fvixxx<T>(w301, w13, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w336 = fvixxx<T>(w303, w6, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w337 = fvixxx<T>(w304, w6, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w338 = fvixxx<T>(w305, w6, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w339 = fvixxx<T>(w306, w5, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w340 = fvixxx<T>(w307, w5, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w341 = fvixxx<T>(w308, w5, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w342 = fvixxx<T>(w309, w4, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w343 = fvixxx<T>(w310, w4, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const wf<T> w344 = fvixxx<T>(w311, w4, g0_0, g0_1, Qs0_4_5_6, T(pe0.m), d0_4_5_6_0);
  const cx<T> amp261 = iovxxx<T>(w327, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp261);
  J[7] = J[7] + (T(0.5) * amp261);
  J[9] = J[9] + (T(0.5) * amp261);
  J[11] = J[11] + (T(-0.5) * amp261);
  J[18] = J[18] + (T(0.16666666666666666) * amp261);
  J[22] = J[22] + (T(-0.16666666666666666) * amp261);
  J[34] = J[34] + (T(-0.16666666666666666) * amp261);
  J[46] = J[46] + (T(0.16666666666666666) * amp261);
  const cx<T> amp262 = iovxxx<T>(w328, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp262);
  J[8] = J[8] + (T(-0.5) * amp262);
  J[10] = J[10] + (T(-0.5) * amp262);
  J[11] = J[11] + (T(0.5) * amp262);
  J[18] = J[18] + (T(-0.16666666666666666) * amp262);
  J[30] = J[30] + (T(0.16666666666666666) * amp262);
  J[42] = J[42] + (T(0.16666666666666666) * amp262);
  J[46] = J[46] + (T(-0.16666666666666666) * amp262);
  const cx<T> amp263 = iovxxx<T>(w329, w1, w7, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp263);
  J[8] = J[8] + (T(0.5) * amp263);
  J[9] = J[9] + (T(-0.5) * amp263);
  J[10] = J[10] + (T(0.5) * amp263);
  J[22] = J[22] + (T(0.16666666666666666) * amp263);
  J[30] = J[30] + (T(-0.16666666666666666) * amp263);
  J[34] = J[34] + (T(0.16666666666666666) * amp263);
  J[42] = J[42] + (T(-0.16666666666666666) * amp263);
  const cx<T> amp264 = iovxxx<T>(w330, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp264);
  J[7] = J[7] + (T(0.5) * amp264);
  J[9] = J[9] + (T(0.5) * amp264);
  J[11] = J[11] + (T(-0.5) * amp264);
  J[18] = J[18] + (T(0.16666666666666666) * amp264);
  J[22] = J[22] + (T(-0.16666666666666666) * amp264);
  J[34] = J[34] + (T(-0.16666666666666666) * amp264);
  J[46] = J[46] + (T(0.16666666666666666) * amp264);
  const cx<T> amp265 = iovxxx<T>(w331, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp265);
  J[8] = J[8] + (T(0.5) * amp265);
  J[10] = J[10] + (T(0.5) * amp265);
  J[11] = J[11] + (T(-0.5) * amp265);
  J[18] = J[18] + (T(0.16666666666666666) * amp265);
  J[30] = J[30] + (T(-0.16666666666666666) * amp265);
  J[42] = J[42] + (T(-0.16666666666666666) * amp265);
  J[46] = J[46] + (T(0.16666666666666666) * amp265);
  const cx<T> amp266 = iovxxx<T>(w332, w1, w7, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp266);
  J[8] = J[8] + (T(0.5) * amp266);
  J[9] = J[9] + (T(-0.5) * amp266);
  J[10] = J[10] + (T(0.5) * amp266);
  J[22] = J[22] + (T(0.16666666666666666) * amp266);
  J[30] = J[30] + (T(-0.16666666666666666) * amp266);
  J[34] = J[34] + (T(0.16666666666666666) * amp266);
  J[42] = J[42] + (T(-0.16666666666666666) * amp266);
  const cx<T> amp267 = iovxxx<T>(w333, w1, w7, g0_0, g0_1);
  J[9] = J[9] + (T(0.5) * amp267);
  J[11] = J[11] + (T(-0.5) * amp267);
  J[34] = J[34] + (T(-0.16666666666666666) * amp267);
  J[46] = J[46] + (T(0.16666666666666666) * amp267);
  const cx<T> amp268 = iovxxx<T>(w334, w1, w7, g0_0, g0_1);
  J[7] = J[7] + (T(0.5) * amp268);
  J[10] = J[10] + (T(-0.5) * amp268);
  J[22] = J[22] + (T(-0.16666666666666666) * amp268);
  J[42] = J[42] + (T(0.16666666666666666) * amp268);
  const cx<T> amp269 = iovxxx<T>(w335, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp269);
  J[8] = J[8] + (T(-0.5) * amp269);
  J[18] = J[18] + (T(-0.16666666666666666) * amp269);
  J[30] = J[30] + (T(0.16666666666666666) * amp269);
  const cx<T> amp270 = iovxxx<T>(w336, w1, w7, g0_0, g0_1);
  J[10] = J[10] + (T(0.5) * amp270);
  J[11] = J[11] + (T(-0.5) * amp270);
  J[42] = J[42] + (T(-0.16666666666666666) * amp270);
  J[46] = J[46] + (T(0.16666666666666666) * amp270);
  const cx<T> amp271 = iovxxx<T>(w337, w1, w7, g0_0, g0_1);
  J[11] = J[11] + (T(-0.5) * amp271);
  J[46] = J[46] + (T(0.16666666666666666) * amp271);
  const cx<T> amp272 = iovxxx<T>(w338, w1, w7, g0_0, g0_1);
  J[10] = J[10] + (T(-0.5) * amp272);
  J[42] = J[42] + (T(0.16666666666666666) * amp272);
  const cx<T> amp273 = iovxxx<T>(w339, w1, w7, g0_0, g0_1);
  J[8] = J[8] + (T(0.5) * amp273);
  J[9] = J[9] + (T(-0.5) * amp273);
  J[30] = J[30] + (T(-0.16666666666666666) * amp273);
  J[34] = J[34] + (T(0.16666666666666666) * amp273);
  const cx<T> amp274 = iovxxx<T>(w340, w1, w7, g0_0, g0_1);
  J[9] = J[9] + (T(-0.5) * amp274);
  J[34] = J[34] + (T(0.16666666666666666) * amp274);
  const cx<T> amp275 = iovxxx<T>(w341, w1, w7, g0_0, g0_1);
  J[8] = J[8] + (T(-0.5) * amp275);
  J[30] = J[30] + (T(0.16666666666666666) * amp275);
  const cx<T> amp276 = iovxxx<T>(w342, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(0.5) * amp276);
  J[7] = J[7] + (T(-0.5) * amp276);
  J[18] = J[18] + (T(-0.16666666666666666) * amp276);
  J[22] = J[22] + (T(0.16666666666666666) * amp276);
  const cx<T> amp277 = iovxxx<T>(w343, w1, w7, g0_0, g0_1);
  J[7] = J[7] + (T(-0.5) * amp277);
  J[22] = J[22] + (T(0.16666666666666666) * amp277);
  const cx<T> amp278 = iovxxx<T>(w344, w1, w7, g0_0, g0_1);
  J[6] = J[6] + (T(-0.5) * amp278);
  J[18] = J[18] + (T(0.16666666666666666) * amp278);
  const mom qs0_2_3_4_5 = pr0 + (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs0_2_3_4_5 = tv<T>(qs0_2_3_4_5);
  const cx<T> d0_2_3_4_5_0 = cvt<T>(inv_denominator(qs0_2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w345 = fvixxx<T>(w0, w83, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const cx<T> amp279 = iovxxx<T>(w345, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(-0.5) * amp279);
  J[39] = J[39] + (T(0.5) * amp279);
  J[43] = J[43] + (T(0.5) * amp279);
  J[47] = J[47] + (T(-0.5) * amp279);
}

// part 7: amplitudes 280 .. 319 (135 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part7(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs4_5 = (-pr4) + (-pr5);
  const vec<T> Qs4_5 = tv<T>(qs4_5);
  const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w13 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
  const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w84 = jgggxx<T, false>(w7, w4, w5, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w85 = jgggxx<T, false>(w5, w7, w4, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w86 = jgggxx<T, false>(w4, w5, w7, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w87 = jvvxxx<T, false>(w32, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w88 = jvvxxx<T, false>(w34, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w89 = jvvxxx<T, false>(w36, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w90 = jvvxxx<T, false>(w49, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w91 = jvvxxx<T, false>(w51, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w92 = jvvxxx<T, false>(w53, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
  const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
  const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w93 = fvoxxx<T>(w2, w13, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w94 = fvoxxx<T>(w33, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w95 = fvoxxx<T>(w50, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
  const wf<T> w96 = jioxxx<T, false>(w3, w93, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w97 = jioxxx<T, false>(w3, w94, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w98 = jioxxx<T, false>(w3, w95, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w99 = jioxxx<T, false>(w35, w50, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w100 = jioxxx<T, false>(w52, w33, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs3_4_5 = (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs3_4_5 = tv<T>(qs3_4_5);
  const cx<T> d3_4_5_3 = cvt<T>(inv_denominator(qs3_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w101 = fvixxx<T>(w3, w13, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w102 = fvixxx<T>(w35, w5, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w103 = fvixxx<T>(w52, w4, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
  const wf<T> w104 = jioxxx<T, false>(w101, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w105 = jioxxx<T, false>(w102, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const wf<T> w106 = jioxxx<T, false>(w103, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
  const mom qs2_3_4_6 = (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs2_3_4_6 = tv<T>(qs2_3_4_6);
  const cx<T> d2_3_4_6_0 = cvt<T>(inv_denominator(qs2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w125 = jvvxxx<T, false>(w7, Qs2_3, w15, Qs4_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w126 = jgggxx<T, false>(w7, w4, w6, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w127 = jgggxx<T, false>(w6, w7, w4, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const mom qs0_5 = pr0 + (-pr5);
  const vec<T> Qs0_5 = tv<T>(qs0_5);
  const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w300 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
  const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w302 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
  const mom qs0_4_5 = pr0 + (-pr4) + (-pr5);
  const vec<T> Qs0_4_5 = tv<T>(qs0_4_5);
  const cx<T> d0_4_5_0 = cvt<T>(inv_denominator(qs0_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w303 = fvixxx<T>(w0, w13, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w304 = fvixxx<T>(w299, w5, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const wf<T> w305 = fvixxx<T>(w300, w4, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
  const mom qs0_2_3_4 = pr0 + (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs0_2_3_4 = tv<T>(qs0_2_3_4);
  const cx<T> d0_2_3_4_0 = cvt<T>(inv_denominator(qs0_2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w312 = fvixxx<T>(w0, w32, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w313 = fvixxx<T>(w0, w34, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w314 = fvixxx<T>(w0, w36, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w315 = fvixxx<T>(w299, w7, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w316 = fvixxx<T>(w302, w4, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const mom qs0_2_3_5 = pr0 + (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs0_2_3_5 = tv<T>(qs0_2_3_5);
  const cx<T> d0_2_3_5_0 = cvt<T>(inv_denominator(qs0_2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w317 = fvixxx<T>(w0, w49, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w318 = fvixxx<T>(w0, w51, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w319 = fvixxx<T>(w0, w53, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w320 = fvixxx<T>(w300, w7, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w321 = fvixxx<T>(w302, w5, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const mom qs0_2_3_4_5 = pr0 + (-pr2) + (-pr3) + (-pr4) + (-pr5);
  const vec<T> Qs0_2_3_4_5 = tv<T>(qs0_2_3_4_5);
  const cx<T> d0_2_3_4_5_0 = cvt<T>(inv_denominator(qs0_2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w346 = fvixxx<T>(w0, w84, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w347 = fvixxx<T>(w0, w85, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w348 = fvixxx<T>(w0, w86, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w349 = fvixxx<T>(w0, w87, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w350 = fvixxx<T>(w0, w88, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w351 = fvixxx<T>(w0, w89, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w352 = fvixxx<T>(w0, w90, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w353 = fvixxx<T>(w0, w91, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w354 = fvixxx<T>(w0, w92, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w355 = fvixxx<T>(w0, w96, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w356 = fvixxx<T>(w0, w97, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w357 = fvixxx<T>(w0, w98, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w358 = fvixxx<T>(w0, w99, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w359 = fvixxx<T>(w0, w100, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w360 = fvixxx<T>(w0, w104, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w361 = fvixxx<T>(w0, w105, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w362 = fvixxx<T>(w0, w106, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w363 = fvixxx<T>(w299, w49, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w364 = fvixxx<T>(w299, w51, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w365 = fvixxx<T>(w299, w53, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w366 = fvixxx<T>(w300, w32, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w367 = fvixxx<T>(w300, w34, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w368 = fvixxx<T>(w300, w36, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w369 = fvixxx<T>(w302, w13, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w370 = fvixxx<T>(w303, w7, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w371 = fvixxx<T>(w304, w7, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w372 = fvixxx<T>(w305, w7, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w373 = fvixxx<T>(w312, w5, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w374 = fvixxx<T>(w313, w5, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w375 = fvixxx<T>(w314, w5, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w376 = fvixxx<T>(w315, w5, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w377 = fvixxx<T>(w316, w5, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w378 = fvixxx<T>(w317, w4, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w379 = fvixxx<T>(w318, w4, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w380 = fvixxx<T>(w319, w4, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w381 = fvixxx<T>(w320, w4, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const wf<T> w382 = fvixxx<T>(w321, w4, g0_0, g0_1, Qs0_2_3_4_5, T(pe0.m), d0_2_3_4_5_0);
  const cx<T> amp280 = iovxxx<T>(w346, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(0.5) * amp280);
  J[41] = J[41] + (T(-0.5) * amp280);
  J[45] = J[45] + (T(-0.5) * amp280);
  J[47] = J[47] + (T(0.5) * amp280);
  const cx<T> amp281 = iovxxx<T>(w347, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(-0.5) * amp281);
  J[41] = J[41] + (T(0.5) * amp281);
  J[43] = J[43] + (T(-0.5) * amp281);
  J[45] = J[45] + (T(0.5) * amp281);
  const cx<T> amp282 = iovxxx<T>(w348, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(-0.5) * amp282);
  J[39] = J[39] + (T(0.5) * amp282);
  J[43] = J[43] + (T(0.5) * amp282);
  J[47] = J[47] + (T(-0.5) * amp282);
  const cx<T> amp283 = iovxxx<T>(w349, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(-0.5) * amp283);
  J[41] = J[41] + (T(0.5) * amp283);
  J[45] = J[45] + (T(0.5) * amp283);
  J[47] = J[47] + (T(-0.5) * amp283);
  const cx<T> amp284 = iovxxx<T>(w350, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(0.5) * amp284);
  J[45] = J[45] + (T(-0.5) * amp284);
  const cx<T> amp285 = iovxxx<T>(w351, w1, w6, g0_0, g0_1);
  J[41] = J[41] + (T(0.5) * amp285);
  J[47] = J[47] + (T(-0.5) * amp285);
  const cx<T> amp286 = iovxxx<T>(w352, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(-0.5) * amp286);
  J[41] = J[41] + (T(0.5) * amp286);
  J[43] = J[43] + (T(-0.5) * amp286);
  J[45] = J[45] + (T(0.5) * amp286);
  const cx<T> amp287 = iovxxx<T>(w353, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(0.5) * amp287);
  J[41] = J[41] + (T(-0.5) * amp287);
  const cx<T> amp288 = iovxxx<T>(w354, w1, w6, g0_0, g0_1);
  J[43] = J[43] + (T(-0.5) * amp288);
  J[45] = J[45] + (T(0.5) * amp288);
  const cx<T> amp289 = iovxxx<T>(w355, w1, w6, g0_0, g0_1);
  J[36] = J[36] + (T(-0.16666666666666666) * amp289);
  J[37] = J[37] + (T(0.16666666666666666) * amp289);
  J[38] = J[38] + (T(0.5) * amp289);
  J[39] = J[39] + (T(-0.5) * amp289);
  const cx<T> amp290 = iovxxx<T>(w356, w1, w6, g0_0, g0_1);
  J[36] = J[36] + (T(0.16666666666666666) * amp290);
  J[38] = J[38] + (T(-0.5) * amp290);
  const cx<T> amp291 = iovxxx<T>(w357, w1, w6, g0_0, g0_1);
  J[37] = J[37] + (T(0.16666666666666666) * amp291);
  J[39] = J[39] + (T(-0.5) * amp291);
  const cx<T> amp292 = iovxxx<T>(w358, w1, w6, g0_0, g0_1);
  J[37] = J[37] + (T(0.16666666666666666) * amp292);
  J[41] = J[41] + (T(-0.5) * amp292);
  const cx<T> amp293 = iovxxx<T>(w359, w1, w6, g0_0, g0_1);
  J[36] = J[36] + (T(0.16666666666666666) * amp293);
  J[45] = J[45] + (T(-0.5) * amp293);
  const cx<T> amp294 = iovxxx<T>(w360, w1, w6, g0_0, g0_1);
  J[36] = J[36] + (T(-0.16666666666666666) * amp294);
  J[37] = J[37] + (T(0.16666666666666666) * amp294);
  J[43] = J[43] + (T(0.5) * amp294);
  J[47] = J[47] + (T(-0.5) * amp294);
  const cx<T> amp295 = iovxxx<T>(w361, w1, w6, g0_0, g0_1);
  J[37] = J[37] + (T(0.16666666666666666) * amp295);
  J[47] = J[47] + (T(-0.5) * amp295);
  const cx<T> amp296 = iovxxx<T>(w362, w1, w6, g0_0, g0_1);
  J[36] = J[36] + (T(0.16666666666666666) * amp296);
  J[43] = J[43] + (T(-0.5) * amp296);
  const cx<T> amp297 = iovxxx<T>(w363, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(0.5) * amp297);
  J[45] = J[45] + (T(-0.5) * amp297);
  const cx<T> amp298 = iovxxx<T>(w364, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(-0.5) * amp298);
  J[40] = J[40] + (T(0.16666666666666666) * amp298);
  const cx<T> amp299 = iovxxx<T>(w365, w1, w6, g0_0, g0_1);
  J[40] = J[40] + (T(0.16666666666666666) * amp299);
  J[45] = J[45] + (T(-0.5) * amp299);
  const cx<T> amp300 = iovxxx<T>(w366, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(0.5) * amp300);
  J[41] = J[41] + (T(-0.5) * amp300);
  const cx<T> amp301 = iovxxx<T>(w367, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(-0.5) * amp301);
  J[44] = J[44] + (T(0.16666666666666666) * amp301);
  const cx<T> amp302 = iovxxx<T>(w368, w1, w6, g0_0, g0_1);
  J[41] = J[41] + (T(-0.5) * amp302);
  J[44] = J[44] + (T(0.16666666666666666) * amp302);
  const cx<T> amp303 = iovxxx<T>(w369, w1, w6, g0_0, g0_1);
  J[42] = J[42] + (T(-0.16666666666666666) * amp303);
  J[43] = J[43] + (T(0.5) * amp303);
  J[46] = J[46] + (T(0.16666666666666666) * amp303);
  J[47] = J[47] + (T(-0.5) * amp303);
  const cx<T> amp304 = iovxxx<T>(w370, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(0.5) * amp304);
  J[39] = J[39] + (T(-0.5) * amp304);
  J[42] = J[42] + (T(-0.16666666666666666) * amp304);
  J[46] = J[46] + (T(0.16666666666666666) * amp304);
  const cx<T> amp305 = iovxxx<T>(w371, w1, w6, g0_0, g0_1);
  J[39] = J[39] + (T(-0.5) * amp305);
  J[46] = J[46] + (T(0.16666666666666666) * amp305);
  const cx<T> amp306 = iovxxx<T>(w372, w1, w6, g0_0, g0_1);
  J[38] = J[38] + (T(-0.5) * amp306);
  J[42] = J[42] + (T(0.16666666666666666) * amp306);
  const cx<T> amp307 = iovxxx<T>(w373, w1, w6, g0_0, g0_1);
  J[45] = J[45] + (T(0.5) * amp307);
  J[47] = J[47] + (T(-0.5) * amp307);
  const cx<T> amp308 = iovxxx<T>(w374, w1, w6, g0_0, g0_1);
  J[44] = J[44] + (T(0.16666666666666666) * amp308);
  J[45] = J[45] + (T(-0.5) * amp308);
  const cx<T> amp309 = iovxxx<T>(w375, w1, w6, g0_0, g0_1);
  J[44] = J[44] + (T(0.16666666666666666) * amp309);
  J[47] = J[47] + (T(-0.5) * amp309);
  const cx<T> amp310 = iovxxx<T>(w376, w1, w6, g0_0, g0_1);
  J[45] = J[45] + (T(-0.5) * amp310);
  J[46] = J[46] + (T(0.16666666666666666) * amp310);
  const cx<T> amp311 = iovxxx<T>(w377, w1, w6, g0_0, g0_1);
  J[46] = J[46] + (T(0.16666666666666666) * amp311);
  J[47] = J[47] + (T(-0.5) * amp311);
  const cx<T> amp312 = iovxxx<T>(w378, w1, w6, g0_0, g0_1);
  J[41] = J[41] + (T(0.5) * amp312);
  J[43] = J[43] + (T(-0.5) * amp312);
  const cx<T> amp313 = iovxxx<T>(w379, w1, w6, g0_0, g0_1);
  J[40] = J[40] + (T(0.16666666666666666) * amp313);
  J[41] = J[41] + (T(-0.5) * amp313);
  const cx<T> amp314 = iovxxx<T>(w380, w1, w6, g0_0, g0_1);
  J[40] = J[40] + (T(0.16666666666666666) * amp314);
  J[43] = J[43] + (T(-0.5) * amp314);
  const cx<T> amp315 = iovxxx<T>(w381, w1, w6, g0_0, g0_1);
  J[41] = J[41] + (T(-0.5) * amp315);
  J[42] = J[42] + (T(0.16666666666666666) * amp315);
  const cx<T> amp316 = iovxxx<T>(w382, w1, w6, g0_0, g0_1);
  J[42] = J[42] + (T(0.16666666666666666) * amp316);
  J[43] = J[43] + (T(-0.5) * amp316);
  const mom qs0_2_3_4_6 = pr0 + (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs0_2_3_4_6 = tv<T>(qs0_2_3_4_6);
  const cx<T> d0_2_3_4_6_0 = cvt<T>(inv_denominator(qs0_2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w383 = fvixxx<T>(w0, w125, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w384 = fvixxx<T>(w0, w126, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w385 = fvixxx<T>(w0, w127, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const cx<T> amp317 = iovxxx<T>(w383, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp317);
  J[27] = J[27] + (T(0.5) * amp317);
  J[31] = J[31] + (T(0.5) * amp317);
  J[35] = J[35] + (T(-0.5) * amp317);
  const cx<T> amp318 = iovxxx<T>(w384, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(0.5) * amp318);
  J[29] = J[29] + (T(-0.5) * amp318);
  J[33] = J[33] + (T(-0.5) * amp318);
  J[35] = J[35] + (T(0.5) * amp318);
  const cx<T> amp319 = iovxxx<T>(w385, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(-0.5) * amp319);
  J[29] = J[29] + (T(0.5) * amp319);
  J[31] = J[31] + (T(-0.5) * amp319);
  J[33] = J[33] + (T(0.5) * amp319);
}

// part 8: amplitudes 320 .. 359 (136 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part8(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const mom qs4_6 = (-pr4) + (-pr6);
  const vec<T> Qs4_6 = tv<T>(qs4_6);
  const cx<T> d4_6_0 = cvt<T>(inv_denominator(qs4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w15 = jvvxxx<T, false>(w4, Qs4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_6_0);
  const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w32 = jvvxxx<T, false>(w7, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_4 = (-pr2) + (-pr4);
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w33 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
  const wf<T> w34 = jioxxx<T, false>(w3, w33, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs3_4 = (-pr3) + (-pr4);
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w35 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
  const wf<T> w36 = jioxxx<T, false>(w35, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_4_6 = (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs2_3_4_6 = tv<T>(qs2_3_4_6);
  const cx<T> d2_3_4_6_0 = cvt<T>(inv_denominator(qs2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w128 = jgggxx<T, false>(w4, w6, w7, g2_0.r, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w129 = jvvxxx<T, false>(w32, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w130 = jvvxxx<T, false>(w34, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w131 = jvvxxx<T, false>(w36, Qs2_3_4, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w132 = jvvxxx<T, false>(w66, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w133 = jvvxxx<T, false>(w68, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w134 = jvvxxx<T, false>(w70, Qs2_3_6, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_4_6 = (-pr2) + (-pr4) + (-pr6);
  const vec<T> Qs2_4_6 = tv<T>(qs2_4_6);
  const cx<T> d2_4_6_3 = cvt<T>(inv_denominator(qs2_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w135 = fvoxxx<T>(w2, w15, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w136 = fvoxxx<T>(w33, w6, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w137 = fvoxxx<T>(w67, w4, g0_0, g0_1, Qs2_4_6, T(pe3.m), d2_4_6_3);
  const wf<T> w138 = jioxxx<T, false>(w3, w135, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w139 = jioxxx<T, false>(w3, w136, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w140 = jioxxx<T, false>(w3, w137, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w141 = jioxxx<T, false>(w35, w67, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w142 = jioxxx<T, false>(w69, w33, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs3_4_6 = (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs3_4_6 = tv<T>(qs3_4_6);
  const cx<T> d3_4_6_3 = cvt<T>(inv_denominator(qs3_4_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w143 = fvixxx<T>(w3, w15, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w144 = fvixxx<T>(w35, w6, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w145 = fvixxx<T>(w69, w4, g0_0, g0_1, Qs3_4_6, T(pe3.m), d3_4_6_3);
  const wf<T> w146 = jioxxx<T, false>(w143, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w147 = jioxxx<T, false>(w144, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const wf<T> w148 = jioxxx<T, false>(w145, w2, g0_0, g0_1, Qs2_3_4_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_6_0);
  const mom qs2_3_5_6 = (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_5_6 = tv<T>(qs2_3_5_6);
  const cx<T> d2_3_5_6_0 = cvt<T>(inv_denominator(qs2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w167 = jvvxxx<T, false>(w7, Qs2_3, w8, Qs5_6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w168 = jgggxx<T, false>(w7, w5, w6, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w169 = jgggxx<T, false>(w6, w7, w5, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w170 = jgggxx<T, false>(w5, w6, w7, g2_0.r, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w171 = jvvxxx<T, false>(w49, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs0_4 = pr0 + (-pr4);
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w299 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
  const mom qs0_6 = pr0 + (-pr6);
  const vec<T> Qs0_6 = tv<T>(qs0_6);
  const cx<T> d0_6_0 = cvt<T>(inv_denominator(qs0_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w301 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_6, T(pe0.m), d0_6_0);
  const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w302 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
  const mom qs0_4_6 = pr0 + (-pr4) + (-pr6);
  const vec<T> Qs0_4_6 = tv<T>(qs0_4_6);
  const cx<T> d0_4_6_0 = cvt<T>(inv_denominator(qs0_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w306 = fvixxx<T>(w0, w15, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w307 = fvixxx<T>(w299, w6, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const wf<T> w308 = fvixxx<T>(w301, w4, g0_0, g0_1, Qs0_4_6, T(pe0.m), d0_4_6_0);
  const mom qs0_2_3_4 = pr0 + (-pr2) + (-pr3) + (-pr4);
  const vec<T> Qs0_2_3_4 = tv<T>(qs0_2_3_4);
  const cx<T> d0_2_3_4_0 = cvt<T>(inv_denominator(qs0_2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w312 = fvixxx<T>(w0, w32, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w313 = fvixxx<T>(w0, w34, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w314 = fvixxx<T>(w0, w36, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w315 = fvixxx<T>(w299, w7, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const wf<T> w316 = fvixxx<T>(w302, w4, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
  const mom qs0_2_3_6 = pr0 + (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs0_2_3_6 = tv<T>(qs0_2_3_6);
  const cx<T> d0_2_3_6_0 = cvt<T>(inv_denominator(qs0_2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w322 = fvixxx<T>(w0, w66, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w323 = fvixxx<T>(w0, w68, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w324 = fvixxx<T>(w0, w70, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w325 = fvixxx<T>(w301, w7, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w326 = fvixxx<T>(w302, w6, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const mom qs0_2_3_4_6 = pr0 + (-pr2) + (-pr3) + (-pr4) + (-pr6);
  const vec<T> Qs0_2_3_4_6 = tv<T>(qs0_2_3_4_6);
  const cx<T> d0_2_3_4_6_0 = cvt<T>(inv_denominator(qs0_2_3_4_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w386 = fvixxx<T>(w0, w128, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w387 = fvixxx<T>(w0, w129, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w388 = fvixxx<T>(w0, w130, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w389 = fvixxx<T>(w0, w131, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w390 = fvixxx<T>(w0, w132, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w391 = fvixxx<T>(w0, w133, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w392 = fvixxx<T>(w0, w134, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w393 = fvixxx<T>(w0, w138, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w394 = fvixxx<T>(w0, w139, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w395 = fvixxx<T>(w0, w140, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w396 = fvixxx<T>(w0, w141, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w397 = fvixxx<T>(w0, w142, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w398 = fvixxx<T>(w0, w146, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w399 = fvixxx<T>(w0, w147, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w400 = fvixxx<T>(w0, w148, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w401 = fvixxx<T>(w299, w66, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w402 = fvixxx<T>(w299, w68, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w403 = fvixxx<T>(w299, w70, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w404 = fvixxx<T>(w301, w32, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w405 = fvixxx<T>(w301, w34, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w406 = fvixxx<T>(w301, w36, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w407 = fvixxx<T>(w302, w15, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w408 = fvixxx<T>(w306, w7, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w409 = fvixxx<T>(w307, w7, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w410 = fvixxx<T>(w308, w7, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w411 = fvixxx<T>(w312, w6, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w412 = fvixxx<T>(w313, w6, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w413 = fvixxx<T>(w314, w6, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w414 = fvixxx<T>(w315, w6, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w415 = fvixxx<T>(w316, w6, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w416 = fvixxx<T>(w322, w4, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w417 = fvixxx<T>(w323, w4, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w418 = fvixxx<T>(w324, w4, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w419 = fvixxx<T>(w325, w4, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const wf<T> w420 = fvixxx<T>(w326, w4, g0_0, g0_1, Qs0_2_3_4_6, T(pe0.m), d0_2_3_4_6_0);
  const cx<T> amp320 = iovxxx<T>(w386, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp320);
  J[27] = J[27] + (T(0.5) * amp320);
  J[31] = J[31] + (T(0.5) * amp320);
  J[35] = J[35] + (T(-0.5) * amp320);
  const cx<T> amp321 = iovxxx<T>(w387, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp321);
  J[29] = J[29] + (T(0.5) * amp321);
  J[33] = J[33] + (T(0.5) * amp321);
  J[35] = J[35] + (T(-0.5) * amp321);
  const cx<T> amp322 = iovxxx<T>(w388, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(0.5) * amp322);
  J[33] = J[33] + (T(-0.5) * amp322);
  const cx<T> amp323 = iovxxx<T>(w389, w1, w5, g0_0, g0_1);
  J[29] = J[29] + (T(0.5) * amp323);
  J[35] = J[35] + (T(-0.5) * amp323);
  const cx<T> amp324 = iovxxx<T>(w390, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(-0.5) * amp324);
  J[29] = J[29] + (T(0.5) * amp324);
  J[31] = J[31] + (T(-0.5) * amp324);
  J[33] = J[33] + (T(0.5) * amp324);
  const cx<T> amp325 = iovxxx<T>(w391, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(0.5) * amp325);
  J[29] = J[29] + (T(-0.5) * amp325);
  const cx<T> amp326 = iovxxx<T>(w392, w1, w5, g0_0, g0_1);
  J[31] = J[31] + (T(-0.5) * amp326);
  J[33] = J[33] + (T(0.5) * amp326);
  const cx<T> amp327 = iovxxx<T>(w393, w1, w5, g0_0, g0_1);
  J[24] = J[24] + (T(-0.16666666666666666) * amp327);
  J[25] = J[25] + (T(0.16666666666666666) * amp327);
  J[26] = J[26] + (T(0.5) * amp327);
  J[27] = J[27] + (T(-0.5) * amp327);
  const cx<T> amp328 = iovxxx<T>(w394, w1, w5, g0_0, g0_1);
  J[24] = J[24] + (T(0.16666666666666666) * amp328);
  J[26] = J[26] + (T(-0.5) * amp328);
  const cx<T> amp329 = iovxxx<T>(w395, w1, w5, g0_0, g0_1);
  J[25] = J[25] + (T(0.16666666666666666) * amp329);
  J[27] = J[27] + (T(-0.5) * amp329);
  const cx<T> amp330 = iovxxx<T>(w396, w1, w5, g0_0, g0_1);
  J[25] = J[25] + (T(0.16666666666666666) * amp330);
  J[29] = J[29] + (T(-0.5) * amp330);
  const cx<T> amp331 = iovxxx<T>(w397, w1, w5, g0_0, g0_1);
  J[24] = J[24] + (T(0.16666666666666666) * amp331);
  J[33] = J[33] + (T(-0.5) * amp331);
  const cx<T> amp332 = iovxxx<T>(w398, w1, w5, g0_0, g0_1);
  J[24] = J[24] + (T(-0.16666666666666666) * amp332);
  J[25] = J[25] + (T(0.16666666666666666) * amp332);
  J[31] = J[31] + (T(0.5) * amp332);
  J[35] = J[35] + (T(-0.5) * amp332);
  const cx<T> amp333 = iovxxx<T>(w399, w1, w5, g0_0, g0_1);
  J[25] = J[25] + (T(0.16666666666666666) * amp333);
  J[35] = J[35] + (T(-0.5) * amp333);
  const cx<T> amp334 = iovxxx<T>(w400, w1, w5, g0_0, g0_1);
  J[24] = J[24] + (T(0.16666666666666666) * amp334);
  J[31] = J[31] + (T(-0.5) * amp334);
  const cx<T> amp335 = iovxxx<T>(w401, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(0.5) * amp335);
  J[33] = J[33] + (T(-0.5) * amp335);
  const cx<T> amp336 = iovxxx<T>(w402, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(-0.5) * amp336);
  J[28] = J[28] + (T(0.16666666666666666) * amp336);
  const cx<T> amp337 = iovxxx<T>(w403, w1, w5, g0_0, g0_1);
  J[28] = J[28] + (T(0.16666666666666666) * amp337);
  J[33] = J[33] + (T(-0.5) * amp337);
  const cx<T> amp338 = iovxxx<T>(w404, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(0.5) * amp338);
  J[29] = J[29] + (T(-0.5) * amp338);
  const cx<T> amp339 = iovxxx<T>(w405, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp339);
  J[32] = J[32] + (T(0.16666666666666666) * amp339);
  const cx<T> amp340 = iovxxx<T>(w406, w1, w5, g0_0, g0_1);
  J[29] = J[29] + (T(-0.5) * amp340);
  J[32] = J[32] + (T(0.16666666666666666) * amp340);
  const cx<T> amp341 = iovxxx<T>(w407, w1, w5, g0_0, g0_1);
  J[30] = J[30] + (T(-0.16666666666666666) * amp341);
  J[31] = J[31] + (T(0.5) * amp341);
  J[34] = J[34] + (T(0.16666666666666666) * amp341);
  J[35] = J[35] + (T(-0.5) * amp341);
  const cx<T> amp342 = iovxxx<T>(w408, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(0.5) * amp342);
  J[27] = J[27] + (T(-0.5) * amp342);
  J[30] = J[30] + (T(-0.16666666666666666) * amp342);
  J[34] = J[34] + (T(0.16666666666666666) * amp342);
  const cx<T> amp343 = iovxxx<T>(w409, w1, w5, g0_0, g0_1);
  J[27] = J[27] + (T(-0.5) * amp343);
  J[34] = J[34] + (T(0.16666666666666666) * amp343);
  const cx<T> amp344 = iovxxx<T>(w410, w1, w5, g0_0, g0_1);
  J[26] = J[26] + (T(-0.5) * amp344);
  J[30] = J[30] + (T(0.16666666666666666) * amp344);
  const cx<T> amp345 = iovxxx<T>(w411, w1, w5, g0_0, g0_1);
  J[33] = J[33] + (T(0.5) * amp345);
  J[35] = J[35] + (T(-0.5) * amp345);
  const cx<T> amp346 = iovxxx<T>(w412, w1, w5, g0_0, g0_1);
  J[32] = J[32] + (T(0.16666666666666666) * amp346);
  J[33] = J[33] + (T(-0.5) * amp346);
  const cx<T> amp347 = iovxxx<T>(w413, w1, w5, g0_0, g0_1);
  J[32] = J[32] + (T(0.16666666666666666) * amp347);
  J[35] = J[35] + (T(-0.5) * amp347);
  const cx<T> amp348 = iovxxx<T>(w414, w1, w5, g0_0, g0_1);
  J[33] = J[33] + (T(-0.5) * amp348);
  J[34] = J[34] + (T(0.16666666666666666) * amp348);
  const cx<T> amp349 = iovxxx<T>(w415, w1, w5, g0_0, g0_1);
  J[34] = J[34] + (T(0.16666666666666666) * amp349);
  J[35] = J[35] + (T(-0.5) * amp349);
  const cx<T> amp350 = iovxxx<T>(w416, w1, w5, g0_0, g0_1);
  J[29] = J[29] + (T(0.5) * amp350);
  J[31] = J[31] + (T(-0.5) * amp350);
  const cx<T> amp351 = iovxxx<T>(w417, w1, w5, g0_0, g0_1);
  J[28] = J[28] + (T(0.16666666666666666) * amp351);
  J[29] = J[29] + (T(-0.5) * amp351);
  const cx<T> amp352 = iovxxx<T>(w418, w1, w5, g0_0, g0_1);
  J[28] = J[28] + (T(0.16666666666666666) * amp352);
  J[31] = J[31] + (T(-0.5) * amp352);
  const cx<T> amp353 = iovxxx<T>(w419, w1, w5, g0_0, g0_1);
  J[29] = J[29] + (T(-0.5) * amp353);
  J[30] = J[30] + (T(0.16666666666666666) * amp353);
  const cx<T> amp354 = iovxxx<T>(w420, w1, w5, g0_0, g0_1);
  J[30] = J[30] + (T(0.16666666666666666) * amp354);
  J[31] = J[31] + (T(-0.5) * amp354);
  const mom qs0_2_3_5_6 = pr0 + (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs0_2_3_5_6 = tv<T>(qs0_2_3_5_6);
  const cx<T> d0_2_3_5_6_0 = cvt<T>(inv_denominator(qs0_2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w421 = fvixxx<T>(w0, w167, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w422 = fvixxx<T>(w0, w168, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w423 = fvixxx<T>(w0, w169, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w424 = fvixxx<T>(w0, w170, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w425 = fvixxx<T>(w0, w171, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const cx<T> amp355 = iovxxx<T>(w421, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp355);
  J[15] = J[15] + (T(0.5) * amp355);
  J[19] = J[19] + (T(0.5) * amp355);
  J[23] = J[23] + (T(-0.5) * amp355);
  const cx<T> amp356 = iovxxx<T>(w422, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp356);
  J[17] = J[17] + (T(-0.5) * amp356);
  J[21] = J[21] + (T(-0.5) * amp356);
  J[23] = J[23] + (T(0.5) * amp356);
  const cx<T> amp357 = iovxxx<T>(w423, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp357);
  J[17] = J[17] + (T(0.5) * amp357);
  J[19] = J[19] + (T(-0.5) * amp357);
  J[21] = J[21] + (T(0.5) * amp357);
  const cx<T> amp358 = iovxxx<T>(w424, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp358);
  J[15] = J[15] + (T(0.5) * amp358);
  J[19] = J[19] + (T(0.5) * amp358);
  J[23] = J[23] + (T(-0.5) * amp358);
  const cx<T> amp359 = iovxxx<T>(w425, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp359);
  J[17] = J[17] + (T(0.5) * amp359);
  J[21] = J[21] + (T(0.5) * amp359);
  J[23] = J[23] + (T(-0.5) * amp359);
}

// part 9: amplitudes 360 .. 392 (113 calls)
template <class T>
__device__ __noinline__ void rows_uu_ttggg_part9(const KernelArgs& a, const int8_t* hh, cx<T>* J) {
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  const mom pr0 = pm_uu_ttggg[opaque_int(0)][threadIdx.x];
  const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
  const mom pr1 = pm_uu_ttggg[opaque_int(1)][threadIdx.x];
  const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
  const mom pr2 = pm_uu_ttggg[opaque_int(2)][threadIdx.x];
  const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
  const mom pr3 = pm_uu_ttggg[opaque_int(3)][threadIdx.x];
  const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
  const mom pr4 = pm_uu_ttggg[opaque_int(4)][threadIdx.x];
  const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
  const mom pr5 = pm_uu_ttggg[opaque_int(5)][threadIdx.x];
  const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
  const mom pr6 = pm_uu_ttggg[opaque_int(6)][threadIdx.x];
  const wf<T> w6 = vxxxxx<T>(tv<T>(pr6), T(pe0.m), hh[6], 1);
  const mom qs2_3 = (-pr2) + (-pr3);
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w7 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
  const mom qs5 = (-pr5);
  const vec<T> Qs5 = tv<T>(qs5);
  const mom qs6 = (-pr6);
  const vec<T> Qs6 = tv<T>(qs6);
  const mom qs5_6 = (-pr5) + (-pr6);
  const vec<T> Qs5_6 = tv<T>(qs5_6);
  const cx<T> d5_6_0 = cvt<T>(inv_denominator(qs5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w8 = jvvxxx<T, false>(w5, Qs5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d5_6_0);
  const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
  const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w49 = jvvxxx<T, false>(w7, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_5 = (-pr2) + (-pr5);
  const vec<T> Qs2_5 = tv<T>(qs2_5);
  const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w50 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
  const wf<T> w51 = jioxxx<T, false>(w3, w50, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs3_5 = (-pr3) + (-pr5);
  const vec<T> Qs3_5 = tv<T>(qs3_5);
  const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w52 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
  const wf<T> w53 = jioxxx<T, false>(w52, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
  const mom qs2_3_6 = (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs2_3_6 = tv<T>(qs2_3_6);
  const cx<T> d2_3_6_0 = cvt<T>(inv_denominator(qs2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w66 = jvvxxx<T, false>(w7, Qs2_3, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_6 = (-pr2) + (-pr6);
  const vec<T> Qs2_6 = tv<T>(qs2_6);
  const cx<T> d2_6_3 = cvt<T>(inv_denominator(qs2_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w67 = fvoxxx<T>(w2, w6, g0_0, g0_1, Qs2_6, T(pe3.m), d2_6_3);
  const wf<T> w68 = jioxxx<T, false>(w3, w67, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs3_6 = (-pr3) + (-pr6);
  const vec<T> Qs3_6 = tv<T>(qs3_6);
  const cx<T> d3_6_3 = cvt<T>(inv_denominator(qs3_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w69 = fvixxx<T>(w3, w6, g0_0, g0_1, Qs3_6, T(pe3.m), d3_6_3);
  const wf<T> w70 = jioxxx<T, false>(w69, w2, g0_0, g0_1, Qs2_3_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_6_0);
  const mom qs2_3_5_6 = (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs2_3_5_6 = tv<T>(qs2_3_5_6);
  const cx<T> d2_3_5_6_0 = cvt<T>(inv_denominator(qs2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w172 = jvvxxx<T, false>(w51, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w173 = jvvxxx<T, false>(w53, Qs2_3_5, w6, Qs6, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w174 = jvvxxx<T, false>(w66, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w175 = jvvxxx<T, false>(w68, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w176 = jvvxxx<T, false>(w70, Qs2_3_6, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs2_5_6 = (-pr2) + (-pr5) + (-pr6);
  const vec<T> Qs2_5_6 = tv<T>(qs2_5_6);
  const cx<T> d2_5_6_3 = cvt<T>(inv_denominator(qs2_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w177 = fvoxxx<T>(w2, w8, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w178 = fvoxxx<T>(w50, w6, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w179 = fvoxxx<T>(w67, w5, g0_0, g0_1, Qs2_5_6, T(pe3.m), d2_5_6_3);
  const wf<T> w180 = jioxxx<T, false>(w3, w177, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w181 = jioxxx<T, false>(w3, w178, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w182 = jioxxx<T, false>(w3, w179, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w183 = jioxxx<T, false>(w52, w67, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w184 = jioxxx<T, false>(w69, w50, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs3_5_6 = (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs3_5_6 = tv<T>(qs3_5_6);
  const cx<T> d3_5_6_3 = cvt<T>(inv_denominator(qs3_5_6, cx<double>{pe3.pole_r, pe3.pole_i}));
  const wf<T> w185 = fvixxx<T>(w3, w8, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w186 = fvixxx<T>(w52, w6, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w187 = fvixxx<T>(w69, w5, g0_0, g0_1, Qs3_5_6, T(pe3.m), d3_5_6_3);
  const wf<T> w188 = jioxxx<T, false>(w185, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w189 = jioxxx<T, false>(w186, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const wf<T> w190 = jioxxx<T, false>(w187, w2, g0_0, g0_1, Qs2_3_5_6, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_6_0);
  const mom qs0_5 = pr0 + (-pr5);
  const vec<T> Qs0_5 = tv<T>(qs0_5);
  const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w300 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
  const mom qs0_6 = pr0 + (-pr6);
  const vec<T> Qs0_6 = tv<T>(qs0_6);
  const cx<T> d0_6_0 = cvt<T>(inv_denominator(qs0_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w301 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_6, T(pe0.m), d0_6_0);
  const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w302 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
  const mom qs0_5_6 = pr0 + (-pr5) + (-pr6);
  const vec<T> Qs0_5_6 = tv<T>(qs0_5_6);
  const cx<T> d0_5_6_0 = cvt<T>(inv_denominator(qs0_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w309 = fvixxx<T>(w0, w8, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const wf<T> w310 = fvixxx<T>(w300, w6, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const wf<T> w311 = fvixxx<T>(w301, w5, g0_0, g0_1, Qs0_5_6, T(pe0.m), d0_5_6_0);
  const mom qs0_2_3_5 = pr0 + (-pr2) + (-pr3) + (-pr5);
  const vec<T> Qs0_2_3_5 = tv<T>(qs0_2_3_5);
  const cx<T> d0_2_3_5_0 = cvt<T>(inv_denominator(qs0_2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w317 = fvixxx<T>(w0, w49, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w318 = fvixxx<T>(w0, w51, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w319 = fvixxx<T>(w0, w53, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w320 = fvixxx<T>(w300, w7, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const wf<T> w321 = fvixxx<T>(w302, w5, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
  const mom qs0_2_3_6 = pr0 + (-pr2) + (-pr3) + (-pr6);
  const vec<T> Qs0_2_3_6 = tv<T>(qs0_2_3_6);
  const cx<T> d0_2_3_6_0 = cvt<T>(inv_denominator(qs0_2_3_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w322 = fvixxx<T>(w0, w66, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w323 = fvixxx<T>(w0, w68, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w324 = fvixxx<T>(w0, w70, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w325 = fvixxx<T>(w301, w7, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const wf<T> w326 = fvixxx<T>(w302, w6, g0_0, g0_1, Qs0_2_3_6, T(pe0.m), d0_2_3_6_0);
  const mom qs0_2_3_5_6 = pr0 + (-pr2) + (-pr3) + (-pr5) + (-pr6);
  const vec<T> Qs0_2_3_5_6 = tv<T>(qs0_2_3_5_6);
  const cx<T> d0_2_3_5_6_0 = cvt<T>(inv_denominator(qs0_2_3_5_6, cx<double>{pe0.pole_r, pe0.pole_i}));
  const wf<T> w426 = fvixxx<T>(w0, w172, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w427 = fvixxx<T>(w0, w173, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w428 = fvixxx<T>(w0, w174, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w429 = fvixxx<T>(w0, w175, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w430 = fvixxx<T>(w0, w176, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w431 = fvixxx<T>(w0, w180, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w432 = fvixxx<T>(w0, w181, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w433 = fvixxx<T>(w0, w182, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w434 = fvixxx<T>(w0, w183, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w435 = fvixxx<T>(w0, w184, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w436 = fvixxx<T>(w0, w188, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w437 = fvixxx<T>(w0, w189, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w438 = fvixxx<T>(w0, w190, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w439 = fvixxx<T>(w300, w66, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w440 = fvixxx<T>(w300, w68, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w441 = fvixxx<T>(w300, w70, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w442 = fvixxx<T>(w301, w49, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w443 = fvixxx<T>(w301, w51, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w444 = fvixxx<T>(w301, w53, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w445 = fvixxx<T>(w302, w8, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w446 = fvixxx<T>(w309, w7, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w447 = fvixxx<T>(w310, w7, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w448 = fvixxx<T>(w311, w7, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w449 = fvixxx<T>(w317, w6, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w450 = fvixxx<T>(w318, w6, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w451 = fvixxx<T>(w319, w6, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w452 = fvixxx<T>(w320, w6, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w453 = fvixxx<T>(w321, w6, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w454 = fvixxx<T>(w322, w5, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w455 = fvixxx<T>(w323, w5, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w456 = fvixxx<T>(w324, w5, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w457 = fvixxx<T>(w325, w5, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const wf<T> w458 = fvixxx<T>(w326, w5, g0_0, g0_1, Qs0_2_3_5_6, T(pe0.m), d0_2_3_5_6_0);
  const mom qs4 = (-pr4);
  const vec<T> Qs4 = tv<T>(qs4);
  const cx<T> amp360 = iovxxx<T>(w426, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp360);
  J[21] = J[21] + (T(-0.5) * amp360);
  const cx<T> amp361 = iovxxx<T>(w427, w1, w4, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp361);
  J[23] = J[23] + (T(-0.5) * amp361);
  const cx<T> amp362 = iovxxx<T>(w428, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp362);
  J[17] = J[17] + (T(0.5) * amp362);
  J[19] = J[19] + (T(-0.5) * amp362);
  J[21] = J[21] + (T(0.5) * amp362);
  const cx<T> amp363 = iovxxx<T>(w429, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(0.5) * amp363);
  J[17] = J[17] + (T(-0.5) * amp363);
  const cx<T> amp364 = iovxxx<T>(w430, w1, w4, g0_0, g0_1);
  J[19] = J[19] + (T(-0.5) * amp364);
  J[21] = J[21] + (T(0.5) * amp364);
  const cx<T> amp365 = iovxxx<T>(w431, w1, w4, g0_0, g0_1);
  J[12] = J[12] + (T(-0.16666666666666666) * amp365);
  J[13] = J[13] + (T(0.16666666666666666) * amp365);
  J[14] = J[14] + (T(0.5) * amp365);
  J[15] = J[15] + (T(-0.5) * amp365);
  const cx<T> amp366 = iovxxx<T>(w432, w1, w4, g0_0, g0_1);
  J[12] = J[12] + (T(0.16666666666666666) * amp366);
  J[14] = J[14] + (T(-0.5) * amp366);
  const cx<T> amp367 = iovxxx<T>(w433, w1, w4, g0_0, g0_1);
  J[13] = J[13] + (T(0.16666666666666666) * amp367);
  J[15] = J[15] + (T(-0.5) * amp367);
  const cx<T> amp368 = iovxxx<T>(w434, w1, w4, g0_0, g0_1);
  J[13] = J[13] + (T(0.16666666666666666) * amp368);
  J[17] = J[17] + (T(-0.5) * amp368);
  const cx<T> amp369 = iovxxx<T>(w435, w1, w4, g0_0, g0_1);
  J[12] = J[12] + (T(0.16666666666666666) * amp369);
  J[21] = J[21] + (T(-0.5) * amp369);
  const cx<T> amp370 = iovxxx<T>(w436, w1, w4, g0_0, g0_1);
  J[12] = J[12] + (T(-0.16666666666666666) * amp370);
  J[13] = J[13] + (T(0.16666666666666666) * amp370);
  J[19] = J[19] + (T(0.5) * amp370);
  J[23] = J[23] + (T(-0.5) * amp370);
  const cx<T> amp371 = iovxxx<T>(w437, w1, w4, g0_0, g0_1);
  J[13] = J[13] + (T(0.16666666666666666) * amp371);
  J[23] = J[23] + (T(-0.5) * amp371);
  const cx<T> amp372 = iovxxx<T>(w438, w1, w4, g0_0, g0_1);
  J[12] = J[12] + (T(0.16666666666666666) * amp372);
  J[19] = J[19] + (T(-0.5) * amp372);
  const cx<T> amp373 = iovxxx<T>(w439, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(0.5) * amp373);
  J[21] = J[21] + (T(-0.5) * amp373);
  const cx<T> amp374 = iovxxx<T>(w440, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp374);
  J[16] = J[16] + (T(0.16666666666666666) * amp374);
  const cx<T> amp375 = iovxxx<T>(w441, w1, w4, g0_0, g0_1);
  J[16] = J[16] + (T(0.16666666666666666) * amp375);
  J[21] = J[21] + (T(-0.5) * amp375);
  const cx<T> amp376 = iovxxx<T>(w442, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp376);
  J[17] = J[17] + (T(-0.5) * amp376);
  const cx<T> amp377 = iovxxx<T>(w443, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp377);
  J[20] = J[20] + (T(0.16666666666666666) * amp377);
  const cx<T> amp378 = iovxxx<T>(w444, w1, w4, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp378);
  J[20] = J[20] + (T(0.16666666666666666) * amp378);
  const cx<T> amp379 = iovxxx<T>(w445, w1, w4, g0_0, g0_1);
  J[18] = J[18] + (T(-0.16666666666666666) * amp379);
  J[19] = J[19] + (T(0.5) * amp379);
  J[22] = J[22] + (T(0.16666666666666666) * amp379);
  J[23] = J[23] + (T(-0.5) * amp379);
  const cx<T> amp380 = iovxxx<T>(w446, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(0.5) * amp380);
  J[15] = J[15] + (T(-0.5) * amp380);
  J[18] = J[18] + (T(-0.16666666666666666) * amp380);
  J[22] = J[22] + (T(0.16666666666666666) * amp380);
  const cx<T> amp381 = iovxxx<T>(w447, w1, w4, g0_0, g0_1);
  J[15] = J[15] + (T(-0.5) * amp381);
  J[22] = J[22] + (T(0.16666666666666666) * amp381);
  const cx<T> amp382 = iovxxx<T>(w448, w1, w4, g0_0, g0_1);
  J[14] = J[14] + (T(-0.5) * amp382);
  J[18] = J[18] + (T(0.16666666666666666) * amp382);
  const cx<T> amp383 = iovxxx<T>(w449, w1, w4, g0_0, g0_1);
  J[21] = J[21] + (T(0.5) * amp383);
  J[23] = J[23] + (T(-0.5) * amp383);
  const cx<T> amp384 = iovxxx<T>(w450, w1, w4, g0_0, g0_1);
  J[20] = J[20] + (T(0.16666666666666666) * amp384);
  J[21] = J[21] + (T(-0.5) * amp384);
  const cx<T> amp385 = iovxxx<T>(w451, w1, w4, g0_0, g0_1);
  J[20] = J[20] + (T(0.16666666666666666) * amp385);
  J[23] = J[23] + (T(-0.5) * amp385);
  const cx<T> amp386 = iovxxx<T>(w452, w1, w4, g0_0, g0_1);
  J[21] = J[21] + (T(-0.5) * amp386);
  J[22] = J[22] + (T(0.16666666666666666) * amp386);
  const cx<T> amp387 = iovxxx<T>(w453, w1, w4, g0_0, g0_1);
  J[22] = J[22] + (T(0.16666666666666666) * amp387);
  J[23] = J[23] + (T(-0.5) * amp387);
  const cx<T> amp388 = iovxxx<T>(w454, w1, w4, g0_0, g0_1);
  J[17] = J[17] + (T(0.5) * amp388);
  J[19] = J[19] + (T(-0.5) * amp388);
  const cx<T> amp389 = iovxxx<T>(w455, w1, w4, g0_0, g0_1);
  J[16] = J[16] + (T(0.16666666666666666) * amp389);
  J[17] = J[17] + (T(-0.5) * amp389);
  const cx<T> amp390 = iovxxx<T>(w456, w1, w4, g0_0, g0_1);
  J[16] = J[16] + (T(0.16666666666666666) * amp390);
  J[19] = J[19] + (T(-0.5) * amp390);
  const cx<T> amp391 = iovxxx<T>(w457, w1, w4, g0_0, g0_1);
  J[17] = J[17] + (T(-0.5) * amp391);
  J[18] = J[18] + (T(0.16666666666666666) * amp391);
  const cx<T> amp392 = iovxxx<T>(w458, w1, w4, g0_0, g0_1);
  J[18] = J[18] + (T(0.16666666666666666) * amp392);
  J[19] = J[19] + (T(-0.5) * amp392);
}

template <class T>
__device__ __forceinline__ void body_uu_ttggg(const KernelArgs& a, int64_t blk) {
  const int64_t i = blk * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  mom p[7];
  double psw = 1.0;   // phase-space weight of a generated event (resonance tree)
  if (active) {
    if (a.mom_in) {
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const double* b = a.mom_in + int64_t(k) * 4 * a.mom_stride + i;
        p[k] = {b[0], b[a.mom_stride], b[2 * a.mom_stride], b[3 * a.mom_stride]};
      }
    } else {
      const double h = 0.5 * a.sqrt_s;
      p[0] = {h, 0.0, 0.0, h};
      p[1] = {h, 0.0, 0.0, -h};
      psw = ps_tree_uu_ttggg(a, a.counter_offset + uint64_t(i), i, p);
    }
    if (a.mom_out) store_momenta<7>(a, i, p);
  } else {
#pragma unroll
    for (int k = 0; k < 7; ++k) p[k] = {1.0, 0.0, 0.0, 1.0};
  }
  const bool pass = active && psw > 0.0 && (!a.cut_enabled || pass_pt_dr<5>(p + 2, a.cut_pt, a.cut_dr));
  // couplings and propagator data (uniform)
  const cx<T> g0_0 = mk<T>(T(a.cpl[0]), T(a.cpl[1]));
  const cx<T> g0_1 = mk<T>(T(a.cpl[2]), T(a.cpl[3]));
  const cx<T> g1_0 = mk<T>(T(a.cpl[4]), T(a.cpl[5]));
  const cx<T> g1_1 = mk<T>(T(a.cpl[6]), T(a.cpl[7]));
  const cx<T> g2_0 = mk<T>(T(a.cpl[8]), T(a.cpl[9]));
  const cx<T> g2_1 = mk<T>(T(a.cpl[10]), T(a.cpl[11]));
  const PropEntry pe0 = a.prop[0];
  const PropEntry pe3 = a.prop[3];
  // momenta flowing into the diagram: +p incoming, -p outgoing (FP64)
  const mom q0 = p[0];
  const mom q1 = p[1];
  const mom q2 = -p[2];
  const mom q3 = -p[3];
  const mom q4 = -p[4];
  const mom q5 = -p[5];
  const mom q6 = -p[6];
  pm_uu_ttggg[0][threadIdx.x] = p[0];
  pm_uu_ttggg[1][threadIdx.x] = p[1];
  pm_uu_ttggg[2][threadIdx.x] = p[2];
  pm_uu_ttggg[3][threadIdx.x] = p[3];
  pm_uu_ttggg[4][threadIdx.x] = p[4];
  pm_uu_ttggg[5][threadIdx.x] = p[5];
  pm_uu_ttggg[6][threadIdx.x] = p[6];
  double me2 = 0.0;
  if (pass) {
    for (int h = 0; h < a.n_hel; ++h) {
      const int8_t* hh = a.hel + h * 7;
      cx<T> J[48];
      for (int f = 0; f < 48; ++f) J[f] = mk<T>(T(0), T(0));
      rows_uu_ttggg_part0<T>(a, hh, J);
      rows_uu_ttggg_part1<T>(a, hh, J);
      rows_uu_ttggg_part2<T>(a, hh, J);
      rows_uu_ttggg_part3<T>(a, hh, J);
      rows_uu_ttggg_part4<T>(a, hh, J);
      rows_uu_ttggg_part5<T>(a, hh, J);
      rows_uu_ttggg_part6<T>(a, hh, J);
      rows_uu_ttggg_part7<T>(a, hh, J);
      rows_uu_ttggg_part8<T>(a, hh, J);
      rows_uu_ttggg_part9<T>(a, hh, J);
      T cs = T(0);
      {
        const cx<T> jf = J[0];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[1]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[2]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[3]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[4]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[5]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[6]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[1];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[2]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[3]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[4]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[5]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[6]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[2];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[3]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[4]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[5]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[6]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[3];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[4]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[5]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[6]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[4];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[5]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[6]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[5];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[6]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[7]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[6];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[7]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[8]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[12]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[7];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[8]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[9]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[12]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[8];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[9]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[10]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[12]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[9];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[10]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[11]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[12]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[10];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[11]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[12]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[11];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[12]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[13]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[12];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[13]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[14]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[13];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[14]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[15]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[17]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[14];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[15]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[16]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[15];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[16]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[18]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[16];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[17]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[19]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[17];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[18]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[20]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[18];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[19]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[21]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[19];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[20]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[22]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[20];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[21]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[23]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[21];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[22]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[22];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[23]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[24]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[23];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[24]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[25]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[24];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[25]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[26]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[25];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[26]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[27]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[29]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[26];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[27]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[28]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[27];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[28]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[30]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[28];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[29]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[31]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[29];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[30]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[32]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(42.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[30];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[31]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[33]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[31];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[32]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[34]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(20.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(60.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[32];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[33]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[35]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[33];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[34]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[34];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[35]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[36]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[35];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[36]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[37]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(2.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(6.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[36];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[37]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[38]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[37];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[38]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[39]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[41]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[38];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[39]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[40]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[39];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[40]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[42]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[40];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[41]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[43]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[41];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[42]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[44]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[42];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[43]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[45]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[43];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[44]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[46]; r += T(-16.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(-48.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[44];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[45]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J[47]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[45];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[46]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[46];
        T r = T(192.0) * norm2(jf);
        { const cx<T> jg = J[47]; r += T(128.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J[47];
        T r = T(192.0) * norm2(jf);
        cs += r;
      }
      me2 += double(cs) * 0.1111111111111111;
    }
  }
  if (a.me2_out && active) a.me2_out[i] = me2;
  if (a.w_out && active) a.w_out[i] = pass ? me2 * a.weight_factor * psw : 0.0;
  if (a.partials) block_partials(a, blk, pass ? me2 * a.weight_factor * psw : 0.0, pass);
}

// one launch: the grid walks the 256-event blocks of the launch (persistent
// kernels: one workspace slot per block), or, for a fused launch of the
// serving engine, the virtual blocks of its batch table
template <class T>
__global__ __launch_bounds__(256) void amp_uu_ttggg(KernelArgs a) {
  const BatchTable* bt = a.batch;
  const int64_t total = bt ? bt->total_blocks : (a.n + 255) / 256;
  const int nseg = bt ? bt->n_seg : 0;
  int s = 0;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    KernelArgs b = a;
    int64_t blk = vb;
    if (bt) {
      while (s + 1 < nseg && bt->seg[s + 1].block_begin <= vb) ++s;
      b = segment_args(a, bt->seg[s]);
      blk = bt->seg[s].block_offset + (vb - bt->seg[s].block_begin);
    }
    body_uu_ttggg<T>(b, blk);
    __syncthreads();
  }
}

// the phase-space step alone (heget_generate): momenta and per-event weights
__global__ __launch_bounds__(256) void gen_uu_ttggg(KernelArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  mom p[7];
  const double w = ps_tree_uu_ttggg(a, a.counter_offset + uint64_t(i), i, p);
  store_momenta<7>(a, i, p);
  if (a.psw_out) a.psw_out[i] = w;
}

}  // namespace

static const GenEntry entry = {0x8e3e43d03eccb7b8ull, "uu_ttggg", 7, reinterpret_cast<const void*>(&amp_uu_ttggg<double>), reinterpret_cast<const void*>(&amp_uu_ttggg<float>), 0, 0, 0, reinterpret_cast<const void*>(&amp_uu_ttggg<double>), reinterpret_cast<const void*>(&amp_uu_ttggg<float>), nullptr, 0, 0, 0, reinterpret_cast<const void*>(&gen_uu_ttggg), 11, 0, nullptr, nullptr, nullptr, nullptr};
static const Registrar reg(&entry);

}  // namespace heget
