// Generated from the process IR 'uu_ttgg' (fingerprint 0xc9d0b9164f81fce4); do not edit.
#include "../generated_common.hpp"

namespace heget {
namespace {

// phase space: the collision and its resonances decay in two bodies (tree of 3 nodes);
// fills p[0 .. n_legs-1] and returns the event's weight dPhi_n
__device__ __forceinline__ double ps_tree_uu_ttgg(const KernelArgs& a, uint64_t event, int64_t i, mom* p) {
#pragma clang fp contract(off)   // each product and sum rounds on its own (plain IEEE)
  double u[8];
  ps_uniforms<8>(a.seed, event, u);
  const double h = 0.5 * a.sqrt_s;
  p[0] = {h, 0.0, 0.0, h};
  p[1] = {h, 0.0, 0.0, -h};
  // adaptive integration: the uniforms through the grid, its Jacobian in the weight
  double w = a.grid ? grid_map<8>(a, i, u) : 1.0;
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
  w *= ps_decay(u[6], u[7], P2, M2, 0.0, 0.0, false, p[4], p[5]);
  return w;
}

// the event's physical momenta, one column per lane, read by every part
__shared__ mom pm_uu_ttgg[6][256];

template <class T>
__device__ __forceinline__ void body_uu_ttgg(const KernelArgs& a, int64_t blk) {
  const int64_t i = blk * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  mom p[6];
  double psw = 1.0;   // phase-space weight of a generated event (resonance tree)
  if (active) {
    if (a.mom_in) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double* b = a.mom_in + int64_t(k) * 4 * a.mom_stride + i;
        p[k] = {b[0], b[a.mom_stride], b[2 * a.mom_stride], b[3 * a.mom_stride]};
      }
    } else {
      const double h = 0.5 * a.sqrt_s;
      p[0] = {h, 0.0, 0.0, h};
      p[1] = {h, 0.0, 0.0, -h};
      psw = ps_tree_uu_ttgg(a, a.counter_offset + uint64_t(i), i, p);
    }
    if (a.mom_out) store_momenta<6>(a, i, p);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = {1.0, 0.0, 0.0, 1.0};
  }
  const bool pass = active && psw > 0.0 && (!a.cut_enabled || pass_pt_dr<4>(p + 2, a.cut_pt, a.cut_dr));
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
  pm_uu_ttgg[0][threadIdx.x] = p[0];
  pm_uu_ttgg[1][threadIdx.x] = p[1];
  pm_uu_ttgg[2][threadIdx.x] = p[2];
  pm_uu_ttgg[3][threadIdx.x] = p[3];
  pm_uu_ttgg[4][threadIdx.x] = p[4];
  pm_uu_ttgg[5][threadIdx.x] = p[5];
  double me2 = 0.0;
  if (pass) {
    for (int h = 0; h < a.n_hel; ++h) {
      const int8_t* hh = a.hel + h * 6;
      cx<T> J0 = mk<T>(T(0), T(0)), J1 = mk<T>(T(0), T(0)), J2 = mk<T>(T(0), T(0)), J3 = mk<T>(T(0), T(0)), J4 = mk<T>(T(0), T(0)), J5 = mk<T>(T(0), T(0)), J6 = mk<T>(T(0), T(0)), J7 = mk<T>(T(0), T(0)), J8 = mk<T>(T(0), T(0)), J9 = mk<T>(T(0), T(0)), J10 = mk<T>(T(0), T(0)), J11 = mk<T>(T(0), T(0));
      const mom pr0 = pm_uu_ttgg[opaque_int(0)][threadIdx.x];
      const wf<T> w0 = cvtw<T>(ixxxxx<double, true>(tv<double>(pr0), pe0.m, hh[0], 1));
      const mom pr1 = pm_uu_ttgg[opaque_int(1)][threadIdx.x];
      const wf<T> w1 = cvtw<T>(oxxxxx<double, true>(tv<double>(pr1), pe0.m, hh[1], -1));
      const mom pr2 = pm_uu_ttgg[opaque_int(2)][threadIdx.x];
      const wf<T> w2 = cvtw<T>(oxxxxx<double, false>(tv<double>(pr2), pe3.m, hh[2], 1));
      const mom pr3 = pm_uu_ttgg[opaque_int(3)][threadIdx.x];
      const wf<T> w3 = cvtw<T>(ixxxxx<double, false>(tv<double>(pr3), pe3.m, hh[3], -1));
      const mom pr4 = pm_uu_ttgg[opaque_int(4)][threadIdx.x];
      const wf<T> w4 = vxxxxx<T>(tv<T>(pr4), T(pe0.m), hh[4], 1);
      const mom pr5 = pm_uu_ttgg[opaque_int(5)][threadIdx.x];
      const wf<T> w5 = vxxxxx<T>(tv<T>(pr5), T(pe0.m), hh[5], 1);
      const mom qs2_3 = (-pr2) + (-pr3);
      const vec<T> Qs2_3 = tv<T>(qs2_3);
      const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w6 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
      const mom qs4 = (-pr4);
      const vec<T> Qs4 = tv<T>(qs4);
      const mom qs5 = (-pr5);
      const vec<T> Qs5 = tv<T>(qs5);
      const mom qs4_5 = (-pr4) + (-pr5);
      const vec<T> Qs4_5 = tv<T>(qs4_5);
      const cx<T> d4_5_0 = cvt<T>(inv_denominator(qs4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w7 = jvvxxx<T, false>(w4, Qs4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d4_5_0);
      const mom qs2_3_4_5 = (-pr2) + (-pr3) + (-pr4) + (-pr5);
      const vec<T> Qs2_3_4_5 = tv<T>(qs2_3_4_5);
      const cx<T> d2_3_4_5_0 = cvt<T>(inv_denominator(qs2_3_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w8 = jvvxxx<T, false>(w6, Qs2_3, w7, Qs4_5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w9 = jgggxx<T, false>(w6, w4, w5, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w10 = jgggxx<T, false>(w5, w6, w4, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w11 = jgggxx<T, false>(w4, w5, w6, g2_0.r, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const mom qs2_3_4 = (-pr2) + (-pr3) + (-pr4);
      const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
      const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w12 = jvvxxx<T, false>(w6, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const mom qs2_4 = (-pr2) + (-pr4);
      const vec<T> Qs2_4 = tv<T>(qs2_4);
      const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w13 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
      const wf<T> w14 = jioxxx<T, false>(w3, w13, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const mom qs3_4 = (-pr3) + (-pr4);
      const vec<T> Qs3_4 = tv<T>(qs3_4);
      const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w15 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
      const wf<T> w16 = jioxxx<T, false>(w15, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const wf<T> w17 = jvvxxx<T, false>(w12, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w18 = jvvxxx<T, false>(w14, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w19 = jvvxxx<T, false>(w16, Qs2_3_4, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const mom qs2_3_5 = (-pr2) + (-pr3) + (-pr5);
      const vec<T> Qs2_3_5 = tv<T>(qs2_3_5);
      const cx<T> d2_3_5_0 = cvt<T>(inv_denominator(qs2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w20 = jvvxxx<T, false>(w6, Qs2_3, w5, Qs5, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
      const mom qs2_5 = (-pr2) + (-pr5);
      const vec<T> Qs2_5 = tv<T>(qs2_5);
      const cx<T> d2_5_3 = cvt<T>(inv_denominator(qs2_5, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w21 = fvoxxx<T>(w2, w5, g0_0, g0_1, Qs2_5, T(pe3.m), d2_5_3);
      const wf<T> w22 = jioxxx<T, false>(w3, w21, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
      const mom qs3_5 = (-pr3) + (-pr5);
      const vec<T> Qs3_5 = tv<T>(qs3_5);
      const cx<T> d3_5_3 = cvt<T>(inv_denominator(qs3_5, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w23 = fvixxx<T>(w3, w5, g0_0, g0_1, Qs3_5, T(pe3.m), d3_5_3);
      const wf<T> w24 = jioxxx<T, false>(w23, w2, g0_0, g0_1, Qs2_3_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_5_0);
      const wf<T> w25 = jvvxxx<T, false>(w20, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w26 = jvvxxx<T, false>(w22, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w27 = jvvxxx<T, false>(w24, Qs2_3_5, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const mom qs2_4_5 = (-pr2) + (-pr4) + (-pr5);
      const vec<T> Qs2_4_5 = tv<T>(qs2_4_5);
      const cx<T> d2_4_5_3 = cvt<T>(inv_denominator(qs2_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w28 = fvoxxx<T>(w2, w7, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
      const wf<T> w29 = fvoxxx<T>(w13, w5, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
      const wf<T> w30 = fvoxxx<T>(w21, w4, g0_0, g0_1, Qs2_4_5, T(pe3.m), d2_4_5_3);
      const wf<T> w31 = jioxxx<T, false>(w3, w28, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w32 = jioxxx<T, false>(w3, w29, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w33 = jioxxx<T, false>(w3, w30, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w34 = jioxxx<T, false>(w15, w21, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w35 = jioxxx<T, false>(w23, w13, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const mom qs3_4_5 = (-pr3) + (-pr4) + (-pr5);
      const vec<T> Qs3_4_5 = tv<T>(qs3_4_5);
      const cx<T> d3_4_5_3 = cvt<T>(inv_denominator(qs3_4_5, cx<double>{pe3.pole_r, pe3.pole_i}));
      const wf<T> w36 = fvixxx<T>(w3, w7, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
      const wf<T> w37 = fvixxx<T>(w15, w5, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
      const wf<T> w38 = fvixxx<T>(w23, w4, g0_0, g0_1, Qs3_4_5, T(pe3.m), d3_4_5_3);
      const wf<T> w39 = jioxxx<T, false>(w36, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w40 = jioxxx<T, false>(w37, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const wf<T> w41 = jioxxx<T, false>(w38, w2, g0_0, g0_1, Qs2_3_4_5, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_5_0);
      const cx<T> amp0 = iovxxx<T>(w0, w1, w8, g0_0, g0_1);
      J2 = J2 + (T(0.5) * amp0);
      J3 = J3 + (T(-0.5) * amp0);
      J7 = J7 + (T(-0.5) * amp0);
      J11 = J11 + (T(0.5) * amp0);
      const cx<T> amp1 = iovxxx<T>(w0, w1, w9, g0_0, g0_1);
      J2 = J2 + (T(-0.5) * amp1);
      J5 = J5 + (T(0.5) * amp1);
      J9 = J9 + (T(0.5) * amp1);
      J11 = J11 + (T(-0.5) * amp1);
      const cx<T> amp2 = iovxxx<T>(w0, w1, w10, g0_0, g0_1);
      J3 = J3 + (T(0.5) * amp2);
      J5 = J5 + (T(-0.5) * amp2);
      J7 = J7 + (T(0.5) * amp2);
      J9 = J9 + (T(-0.5) * amp2);
      const cx<T> amp3 = iovxxx<T>(w0, w1, w11, g0_0, g0_1);
      J2 = J2 + (T(0.5) * amp3);
      J3 = J3 + (T(-0.5) * amp3);
      J7 = J7 + (T(-0.5) * amp3);
      J11 = J11 + (T(0.5) * amp3);
      const cx<T> amp4 = iovxxx<T>(w0, w1, w17, g0_0, g0_1);
      J2 = J2 + (T(0.5) * amp4);
      J5 = J5 + (T(-0.5) * amp4);
      J9 = J9 + (T(-0.5) * amp4);
      J11 = J11 + (T(0.5) * amp4);
      const cx<T> amp5 = iovxxx<T>(w0, w1, w18, g0_0, g0_1);
      J2 = J2 + (T(-0.5) * amp5);
      J9 = J9 + (T(0.5) * amp5);
      const cx<T> amp6 = iovxxx<T>(w0, w1, w19, g0_0, g0_1);
      J5 = J5 + (T(-0.5) * amp6);
      J11 = J11 + (T(0.5) * amp6);
      const cx<T> amp7 = iovxxx<T>(w0, w1, w25, g0_0, g0_1);
      J3 = J3 + (T(0.5) * amp7);
      J5 = J5 + (T(-0.5) * amp7);
      J7 = J7 + (T(0.5) * amp7);
      J9 = J9 + (T(-0.5) * amp7);
      const cx<T> amp8 = iovxxx<T>(w0, w1, w26, g0_0, g0_1);
      J3 = J3 + (T(-0.5) * amp8);
      J5 = J5 + (T(0.5) * amp8);
      const cx<T> amp9 = iovxxx<T>(w0, w1, w27, g0_0, g0_1);
      J7 = J7 + (T(0.5) * amp9);
      J9 = J9 + (T(-0.5) * amp9);
      const cx<T> amp10 = iovxxx<T>(w0, w1, w31, g0_0, g0_1);
      J0 = J0 + (T(0.16666666666666666) * amp10);
      J1 = J1 + (T(-0.16666666666666666) * amp10);
      J2 = J2 + (T(-0.5) * amp10);
      J3 = J3 + (T(0.5) * amp10);
      const cx<T> amp11 = iovxxx<T>(w0, w1, w32, g0_0, g0_1);
      J0 = J0 + (T(-0.16666666666666666) * amp11);
      J2 = J2 + (T(0.5) * amp11);
      const cx<T> amp12 = iovxxx<T>(w0, w1, w33, g0_0, g0_1);
      J1 = J1 + (T(-0.16666666666666666) * amp12);
      J3 = J3 + (T(0.5) * amp12);
      const cx<T> amp13 = iovxxx<T>(w0, w1, w34, g0_0, g0_1);
      J1 = J1 + (T(-0.16666666666666666) * amp13);
      J5 = J5 + (T(0.5) * amp13);
      const cx<T> amp14 = iovxxx<T>(w0, w1, w35, g0_0, g0_1);
      J0 = J0 + (T(-0.16666666666666666) * amp14);
      J9 = J9 + (T(0.5) * amp14);
      const cx<T> amp15 = iovxxx<T>(w0, w1, w39, g0_0, g0_1);
      J0 = J0 + (T(0.16666666666666666) * amp15);
      J1 = J1 + (T(-0.16666666666666666) * amp15);
      J7 = J7 + (T(-0.5) * amp15);
      J11 = J11 + (T(0.5) * amp15);
      const cx<T> amp16 = iovxxx<T>(w0, w1, w40, g0_0, g0_1);
      J1 = J1 + (T(-0.16666666666666666) * amp16);
      J11 = J11 + (T(0.5) * amp16);
      const cx<T> amp17 = iovxxx<T>(w0, w1, w41, g0_0, g0_1);
      J0 = J0 + (T(-0.16666666666666666) * amp17);
      J7 = J7 + (T(0.5) * amp17);
      const mom qs0_4 = pr0 + (-pr4);
      const vec<T> Qs0_4 = tv<T>(qs0_4);
      const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w42 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
      const cx<T> amp18 = iovxxx<T>(w42, w1, w20, g0_0, g0_1);
      J3 = J3 + (T(-0.5) * amp18);
      J9 = J9 + (T(0.5) * amp18);
      const cx<T> amp19 = iovxxx<T>(w42, w1, w22, g0_0, g0_1);
      J3 = J3 + (T(0.5) * amp19);
      J4 = J4 + (T(-0.16666666666666666) * amp19);
      const cx<T> amp20 = iovxxx<T>(w42, w1, w24, g0_0, g0_1);
      J4 = J4 + (T(-0.16666666666666666) * amp20);
      J9 = J9 + (T(0.5) * amp20);
      const mom qs0_5 = pr0 + (-pr5);
      const vec<T> Qs0_5 = tv<T>(qs0_5);
      const cx<T> d0_5_0 = cvt<T>(inv_denominator(qs0_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w43 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_5, T(pe0.m), d0_5_0);
      const cx<T> amp21 = iovxxx<T>(w43, w1, w12, g0_0, g0_1);
      J2 = J2 + (T(-0.5) * amp21);
      J5 = J5 + (T(0.5) * amp21);
      const cx<T> amp22 = iovxxx<T>(w43, w1, w14, g0_0, g0_1);
      J2 = J2 + (T(0.5) * amp22);
      J8 = J8 + (T(-0.16666666666666666) * amp22);
      const cx<T> amp23 = iovxxx<T>(w43, w1, w16, g0_0, g0_1);
      J5 = J5 + (T(0.5) * amp23);
      J8 = J8 + (T(-0.16666666666666666) * amp23);
      const mom qs0_2_3 = pr0 + (-pr2) + (-pr3);
      const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
      const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w44 = fvixxx<T>(w0, w6, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
      const cx<T> amp24 = iovxxx<T>(w44, w1, w7, g0_0, g0_1);
      J6 = J6 + (T(0.16666666666666666) * amp24);
      J7 = J7 + (T(-0.5) * amp24);
      J10 = J10 + (T(-0.16666666666666666) * amp24);
      J11 = J11 + (T(0.5) * amp24);
      const mom qs0_4_5 = pr0 + (-pr4) + (-pr5);
      const vec<T> Qs0_4_5 = tv<T>(qs0_4_5);
      const cx<T> d0_4_5_0 = cvt<T>(inv_denominator(qs0_4_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w45 = fvixxx<T>(w0, w7, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
      const wf<T> w46 = fvixxx<T>(w42, w5, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
      const wf<T> w47 = fvixxx<T>(w43, w4, g0_0, g0_1, Qs0_4_5, T(pe0.m), d0_4_5_0);
      const cx<T> amp25 = iovxxx<T>(w45, w1, w6, g0_0, g0_1);
      J2 = J2 + (T(-0.5) * amp25);
      J3 = J3 + (T(0.5) * amp25);
      J6 = J6 + (T(0.16666666666666666) * amp25);
      J10 = J10 + (T(-0.16666666666666666) * amp25);
      const cx<T> amp26 = iovxxx<T>(w46, w1, w6, g0_0, g0_1);
      J3 = J3 + (T(0.5) * amp26);
      J10 = J10 + (T(-0.16666666666666666) * amp26);
      const cx<T> amp27 = iovxxx<T>(w47, w1, w6, g0_0, g0_1);
      J2 = J2 + (T(0.5) * amp27);
      J6 = J6 + (T(-0.16666666666666666) * amp27);
      const mom qs0_2_3_4 = pr0 + (-pr2) + (-pr3) + (-pr4);
      const vec<T> Qs0_2_3_4 = tv<T>(qs0_2_3_4);
      const cx<T> d0_2_3_4_0 = cvt<T>(inv_denominator(qs0_2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w48 = fvixxx<T>(w0, w12, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
      const wf<T> w49 = fvixxx<T>(w0, w14, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
      const wf<T> w50 = fvixxx<T>(w0, w16, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
      const wf<T> w51 = fvixxx<T>(w42, w6, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
      const wf<T> w52 = fvixxx<T>(w44, w4, g0_0, g0_1, Qs0_2_3_4, T(pe0.m), d0_2_3_4_0);
      const cx<T> amp28 = iovxxx<T>(w48, w1, w5, g0_0, g0_1);
      J9 = J9 + (T(-0.5) * amp28);
      J11 = J11 + (T(0.5) * amp28);
      const cx<T> amp29 = iovxxx<T>(w49, w1, w5, g0_0, g0_1);
      J8 = J8 + (T(-0.16666666666666666) * amp29);
      J9 = J9 + (T(0.5) * amp29);
      const cx<T> amp30 = iovxxx<T>(w50, w1, w5, g0_0, g0_1);
      J8 = J8 + (T(-0.16666666666666666) * amp30);
      J11 = J11 + (T(0.5) * amp30);
      const cx<T> amp31 = iovxxx<T>(w51, w1, w5, g0_0, g0_1);
      J9 = J9 + (T(0.5) * amp31);
      J10 = J10 + (T(-0.16666666666666666) * amp31);
      const cx<T> amp32 = iovxxx<T>(w52, w1, w5, g0_0, g0_1);
      J10 = J10 + (T(-0.16666666666666666) * amp32);
      J11 = J11 + (T(0.5) * amp32);
      const mom qs0_2_3_5 = pr0 + (-pr2) + (-pr3) + (-pr5);
      const vec<T> Qs0_2_3_5 = tv<T>(qs0_2_3_5);
      const cx<T> d0_2_3_5_0 = cvt<T>(inv_denominator(qs0_2_3_5, cx<double>{pe0.pole_r, pe0.pole_i}));
      const wf<T> w53 = fvixxx<T>(w0, w20, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
      const wf<T> w54 = fvixxx<T>(w0, w22, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
      const wf<T> w55 = fvixxx<T>(w0, w24, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
      const wf<T> w56 = fvixxx<T>(w43, w6, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
      const wf<T> w57 = fvixxx<T>(w44, w5, g0_0, g0_1, Qs0_2_3_5, T(pe0.m), d0_2_3_5_0);
      const cx<T> amp33 = iovxxx<T>(w53, w1, w4, g0_0, g0_1);
      J5 = J5 + (T(-0.5) * amp33);
      J7 = J7 + (T(0.5) * amp33);
      const cx<T> amp34 = iovxxx<T>(w54, w1, w4, g0_0, g0_1);
      J4 = J4 + (T(-0.16666666666666666) * amp34);
      J5 = J5 + (T(0.5) * amp34);
      const cx<T> amp35 = iovxxx<T>(w55, w1, w4, g0_0, g0_1);
      J4 = J4 + (T(-0.16666666666666666) * amp35);
      J7 = J7 + (T(0.5) * amp35);
      const cx<T> amp36 = iovxxx<T>(w56, w1, w4, g0_0, g0_1);
      J5 = J5 + (T(0.5) * amp36);
      J6 = J6 + (T(-0.16666666666666666) * amp36);
      const cx<T> amp37 = iovxxx<T>(w57, w1, w4, g0_0, g0_1);
      J6 = J6 + (T(-0.16666666666666666) * amp37);
      J7 = J7 + (T(0.5) * amp37);
      T cs = T(0);
      {
        const cx<T> jf = J0;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J1; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J2; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J3; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J5; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J6; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J7; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J9; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J1;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J2; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J3; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J5; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J6; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J7; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J9; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J2;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J3; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J4; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J6; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J7; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J8; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J3;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J4; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J6; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J7; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J8; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J4;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J5; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J7; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J8; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J9; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J5;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J6; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J8; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J9; r += T(12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J6;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J7; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J9; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J7;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J8; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J10; r += T(-4.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(-12.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J8;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J9; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J11; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J9;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J10; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J10;
        T r = T(48.0) * norm2(jf);
        { const cx<T> jg = J11; r += T(32.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J11;
        T r = T(48.0) * norm2(jf);
        cs += r;
      }
      me2 += double(cs) * 0.3333333333333333;
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
__global__ __launch_bounds__(256) void amp_uu_ttgg(KernelArgs a) {
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
    body_uu_ttgg<T>(b, blk);
    __syncthreads();
  }
}

// the phase-space step alone (heget_generate): momenta and per-event weights
__global__ __launch_bounds__(256) void gen_uu_ttgg(KernelArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  mom p[6];
  const double w = ps_tree_uu_ttgg(a, a.counter_offset + uint64_t(i), i, p);
  store_momenta<6>(a, i, p);
  if (a.psw_out) a.psw_out[i] = w;
}

}  // namespace

static const GenEntry entry = {0xc9d0b9164f81fce4ull, "uu_ttgg", 6, reinterpret_cast<const void*>(&amp_uu_ttgg<double>), reinterpret_cast<const void*>(&amp_uu_ttgg<float>), 0, 0, 0, reinterpret_cast<const void*>(&amp_uu_ttgg<double>), reinterpret_cast<const void*>(&amp_uu_ttgg<float>), nullptr, 0, 0, 0, reinterpret_cast<const void*>(&gen_uu_ttgg), 8, 0, nullptr, nullptr, nullptr, nullptr};
static const Registrar reg(&entry);

}  // namespace heget
