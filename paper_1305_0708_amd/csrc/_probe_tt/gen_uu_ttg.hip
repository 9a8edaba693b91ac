// Generated from the process IR 'uu_ttg' (fingerprint 0x49875fd400262df3); do not edit.
#include "../generated_common.hpp"

namespace heget {
namespace {

// phase space: the collision and its resonances decay in two bodies (tree of 2 nodes);
// fills p[0 .. n_legs-1] and returns the event's weight dPhi_n
__device__ __forceinline__ double ps_tree_uu_ttg(const KernelArgs& a, uint64_t event, int64_t i, mom* p) {
#pragma clang fp contract(off)   // each product and sum rounds on its own (plain IEEE)
  double u[5];
  ps_uniforms<5>(a.seed, event, u);
  const double h = 0.5 * a.sqrt_s;
  p[0] = {h, 0.0, 0.0, h};
  p[1] = {h, 0.0, 0.0, -h};
  // adaptive integration: the uniforms through the grid, its Jacobian in the weight
  double w = a.grid ? grid_map<5>(a, i, u) : 1.0;
  const double M0 = a.sqrt_s;
  const mom P0 = {a.sqrt_s, 0.0, 0.0, 0.0};
  double s1;
  w *= ps_mass(u[0], (a.prop[3].m) * (a.prop[3].m), (M0 - a.prop[3].m) * (M0 - a.prop[3].m), a.prop[0].m, a.prop[0].w, false, 20.0, s1);
  const double M1 = sqrt(s1);
  mom P1;
  w *= ps_decay(u[1], u[2], P0, M0, a.prop[3].m, M1, true, p[2], P1);
  w *= ps_decay(u[3], u[4], P1, M1, a.prop[3].m, 0.0, false, p[3], p[4]);
  return w;
}

template <class T>
__device__ __forceinline__ void body_uu_ttg(const KernelArgs& a, int64_t blk) {
  const int64_t i = blk * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  mom p[5];
  double psw = 1.0;   // phase-space weight of a generated event (resonance tree)
  if (active) {
    if (a.mom_in) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const double* b = a.mom_in + int64_t(k) * 4 * a.mom_stride + i;
        p[k] = {b[0], b[a.mom_stride], b[2 * a.mom_stride], b[3 * a.mom_stride]};
      }
    } else {
      const double h = 0.5 * a.sqrt_s;
      p[0] = {h, 0.0, 0.0, h};
      p[1] = {h, 0.0, 0.0, -h};
      psw = ps_tree_uu_ttg(a, a.counter_offset + uint64_t(i), i, p);
    }
    if (a.mom_out) store_momenta<5>(a, i, p);
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k) p[k] = {1.0, 0.0, 0.0, 1.0};
  }
  const bool pass = active && psw > 0.0 && (!a.cut_enabled || pass_pt_dr<3>(p + 2, a.cut_pt, a.cut_dr));
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
  const vec<T> Qs4 = tv<T>(q4);
  const mom qs2_3 = q2 + q3;
  const vec<T> Qs2_3 = tv<T>(qs2_3);
  const cx<T> d2_3_0 = cvt<T>(inv_denominator(qs2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const mom qs2_3_4 = q2 + q3 + q4;
  const vec<T> Qs2_3_4 = tv<T>(qs2_3_4);
  const cx<T> d2_3_4_0 = cvt<T>(inv_denominator(qs2_3_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const mom qs2_4 = q2 + q4;
  const vec<T> Qs2_4 = tv<T>(qs2_4);
  const cx<T> d2_4_3 = cvt<T>(inv_denominator(qs2_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const mom qs3_4 = q3 + q4;
  const vec<T> Qs3_4 = tv<T>(qs3_4);
  const cx<T> d3_4_3 = cvt<T>(inv_denominator(qs3_4, cx<double>{pe3.pole_r, pe3.pole_i}));
  const mom qs0_4 = q0 + q4;
  const vec<T> Qs0_4 = tv<T>(qs0_4);
  const cx<T> d0_4_0 = cvt<T>(inv_denominator(qs0_4, cx<double>{pe0.pole_r, pe0.pole_i}));
  const mom qs0_2_3 = q0 + q2 + q3;
  const vec<T> Qs0_2_3 = tv<T>(qs0_2_3);
  const cx<T> d0_2_3_0 = cvt<T>(inv_denominator(qs0_2_3, cx<double>{pe0.pole_r, pe0.pole_i}));
  const MLF<T> e0 = mlf_pre<T>(p[0]);
  const MLF<T> e1 = mlf_pre<T>(p[1]);
  const wf<T> e2m = cvtw<T>(oxxxxx<double, false>(tv<double>(p[2]), pe3.m, -1, 1));
  const wf<T> e2p = cvtw<T>(oxxxxx<double, false>(tv<double>(p[2]), pe3.m, 1, 1));
  const wf<T> e3m = cvtw<T>(ixxxxx<double, false>(tv<double>(p[3]), pe3.m, -1, -1));
  const wf<T> e3p = cvtw<T>(ixxxxx<double, false>(tv<double>(p[3]), pe3.m, 1, -1));
  const vec<T> P4 = tv<T>(p[4]);
  const VPol<T> V4 = vpol_pre<T>(p[4]);
  double me2 = 0.0;
  if (pass && a.hel_nest) {
    // helicity loop nest, outermost leg first: [2, 4, 3, 0, 1]
    // kinematics used only inside the helicity loops wait in LDS and are read
    // back in the loop that first needs them, instead of occupying registers
    __shared__ T stash[61][256];
    stash_put(stash, 0, e2m);
    stash_put(stash, 8, e2p);
    stash_put(stash, 16, Qs2_4);
    stash_put(stash, 20, d2_4_3);
    stash_put(stash, 22, V4);
    stash_put(stash, 27, Qs4);
    stash_put(stash, 31, Qs2_3);
    stash_put(stash, 35, d2_3_0);
    stash_put(stash, 37, Qs2_3_4);
    stash_put(stash, 41, d2_3_4_0);
    stash_put(stash, 43, Qs3_4);
    stash_put(stash, 47, d3_4_3);
    stash_put(stash, 49, Qs0_4);
    stash_put(stash, 53, d0_4_0);
    stash_put(stash, 55, Qs0_2_3);
    stash_put(stash, 59, d0_2_3_0);
    #pragma unroll 1
    for (int c2 = 0; c2 < 2; ++c2) {
      const int hh2 = 2 * c2 - 1;
      const wf<T> e2m = stash_get<wf<T>>(stash, 0);
      const wf<T> e2p = stash_get<wf<T>>(stash, 8);
      const wf<T> w2 = hh2 > 0 ? e2p : e2m;
      #pragma unroll 1
      for (int c4 = 0; c4 < 2; ++c4) {
        const int hh4 = 2 * c4 - 1;
        const vec<T> Qs2_4 = stash_get<vec<T>>(stash, 16);
        const cx<T> d2_4_3 = stash_get<cx<T>>(stash, 20);
        const VPol<T> V4 = stash_get<VPol<T>>(stash, 22);
        const wf<T> w4 = vxxxxx0<T>(V4, hh4, 1);
        const wf<T> w7 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
        #pragma unroll
        for (int c3 = 0; c3 < 2; ++c3) {
          const int hh3 = 2 * c3 - 1;
          const vec<T> Qs4 = stash_get<vec<T>>(stash, 27);
          const vec<T> Qs2_3 = stash_get<vec<T>>(stash, 31);
          const cx<T> d2_3_0 = stash_get<cx<T>>(stash, 35);
          const vec<T> Qs2_3_4 = stash_get<vec<T>>(stash, 37);
          const cx<T> d2_3_4_0 = stash_get<cx<T>>(stash, 41);
          const vec<T> Qs3_4 = stash_get<vec<T>>(stash, 43);
          const cx<T> d3_4_3 = stash_get<cx<T>>(stash, 47);
          const wf<T> w3 = hh3 > 0 ? e3p : e3m;
          const wf<T> w5 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
          const wf<T> w6 = jvvxxx<T, false>(w5, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
          const wf<T> w8 = jioxxx<T, false>(w3, w7, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
          const wf<T> w9 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
          const wf<T> w10 = jioxxx<T, false>(w9, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
          #pragma unroll
          for (int c0 = 0; c0 < 2; ++c0) {
            const int hh0 = 2 * c0 - 1;
            const vec<T> Qs0_4 = stash_get<vec<T>>(stash, 49);
            const cx<T> d0_4_0 = stash_get<cx<T>>(stash, 53);
            const vec<T> Qs0_2_3 = stash_get<vec<T>>(stash, 55);
            const cx<T> d0_2_3_0 = stash_get<cx<T>>(stash, 59);
            const wf<T> w0 = ixxxxx0<T>(e0, hh0, 1);
            const wf<T> w11 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
            const wf<T> w12 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
            #pragma unroll
            for (int c1 = 0; c1 < 2; ++c1) {
              const int hh1 = 2 * c1 - 1;
              const wf<T> w1 = oxxxxx0<T>(e1, hh1, -1);
              const cx<T> amp0 = iovxxx<T>(w0, w1, w6, g0_0, g0_1);
              const cx<T> amp1 = iovxxx<T>(w0, w1, w8, g0_0, g0_1);
              const cx<T> amp2 = iovxxx<T>(w0, w1, w10, g0_0, g0_1);
              const cx<T> amp3 = iovxxx<T>(w11, w1, w5, g0_0, g0_1);
              const cx<T> amp4 = iovxxx<T>(w12, w1, w4, g0_0, g0_1);
              const cx<T> K0_0 = (T(0.16666666666666666) * amp1) + (T(0.16666666666666666) * amp2);
              const cx<T> J0 = K0_0;
              const cx<T> K1_0 = (T(0.5) * amp0) + (T(-0.5) * amp1) + (T(-0.5) * amp3);
              const cx<T> J1 = K1_0;
              const cx<T> K2_0 = (T(0.16666666666666666) * amp3) + (T(0.16666666666666666) * amp4);
              const cx<T> J2 = K2_0;
              const cx<T> K3_0 = (T(-0.5) * amp0) + (T(-0.5) * amp2) + (T(-0.5) * amp4);
              const cx<T> J3 = K3_0;
              T cs = T(0);
              {
                const cx<T> jf = J0;
                T r = T(12.0) * norm2(jf);
                { const cx<T> jg = J1; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
                { const cx<T> jg = J3; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
                cs += r;
              }
              {
                const cx<T> jf = J1;
                T r = T(12.0) * norm2(jf);
                { const cx<T> jg = J2; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
                cs += r;
              }
              {
                const cx<T> jf = J2;
                T r = T(12.0) * norm2(jf);
                { const cx<T> jg = J3; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
                cs += r;
              }
              {
                const cx<T> jf = J3;
                T r = T(12.0) * norm2(jf);
                cs += r;
              }
              me2 += double(cs) * 1.0;
            }
          }
        }
      }
    }
  } else if (pass) {
    // an arbitrary helicity table (filtered, reordered or gauge-test rows)
    for (int h = 0; h < a.n_hel; ++h) {
      const int8_t* hh = a.hel + h * 5;
      const wf<T> w0 = ixxxxx0<T>(e0, hh[0], 1);
      const wf<T> w1 = oxxxxx0<T>(e1, hh[1], -1);
      const wf<T> w2 = hh[2] > 0 ? e2p : e2m;
      const wf<T> w3 = hh[3] > 0 ? e3p : e3m;
      const wf<T> w4 = vxxxxx<T>(P4, T(pe0.m), hh[4], 1);
      const wf<T> w5 = jioxxx<T, false>(w3, w2, g0_0, g0_1, Qs2_3, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_0);
      const wf<T> w6 = jvvxxx<T, false>(w5, Qs2_3, w4, Qs4, g1_0.r, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const wf<T> w7 = fvoxxx<T>(w2, w4, g0_0, g0_1, Qs2_4, T(pe3.m), d2_4_3);
      const wf<T> w8 = jioxxx<T, false>(w3, w7, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const wf<T> w9 = fvixxx<T>(w3, w4, g0_0, g0_1, Qs3_4, T(pe3.m), d3_4_3);
      const wf<T> w10 = jioxxx<T, false>(w9, w2, g0_0, g0_1, Qs2_3_4, mk<T>(T(pe0.inum_r), T(pe0.inum_i)), d2_3_4_0);
      const cx<T> amp0 = iovxxx<T>(w0, w1, w6, g0_0, g0_1);
      const cx<T> amp1 = iovxxx<T>(w0, w1, w8, g0_0, g0_1);
      const cx<T> amp2 = iovxxx<T>(w0, w1, w10, g0_0, g0_1);
      const wf<T> w11 = fvixxx<T>(w0, w4, g0_0, g0_1, Qs0_4, T(pe0.m), d0_4_0);
      const cx<T> amp3 = iovxxx<T>(w11, w1, w5, g0_0, g0_1);
      const wf<T> w12 = fvixxx<T>(w0, w5, g0_0, g0_1, Qs0_2_3, T(pe0.m), d0_2_3_0);
      const cx<T> amp4 = iovxxx<T>(w12, w1, w4, g0_0, g0_1);
      const cx<T> J0 = (T(0.16666666666666666) * amp1) + (T(0.16666666666666666) * amp2);
      const cx<T> J1 = (T(0.5) * amp0) + (T(-0.5) * amp1) + (T(-0.5) * amp3);
      const cx<T> J2 = (T(0.16666666666666666) * amp3) + (T(0.16666666666666666) * amp4);
      const cx<T> J3 = (T(-0.5) * amp0) + (T(-0.5) * amp2) + (T(-0.5) * amp4);
      T cs = T(0);
      {
        const cx<T> jf = J0;
        T r = T(12.0) * norm2(jf);
        { const cx<T> jg = J1; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
        { const cx<T> jg = J3; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J1;
        T r = T(12.0) * norm2(jf);
        { const cx<T> jg = J2; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J2;
        T r = T(12.0) * norm2(jf);
        { const cx<T> jg = J3; r += T(8.0) * (jf.r * jg.r + jf.i * jg.i); }
        cs += r;
      }
      {
        const cx<T> jf = J3;
        T r = T(12.0) * norm2(jf);
        cs += r;
      }
      me2 += double(cs) * 1.0;
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
__global__ __launch_bounds__(256) void amp_uu_ttg(KernelArgs a) {
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
    body_uu_ttg<T>(b, blk);
    __syncthreads();
  }
}

// the phase-space step alone (heget_generate): momenta and per-event weights
__global__ __launch_bounds__(256) void gen_uu_ttg(KernelArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  mom p[5];
  const double w = ps_tree_uu_ttg(a, a.counter_offset + uint64_t(i), i, p);
  store_momenta<5>(a, i, p);
  if (a.psw_out) a.psw_out[i] = w;
}

}  // namespace

// the full helicity product in canonical order: tables equal to it run the loop nest
static const int8_t hel_canon[] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, 1, -1, -1, -1, 1, -1, -1, -1, -1, 1, 1, -1, -1, 1, -1, -1, -1, -1, 1, -1, 1, -1, -1, 1, 1, -1, -1, -1, 1, 1, 1, -1, 1, -1, -1, -1, -1, 1, -1, -1, 1, -1, 1, -1, 1, -1, -1, 1, -1, 1, 1, -1, 1, 1, -1, -1, -1, 1, 1, -1, 1, -1, 1, 1, 1, -1, -1, 1, 1, 1, 1, 1, -1, -1, -1, -1, 1, -1, -1, -1, 1, 1, -1, -1, 1, -1, 1, -1, -1, 1, 1, 1, -1, 1, -1, -1, 1, -1, 1, -1, 1, 1, -1, 1, 1, -1, 1, -1, 1, 1, 1, 1, 1, -1, -1, -1, 1, 1, -1, -1, 1, 1, 1, -1, 1, -1, 1, 1, -1, 1, 1, 1, 1, 1, -1, -1, 1, 1, 1, -1, 1, 1, 1, 1, 1, -1, 1, 1, 1, 1, 1};
static const GenEntry entry = {0x49875fd400262df3ull, "uu_ttg", 5, reinterpret_cast<const void*>(&amp_uu_ttg<double>), reinterpret_cast<const void*>(&amp_uu_ttg<float>), 0, 0, 0, reinterpret_cast<const void*>(&amp_uu_ttg<double>), reinterpret_cast<const void*>(&amp_uu_ttg<float>), hel_canon, 32, 0, 0, reinterpret_cast<const void*>(&gen_uu_ttg), 5, 0, nullptr, nullptr, nullptr, nullptr};
static const Registrar reg(&entry);

}  // namespace heget
