// HEGET-style helicity-amplitude building blocks for gfx950 (device code).
//
// One event per lane: every function works on one lane's registers; nothing
// here touches memory.  Each function implements the output the paper defines
// for the HEGET/HELAS function of the same role (Sec. 4, Tables of external
// lines and vertices, App. C), derived from the vertex Lagrangians of Sec. 4.2
// in the chiral (Weyl) representation:
//   gamma^mu = [[0, s^mu], [sb^mu, 0]],  s^mu = (1, sigma),  sb^mu = (1, -sigma),
//   gamma5 = diag(-1, -1, 1, 1),  P_L = diag(1, 1, 0, 0).
//
// Conventions shared by the whole path:
//  * T is the arithmetic type of wavefunction components (double or float).
//    Momenta are always carried in FP64 (type mom), and propagator
//    denominators are formed in FP64 by the caller and passed in as 1/D.
//  * A wavefunction's momentum q is the momentum flowing INTO the vertex where
//    it is consumed (incoming external particle: +p, outgoing: -p).  An
//    off-shell current built from inputs q_i carries q = sum q_i.
//  * Vertex functions return the Feynman rule divided by i (the Lagrangian
//    coefficient contracted with the wavefunctions; derivatives -> -i q).
//  * Off-shell currents carry the factor -N/D of their propagator (N the
//    numerator of the i-stripped propagator), so that a tree amplitude is the
//    plain product of vertex values and currents.
//  * Fermion momenta along the fermion arrow are +q for flowing-in (|fi>) and
//    -q for flowing-out (<fo|) wavefunctions.
#pragma once
#include <hip/hip_runtime.h>

namespace heget {

template <class T>
struct cx {
  T r, i;
};

template <class T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return {r, i}; }
template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {s * a.r, s * a.i}; }
template <class T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
template <class T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }   // i a
template <class T>
__device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }  // -i a
template <class T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.r * a.r + a.i * a.i; }
template <class T, class S>
__device__ __forceinline__ cx<T> cvt(cx<S> a) { return {T(a.r), T(a.i)}; }

// FP64 four-momentum (E, px, py, pz)
struct mom {
  double e, x, y, z;
};
__device__ __forceinline__ mom operator+(mom a, mom b) { return {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ mom operator-(mom a) { return {-a.e, -a.x, -a.y, -a.z}; }

// FP64 square root and reciprocal for the kinematics, from the hardware
// estimates (v_rsq_f64, v_rcp_f64, about 23 bits) refined in FMA: the square
// root by the coupled Newton iteration for sqrt(x) and 1/(2 sqrt(x)) followed by
// two residual corrections (Goldschmidt's method as Markstein arranges it, IA-64
// and Elementary Functions, 2000), the reciprocal by two Newton steps.  Within
// one unit in the last place; they skip the IEEE library's scaling of tiny and
// huge arguments, which kinematics never produce.  sqrt_pos returns 0 for x <= 0.
// The FP32 overloads are the library's.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}
__device__ __forceinline__ float sqrt_pos(float x) { return sqrtf(x); }
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ float recip(float d) { return 1.0f / d; }
// a / b: the reciprocal times a, and one correction of the quotient
__device__ __forceinline__ double quot(double a, double b) {
  const double r = recip(b);
  const double q = a * r;
  return fma(r, fma(-b, q, a), q);
}
__device__ __forceinline__ float quot(float a, float b) { return a / b; }
// The same momentum, opaque to the optimiser: kinematics computed from it
// inside a loop stay in that loop (recomputed) instead of being hoisted out and
// held in registers across it.
__device__ __forceinline__ mom opaque_mom(mom a) {
  asm volatile("" : "+v"(a.e), "+v"(a.x), "+v"(a.y), "+v"(a.z));
  return a;
}
// An integer opaque to the optimiser (same value): addresses built from it
// inside a loop keep their loads in that loop.
__device__ __forceinline__ int opaque_int(int x) {
  asm volatile("" : "+s"(x));
  return x;
}
__device__ __forceinline__ double msq(mom a) { return a.e * a.e - a.x * a.x - a.y * a.y - a.z * a.z; }

// four-momentum in the arithmetic type of the wavefunctions
template <class T>
struct vec {
  T e, x, y, z;
};
template <class T>
__device__ __forceinline__ vec<T> tv(mom a) { return {T(a.e), T(a.x), T(a.y), T(a.z)}; }

// Four complex components: a Dirac spinor (|fi> column or <fo| row) or a
// contravariant polarisation / current vector.
template <class T>
struct wf {
  cx<T> c[4];
};

template <class T, class S>
__device__ __forceinline__ wf<T> cvtw(const wf<S>& a) {
  return {{cvt<T>(a.c[0]), cvt<T>(a.c[1]), cvt<T>(a.c[2]), cvt<T>(a.c[3])}};
}

template <class T>
__device__ __forceinline__ wf<T> wscale(cx<T> s, const wf<T>& a) {
  return {{s * a.c[0], s * a.c[1], s * a.c[2], s * a.c[3]}};
}

template <class T>
__device__ __forceinline__ wf<T> waxpy(T s, const wf<T>& x, const wf<T>& y) {
  return {{s * x.c[0] + y.c[0], s * x.c[1] + y.c[1], s * x.c[2] + y.c[2], s * x.c[3] + y.c[3]}};
}

template <class T>
__device__ __forceinline__ wf<T> vadd(const wf<T>& a, const wf<T>& b) {
  return {{a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2], a.c[3] + b.c[3]}};
}
template <class T>
__device__ __forceinline__ wf<T> vsub(const wf<T>& a, const wf<T>& b) {
  return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2], a.c[3] - b.c[3]}};
}

// Minkowski product of two complex vectors (no conjugation)
template <class T>
__device__ __forceinline__ cx<T> dot(const wf<T>& a, const wf<T>& b) {
  return a.c[0] * b.c[0] - a.c[1] * b.c[1] - a.c[2] * b.c[2] - a.c[3] * b.c[3];
}
template <class T>
__device__ __forceinline__ cx<T> dot(const wf<T>& a, vec<T> q) {
  return q.e * a.c[0] - q.x * a.c[1] - q.y * a.c[2] - q.z * a.c[3];
}

// 1 / (q^2 - pole) in FP64 for a complex pole (m^2 - i m Gamma, or the complex mass)
__device__ __forceinline__ cx<double> inv_denominator(mom q, cx<double> pole) {
  const double a = msq(q) - pole.r, b = -pole.i;
  const double n = recip(a * a + b * b);
  return {a * n, -b * n};
}

// --------------------------------------------------------------- external lines
// Two-component helicity eigenstates chi_lam of sigma.phat (unit norm), written
// with sqrt(2|p|(|p|+pz)); for a momentum along -z: chi_+ = (0,1), chi_- = (-1,0).
// |p| + p_z without cancellation: for p_z < 0 it equals p_T^2 / (|p| - p_z)
template <class T>
__device__ __forceinline__ T pp_plus_pz(vec<T> p, T pp) {
  return p.z >= T(0) ? pp + p.z : quot(p.x * p.x + p.y * p.y, pp - p.z);
}

template <class T>
__device__ __forceinline__ void chi2(vec<T> p, T pp, int lam, cx<T>& a, cx<T>& b) {
  const T s = pp_plus_pz(p, pp);
  if (s > T(0)) {
    const T n = recip(sqrt_pos(T(2) * pp * s));
    if (lam > 0) {
      a = mk<T>(s * n, T(0));
      b = mk<T>(p.x * n, p.y * n);
    } else {
      a = mk<T>(-p.x * n, p.y * n);
      b = mk<T>(s * n, T(0));
    }
  } else {
    if (lam > 0) {
      a = mk<T>(T(0), T(0));
      b = mk<T>(T(1), T(0));
    } else {
      a = mk<T>(T(-1), T(0));
      b = mk<T>(T(0), T(0));
    }
  }
}

// Massless Weyl factor sqrt(2E) chi_lam in the sqrt(E+pz) form (exact zeros in
// the opposite chirality):  lam = +1: (sqrt(E+pz), (px + i py)/sqrt(E+pz)),
// lam = -1: ((-px + i py)/sqrt(E+pz), sqrt(E+pz)).  E is taken as |p| of the
// three-momentum, so that a momentum that is massless only up to rounding
// still defines an exactly massless state.
template <class T>
__device__ __forceinline__ void weyl0(vec<T> p, int lam, cx<T>& a, cx<T>& b) {
  const T pp = sqrt_pos(p.x * p.x + p.y * p.y + p.z * p.z);
  const T s = pp_plus_pz(p, pp);
  if (s > T(0)) {
    const T r = sqrt_pos(s), ir = recip(r);
    if (lam > 0) {
      a = mk<T>(r, T(0));
      b = mk<T>(p.x * ir, p.y * ir);
    } else {
      a = mk<T>(-p.x * ir, p.y * ir);
      b = mk<T>(r, T(0));
    }
  } else {
    const T r = sqrt_pos(T(2) * pp);
    if (lam > 0) {
      a = mk<T>(T(0), T(0));
      b = mk<T>(r, T(0));
    } else {
      a = mk<T>(-r, T(0));
      b = mk<T>(T(0), T(0));
    }
  }
}

// |fi> for a flowing-in fermion: u(p, lam) (nsf = +1, incoming particle) or
// v(p, lam) (nsf = -1, outgoing antiparticle of helicity lam).
//   u = ( sqrt(E - lam|p|) chi_lam ; sqrt(E + lam|p|) chi_lam )
//   v = ( -lam sqrt(E + lam|p|) chi_-lam ; lam sqrt(E - lam|p|) chi_-lam )
template <class T, bool MASSLESS>
__device__ __forceinline__ wf<T> ixxxxx(vec<T> p, T m, int lam, int nsf) {
  wf<T> f;
  const cx<T> z = mk<T>(T(0), T(0));
  if (MASSLESS) {
    cx<T> a, b;
    if (nsf > 0) {
      weyl0(p, lam, a, b);
      if (lam > 0) {
        f.c[0] = z; f.c[1] = z; f.c[2] = a; f.c[3] = b;
      } else {
        f.c[0] = a; f.c[1] = b; f.c[2] = z; f.c[3] = z;
      }
    } else {
      weyl0(p, -lam, a, b);
      const T l = T(lam);
      if (lam > 0) {
        f.c[0] = -l * a; f.c[1] = -l * b; f.c[2] = z; f.c[3] = z;
      } else {
        f.c[0] = z; f.c[1] = z; f.c[2] = l * a; f.c[3] = l * b;
      }
    }
    return f;
  }
  const T pp = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  const T E = sqrt(pp * pp + m * m);
  cx<T> a, b;
  const T l = T(lam);
  if (nsf > 0) {
    chi2(p, pp, lam, a, b);
    const T wm = sqrt(E - l * pp), wp = sqrt(E + l * pp);
    f.c[0] = wm * a; f.c[1] = wm * b; f.c[2] = wp * a; f.c[3] = wp * b;
  } else {
    chi2(p, pp, -lam, a, b);
    const T wp = sqrt(E + l * pp), wm = sqrt(E - l * pp);
    f.c[0] = (-l * wp) * a; f.c[1] = (-l * wp) * b; f.c[2] = (l * wm) * a; f.c[3] = (l * wm) * b;
  }
  return f;
}

// Helicity-independent part of a massless external fermion: sqrt(2E) chi_+ and
// sqrt(2E) chi_- formed once per event in FP64 (the sqrt(E+pz) form loses
// precision in FP32 for momenta near -z), stored in the arithmetic type T.
template <class T>
struct MLF {
  cx<T> ap, bp, am, bm;
};
template <class T>
__device__ __forceinline__ MLF<T> mlf_pre(mom p) {
  const vec<double> q = {p.e, p.x, p.y, p.z};
  cx<double> ap, bp, am, bm;
  weyl0(q, +1, ap, bp);
  weyl0(q, -1, am, bm);
  return {cvt<T>(ap), cvt<T>(bp), cvt<T>(am), cvt<T>(bm)};
}
// |fi> of a massless fermion from its precomputed Weyl factors (same
// conventions as ixxxxx<T, true>)
template <class T>
__device__ __forceinline__ wf<T> ixxxxx0(const MLF<T>& e, int lam, int nsf) {
  const cx<T> z = mk<T>(T(0), T(0));
  wf<T> f;
  if (nsf > 0) {
    if (lam > 0) {
      f.c[0] = z; f.c[1] = z; f.c[2] = e.ap; f.c[3] = e.bp;
    } else {
      f.c[0] = e.am; f.c[1] = e.bm; f.c[2] = z; f.c[3] = z;
    }
  } else {
    if (lam > 0) {
      f.c[0] = -e.am; f.c[1] = -e.bm; f.c[2] = z; f.c[3] = z;
    } else {
      f.c[0] = z; f.c[1] = z; f.c[2] = -e.ap; f.c[3] = -e.bp;
    }
  }
  return f;
}
template <class T>
__device__ __forceinline__ wf<T> oxxxxx0(const MLF<T>& e, int lam, int nsf) {
  const wf<T> s = ixxxxx0(e, lam, nsf);
  wf<T> f;
  f.c[0] = conj(s.c[2]);
  f.c[1] = conj(s.c[3]);
  f.c[2] = conj(s.c[0]);
  f.c[3] = conj(s.c[1]);
  return f;
}

// <fo| for a flowing-out fermion: ubar(p, lam) (nsf = +1, outgoing particle) or
// vbar(p, lam) (nsf = -1, incoming antiparticle).  psibar = psi^dagger gamma^0,
// which in the chiral basis swaps the two Weyl halves and conjugates.
template <class T, bool MASSLESS>
__device__ __forceinline__ wf<T> oxxxxx(vec<T> p, T m, int lam, int nsf) {
  const wf<T> s = ixxxxx<T, MASSLESS>(p, m, lam, nsf);
  wf<T> f;
  f.c[0] = conj(s.c[2]);
  f.c[1] = conj(s.c[3]);
  f.c[2] = conj(s.c[0]);
  f.c[3] = conj(s.c[1]);
  return f;
}

// Polarisation vector: eps(k, lam) for an incoming vector (nsv = -1) and
// eps(k, lam)^* for an outgoing one (nsv = +1).  Transverse lam = +-1:
// (1/sqrt2)(-lam e1 - i e2), e1 = (0, cos th cos ph, cos th sin ph, -sin th),
// e2 = (0, -sin ph, cos ph, 0); lam = 0: (|k|, E khat)/m.  lam = 4 gives the
// gauge-check vector k/k^0.
template <class T>
__device__ __forceinline__ wf<T> vxxxxx(vec<T> k, T m, int lam, int nsv) {
  wf<T> v;
  if (lam == 4) {
    const T r = T(1) / k.e;
    v.c[0] = mk<T>(T(1), T(0));
    v.c[1] = mk<T>(k.x * r, T(0));
    v.c[2] = mk<T>(k.y * r, T(0));
    v.c[3] = mk<T>(k.z * r, T(0));
    return v;
  }
  const T pt2 = k.x * k.x + k.y * k.y;
  // the library's sqrt and division here: the gluon templates form this vector
  // inside their loops, and the FMA forms moved those kernels' spills into the loops
  const T pt = sqrt(pt2);
  const T pp = sqrt(pt2 + k.z * k.z);
  T ct, st, cp, sp;
  if (pp > T(0)) {
    const T ipp = T(1) / pp;
    ct = k.z * ipp;
    st = pt * ipp;
  } else {
    ct = T(1);
    st = T(0);
  }
  if (pt > T(0)) {
    const T ipt = T(1) / pt;
    cp = k.x * ipt;
    sp = k.y * ipt;
  } else {
    cp = T(1);
    sp = T(0);
  }
  if (lam == 0) {
    const T E = sqrt(pp * pp + m * m);
    const T im = T(1) / m;
    v.c[0] = mk<T>(pp * im, T(0));
    v.c[1] = mk<T>(E * im * st * cp, T(0));
    v.c[2] = mk<T>(E * im * st * sp, T(0));
    v.c[3] = mk<T>(E * im * ct, T(0));
    return v;
  }
  const T h = T(0.70710678118654752440);
  const T hl = h * T(lam);
  // eps = h(-lam e1 - i e2); the outgoing (conjugated) vector flips the imaginary parts
  const T si = nsv > 0 ? -h : h;
  v.c[0] = mk<T>(T(0), T(0));
  v.c[1] = mk<T>(-hl * ct * cp, si * sp);
  v.c[2] = mk<T>(-hl * ct * sp, -si * cp);
  v.c[3] = mk<T>(hl * st, T(0));
  return v;
}

// Helicity-independent part of a massless vector's transverse polarisations:
// (1/sqrt2) x (cos th cos ph, cos th sin ph, sin th, sin ph, cos ph), formed
// in FP64 from the FP64 momentum exactly as vxxxxx forms them.
template <class T>
struct VPol {
  T a, b, c, d, e;
};
template <class T>
__device__ __forceinline__ VPol<T> vpol_pre(mom p) {
  const double pt2 = p.x * p.x + p.y * p.y;
  const double pt = sqrt_pos(pt2);
  const double pp = sqrt_pos(pt2 + p.z * p.z);
  double ct = 1.0, st = 0.0, cp = 1.0, sp = 0.0;
  if (pp > 0.0) {
    const double ipp = recip(pp);
    ct = p.z * ipp;
    st = pt * ipp;
  }
  if (pt > 0.0) {
    const double ipt = recip(pt);
    cp = p.x * ipt;
    sp = p.y * ipt;
  }
  const double h = 0.70710678118654752440;
  return {T(h * ct * cp), T(h * ct * sp), T(h * st), T(h * sp), T(h * cp)};
}
// eps(k, lam), lam = +-1, of a massless vector from its precomputed factors
// (the same vector as vxxxxx(k, 0, lam, nsv))
template <class T>
__device__ __forceinline__ wf<T> vxxxxx0(const VPol<T>& q, int lam, int nsv) {
  const T l = T(lam);
  const T s = nsv > 0 ? T(-1) : T(1);
  wf<T> v;
  v.c[0] = mk<T>(T(0), T(0));
  v.c[1] = mk<T>(-l * q.a, s * q.d);
  v.c[2] = mk<T>(-l * q.b, -s * q.e);
  v.c[3] = mk<T>(l * q.c, T(0));
  return v;
}

// Scalar external line: the component is 1.
template <class T>
__device__ __forceinline__ cx<T> sxxxxx() { return mk<T>(T(1), T(0)); }

// ------------------------------------------------------------ Weyl helpers
// s.V = s^mu V_mu and sb.V acting on a 2-spinor (x0, x1), V contravariant.
//   s.V  = [[V0 - V3, -(V1 - i V2)], [-(V1 + i V2), V0 + V3]]
//   sb.V = [[V0 + V3,   V1 - i V2 ], [  V1 + i V2,  V0 - V3 ]]
template <class T>
__device__ __forceinline__ void sV(const cx<T>* V, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> vm = V[1] - times_i(V[2]), vp = V[1] + times_i(V[2]);
  y0 = (V[0] - V[3]) * x0 - vm * x1;
  y1 = (V[0] + V[3]) * x1 - vp * x0;
}
template <class T>
__device__ __forceinline__ void sbV(const cx<T>* V, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> vm = V[1] - times_i(V[2]), vp = V[1] + times_i(V[2]);
  y0 = (V[0] + V[3]) * x0 + vm * x1;
  y1 = vp * x0 + (V[0] - V[3]) * x1;
}
// row 2-spinor times s.V / sb.V
template <class T>
__device__ __forceinline__ void rsV(const cx<T>* V, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> vm = V[1] - times_i(V[2]), vp = V[1] + times_i(V[2]);
  y0 = x0 * (V[0] - V[3]) - x1 * vp;
  y1 = -(x0 * vm) + x1 * (V[0] + V[3]);
}
template <class T>
__device__ __forceinline__ void rsbV(const cx<T>* V, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> vm = V[1] - times_i(V[2]), vp = V[1] + times_i(V[2]);
  y0 = x0 * (V[0] + V[3]) + x1 * vp;
  y1 = x0 * vm + x1 * (V[0] - V[3]);
}
// the same with a real momentum
template <class T>
__device__ __forceinline__ void sq(vec<T> q, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> qm = mk<T>(q.x, -q.y), qp = mk<T>(q.x, q.y);
  y0 = (q.e - q.z) * x0 - qm * x1;
  y1 = (q.e + q.z) * x1 - qp * x0;
}
template <class T>
__device__ __forceinline__ void sbq(vec<T> q, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> qm = mk<T>(q.x, -q.y), qp = mk<T>(q.x, q.y);
  y0 = (q.e + q.z) * x0 + qm * x1;
  y1 = qp * x0 + (q.e - q.z) * x1;
}
template <class T>
__device__ __forceinline__ void rsq(vec<T> q, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> qm = mk<T>(q.x, -q.y), qp = mk<T>(q.x, q.y);
  y0 = (q.e - q.z) * x0 - qp * x1;
  y1 = (q.e + q.z) * x1 - qm * x0;
}
template <class T>
__device__ __forceinline__ void rsbq(vec<T> q, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> qm = mk<T>(q.x, -q.y), qp = mk<T>(q.x, q.y);
  y0 = (q.e + q.z) * x0 + qp * x1;
  y1 = qm * x0 + (q.e - q.z) * x1;
}

// -------------------------------------------------------------------- FFV
// L = psibar_1 gamma^mu [g0 P_L + g1 P_R] psi_2 V*_mu  (Sec. 4.2.1)

// amplitude <fo| Vslash (g0 P_L + g1 P_R) |fi>
template <class T>
__device__ __forceinline__ cx<T> iovxxx(const wf<T>& fi, const wf<T>& fo, const wf<T>& vc, cx<T> g0, cx<T> g1) {
  cx<T> a0, a1, b0, b1;
  sbV(vc.c, fi.c[0], fi.c[1], a0, a1);   // lower rows of Vslash P_L |fi>
  sV(vc.c, fi.c[2], fi.c[3], b0, b1);    // upper rows of Vslash P_R |fi>
  return g0 * (fo.c[2] * a0 + fo.c[3] * a1) + g1 * (fo.c[0] * b0 + fo.c[1] * b1);
}

// The row spinor <fo| Vslash (g0 P_L + g1 P_R): iovxxx(fi, fo, V) = spinor_dot(ffv_bra(fo, V), fi).
// Lets a loop nest form it once per (fo, V) and contract it with many fi.
template <class T>
__device__ __forceinline__ wf<T> ffv_bra(const wf<T>& fo, const wf<T>& vc, cx<T> g0, cx<T> g1) {
  cx<T> u0, u1, l0, l1;
  rsbV(vc.c, fo.c[2], fo.c[3], u0, u1);  // acts on the upper (left-handed) components of fi
  rsV(vc.c, fo.c[0], fo.c[1], l0, l1);   // acts on the lower (right-handed) components of fi
  return {{g0 * u0, g0 * u1, g1 * l0, g1 * l1}};
}

// row spinor times column spinor
template <class T>
__device__ __forceinline__ cx<T> spinor_dot(const wf<T>& b, const wf<T>& f) {
  return b.c[0] * f.c[0] + b.c[1] * f.c[1] + b.c[2] * f.c[2] + b.c[3] * f.c[3];
}

// contravariant current v^mu = <fo| gamma^mu (g0 P_L + g1 P_R) |fi>
template <class T>
__device__ __forceinline__ wf<T> ffv_current(const wf<T>& fi, const wf<T>& fo, cx<T> g0, cx<T> g1) {
  // L part: fo_low sb^mu fi_up ; R part: fo_up s^mu fi_low
  const cx<T> l0 = fo.c[2] * fi.c[0], l1 = fo.c[2] * fi.c[1], l2 = fo.c[3] * fi.c[0], l3 = fo.c[3] * fi.c[1];
  const cx<T> r0 = fo.c[0] * fi.c[2], r1 = fo.c[0] * fi.c[3], r2 = fo.c[1] * fi.c[2], r3 = fo.c[1] * fi.c[3];
  wf<T> v;
  v.c[0] = g0 * (l0 + l3) + g1 * (r0 + r3);
  v.c[1] = g1 * (r1 + r2) - g0 * (l1 + l2);
  v.c[2] = times_i(g0 * (l1 - l2)) - times_i(g1 * (r1 - r2));
  v.c[3] = g1 * (r0 - r3) - g0 * (l0 - l3);
  return v;
}

// Apply the vector propagator -N/D to a contravariant vertex vector A:
// massive (unitary gauge): (A - q (q.A) / M2) / D;  massless: A / D.
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> vector_prop(wf<T> A, vec<T> q, cx<T> inv_m2, cx<T> dinv) {
  if (MASSIVE) {
    const cx<T> k = dot(A, q) * inv_m2;
    A.c[0] = A.c[0] - q.e * k;
    A.c[1] = A.c[1] - q.x * k;
    A.c[2] = A.c[2] - q.y * k;
    A.c[3] = A.c[3] - q.z * k;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) A.c[m] = A.c[m] * dinv;
  return A;
}

// off-shell vector current from a fermion pair (jioxxx); q = q_fi + q_fo
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jioxxx(const wf<T>& fi, const wf<T>& fo, cx<T> g0, cx<T> g1, vec<T> q,
                                        cx<T> inv_m2, cx<T> dinv) {
  return vector_prop<T, MASSIVE>(ffv_current(fi, fo, g0, g1), q, inv_m2, dinv);
}

// off-shell flowing-in fermion (fvixxx): -(qslash + m) Vslash (g0 P_L + g1 P_R) |fi> / D
template <class T>
__device__ __forceinline__ wf<T> fvixxx(const wf<T>& fi, const wf<T>& vc, cx<T> g0, cx<T> g1, vec<T> q, T m,
                                        cx<T> dinv) {
  cx<T> u0, u1, l0, l1;
  sV(vc.c, fi.c[2], fi.c[3], u0, u1);    // upper: s.V fi_R
  sbV(vc.c, fi.c[0], fi.c[1], l0, l1);   // lower: sb.V fi_L
  u0 = g1 * u0; u1 = g1 * u1;
  l0 = g0 * l0; l1 = g0 * l1;
  cx<T> a0, a1, b0, b1;
  sq(q, l0, l1, a0, a1);                 // upper: s.q psi_low + m psi_up
  sbq(q, u0, u1, b0, b1);                // lower: sb.q psi_up + m psi_low
  const cx<T> md = -(m * dinv), nd = -dinv;
  wf<T> f;
  f.c[0] = nd * a0 + md * u0;
  f.c[1] = nd * a1 + md * u1;
  f.c[2] = nd * b0 + md * l0;
  f.c[3] = nd * b1 + md * l1;
  return f;
}

// off-shell flowing-out fermion (fvoxxx): -<fo| Vslash (g0 P_L + g1 P_R) (-qslash + m) / D
template <class T>
__device__ __forceinline__ wf<T> fvoxxx(const wf<T>& fo, const wf<T>& vc, cx<T> g0, cx<T> g1, vec<T> q, T m,
                                        cx<T> dinv) {
  cx<T> u0, u1, l0, l1;
  rsbV(vc.c, fo.c[2], fo.c[3], u0, u1);  // row components 0,1: g0 fo_low sb.V
  rsV(vc.c, fo.c[0], fo.c[1], l0, l1);   // row components 2,3: g1 fo_up s.V
  u0 = g0 * u0; u1 = g0 * u1;
  l0 = g1 * l0; l1 = g1 * l1;
  // row (u, l) times (k.gamma + m) with k = -q: (m u + l sb.k ; u s.k + m l)
  cx<T> a0, a1, b0, b1;
  rsbq(q, l0, l1, a0, a1);
  rsq(q, u0, u1, b0, b1);
  const cx<T> md = -(m * dinv);
  wf<T> f;
  f.c[0] = dinv * a0 + md * u0;   // -(-l sb.q)/D
  f.c[1] = dinv * a1 + md * u1;
  f.c[2] = dinv * b0 + md * l0;
  f.c[3] = dinv * b1 + md * l1;
  return f;
}

// -------------------------------------------------------------------- FFS
// L = psibar_1 [g0 P_L + g1 P_R] psi_2 S*  (Sec. 4.2.2)
template <class T>
__device__ __forceinline__ cx<T> iosxxx(const wf<T>& fi, const wf<T>& fo, cx<T> sc, cx<T> g0, cx<T> g1) {
  return sc * (g0 * (fo.c[0] * fi.c[0] + fo.c[1] * fi.c[1]) + g1 * (fo.c[2] * fi.c[2] + fo.c[3] * fi.c[3]));
}
// scalar current (hioxxx): -<fo|(g0 P_L + g1 P_R)|fi> / D
template <class T>
__device__ __forceinline__ cx<T> hioxxx(const wf<T>& fi, const wf<T>& fo, cx<T> g0, cx<T> g1, cx<T> dinv) {
  return -(dinv * (g0 * (fo.c[0] * fi.c[0] + fo.c[1] * fi.c[1]) + g1 * (fo.c[2] * fi.c[2] + fo.c[3] * fi.c[3])));
}
// off-shell flowing-in fermion (fsixxx): -S (qslash + m)(g0 P_L + g1 P_R)|fi> / D
template <class T>
__device__ __forceinline__ wf<T> fsixxx(const wf<T>& fi, cx<T> sc, cx<T> g0, cx<T> g1, vec<T> q, T m, cx<T> dinv) {
  const cx<T> u0 = g0 * fi.c[0], u1 = g0 * fi.c[1], l0 = g1 * fi.c[2], l1 = g1 * fi.c[3];
  cx<T> a0, a1, b0, b1;
  sq(q, l0, l1, a0, a1);
  sbq(q, u0, u1, b0, b1);
  const cx<T> nd = -(sc * dinv), md = m * nd;
  wf<T> f;
  f.c[0] = nd * a0 + md * u0;
  f.c[1] = nd * a1 + md * u1;
  f.c[2] = nd * b0 + md * l0;
  f.c[3] = nd * b1 + md * l1;
  return f;
}
// off-shell flowing-out fermion (fsoxxx): -S <fo|(g0 P_L + g1 P_R)(-qslash + m) / D
template <class T>
__device__ __forceinline__ wf<T> fsoxxx(const wf<T>& fo, cx<T> sc, cx<T> g0, cx<T> g1, vec<T> q, T m, cx<T> dinv) {
  const cx<T> u0 = g0 * fo.c[0], u1 = g0 * fo.c[1], l0 = g1 * fo.c[2], l1 = g1 * fo.c[3];
  cx<T> a0, a1, b0, b1;
  rsbq(q, l0, l1, a0, a1);
  rsq(q, u0, u1, b0, b1);
  const cx<T> sd = sc * dinv, md = -(m * sd);
  wf<T> f;
  f.c[0] = sd * a0 + md * u0;
  f.c[1] = sd * a1 + md * u1;
  f.c[2] = sd * b0 + md * l0;
  f.c[3] = sd * b1 + md * l1;
  return f;
}

// -------------------------------------------------------------------- VVV
// L = -i g {(d_mu V1*_nu)(V2*^mu V3*^nu - V2*^nu V3*^mu) + cyclic}  (Sec. 4.2.3)
// with d -> -i q (q incoming):
//   vertex = -g [ (V1.V2)(q2-q1).V3 + (V2.V3)(q3-q2).V1 + (V3.V1)(q1-q3).V2 ]
template <class T>
__device__ __forceinline__ cx<T> vvvxxx(const wf<T>& v1, vec<T> q1, const wf<T>& v2, vec<T> q2, const wf<T>& v3,
                                        vec<T> q3, T g) {
  const vec<T> a = {q2.e - q1.e, q2.x - q1.x, q2.y - q1.y, q2.z - q1.z};
  const vec<T> b = {q3.e - q2.e, q3.x - q2.x, q3.y - q2.y, q3.z - q2.z};
  const vec<T> c = {q1.e - q3.e, q1.x - q3.x, q1.y - q3.y, q1.z - q3.z};
  return -g * (dot(v1, v2) * dot(v3, a) + dot(v2, v3) * dot(v1, b) + dot(v3, v1) * dot(v2, c));
}
// off-shell V3 current (jvvxxx), q = q1 + q2 flows out to the next vertex (q3 = -q):
//   A = -g [ (V1.V2)(q2 - q1) - ((q1 + 2 q2).V1) V2 + ((2 q1 + q2).V2) V1 ]
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jvvxxx(const wf<T>& v1, vec<T> q1, const wf<T>& v2, vec<T> q2, T g, cx<T> inv_m2,
                                        cx<T> dinv) {
  const vec<T> d = {q2.e - q1.e, q2.x - q1.x, q2.y - q1.y, q2.z - q1.z};
  const vec<T> e1 = {q1.e + T(2) * q2.e, q1.x + T(2) * q2.x, q1.y + T(2) * q2.y, q1.z + T(2) * q2.z};
  const vec<T> e2 = {T(2) * q1.e + q2.e, T(2) * q1.x + q2.x, T(2) * q1.y + q2.y, T(2) * q1.z + q2.z};
  const cx<T> v12 = dot(v1, v2), a1 = dot(v1, e1), a2 = dot(v2, e2);
  wf<T> A;
  A.c[0] = -g * (d.e * v12 - a1 * v2.c[0] + a2 * v1.c[0]);
  A.c[1] = -g * (d.x * v12 - a1 * v2.c[1] + a2 * v1.c[1]);
  A.c[2] = -g * (d.y * v12 - a1 * v2.c[2] + a2 * v1.c[2]);
  A.c[3] = -g * (d.z * v12 - a1 * v2.c[3] + a2 * v1.c[3]);
  const vec<T> q = {q1.e + q2.e, q1.x + q2.x, q1.y + q2.y, q1.z + q2.z};
  return vector_prop<T, MASSIVE>(A, q, inv_m2, dinv);
}

// vvvxxx is linear in V3: vvvxxx(v1, q1, v2, q2, v3, q3, g) = dot(v3, vvv_r3(v1, q1, v2, q2, q3, g)).
// Lets a loop over V3's helicity reuse the rest.
template <class T>
__device__ __forceinline__ wf<T> vvv_r3(const wf<T>& v1, vec<T> q1, const wf<T>& v2, vec<T> q2, vec<T> q3, T g) {
  const vec<T> a = {q2.e - q1.e, q2.x - q1.x, q2.y - q1.y, q2.z - q1.z};
  const vec<T> b = {q3.e - q2.e, q3.x - q2.x, q3.y - q2.y, q3.z - q2.z};
  const vec<T> c = {q1.e - q3.e, q1.x - q3.x, q1.y - q3.y, q1.z - q3.z};
  const cx<T> v12 = -g * dot(v1, v2), v1b = -g * dot(v1, b), v2c = -g * dot(v2, c);
  wf<T> r;
  r.c[0] = a.e * v12 + v1b * v2.c[0] + v2c * v1.c[0];
  r.c[1] = a.x * v12 + v1b * v2.c[1] + v2c * v1.c[1];
  r.c[2] = a.y * v12 + v1b * v2.c[2] + v2c * v1.c[2];
  r.c[3] = a.z * v12 + v1b * v2.c[3] + v2c * v1.c[3];
  return r;
}

// ------------------------------------------------------------------- VVVV
// L = gg {(V1*.V4*)(V2*.V3*) - (V1*.V3*)(V2*.V4*)}  (Sec. 4.2.4); for gluons the
// effective strength gg is g_s^2 (passed already squared).
template <class T>
__device__ __forceinline__ cx<T> ggggxx(const wf<T>& v1, const wf<T>& v2, const wf<T>& v3, const wf<T>& v4, T gg) {
  return gg * (dot(v1, v4) * dot(v2, v3) - dot(v1, v3) * dot(v2, v4));
}
// ggggxx is linear in each input: ggggxx(v1, v2, v3, v4) = dot(v4, gggg_r4(v1, v2, v3))
// = dot(v2, gggg_r2(v1, v3, v4)).
template <class T>
__device__ __forceinline__ wf<T> gggg_r4(const wf<T>& v1, const wf<T>& v2, const wf<T>& v3, T gg) {
  const cx<T> a = gg * dot(v2, v3), b = gg * dot(v1, v3);
  return {{a * v1.c[0] - b * v2.c[0], a * v1.c[1] - b * v2.c[1], a * v1.c[2] - b * v2.c[2],
           a * v1.c[3] - b * v2.c[3]}};
}
template <class T>
__device__ __forceinline__ wf<T> gggg_r2(const wf<T>& v1, const wf<T>& v3, const wf<T>& v4, T gg) {
  const cx<T> a = gg * dot(v1, v4), b = gg * dot(v1, v3);
  return {{a * v3.c[0] - b * v4.c[0], a * v3.c[1] - b * v4.c[1], a * v3.c[2] - b * v4.c[2],
           a * v3.c[3] - b * v4.c[3]}};
}
// V4 current (jgggxx): A = gg {V1 (V2.V3) - V2 (V1.V3)}, propagated
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jgggxx(const wf<T>& v1, const wf<T>& v2, const wf<T>& v3, T gg, vec<T> q,
                                        cx<T> inv_m2, cx<T> dinv) {
  const cx<T> a = gg * dot(v2, v3), b = gg * dot(v1, v3);
  wf<T> A;
#pragma unroll
  for (int m = 0; m < 4; ++m) A.c[m] = a * v1.c[m] - b * v2.c[m];
  return vector_prop<T, MASSIVE>(A, q, inv_m2, dinv);
}
// Weak quartic vertex as the sum of two identical-field terms (Sec. 4.2.4):
// Gamma(gw2; V1, V2, V3, V4) + Gamma(gw2; V1, V4, V3, V2) with the overall
// coupling gw2 (-g_W^2 for W-W+W-W+, +g_W^2 for W-W3W+W3 channels)
template <class T>
__device__ __forceinline__ cx<T> wwwwxx(const wf<T>& v1, const wf<T>& v2, const wf<T>& v3, const wf<T>& v4, T gw2) {
  return ggggxx(v1, v2, v3, v4, gw2) + ggggxx(v1, v4, v3, v2, gw2);
}
// current of leg 4 from the same two terms
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jwwwxx(const wf<T>& v1, const wf<T>& v2, const wf<T>& v3, T gw2, vec<T> q,
                                        cx<T> inv_m2, cx<T> dinv) {
  // d/dV4 of gw2[(V1.V4)(V2.V3) - (V1.V3)(V2.V4)] + gw2[(V1.V2)(V4.V3) - (V1.V3)(V4.V2)]
  const cx<T> v23 = dot(v2, v3), v13 = dot(v1, v3), v12 = dot(v1, v2);
  wf<T> A;
#pragma unroll
  for (int m = 0; m < 4; ++m)
    A.c[m] = gw2 * (v23 * v1.c[m] - v13 * v2.c[m] + v12 * v3.c[m] - v13 * v2.c[m]);
  return vector_prop<T, MASSIVE>(A, q, inv_m2, dinv);
}

// -------------------------------------------------------------------- VVS
// L = gc (V1*.V2*) S*  (Sec. 4.2.5)
template <class T>
__device__ __forceinline__ cx<T> vvsxxx(const wf<T>& v1, const wf<T>& v2, cx<T> sc, cx<T> gc) {
  return gc * dot(v1, v2) * sc;
}
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jvsxxx(const wf<T>& vc, cx<T> sc, cx<T> gc, vec<T> q, cx<T> inv_m2, cx<T> dinv) {
  const cx<T> k = gc * sc;
  wf<T> A;
#pragma unroll
  for (int m = 0; m < 4; ++m) A.c[m] = k * vc.c[m];
  return vector_prop<T, MASSIVE>(A, q, inv_m2, dinv);
}
template <class T>
__device__ __forceinline__ cx<T> hvvxxx(const wf<T>& v1, const wf<T>& v2, cx<T> gc, cx<T> dinv) {
  return -(gc * dot(v1, v2) * dinv);
}

// ------------------------------------------------------------------- VVSS
// L = gc (V1*.V2*) S3* S4*  (Sec. 4.2.6)
template <class T>
__device__ __forceinline__ cx<T> vvssxx(const wf<T>& v1, const wf<T>& v2, cx<T> s1, cx<T> s2, cx<T> gc) {
  return gc * dot(v1, v2) * s1 * s2;
}
// The vector bra of a VVS or VVSS amplitude: vvsxxx(v1, v2, s, gc) =
// vec_dot(vs_bra(v1, gc s), v2) and vvssxx(v1, v2, s1, s2, gc) =
// vec_dot(vs_bra(v1, gc s1 s2), v2).  Lets a loop nest form k v1 once in an
// outer loop and contract it (or a sum of such bras) with many v2.
template <class T>
__device__ __forceinline__ wf<T> vs_bra(const wf<T>& v, cx<T> k) {
  return {{k * v.c[0], k * v.c[1], k * v.c[2], k * v.c[3]}};
}
template <class T>
__device__ __forceinline__ cx<T> vec_dot(const wf<T>& b, const wf<T>& v) {
  return dot(b, v);
}
template <class T, bool MASSIVE>
__device__ __forceinline__ wf<T> jvssxx(const wf<T>& vc, cx<T> s1, cx<T> s2, cx<T> gc, vec<T> q, cx<T> inv_m2,
                                        cx<T> dinv) {
  const cx<T> k = gc * s1 * s2;
  wf<T> A;
#pragma unroll
  for (int m = 0; m < 4; ++m) A.c[m] = k * vc.c[m];
  return vector_prop<T, MASSIVE>(A, q, inv_m2, dinv);
}
template <class T>
__device__ __forceinline__ cx<T> hvvsxx(const wf<T>& v1, const wf<T>& v2, cx<T> sc, cx<T> gc, cx<T> dinv) {
  return -(gc * dot(v1, v2) * sc * dinv);
}

// ------------------------------------------------------------ SSS and SSSS
// L = gc S1* S2* S3*  and  L = gc S1* S2* S3* S4*  (Sec. 4.2.7, 4.2.8)
template <class T>
__device__ __forceinline__ cx<T> sssxxx(cx<T> s1, cx<T> s2, cx<T> s3, cx<T> gc) { return gc * s1 * s2 * s3; }
template <class T>
__device__ __forceinline__ cx<T> hssxxx(cx<T> s1, cx<T> s2, cx<T> gc, cx<T> dinv) { return -(gc * s1 * s2 * dinv); }
template <class T>
__device__ __forceinline__ cx<T> ssssxx(cx<T> s1, cx<T> s2, cx<T> s3, cx<T> s4, cx<T> gc) {
  return gc * s1 * s2 * s3 * s4;
}
template <class T>
__device__ __forceinline__ cx<T> hsssxx(cx<T> s1, cx<T> s2, cx<T> s3, cx<T> gc, cx<T> dinv) {
  return -(gc * s1 * s2 * s3 * dinv);
}

}  // namespace heget
