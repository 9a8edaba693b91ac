"""Process IR -> straight-line HIP kernel for gfx950.

The generated kernel evaluates one event per lane (the paper's one
phase-space point per thread, Sec. 3): momenta (loaded, or Philox + RAMBO),
the generation cut, then the helicity loop with the call list unrolled as
straight-line code, the jamps and the colour quadratic form (Sec. 5.4).

Choices made here rather than in the paper's generated CUDA:
 * momenta, internal-line momenta and every propagator denominator depend on
   the event but not on the helicity, so they are formed once per event in FP64
   before the helicity loop (in both precisions);
 * temporaries are plain SSA values, so the compiler's register allocator does
   the recycling of temporary wavefunctions the paper did by hand (Sec. 5.5);
 * colour factors and the colour matrix are compile-time constants.

Usage:  python -m paper_1305_0708_amd.codegen <out_dir>   (writes one .hip per process)
"""
import os
import sys
from fractions import Fraction

from . import ir
from .ir import F, V, S, AMP_OPS, P_ZERO, P_W, P_Z, P_TOP, P_H

MASSIVE_VECTORS = {P_W, P_Z}


def _c(x):
    return repr(float(x))


def _coef_expr(c, a):
    """coefficient * amplitude with the trivial cases spelled out"""
    c = complex(c)
    if c == 1:
        return a
    if c == -1:
        return f"(-{a})"
    if c == 1j:
        return f"times_i({a})"
    if c == -1j:
        return f"times_mi({a})"
    if c.imag == 0:
        return f"(T({_c(c.real)}) * {a})"
    return f"(mk<T>(T({_c(c.real)}), T({_c(c.imag)})) * {a})"


class Gen:
    def __init__(self, proc: ir.Process):
        self.p = proc
        self.nl = proc.n_legs
        self.nout = proc.n_legs - 2
        self.kind = {i: leg.kind for i, leg in enumerate(proc.legs)}
        self.prop = {}
        for c in proc.calls:
            if c.op not in AMP_OPS:
                self.kind[c.out] = ir.OUT_KIND[c.op]
                self.prop[c.out] = c.prop
        # momentum of each slot as a set of external legs (q = sum over legs of q_leg)
        self.legs_of = {i: (i,) for i in range(self.nl)}
        for c in proc.calls:
            if c.op not in AMP_OPS:
                s = []
                for x in c.ins:
                    s.extend(self.legs_of[x])
                self.legs_of[c.out] = tuple(sorted(s))
        # slots whose vec<T> momentum is needed inside the helicity loop
        self.need_q = set()
        for c in proc.calls:
            if c.op in ("fvi", "fvo", "fsi", "fso", "jio", "jvv", "jggg", "jwww", "jvs", "jvss"):
                self.need_q.add(c.out)
            if c.op in ("vvv", "jvv"):
                self.need_q.update(c.ins)

    # ------------------------------------------------------------ emission
    def name(self):
        return self.p.name

    def emit(self):
        p = self.p
        L = []
        w = L.append
        fp = p.fingerprint()
        w(f"// Generated from the process IR '{p.name}' (fingerprint 0x{fp:016x}); do not edit.")
        w('#include "../generated_common.hpp"')
        w("")
        w("namespace heget {")
        w("namespace {")
        w("")
        w("template <class T>")
        w(f"__global__ __launch_bounds__(256) void amp_{p.name}(KernelArgs a) {{")
        w("  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;")
        w("  const bool active = i < a.n;")
        w(f"  mom p[{self.nl}];")
        w("  if (active) {")
        w("    if (a.mom_in) {")
        w(f"#pragma unroll")
        w(f"      for (int k = 0; k < {self.nl}; ++k) {{")
        w("        const double* b = a.mom_in + int64_t(k) * 4 * a.mom_stride + i;")
        w("        p[k] = {b[0], b[a.mom_stride], b[2 * a.mom_stride], b[3 * a.mom_stride]};")
        w("      }")
        w("    } else {")
        w("      const double h = 0.5 * a.sqrt_s;")
        w("      p[0] = {h, 0.0, 0.0, h};")
        w("      p[1] = {h, 0.0, 0.0, -h};")
        w(f"      rambo<{self.nout}>(a.seed, a.counter_offset + uint64_t(i), a.sqrt_s, p + 2);")
        w("    }")
        w("    if (a.mom_out) store_momenta<%d>(a, i, p);" % self.nl)
        w("  } else {")
        w(f"#pragma unroll")
        w(f"    for (int k = 0; k < {self.nl}; ++k) p[k] = {{1.0, 0.0, 0.0, 1.0}};")
        w("  }")
        if p.cut_enabled:
            w(f"  const bool pass = active && (!a.cut_enabled || pass_pt_dr<{self.nout}>(p + 2, a.cut_pt, a.cut_dr));")
        else:
            w("  const bool pass = active;")
        # couplings (uniform values, loaded once)
        w("  // couplings (uniform)")
        for k, c in enumerate(p.couplings):
            w(f"  const cx<T> g{k}_0 = mk<T>(T(a.cpl[{4 * k}]), T(a.cpl[{4 * k + 1}]));")
            w(f"  const cx<T> g{k}_1 = mk<T>(T(a.cpl[{4 * k + 2}]), T(a.cpl[{4 * k + 3}]));")
        used_parts = sorted({pp for pp in self.prop.values()} | {leg.particle for leg in p.legs})
        for pid in used_parts:
            w(f"  const PropEntry pe{pid} = a.prop[{pid}];")
        # momenta flowing into the diagram: q = p (incoming) or -p (outgoing)
        w("  // incoming-flow momenta of every slot (FP64) and inverse denominators")
        for k, leg in enumerate(p.legs):
            w(f"  const mom q{k} = {'p[%d]' % k if leg.incoming else '-p[%d]' % k};")
        for c in p.calls:
            if c.op in AMP_OPS:
                continue
            s = c.out
            terms = " + ".join(f"q{x}" for x in c.ins)
            w(f"  const mom q{s} = {terms};")
            pid = c.prop
            w(f"  const cx<T> d{s} = cvt<T>(inv_denominator(q{s}, cx<double>{{pe{pid}.pole_r, pe{pid}.pole_i}}));")
        for s in sorted(self.need_q):
            w(f"  const vec<T> Q{s} = tv<T>(q{s});")
        for k, leg in enumerate(p.legs):
            if leg.kind == F and leg.particle == P_ZERO:
                # helicity-independent Weyl factors, formed in FP64
                w(f"  const MLF<T> e{k} = mlf_pre<T>(p[{k}]);")
            elif leg.kind == F:
                # massive external fermion: both helicity states in FP64
                fn = "ixxxxx" if self._flowing_in(leg) else "oxxxxx"
                for lam, tag in ((-1, "m"), (1, "p")):
                    w(f"  const wf<T> e{k}{tag} = cvtw<T>({fn}<double, false>(tv<double>(p[{k}]), "
                      f"pe{leg.particle}.m, {lam}, {leg.flow}));")
            elif leg.kind == V:
                w(f"  const vec<T> P{k} = tv<T>(p[{k}]);")
        w("  double me2 = 0.0;")
        w("  if (pass) {")
        w("    for (int h = 0; h < a.n_hel; ++h) {")
        w(f"      const int8_t* hh = a.hel + h * {self.nl};")
        for k, leg in enumerate(p.legs):
            self._external(w, k, leg)
        for c in p.calls:
            self._call(w, c)
        self._colour(w)
        w("    }")
        w("  }")
        w("  if (a.me2_out && active) a.me2_out[i] = me2;")
        w("  if (a.partials) block_partials(a, pass ? me2 * a.weight_factor : 0.0, pass);")
        w("}")
        w("")
        w("}  // namespace")
        w("")
        cfg = (f'static const GenEntry entry = {{0x{fp:016x}ull, "{p.name}", {self.nl}, '
               f'reinterpret_cast<const void*>(&amp_{p.name}<double>), '
               f'reinterpret_cast<const void*>(&amp_{p.name}<float>)}};')
        w(cfg)
        w("static const Registrar reg(&entry);")
        w("")
        w("}  // namespace heget")
        return "\n".join(L) + "\n"

    @staticmethod
    def _flowing_in(leg):
        return (leg.incoming and leg.flow > 0) or ((not leg.incoming) and leg.flow < 0)

    def _external(self, w, k, leg):
        if leg.kind == F:
            if leg.particle == P_ZERO:
                fn = "ixxxxx0" if self._flowing_in(leg) else "oxxxxx0"
                w(f"      const wf<T> w{k} = {fn}<T>(e{k}, hh[{k}], {leg.flow});")
            else:
                w(f"      const wf<T> w{k} = hh[{k}] > 0 ? e{k}p : e{k}m;")
        elif leg.kind == V:
            nsv = -1 if leg.incoming else 1
            w(f"      const wf<T> w{k} = vxxxxx<T>(P{k}, T(pe{leg.particle}.m), hh[{k}], {nsv});")
        else:
            w(f"      const cx<T> w{k} = sxxxxx<T>();")

    def _call(self, w, c):
        op, ins, o = c.op, c.ins, c.out
        g0, g1 = f"g{c.cpl}_0", f"g{c.cpl}_1"
        gr = f"g{c.cpl}_0.r"
        pid = c.prop
        mass = f"T(pe{pid}.m)"
        inum = f"mk<T>(T(pe{pid}.inum_r), T(pe{pid}.inum_i))"
        massive = "true" if pid in MASSIVE_VECTORS else "false"
        a = [f"w{x}" for x in ins]
        if op in AMP_OPS:
            lhs = f"      const cx<T> amp{o} = "
        elif ir.OUT_KIND[op] == S:
            lhs = f"      const cx<T> w{o} = "
        else:
            lhs = f"      const wf<T> w{o} = "
        d = f"d{o}"
        if op == "iov":
            rhs = f"iovxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {g1})"
        elif op == "fvi":
            rhs = f"fvixxx<T>({a[0]}, {a[1]}, {g0}, {g1}, Q{o}, {mass}, {d})"
        elif op == "fvo":
            rhs = f"fvoxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, Q{o}, {mass}, {d})"
        elif op == "jio":
            rhs = f"jioxxx<T, {massive}>({a[0]}, {a[1]}, {g0}, {g1}, Q{o}, {inum}, {d})"
        elif op == "ios":
            rhs = f"iosxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {g1})"
        elif op == "fsi":
            rhs = f"fsixxx<T>({a[0]}, {a[1]}, {g0}, {g1}, Q{o}, {mass}, {d})"
        elif op == "fso":
            rhs = f"fsoxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, Q{o}, {mass}, {d})"
        elif op == "hio":
            rhs = f"hioxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {d})"
        elif op == "vvv":
            q = [f"Q{x}" for x in ins]
            rhs = f"vvvxxx<T>({a[0]}, {q[0]}, {a[1]}, {q[1]}, {a[2]}, {q[2]}, {gr})"
        elif op == "jvv":
            q = [f"Q{x}" for x in ins]
            rhs = f"jvvxxx<T, {massive}>({a[0]}, {q[0]}, {a[1]}, {q[1]}, {gr}, {inum}, {d})"
        elif op == "gggg":
            rhs = f"ggggxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {gr})"
        elif op == "jggg":
            rhs = f"jgggxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {gr}, Q{o}, {inum}, {d})"
        elif op == "wwww":
            rhs = f"wwwwxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {gr})"
        elif op == "jwww":
            rhs = f"jwwwxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {gr}, Q{o}, {inum}, {d})"
        elif op == "vvs":
            rhs = f"vvsxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0})"
        elif op == "jvs":
            rhs = f"jvsxxx<T, {massive}>({a[0]}, {a[1]}, {g0}, Q{o}, {inum}, {d})"
        elif op == "hvv":
            rhs = f"hvvxxx<T>({a[0]}, {a[1]}, {g0}, {d})"
        elif op == "vvss":
            rhs = f"vvssxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {g0})"
        elif op == "jvss":
            rhs = f"jvssxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {g0}, Q{o}, {inum}, {d})"
        elif op == "hvvs":
            rhs = f"hvvsxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {d})"
        elif op == "sss":
            rhs = f"sssxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0})"
        elif op == "hss":
            rhs = f"hssxxx<T>({a[0]}, {a[1]}, {g0}, {d})"
        elif op == "ssss":
            rhs = f"ssssxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {g0})"
        elif op == "hsss":
            rhs = f"hsssxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {d})"
        else:
            raise ValueError(op)
        w(lhs + rhs + ";")

    def _colour(self, w):
        p = self.p
        for f, terms in enumerate(p.jamp):
            expr = " + ".join(_coef_expr(cc, f"amp{ai}") for ai, cc in terms) or "mk<T>(T(0), T(0))"
            w(f"      const cx<T> J{f} = {expr};")
        den = p.colour_denominator()
        parts = []
        n = p.n_flows
        for f in range(n):
            cff = Fraction(p.colour[f][f]) * den
            parts.append(f"T({_c(cff)}) * norm2(J{f})")
            for g in range(f + 1, n):
                cfg = Fraction(p.colour[f][g]) * den
                if cfg != 0:
                    parts.append(f"T({_c(2 * cfg)}) * (J{f}.r * J{g}.r + J{f}.i * J{g}.i)")
        w(f"      const T cs = {' + '.join(parts)};")
        w(f"      me2 += double(cs) * {_c(Fraction(1, den))};")


def generate(proc, out_dir):
    g = Gen(proc)
    src = g.emit()
    path = os.path.join(out_dir, f"gen_{proc.name}.hip")
    old = open(path).read() if os.path.exists(path) else None
    if old != src:
        with open(path, "w") as f:
            f.write(src)
    return path


def main(argv):
    from . import processes
    out = argv[1] if len(argv) > 1 else os.path.join(os.path.dirname(__file__), "csrc", "gen")
    os.makedirs(out, exist_ok=True)
    for name in ("ee_mumu", "gg_ttbar_6f", "ud_udhh_4b"):
        print(generate(processes.by_name(name), out))


if __name__ == "__main__":
    main(sys.argv)
