"""Process IR -> HIP kernel for gfx950.

The generated kernel evaluates one event per lane (the paper's one
phase-space point per thread, Sec. 3): momenta (loaded, or Philox + RAMBO),
the generation cut, then the helicity loop over the IR's calls, the jamps and
the colour quadratic form (Sec. 5.4).

Two forms:
 * straight-line: every call of the IR unrolled once per helicity; the
   momenta of internal lines and every propagator denominator are event
   properties, formed once in FP64 before the helicity loop;
 * ordering template (colour-ordered processes): the calls are a template over
   leg positions, run once per ordering inside a non-unrolled loop with the
   positions bound to the permuted external wavefunctions; each ordering's
   jamp is staged in LDS and the colour form reads them back.  This bounds the
   code size and the live currents to those of one ordering, where the paper
   split long amplitude programs into successive calls (Sec. 5.3).

Temporaries are SSA values, so the compiler's register allocator recycles
them (the paper did this by hand, Sec. 5.5).  Colour factors and the colour
matrix are compile-time constants.
"""
import os
import sys
from fractions import Fraction

from . import ir, nest
from .ir import F, V, S, AMP_OPS, LINEAR_OPS, P_ZERO, P_W, P_Z

MASSIVE_VECTORS = {P_W, P_Z}
# ordering templates: recompute the momenta and denominators a call needs in
# the loop of the call instead of carrying them from the loop that first formed them
TEMPLATE_KIN_PER_LEVEL = True
# ordering templates: per-lane LDS words (in the arithmetic type) for currents
# that outer helicity loops form and inner loops read (shared with the colour
# form's amplitude rows, which are used after the orderings).  FP64 only: the
# FP32 kernels hold these currents in registers without spilling, and there
# the opaque reads cost more than they save.
TEMPLATE_STASH_WORDS = 48
# ordering templates: each vertex vector of the running sum R is added right
# after the last of its operands is formed in the sum's loop (first, when all
# come from outer loops), so that the currents it reads can die early
TEMPLATE_EARLY_VERTEX_SUM = True
# ordering templates: the same for the sums of partial currents (vadd, vsub) in
# every loop, so that a current's terms are accumulated as they are formed
TEMPLATE_EARLY_CURRENT_SUMS = True
# MFMA colour form: 16-event chunks of a wave per pass (each fragment load serves them all)
COLOUR_CHUNKS = 2
# MFMA colour form: the fragments of the triangle held in registers for the whole
# colour-form phase (loaded once per block of events) instead of streamed from L2
# for every chunk and helicity
COLOUR_RESIDENT = True
# amplitude rows of the MFMA colour form above this many bytes (FP64) are not
# staged in LDS: the workspace holds them in the colour form's layout
DIRECT_ROWS_BYTES = 128 * 1024
# per-lane LDS words (in the arithmetic type) of the helicity nest's stash of
# event kinematics: 64 words are 128 KiB per 256-lane block in FP64
STASH_WORDS = 64
# per-lane LDS words (arithmetic type) of the inner table of the FP32 kernels:
# the values of the unrolled innermost loops that depend on no real loop,
# formed once before the loops for every combination of the unrolled
# helicities and read from LDS inside them (the FP64 kernels leave them to the
# compiler, which hoists them into registers: faster there); the stash takes
# what is left of NEST_LDS_WORDS
INNER_TABLE_WORDS = 64
NEST_LDS_WORDS = 72
_KIN_WORDS = {"vec<T>": 4, "cx<T>": 2, "MLF<T>": 8, "wf<T>": 8, "VPol<T>": 5}


def _c(x):
    return repr(float(x))


def _coef_expr(c, a):
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


def _coupling_decls(k, kind, ind="  "):
    """the two coupling values of coupling k, with the parts that the
    library's coupling of this kind fixes at zero (or equal) as constants"""
    im = lambda j: f"T(a.cpl[{4 * k + j}])" if kind in ir.CPL_COMPLEX else "T(0)"
    g0 = f"{ind}const cx<T> g{k}_0 = mk<T>(T(a.cpl[{4 * k}]), {im(1)});"
    if kind in ir.CPL_G1_EQ_G0:
        g1 = f"{ind}const cx<T> g{k}_1 = g{k}_0;"
    elif kind in ir.CPL_G1_FREE:
        g1 = f"{ind}const cx<T> g{k}_1 = mk<T>(T(a.cpl[{4 * k + 2}]), {im(3)});"
    else:
        g1 = f"{ind}const cx<T> g{k}_1 = mk<T>(T(0), T(0));"
    return [g0, g1]


def _flowing_in(leg):
    return (leg.incoming and leg.flow > 0) or ((not leg.incoming) and leg.flow < 0)


class Gen:
    def __init__(self, proc: ir.Process):
        self.p = proc
        self._scope, self._opaque = None, set()
        self._kin = {}       # event kinematics formed before the helicity loops: name -> type
        self.nl = proc.n_legs
        self.nout = proc.n_legs - 2
        self.ordered = proc.orderings is not None
        # a linear combination carries the momentum of its first input
        self.mslot = {}
        for c in proc.calls:
            if c.op in LINEAR_OPS:
                self.mslot[c.out] = self.mslot.get(c.ins[0], c.ins[0])
        # external legs (or positions) whose momenta a slot carries
        self.subset = {k: (k,) for k in range(self.nl)}
        for c in proc.calls:
            if c.op in LINEAR_OPS:
                self.subset[c.out] = self.subset[c.ins[0]]
            elif c.op not in AMP_OPS:
                self.subset[c.out] = tuple(sorted(x for i in c.ins for x in self.subset[i]))
        self.need_q = set()    # subsets whose vec<T> momentum the calls use
        for c in proc.calls:
            if c.op in ("fvi", "fvo", "fsi", "fso", "jio", "jvv", "jggg", "jwww", "jvs", "jvss"):
                self.need_q.add(self.subset[c.out])
            if c.op in ("vvv", "jvv"):
                self.need_q.update(self.subset[x] for x in c.ins)

    def cterm_cap(self):
        """words of the MFMA colour form's term table: flows sorted (stably) by
        their number of flow-map terms, each k-step of four flows padded to its
        longest row, four words per term row"""
        p = self.p
        rows = p.flow_map if p.flow_map is not None else [[1 if o == f else 0 for o in range(len(p.orderings))]
                                                          for f in range(p.n_flows)]
        nnz = sorted(sum(1 for x in r if x) for r in rows)
        return 4 * sum(max(nnz[4 * s:4 * s + 4]) for s in range((len(nnz) + 3) // 4))

    def m(self, s):
        return self.mslot.get(s, s)

    @staticmethod
    def sname(sub):
        return "_".join(str(x) for x in sub)

    # ---------------------------------------------------------------- common
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
        tree = p.ps_tree is not None
        if tree:
            self._emit_ps_tree(w)
        if p.helicity_schedule == "rows":
            self._emit_row_parts(w)
        split = p.division == "split"
        self._split = split
        if split:
            w("// PHASE 0: the whole program; 1: the orderings' amplitudes only (to the")
            w("// workspace); 2: the colour form and the outputs only (from the workspace)")
            w("template <class T, int PHASE = 0>")
        else:
            w("template <class T>")
        w(f"__device__ __forceinline__ void body_{p.name}(const KernelArgs& a, int64_t blk) {{")
        w("  const int64_t i = blk * blockDim.x + threadIdx.x;")
        w("  const bool active = i < a.n;")
        w(f"  mom p[{self.nl}];")
        if tree:
            w("  double psw = 1.0;   // phase-space weight of a generated event (resonance tree)")
        w("  if (active) {")
        w("    if (a.mom_in) {")
        w("#pragma unroll")
        w(f"      for (int k = 0; k < {self.nl}; ++k) {{")
        w("        const double* b = a.mom_in + int64_t(k) * 4 * a.mom_stride + i;")
        w("        p[k] = {b[0], b[a.mom_stride], b[2 * a.mom_stride], b[3 * a.mom_stride]};")
        w("      }")
        w("    } else {")
        w("      const double h = 0.5 * a.sqrt_s;")
        w("      p[0] = {h, 0.0, 0.0, h};")
        w("      p[1] = {h, 0.0, 0.0, -h};")
        if tree:
            w(f"      psw = ps_tree_{p.name}(a, a.counter_offset + uint64_t(i), i, p);")
        else:
            w(f"      rambo<{self.nout}>(a.seed, a.counter_offset + uint64_t(i), a.sqrt_s, p + 2);")
        w("    }")
        if split:
            w("    if (PHASE != 2 && a.mom_out) store_momenta<%d>(a, i, p);" % self.nl)
        else:
            w("    if (a.mom_out) store_momenta<%d>(a, i, p);" % self.nl)
        w("  } else {")
        w("#pragma unroll")
        w(f"    for (int k = 0; k < {self.nl}; ++k) p[k] = {{1.0, 0.0, 0.0, 1.0}};")
        w("  }")
        live = "active && psw > 0.0" if tree else "active"
        if p.cut_enabled:
            w(f"  const bool pass = {live} && (!a.cut_enabled || pass_pt_dr<{self.nout}>(p + 2, a.cut_pt, a.cut_dr));")
        else:
            w(f"  const bool pass = {live};")
        w("  // couplings and propagator data (uniform)")
        for k, c in enumerate(p.couplings):
            for line in _coupling_decls(k, c.kind):
                w(line)
        used = sorted({c.prop for c in p.calls} | {leg.particle for leg in p.legs} | {P_ZERO})
        for pid in used:
            w(f"  const PropEntry pe{pid} = a.prop[{pid}];")
        w("  // momenta flowing into the diagram: +p incoming, -p outgoing (FP64)")
        for k, leg in enumerate(p.legs):
            w(f"  const mom q{k} = {'p[%d]' % k if leg.incoming else '-p[%d]' % k};")
        if self.ordered:
            w(f"  // the event's momenta flowing into the diagram, in LDS: read per ordering and")
            w(f"  // loop, not held in registers")
            w(f"  __shared__ mom pm[{self.nl}][256];")
            for k in range(self.nl):
                w(f"  pm[{k}][threadIdx.x] = q{k};")
            self._emit_ordered(w)
        else:
            self._emit_straight(w)
        if split:
            w("  if constexpr (PHASE != 1) {")
        w("  if (a.me2_out && active) a.me2_out[i] = me2;")
        if tree:
            w("  if (a.w_out && active) a.w_out[i] = pass ? me2 * a.weight_factor * psw : 0.0;")
        w(f"  if (a.partials) block_partials(a, blk, pass ? me2 * a.weight_factor{' * psw' if tree else ''} : 0.0, pass);")
        if split:
            w("  }")
        w("}")
        w("")
        # One kernel per arithmetic type serves a launch of one request and the
        # serving engine's fused launches: a grid-stride loop over virtual blocks
        # takes the launch's own blocks, or the batch table's segments when the
        # launch carries one.  The body has this single call site, so a request
        # gets the same compiled code, and the same bits, alone and in a mix.
        w("// one launch: the grid walks the 256-event blocks of the launch (persistent")
        w("// kernels: one workspace slot per block), or, for a fused launch of the")
        w("// serving engine, the virtual blocks of its batch table")
        w("template <class T>")
        w64, w32 = p.waves_per_simd, p.waves_per_simd_mixed or p.waves_per_simd
        if w64 != w32:
            # the FP64 and the FP32 kernel compiled for different occupancies
            lb = f"256, sizeof(T) == 8 ? {w64} : {w32}"
        else:
            lb = f"256, {w64}" if w64 > 1 else "256"
        w(f"__global__ __launch_bounds__({lb}) void amp_{p.name}(KernelArgs a) {{")
        if p.uses_colour_mfma():
            w(f"  colour_stage<T, {(p.n_flows + 3) // 4}, {(p.n_flows + 15) // 16}, {self.cterm_cap()}>(a);")
        w("  const BatchTable* bt = a.batch;")
        w("  const int64_t total = bt ? bt->total_blocks : (a.n + 255) / 256;")
        w("  const int nseg = bt ? bt->n_seg : 0;")
        w("  int s = 0;")
        w("  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {")
        w("    KernelArgs b = a;")
        w("    int64_t blk = vb;")
        w("    if (bt) {")
        w("      while (s + 1 < nseg && bt->seg[s + 1].block_begin <= vb) ++s;")
        w("      b = segment_args(a, bt->seg[s]);")
        w("      blk = bt->seg[s].block_offset + (vb - bt->seg[s].block_begin);")
        w("    }")
        w(f"    body_{p.name}<T>(b, blk);")
        w("    __syncthreads();")
        w("  }")
        w("}")
        if split:
            w("")
            w("// split division: block b of a round evaluates block block_base + b of the")
            w("// launch into workspace slot b (the orderings' amplitudes), then the")
            w("// colour-form kernel of the same round reads that slot")
            w("template <class T>")
            w(f"__global__ __launch_bounds__(256) void amp_{p.name}_chain(KernelArgs a) {{")
            w(f"  body_{p.name}<T, 1>(a, a.block_base + blockIdx.x);")
            w("}")
            w("template <class T>")
            w(f"__global__ __launch_bounds__(256) void amp_{p.name}_colour(KernelArgs a) {{")
            if p.uses_colour_mfma():
                w(f"  colour_stage<T, {(p.n_flows + 3) // 4}, {(p.n_flows + 15) // 16}, {self.cterm_cap()}>(a);")
            w(f"  body_{p.name}<T, 2>(a, a.block_base + blockIdx.x);")
            w("}")
        w("")
        if tree:
            w("// the phase-space step alone (heget_generate): momenta and per-event weights")
            w(f"__global__ __launch_bounds__(256) void gen_{p.name}(KernelArgs a) {{")
            w("  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;")
            w("  if (i >= a.n) return;")
            w(f"  mom p[{self.nl}];")
            w(f"  const double w = ps_tree_{p.name}(a, a.counter_offset + uint64_t(i), i, p);")
            w(f"  store_momenta<{self.nl}>(a, i, p);")
            w("  if (a.psw_out) a.psw_out[i] = w;")
            w("}")
            w("")
        w("}  // namespace")
        w("")
        mf = p.uses_colour_mfma()
        nks, nfo = ((p.n_flows + 3) // 4, (p.n_flows + 15) // 16) if mf else (0, 0)
        if p.helicity_schedule == "rows":
            # no loop nest: every table is summed row by row
            canon, n_canon = "nullptr", 0
        else:
            rows = ir.all_helicities(p.legs)
            flat = ", ".join(str(h) for row in rows for h in row)
            w(f"// the full helicity product in canonical order: tables equal to it run the loop nest")
            w(f"static const int8_t hel_canon[] = {{{flat}}};")
            canon, n_canon = "hel_canon", len(rows)
        w(f'static const GenEntry entry = {{0x{fp:016x}ull, "{p.name}", {self.nl}, '
          f'reinterpret_cast<const void*>(&amp_{p.name}<double>), '
          f'reinterpret_cast<const void*>(&amp_{p.name}<float>), {int(mf)}, {nks}, {nfo}, '
          f'reinterpret_cast<const void*>(&amp_{p.name}<double>), '
          f'reinterpret_cast<const void*>(&amp_{p.name}<float>), {canon}, {n_canon}, '
          f'{int(self.ordered)}, {self.cterm_cap() if mf else 0}, '
          f'{f"reinterpret_cast<const void*>(&gen_{p.name})" if tree else "nullptr"}, {self.ps_dims()}, '
          f'{int(p.mixed_uses_mfma())}, '
          + (f'reinterpret_cast<const void*>(&amp_{p.name}_chain<double>), '
             f'reinterpret_cast<const void*>(&amp_{p.name}_chain<float>), '
             f'reinterpret_cast<const void*>(&amp_{p.name}_colour<double>), '
             f'reinterpret_cast<const void*>(&amp_{p.name}_colour<float>)'
             if p.division == "split" else 'nullptr, nullptr, nullptr, nullptr') + '};')
        w("static const Registrar reg(&entry);")
        w("")
        w("}  // namespace heget")
        return "\n".join(L) + "\n"

    def ps_dims(self):
        """uniforms per event of the resonance tree (0 without one)"""
        tree = self.p.ps_tree
        if tree is None:
            return 0
        return sum(1 for node in tree for d in node[2:4] if d < 0) + 2 * len(tree) + (2 if self.p.ps_hadronic else 0)

    def _emit_ps_tree(self, w):
        """the process's resonance phase space as straight-line device code:
        per node in index order, the invariant masses of its resonant
        daughters (first daughter first; ranges from the final legs' masses
        below each), then its two-body decay"""
        p = self.p
        tree = p.ps_tree
        nu = self.ps_dims()
        had = p.ps_hadronic
        if had:
            w(f"// phase space: a parton collision at a hadron collider (parton densities 1) and the two-body")
            w(f"// decays of its resonances (tree of {len(tree)} nodes); fills p[0 .. n_legs-1] and returns the")
            w("// event's weight dSigma_n / (2 s_hat)")
        else:
            w(f"// phase space: the collision and its resonances decay in two bodies (tree of {len(tree)} nodes);")
            w("// fills p[0 .. n_legs-1] and returns the event's weight dPhi_n")
        w(f"__device__ __forceinline__ double ps_tree_{p.name}(const KernelArgs& a, uint64_t event, int64_t i, mom* p) {{")
        w("#pragma clang fp contract(off)   // each product and sum rounds on its own (plain IEEE)")
        w(f"  double u[{nu}];")
        w(f"  ps_uniforms<{nu}>(a.seed, event, u);")
        beams = [p.legs[k].particle for k in (0, 1)]
        if all(b == P_ZERO for b in beams):
            w("  const double h = 0.5 * a.sqrt_s;")
            w("  p[0] = {h, 0.0, 0.0, h};")
            w("  p[1] = {h, 0.0, 0.0, -h};")
        else:
            # massive beams along +-z in the collision frame
            ma, mb = (f"a.prop[{b}].m" if b != P_ZERO else "0.0" for b in beams)
            w(f"  const double ma = {ma}, mb = {mb}, s0 = a.sqrt_s * a.sqrt_s;")
            w("  const double pz = sqrt(fmax((s0 - (ma + mb) * (ma + mb)) * (s0 - (ma - mb) * (ma - mb)), 0.0)) / "
              "(2.0 * a.sqrt_s);")
            w("  p[0] = {(s0 + ma * ma - mb * mb) / (2.0 * a.sqrt_s), 0.0, 0.0, pz};")
            w("  p[1] = {(s0 + mb * mb - ma * ma) / (2.0 * a.sqrt_s), 0.0, 0.0, -pz};")
        w("  // adaptive integration: the uniforms through the grid, its Jacobian in the weight")
        w(f"  double w = a.grid ? grid_map<{nu}>(a, i, u) : 1.0;")
        w("  const double M0 = a.sqrt_s;")
        w("  const mom P0 = {a.sqrt_s, 0.0, 0.0, 0.0};")
        def leg_mass(L):
            part = p.legs[L].particle
            return "0.0" if part == P_ZERO else f"a.prop[{part}].m"

        def min_mass(d):
            """minimal invariant mass of daughter d (final leg or node) as a sum of leg masses"""
            if d >= 0:
                return [leg_mass(d)] if leg_mass(d) != "0.0" else []
            node = tree[-1 - d]
            return min_mass(node[2]) + min_mass(node[3])

        def total(terms):
            return "(" + " + ".join(terms) + ")" if terms else "0.0"
        iu = 0
        for k, (_, _, d0, d1) in enumerate(tree):
            dm = {}
            for j, d in enumerate((d0, d1)):
                if d >= 0:
                    dm[j] = leg_mass(d)
                    continue
                nd = -1 - d
                part, mapping = tree[nd][0], tree[nd][1]
                other = dm[0] if j == 1 else total(min_mass(d1))
                hi = f"M{k} * M{k}" if other == "0.0" else f"(M{k} - {other}) * (M{k} - {other})"
                mine = total(min_mass(d))
                lo = "0.0" if mine == "0.0" else f"{mine} * {mine}"
                bw = "true" if mapping == ir.PS_BREIT_WIGNER else "false"
                w(f"  double s{nd};")
                w(f"  w *= ps_mass(u[{iu}], {lo}, {hi}, a.prop[{part}].m, a.prop[{part}].w, {bw}, "
                  f"{_c(p.ps_window)}, s{nd});")
                w(f"  const double M{nd} = sqrt(s{nd});")
                w(f"  mom P{nd};")
                dm[j] = f"M{nd}"
                iu += 1
            outs = [f"p[{d}]" if d >= 0 else f"P{-1 - d}" for d in (d0, d1)]
            if k == 0 and had:
                w(f"  w *= ps_hadronic(u + {iu}, a.sqrt_s, {dm[0]}, {dm[1]}, {_c(had[0])}, {_c(had[1])}, "
                  f"{outs[0]}, {outs[1]}, p[0], p[1]);")
                iu += 4
                continue
            w(f"  w *= ps_decay(u[{iu}], u[{iu + 1}], P{k}, M{k}, {dm[0]}, {dm[1]}, {'true' if k == 0 else 'false'}, "
              f"{outs[0]}, {outs[1]});")
            iu += 2
        assert iu == nu
        w("  return w;")
        w("}")
        w("")

    def _ext_pre(self, w):
        """helicity-independent pieces of the external wavefunctions"""
        for k, leg in enumerate(self.p.legs):
            if leg.kind == F and leg.particle == P_ZERO:
                w(f"  const MLF<T> e{k} = mlf_pre<T>(p[{k}]);")
                self._kin[f"e{k}"] = "MLF<T>"
            elif leg.kind == F:
                fn = "ixxxxx" if _flowing_in(leg) else "oxxxxx"
                for lam, tag in ((-1, "m"), (1, "p")):
                    w(f"  const wf<T> e{k}{tag} = cvtw<T>({fn}<double, false>(tv<double>(p[{k}]), "
                      f"pe{leg.particle}.m, {lam}, {leg.flow}));")
                    self._kin[f"e{k}{tag}"] = "wf<T>"
            elif leg.kind == V:
                w(f"  const vec<T> P{k} = tv<T>(p[{k}]);")
                self._kin[f"P{k}"] = "vec<T>"
                if leg.particle == P_ZERO:
                    w(f"  const VPol<T> V{k} = vpol_pre<T>(p[{k}]);")
                    self._kin[f"V{k}"] = "VPol<T>"

    def _external(self, k, leg, name, hel=None, nest=False):
        """external wavefunction; in the helicity nest a massless vector is
        built from its precomputed polarisation factors (helicities +-1 only)"""
        hel = hel or f"hh[{k}]"
        if leg.kind == F:
            if leg.particle == P_ZERO:
                fn = "ixxxxx0" if _flowing_in(leg) else "oxxxxx0"
                return f"const wf<T> {name} = {fn}<T>(e{k}, {hel}, {leg.flow});"
            return f"const wf<T> {name} = {hel} > 0 ? e{k}p : e{k}m;"
        if leg.kind == V:
            nsv = -1 if leg.incoming else 1
            if nest and leg.particle == P_ZERO:
                return f"const wf<T> {name} = vxxxxx0<T>(V{k}, {hel}, {nsv});"
            return f"const wf<T> {name} = vxxxxx<T>(P{k}, T(pe{leg.particle}.m), {hel}, {nsv});"
        return f"const cx<T> {name} = sxxxxx<T>();"

    def _current_momenta(self, w, ind, qname):
        """FP64 momentum of every leg subset an internal line carries (summed in
        leg order, once per subset) and its inverse denominator per propagator"""
        done_q, done_d = set(), set()
        for c in self.p.calls:
            if c.op in AMP_OPS or c.op in LINEAR_OPS:
                continue
            sub = self.subset[c.out]
            n = self.sname(sub)
            if sub not in done_q:
                done_q.add(sub)
                w(f"{ind}const mom qs{n} = {' + '.join(qname(x) for x in sub)};")
                if sub in self.need_q:
                    w(f"{ind}const vec<T> Qs{n} = tv<T>(qs{n});")
                    self._kin[f"Qs{n}"] = "vec<T>"
            if (sub, c.prop) not in done_d:
                done_d.add((sub, c.prop))
                pid = c.prop
                w(f"{ind}const cx<T> d{n}_{pid} = cvt<T>(inv_denominator(qs{n}, cx<double>{{pe{pid}.pole_r, pe{pid}.pole_i}}));")
                self._kin[f"d{n}_{pid}"] = "cx<T>"

    # ---------------------------------------------------------- straight-line
    def _row_groups(self, parts):
        """the amplitude calls of the rows schedule in groups of consecutive
        amplitudes, one per part of the function division (one group: no
        division)"""
        amps = [i for i, c in enumerate(self.p.calls) if c.op in AMP_OPS]
        size = -(-len(amps) // max(1, parts))
        return [amps[i:i + size] for i in range(0, len(amps), size)]

    def _row_divisions(self):
        """(precision test, function-name tag, groups) of the FP64 and FP32
        kernels: one division for both when they have the same number of parts"""
        p = self.p
        n64, n32 = p.row_parts, p.row_parts_mixed or p.row_parts
        if n64 == n32:
            return [("true", "", self._row_groups(n64))]
        return [("sizeof(T) == 8", "d", self._row_groups(n64)), ("sizeof(T) == 4", "f", self._row_groups(n32))]

    def _closure(self, idxs):
        """the calls that the given calls need, in IR order"""
        calls = self.p.calls
        producer = {c.out: i for i, c in enumerate(calls) if c.op not in AMP_OPS}
        need, stack = set(), list(idxs)
        while stack:
            i = stack.pop()
            if i in need:
                continue
            need.add(i)
            stack.extend(producer[x] for x in calls[i].ins if x in producer)
        return sorted(need)

    def _emit_row_calls(self, w, ind, idxs, acc):
        """one helicity row's calls idxs (IR order) with the external states,
        momentum sums and denominators they need, formed in place from the LDS
        momenta behind an opaque index (not hoisted out of the row loop); each
        amplitude is added to its flows, acc(f), as soon as it is formed"""
        p, nl = self.p, self.nl
        flows_of = {}
        for f, terms in enumerate(p.jamp):
            for ai, cc in terms:
                flows_of.setdefault(ai, []).append((f, cc))
        loaded, done = set(), set()

        def phys(k):
            if k not in loaded:
                loaded.add(k)
                w(f"{ind}const mom pr{k} = pm_{p.name}[opaque_int({k})][threadIdx.x];")
            return f"pr{k}"

        def qsum(sub):
            n = self.sname(sub)
            if f"qs{n}" not in done:
                done.add(f"qs{n}")
                terms = (phys(x) if p.legs[x].incoming else f"(-{phys(x)})" for x in sub)
                w(f"{ind}const mom qs{n} = {' + '.join(terms)};")
            return f"qs{n}"

        legs = sorted({x for i in idxs for x in p.calls[i].ins if x < nl})
        for k in legs:
            leg = p.legs[k]
            pk = phys(k)
            if leg.kind == F:
                fn = "ixxxxx" if _flowing_in(leg) else "oxxxxx"
                massless = "true" if leg.particle == P_ZERO else "false"
                w(f"{ind}const wf<T> w{k} = cvtw<T>({fn}<double, {massless}>(tv<double>({pk}), pe{leg.particle}.m, "
                  f"hh[{k}], {leg.flow}));")
            elif leg.kind == V:
                nsv = -1 if leg.incoming else 1
                w(f"{ind}const wf<T> w{k} = vxxxxx<T>(tv<T>({pk}), T(pe{leg.particle}.m), hh[{k}], {nsv});")
            else:
                w(f"{ind}const cx<T> w{k} = sxxxxx<T>();")
        for i in idxs:
            c = p.calls[i]
            subs = [self.subset[x] for x in c.ins]
            if c.op not in AMP_OPS and c.op not in LINEAR_OPS:
                subs.append(self.subset[c.out])
            for sub in subs:
                n = self.sname(sub)
                if sub in self.need_q and f"Qs{n}" not in done:
                    done.add(f"Qs{n}")
                    w(f"{ind}const vec<T> Qs{n} = tv<T>({qsum(sub)});")
            if c.op not in AMP_OPS and c.op not in LINEAR_OPS:
                sub, pid = self.subset[c.out], c.prop
                n = self.sname(sub)
                if f"d{n}_{pid}" not in done:
                    done.add(f"d{n}_{pid}")
                    w(f"{ind}const cx<T> d{n}_{pid} = cvt<T>(inv_denominator({qsum(sub)}, "
                      f"cx<double>{{pe{pid}.pole_r, pe{pid}.pole_i}}));")
            self._call(w, c, ind)
            if c.op in AMP_OPS:
                for f, cc in flows_of.get(c.out, []):
                    w(f"{ind}{acc(f)} = {acc(f)} + {_coef_expr(cc, f'amp{c.out}')};")

    def _emit_row_parts(self, w):
        """the function division of the rows schedule (the paper's Sec. 5.3):
        each group of amplitudes in a device function of its own, not inlined,
        that forms the currents its amplitudes need (a current two groups share
        is formed in each) and adds the amplitudes to the flows J (in the
        caller's memory).  Each part is compiled and register-allocated alone."""
        p = self.p
        w(f"// the event's physical momenta, one column per lane, read by every part")
        w(f"__shared__ mom pm_{p.name}[{self.nl}][256];")
        w("")
        for _, tag, groups in self._row_divisions():
            if len(groups) > 1:
                self._emit_parts_of(w, tag, groups)

    def _emit_parts_of(self, w, tag, groups):
        p = self.p
        for k, grp in enumerate(groups):
            idxs = self._closure(grp)
            w(f"// part {k}{f' ({tag})' if tag else ''}: amplitudes {p.calls[grp[0]].out} .. {p.calls[grp[-1]].out} "
              f"({len(idxs)} calls)")
            w("template <class T>")
            w(f"__device__ __noinline__ void rows_{p.name}{tag}_part{k}(const KernelArgs& a, const int8_t* hh, cx<T>* J) {{")
            cpls = sorted({p.calls[i].cpl for i in idxs if p.calls[i].cpl >= 0})
            for c in cpls:
                for line in _coupling_decls(c, p.couplings[c].kind):
                    w(line)
            pids = sorted({p.calls[i].prop for i in idxs} | {leg.particle for leg in p.legs} | {P_ZERO})
            for pid in pids:
                w(f"  const PropEntry pe{pid} = a.prop[{pid}];")
            self._emit_row_calls(w, "  ", idxs, lambda f: f"J[{f}]")
            w("}")
            w("")

    def _emit_rows(self, w):
        """the helicity table row by row (the rows schedule): the momenta are
        copied to LDS, then per row the calls run in IR order, in one piece or
        as the parts of the function division, and the colour form sums the
        row's flows"""
        p, nl = self.p, self.nl
        for k in range(nl):
            w(f"  pm_{p.name}[{k}][threadIdx.x] = p[{k}];")
        w("  double me2 = 0.0;")
        w("  if (pass) {")
        w("    for (int h = 0; h < a.n_hel; ++h) {")
        w(f"      const int8_t* hh = a.hel + h * {nl};")
        for cond, tag, groups in self._row_divisions():
            w(f"      if constexpr ({cond}) {{")
            if len(groups) < 2:
                w(f"        cx<T> {', '.join(f'J{f} = mk<T>(T(0), T(0))' for f in range(p.n_flows))};")
                self._emit_row_calls(w, "        ", list(range(len(p.calls))), lambda f: f"J{f}")
                self._colour_form(w, lambda f: f"J{f}", "        ")
            else:
                w(f"        cx<T> J[{p.n_flows}];")
                w(f"        for (int f = 0; f < {p.n_flows}; ++f) J[f] = mk<T>(T(0), T(0));")
                for k in range(len(groups)):
                    w(f"        rows_{p.name}{tag}_part{k}<T>(a, hh, J);")
                self._colour_form(w, lambda f: f"J[{f}]", "        ")
            w("      }")
        w("    }")
        w("  }")

    def _emit_straight(self, w):
        p = self.p
        self._kin = {}
        if p.helicity_schedule == "rows":
            self._emit_rows(w)
            return
        for k in range(self.nl):
            if (k,) in self.need_q:
                w(f"  const vec<T> Qs{k} = tv<T>(q{k});")
                self._kin[f"Qs{k}"] = "vec<T>"
        self._current_momenta(w, "  ", lambda x: f"q{x}")
        self._ext_pre(w)
        w("  double me2 = 0.0;")
        w("  if (pass && a.hel_nest) {")
        self._emit_nest(w)
        w("  } else if (pass) {")
        w("    // an arbitrary helicity table (filtered, reordered or gauge-test rows)")
        w("    for (int h = 0; h < a.n_hel; ++h) {")
        w(f"      const int8_t* hh = a.hel + h * {self.nl};")
        for k, leg in enumerate(p.legs):
            w("      " + self._external(k, leg, f"w{k}"))
        for c in p.calls:
            self._call(w, c, "      ")
        self._jamps(w, "      ")
        self._colour_form(w, lambda f: f"J{f}")
        w("    }")
        w("  }")

    def _jamps(self, w, ind):
        for f, terms in enumerate(self.p.jamp):
            expr = " + ".join(_coef_expr(cc, f"amp{ai}") for ai, cc in terms) or "mk<T>(T(0), T(0))"
            w(f"{ind}const cx<T> J{f} = {expr};")

    def _emit_nest(self, w):
        """the full helicity product as one loop per leg (nest.schedule): each
        wavefunction, call, bra, amplitude core and jamp sits in the
        innermost loop its inputs need; an FP32 variant with the inner table
        where the process has one"""
        sc = nest.schedule(self.p)
        if self._inner_table_plan(sc, nest.unrolled_levels(sc), INNER_TABLE_WORDS)[0]:
            w("    if constexpr (sizeof(T) == 4) {")
            self._emit_nest_body(w, INNER_TABLE_WORDS, "  ")
            w("    } else {")
            self._emit_nest_body(w, 0, "  ")
            w("    }")
        else:
            self._emit_nest_body(w, 0, "")

    def _emit_nest_body(self, w, inner_words, extra):
        p = self.p
        sc = nest.schedule(p)
        by_level = {}
        for it in sc.items:
            by_level.setdefault(it.level, []).append(it)
        ind = "    " + extra
        w(f"{ind}// helicity loop nest, outermost leg first: {sc.order}")
        for it in by_level.get(-1, []):
            self._nest_item(w, it, ind)
        # the innermost loops (up to 8 combinations) are unrolled: constant
        # helicities there let the compiler specialise the external states and
        # interleave the independent iterations
        unrolled = nest.unrolled_levels(sc)
        tables = self._tables(sc, unrolled)
        inner, hoisted, iwords = self._inner_table_plan(sc, unrolled, inner_words)
        loads = self._stash_plan(sc, unrolled, tables, inner_words=iwords)
        if loads:
            words = sum(_KIN_WORDS[self._kin[nm]] for L in loads.values() for nm, _ in L)
            w(f"{ind}// kinematics used only inside the helicity loops wait in LDS and are read")
            w(f"{ind}// back in the loop that first needs them, instead of occupying registers")
            w(f"{ind}__shared__ T stash[{words}][256];")
            for L in loads.values():
                for nm, off in L:
                    w(f"{ind}stash_put(stash, {off}, {nm});")
        self._emit_tables(w, sc, tables, ind, -1)
        if inner:
            self._emit_inner_table(w, sc, unrolled, inner, hoisted, iwords, ind)
        for lvl, L in enumerate(sc.order):
            ch = sc.choices[L]
            if len(ch) == 1:
                w(f"{ind}const int hh{L} = {ch[0]};")
            else:
                w(f"{ind}#pragma unroll{'' if lvl in unrolled else ' 1'}")
                w(f"{ind}for (int c{L} = 0; c{L} < {len(ch)}; ++c{L}) {{")
                ind += "  "
                if ch == (-1, 1):
                    w(f"{ind}const int hh{L} = 2 * c{L} - 1;")
                elif ch == (-1, 0, 1):
                    w(f"{ind}const int hh{L} = c{L} - 1;")
                else:
                    raise NotImplementedError(f"helicity states {ch}")
            for nm, off in loads.get(lvl, []):
                w(f"{ind}const {self._kin[nm]} {nm} = stash_get<{self._kin[nm]}>(stash, {off});")
            for it in by_level.get(lvl, []):
                if id(it) in tables:
                    w(ind + self._table_select(it, tables[id(it)]))
                elif id(it) in hoisted:
                    for nm, (typ, off, legs) in inner.items():
                        if hoisted[id(it)] == nm:
                            n = _KIN_WORDS[typ]
                            idx = " + ".join(f"{1 << (len(legs) - 1 - j)} * c{L}" for j, L in enumerate(legs))
                            w(f"{ind}const {typ} {nm} = stash_get<{typ}>(itab, {off} + {n} * ({idx}));")
                else:
                    self._nest_item(w, it, ind)
            self._emit_tables(w, sc, tables, ind, lvl)
        self._colour_form(w, lambda f: f"J{f}", ind)
        for L in reversed(sc.order):
            if len(sc.choices[L]) > 1:
                ind = ind[:-2]
                w(f"{ind}}}")

    def _tables(self, sc, unrolled):
        return {key: (t[0], t[1]) for key, t in nest.tables(self.p, sc, unrolled).items()}

    def _emit_tables(self, w, sc, tables, ind, level):
        """the tables formed at this loop level (-1: before the loops)"""
        import itertools
        p = self.p
        mine = [it for it in sc.items if id(it) in tables and tables[id(it)][0] == level]
        if not mine:
            return
        w(f"{ind}// calls tabulated over the helicities of deeper external legs")
        done = set()
        for it in mine:
            legs = tables[id(it)][1]
            for L in legs:
                for h, tag in ((-1, "m"), (1, "p")):
                    if (L, h) not in done:
                        done.add((L, h))
                        w(ind + self._external(L, p.legs[L], f"x{L}{tag}", str(h), nest=True))
            k, args = it.data
            o = p.calls[k].out
            for j, hs in enumerate(itertools.product((-1, 1), repeat=len(legs))):
                tag = {L: ("m" if h < 0 else "p") for L, h in zip(legs, hs)}
                buf = []
                argv = []
                for a in args:
                    if a is nest.ONE:
                        argv.append("mk<T>(T(1), T(0))")
                    elif a[1] in tag:
                        argv.append(f"x{a[1]}{tag[a[1]]}")
                    else:
                        argv.append(f"w{a[1]}")
                self._call(buf.append, p.calls[k], ind, args=argv)
                line = buf[0]
                assert f" w{o} = " in line, line
                w(line.replace(f" w{o} = ", f" t{o}_{j} = ", 1))

    def _table_select(self, it, table):
        legs = table[1]
        o = self.p.calls[it.data[0]].out

        def sel(k, j):
            if k == len(legs):
                return f"t{o}_{j}"
            return f"(c{legs[k]} ? {sel(k + 1, 2 * j + 1)} : {sel(k + 1, 2 * j)})"
        kind = "cx<T>" if ir.OUT_KIND[self.p.calls[it.data[0]].op] == S else "wf<T>"
        return f"const {kind} w{o} = {sel(0, 0)};"

    def _hoistable(self, sc, unrolled):
        """items of the unrolled levels that depend on no real loop, with the
        names they define and the names of all items' uses"""
        import re
        real = [lvl for lvl, L in enumerate(sc.order) if len(sc.choices[L]) > 1 and lvl not in unrolled]
        real_hh = {f"hh{sc.order[lvl]}" for lvl in real}
        varying, info = set(), []
        for it in sc.items:
            buf = []
            self._nest_item(buf.append, it, "")
            code = "\n".join(buf)
            toks = set(re.findall(r"[A-Za-z_]\w*", code))
            defined = re.findall(r"const (\S+) (\w+) =", code)
            rv = bool(toks & (varying | real_hh))
            if rv:
                varying |= {nm for _, nm in defined}
            info.append((it, rv, defined, toks))
        return info

    def _inner_table_plan(self, sc, unrolled, budget):
        """The inner table: values defined by hoistable items (unrolled level,
        no real loop) and used by items that are not hoistable, one entry per
        combination of the unrolled helicities up to the value's level.
        Returns ({name: (type, word offset, legs)}, {id(item): name}, words)."""
        if not budget or not unrolled:
            return {}, {}, 0
        info = self._hoistable(sc, unrolled)
        # calls only: external states are cheap to form again inside the loops
        hoist = {id(it) for it, rv, _, _ in info if it.level in unrolled and not rv and it.kind == "call"}
        self._inner_pre = {id(it) for it, rv, _, _ in info
                           if it.level in unrolled and not rv and it.kind in ("ext", "call")}
        used_outside = set()
        for it, rv, defined, toks in info:
            if id(it) not in hoist:
                used_outside |= toks
        inner, hoisted, off = {}, {}, 0
        for it, rv, defined, toks in info:
            if id(it) not in hoist:
                continue
            for typ, nm in defined:
                if nm in used_outside and typ in _KIN_WORDS:
                    legs = [sc.order[lvl] for lvl in sorted(unrolled) if lvl <= it.level]
                    n = _KIN_WORDS[typ] * 2 ** len(legs)
                    if off + n > budget:
                        return {}, {}, 0
                    inner[nm] = (typ, off, legs)
                    hoisted[id(it)] = nm
                    off += n
        # the other hoistable items are formed only in the table's loops
        for it, rv, defined, toks in info:
            if id(it) in hoist and id(it) not in hoisted:
                hoisted[id(it)] = None
        return inner, hoisted, off

    def _emit_inner_table(self, w, sc, unrolled, inner, hoisted, words, ind):
        """the inner table's loops before the nest: the hoistable items for
        every combination of the unrolled helicities, the table values to LDS"""
        items = {id(it): it for it in sc.items}
        w(f"{ind}// values of the unrolled loops that no outer loop changes, for every combination")
        w(f"{ind}// of the unrolled helicities, in LDS (read back inside the loops)")
        w(f"{ind}__shared__ T itab[{words}][256];")
        ind0 = ind
        for lvl in sorted(unrolled):
            L = sc.order[lvl]
            w(f"{ind}#pragma unroll")
            w(f"{ind}for (int c{L} = 0; c{L} < 2; ++c{L}) {{")
            ind += "  "
            w(f"{ind}const int hh{L} = 2 * c{L} - 1;")
            for it in sc.items:
                if it.level == lvl and id(it) in self._inner_pre:
                    self._nest_item(w, it, ind)
                    nm = hoisted.get(id(it))
                    if nm is not None:
                        typ, off, legs = inner[nm]
                        n = _KIN_WORDS[typ]
                        idx = " + ".join(f"{1 << (len(legs) - 1 - j)} * c{L2}" for j, L2 in enumerate(legs))
                        w(f"{ind}stash_put(itab, {off} + {n} * ({idx}), {nm});")
        for _ in sorted(unrolled):
            ind = ind[:-2]
            w(f"{ind}}}")
        assert ind == ind0

    def _stash_plan(self, sc, unrolled, tables=None, inner_words=0):
        """Which event kinematics go to the LDS stash, and the loop level that
        reads each back: a value qualifies when every item using it sits inside
        a real (not unrolled) helicity loop or depends on one.  Values that feed
        items depending only on unrolled legs stay in registers (the compiler
        hoists those items out of the loops).  Outer loops first, up to
        STASH_WORDS words.  Returns {level: [(name, word offset), ...]}."""
        import re
        real = [lvl for lvl, L in enumerate(sc.order) if len(sc.choices[L]) > 1 and lvl not in unrolled]
        if not real or not self._kin:
            return {}
        first_real, last_real = real[0], real[-1]
        real_hh = {f"hh{sc.order[lvl]}" for lvl in real}
        varying = set()
        uses = {}
        tables = tables or {}
        for it in sc.items:
            buf = []
            self._nest_item(buf.append, it, "")
            code = "\n".join(buf)
            toks = set(re.findall(r"[A-Za-z_]\w*", code))
            defined = set(re.findall(r"const \S+ (\w+) =", code))
            if id(it) in tables:
                varying |= defined
                tlev = tables[id(it)][0]
                for nm in toks & self._kin.keys():
                    uses.setdefault(nm, []).append((tlev, tlev >= 0))
                continue
            rv = bool(toks & (varying | real_hh))
            if rv:
                varying |= defined
            for nm in toks & self._kin.keys():
                uses.setdefault(nm, []).append((it.level, rv))
        cand = []
        for nm, us in uses.items():
            if all(rv and lvl >= first_real for lvl, rv in us):
                cand.append((min(lvl for lvl, _ in us), nm))
        loads, off = {}, 0
        cap = min(STASH_WORDS, self.p.stash_words)
        budget = min(cap, NEST_LDS_WORDS - inner_words) if inner_words else cap
        for lvl, nm in sorted(cand, key=lambda c: (c[0], list(self._kin).index(c[1]))):
            n = _KIN_WORDS[self._kin[nm]]
            if off + n > budget:
                continue
            loads.setdefault(lvl, []).append((nm, off))
            off += n
        return loads

    @staticmethod
    def _nest_arg(a):
        if a is nest.ONE:
            return "mk<T>(T(1), T(0))"
        return f"w{a[1]}" if a[0] == "w" else a[1]

    def _nest_item(self, w, it, ind):
        p = self.p
        if it.kind == "ext":
            (L,) = it.data
            w(ind + self._external(L, p.legs[L], f"w{L}", f"hh{L}", nest=True))
        elif it.kind == "call":
            k, args = it.data
            self._call(w, p.calls[k], ind, args=[self._nest_arg(a) for a in args])
        elif it.kind == "mat":
            name, x, facs = it.data
            prod = " * ".join(f"w{s}" for s in facs)
            w(f"{ind}const wf<T> {name} = wscale<T>({prod}, w{x});")
        elif it.kind == "bra":
            k, fo, vc = it.data
            c = p.calls[k]
            w(f"{ind}const wf<T> bra{c.out} = ffv_bra<T>({self._nest_arg(fo)}, {self._nest_arg(vc)}, "
              f"g{c.cpl}_0, g{c.cpl}_1);")
        elif it.kind == "dot":
            k, fi = it.data
            c = p.calls[k]
            w(f"{ind}const cx<T> amp{c.out} = spinor_dot(bra{c.out}, {self._nest_arg(fi)});")
        elif it.kind == "vbra":
            k, vo, scal = it.data
            c = p.calls[k]
            kfac = " * ".join([f"g{c.cpl}_0"] + [self._nest_arg(a) for a in scal])
            w(f"{ind}const wf<T> bra{c.out} = vs_bra<T>({self._nest_arg(vo)}, {kfac});")
        elif it.kind == "vdot":
            k, v = it.data
            c = p.calls[k]
            w(f"{ind}const cx<T> amp{c.out} = vec_dot(bra{c.out}, {self._nest_arg(v)});")
        elif it.kind == "ksum":
            f, g, members = it.data
            expr = " + ".join(_coef_expr(cc, f"amp{a}") for a, cc in members)
            w(f"{ind}const cx<T> K{f}_{g} = {expr};")
        elif it.kind == "bsum":
            f, g, members = it.data
            comps = [" + ".join(_coef_expr(cc, f"bra{a}.c[{m}]") for a, cc in members) for m in range(4)]
            w(f"{ind}const wf<T> bj{f}_{g} = {{{{{', '.join(comps)}}}}};")
        elif it.kind == "bacc":
            f, g, a, cc, j, last = it.data
            name = f"bj{f}_{g}" if last else f"bj{f}_{g}_{j}"
            comps = [(f"bj{f}_{g}_{j - 1}.c[{m}] + " if j else "") + _coef_expr(cc, f"bra{a}.c[{m}]") for m in range(4)]
            w(f"{ind}const wf<T> {name} = {{{{{', '.join(comps)}}}}};")
        elif it.kind == "kdot":
            f, g, ket, vector = it.data
            prod = "vec_dot" if vector else "spinor_dot"
            w(f"{ind}const cx<T> K{f}_{g} = {prod}(bj{f}_{g}, {self._nest_arg(ket)});")
        elif it.kind == "jamp":
            f, parts = it.data
            terms = [(" * ".join([f"w{s}" for s in facs] + [f"K{f}_{g}"])) for g, facs in parts]
            w(f"{ind}const cx<T> J{f} = {' + '.join(terms) or 'mk<T>(T(0), T(0))'};")
        else:
            raise ValueError(it.kind)

    # ------------------------------------------------------ ordering template
    def _emit_ordered(self, w):
        """Ordering templates, two phases per block of 256 events:
        1. for every ordering, the helicity sum's amplitudes A_o(h) of the
           lane's event (a loop nest over the positions' helicities, or the
           table row by row) go to the block's workspace slot [o][h][256];
        2. for every helicity, the colour form over the orderings' amplitudes
           (read back from the workspace; on MFMA through LDS for large bases)."""
        p = self.p
        nl, no = self.nl, len(p.orderings)
        if any(leg.kind == F for leg in p.legs):
            raise NotImplementedError("ordering templates support vector and scalar legs")
        mf = p.uses_colour_mfma()
        # the colour form's amplitude rows ([2 o][256] per helicity): staged in LDS,
        # or, when they would not fit, laid out that way in the workspace itself
        self._direct_rows = mf and 2 * no * 256 * 8 > DIRECT_ROWS_BYTES
        self._template_stash_plan()
        rows = 2 * no if mf and not self._direct_rows else 0
        if self._tstash_words or rows:
            w("  // per-lane LDS rows (column = lane): the helicity nest's stash of outer")
            w("  // currents while the orderings run (FP64), then the amplitude rows of the colour form")
            w(f"  constexpr bool kStash = {'sizeof(T) == 8' if self._tstash_words else 'false'};")
            w(f"  __shared__ T lds_rows[kStash ? {max(rows, self._tstash_words)} : {max(rows, 1)}][256];")
        for k, L in sorted(self._fixed_vector_positions().items()):
            w(f"  const VPol<T> VP{k} = vpol_pre<T>(p[{L}]);   // position {k} is leg {L} in every ordering")
        if self._direct_rows:
            w("  // this block's workspace slot: per helicity h, the real and imaginary rows")
            w(f"  // [2 o][256] of the orderings' amplitudes (h * {2 * no * 256} + (2 o) * 256 + lane)")
        else:
            w("  // this block's workspace slot: A[o][h][256] of its events")
        w("  cx<T>* const work = static_cast<cx<T>*>(a.work) + size_t(blockIdx.x) * size_t(a.work_stride);")
        w("  const int nh = a.n_hel;")
        if self._split:
            w("  if constexpr (PHASE != 2) {")
        w("  if (pass) {")
        w("#pragma unroll 1")
        w(f"    for (int o = 0; o < {no}; ++o) {{")
        w(f"      const int8_t* ord = a.ord + o * {nl};")
        ind = "      "
        self._bind_positions(w, ind)
        w(f"{ind}if (a.hel_nest) {{")
        if self._tstash_words:
            w(f"{ind}  if constexpr (kStash) {{")
            self._emit_template_nest(w, ind + "    ")
            w(f"{ind}  }} else {{")
            self._emit_template_nest(w, ind + "    ", use_stash=False)
            w(f"{ind}  }}")
        else:
            self._emit_template_nest(w, ind + "  ")
        w(f"{ind}}} else {{")
        w(f"{ind}  for (int h = 0; h < nh; ++h) {{")
        w(f"{ind}    const int8_t* hh = a.hel + h * {nl};")
        done = set()
        self._scope, self._opaque = "h", set()
        self._w, self._ind = w, ind + "    "
        for k in range(nl):
            w(f"{ind}    const int hp{k} = hh[lk{k}];")
            w(f"{ind}    " + self._position_external(k))
        for c in p.calls:
            self._lazy_kinematics(w, ind + "    ", c, done)
            self._call(w, c, ind + "    ")
        self._scope = None
        expr = " + ".join(_coef_expr(cc, f"amp{ai}") for ai, cc in p.jamp[0])
        w(f"{ind}    {self._work_store('h', expr)}")
        w(f"{ind}  }}")
        w(f"{ind}}}")
        w("    }")
        if self._direct_rows:
            w("  } else {")
            w("    // the colour form reads every lane of the wave: a failed lane's rows are zero")
            w("    T* const wr = reinterpret_cast<T*>(work) + threadIdx.x;")
            w("    for (int h = 0; h < nh; ++h)")
            w(f"      for (int r = 0; r < {2 * no}; ++r) wr[(size_t(h) * {2 * no} + r) * 256] = T(0);")
        w("  }")
        if self._split:
            w("  }")
        w("  double me2 = 0.0;")
        if self._split:
            w("  if constexpr (PHASE != 1) {")
        self._emit_colour_phase(w, mf, no)
        if self._split:
            w("  }")

    def _emit_colour_phase(self, w, mf, no):
        """phase 2 of an ordering template: the colour form per helicity over the
        orderings' amplitudes in the workspace"""
        p = self.p
        if mf and p.colour_form == "compressed":
            # FP32: the compressed colour form on VALU (no MFMA in the FP32 kernel);
            # FP64: the dense MFMA form (the flows' FP64 values would not fit registers)
            w("  if constexpr (sizeof(T) == 4) {")
            self._emit_valu_colour_from_work(w)
            w("  } else {")
            self._emit_mfma_colour(w)
            w("  }")
        elif mf:
            self._emit_mfma_colour(w)
        else:
            w("  if (pass) {")
            w("    for (int h = 0; h < nh; ++h) {")
            for o in range(no):
                w(f"      const cx<T> A{o} = work[(size_t({o}) * nh + h) * 256 + threadIdx.x];")
            self._colour_form(w, lambda f: f"A{f}")
            w("    }")
            w("  }")

    def _emit_mfma_colour(self, w):
        """the MFMA colour form over the orderings' amplitudes in the workspace
        (direct rows) or staged per helicity in LDS rows"""
        p = self.p
        no = len(p.orderings)
        if self._direct_rows:
            nks, nfo = (p.n_flows + 3) // 4, (p.n_flows + 15) // 16
            w("  // the MFMA colour form needs every lane of the wavefront; it reads the wave's")
            w("  // columns of the workspace rows, written above by the wave's own lanes")
            w("  if (__any(pass)) {")
            w("    __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"workgroup\");")
            w("    __builtin_amdgcn_wave_barrier();")
            w("    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"workgroup\");")
            w("    const T* const rows = reinterpret_cast<const T*>(work);")
            if COLOUR_RESIDENT:
                w(f"    ResidentFrags<T, {nks}, {nfo}> fr;")
                w("    fr.load(a.cfrag);")
                w("    for (int h = 0; h < nh; ++h)")
                w(f"      me2 += double(colour_form_resident<T, {nks}, {nfo}, {self.cterm_cap()}>"
                  f"(fr, rows + size_t(h) * {2 * no * 256}, a.cstep));")
            else:
                w("    for (int h = 0; h < nh; ++h)")
                w(f"      me2 += double(colour_form_mfma<T, {nks}, {nfo}, {self.cterm_cap()}, {COLOUR_CHUNKS}>"
                  f"(rows + size_t(h) * {2 * no * 256}, a.cstep, a));")
            w("  }")
        else:
            nks, nfo = (p.n_flows + 3) // 4, (p.n_flows + 15) // 16
            w("  // the MFMA colour form needs every lane of the wavefront: failed lanes take part with zeros")
            w("  if (__any(pass)) {")
            if COLOUR_RESIDENT:
                w(f"    ResidentFrags<T, {nks}, {nfo}> fr;")
                w("    fr.load(a.cfrag);")
            w("    for (int h = 0; h < nh; ++h) {")
            w(f"      for (int o = 0; o < {no}; ++o) {{")
            w("        const cx<T> v = pass ? work[(size_t(o) * nh + h) * 256 + threadIdx.x] : cx<T>{T(0), T(0)};")
            w("        lds_rows[2 * o][threadIdx.x] = v.r;")
            w("        lds_rows[2 * o + 1][threadIdx.x] = v.i;")
            w("      }")
            w("      __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\");")
            w("      __builtin_amdgcn_wave_barrier();")
            w("      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"wavefront\");")
            if COLOUR_RESIDENT:
                w(f"      me2 += double(colour_form_resident<T, {nks}, {nfo}, {self.cterm_cap()}>"
                  f"(fr, &lds_rows[0][0], a.cstep));")
            else:
                w(f"      me2 += double(colour_form_mfma<T, {nks}, {nfo}, {self.cterm_cap()}, {COLOUR_CHUNKS}>"
                  f"(&lds_rows[0][0], a.cstep, a));")
            w("      __builtin_amdgcn_wave_barrier();")
            w("    }")
            w("  }")

    def _emit_valu_colour_from_work(self, w):
        """the VALU colour form of the IR over the orderings' amplitudes in the
        workspace, flows formed through the flow map (FP32 kernels of MFMA-sized
        bases with the compressed form)"""
        p = self.p
        no = len(p.orderings)
        w("    if (pass) {")
        w("      const T* const rows = reinterpret_cast<const T*>(work);")
        w("      for (int h = 0; h < nh; ++h) {")
        for o in range(no):
            if self._direct_rows:
                w(f"        const cx<T> A{o} = {{rows[(size_t(h) * {2 * no} + {2 * o}) * 256 + threadIdx.x], "
                  f"rows[(size_t(h) * {2 * no} + {2 * o + 1}) * 256 + threadIdx.x]}};")
            else:
                w(f"        const cx<T> A{o} = work[(size_t({o}) * nh + h) * 256 + threadIdx.x];")
        if p.flow_map is not None:
            for f, row in enumerate(p.flow_map):
                terms = [_coef_expr(c, f"A{o}") for o, c in enumerate(row) if c]
                w(f"        const cx<T> J{f} = {' + '.join(terms)};")
            J = lambda f: f"J{f}"
        else:
            J = lambda f: f"A{f}"
        self._colour_form(w, J, ind="        ")
        w("      }")
        w("    }")

    def _work_store(self, h, value):
        """store of ordering o's amplitude at helicity h in the workspace slot"""
        if not self._direct_rows:
            return f"work[(size_t(o) * nh + {h}) * 256 + threadIdx.x] = {value};"
        no = len(self.p.orderings)
        return (f"{{ const cx<T> v_ = {value}; T* const r_ = reinterpret_cast<T*>(work) + "
                f"(size_t({h}) * {2 * no} + 2 * o) * 256 + threadIdx.x; r_[0] = v_.r; r_[256] = v_.i; }}")

    def _bind_positions(self, w, ind):
        """bind every position to the ordering's leg (uniform over the wave):
        leg index, flow sign and vector sign.  Momenta are read from the LDS
        copy where they are used."""
        p = self.p
        nl = self.nl
        self._pos_nsv, self._pos_sign = {}, {}
        for k in range(nl):
            cand = sorted({o[k] for o in p.orderings})
            L0 = cand[0]
            w(f"{ind}const int lk{k} = {L0 if len(cand) == 1 else f'ord[{k}]'};")
            signs = {p.legs[L].incoming for L in cand}
            if len(signs) == 1:
                self._pos_sign[k] = "+" if p.legs[L0].incoming else "-"
            else:
                w(f"{ind}const double sg{k} = lk{k} < 2 ? 1.0 : -1.0;")
                self._pos_sign[k] = f"sg{k}"
            legs = [p.legs[L] for L in cand]
            assert len({l.kind for l in legs}) == 1 and len({l.particle for l in legs}) == 1, \
                "a position must hold one kind of particle"
            if legs[0].kind == V:
                if len(signs) == 1:
                    self._pos_nsv[k] = "-1" if legs[0].incoming else "1"
                else:
                    w(f"{ind}const int nsv{k} = lk{k} < 2 ? -1 : 1;")
                    self._pos_nsv[k] = f"nsv{k}"

    def _pmom(self, k, w, ind):
        """momentum flowing into the diagram at position k in the current loop
        scope (an LDS read behind an opaque leg index, so that it is not
        hoisted); the LDS copy holds +p for incoming and -p for outgoing legs"""
        key = (k, self._scope)
        if key not in self._opaque:
            self._opaque.add(key)
            w(f"{ind}const mom pl{k}_{self._scope} = pm[opaque_int(lk{k})][threadIdx.x];")
        return f"pl{k}_{self._scope}"

    def _qterm(self, k, w, ind):
        """momentum of position k flowing into the diagram"""
        return self._pmom(k, w, ind)

    def _physical(self, k, w, ind):
        """physical momentum of position k"""
        name = self._pmom(k, w, ind)
        sg = self._pos_sign[k]
        if sg == "+":
            return name
        if sg == "-":
            return f"-{name}"
        return f"mom{{{sg} * {name}.e, {sg} * {name}.x, {sg} * {name}.y, {sg} * {name}.z}}"

    def _lazy_kinematics(self, w, ind, c, done):
        """the momenta (FP64, and as T where the call uses them) and the
        propagator denominator call c needs, each emitted once in scope"""
        subs = [self.subset[x] for x in c.ins]
        if c.op not in AMP_OPS and c.op not in LINEAR_OPS:
            subs.append(self.subset[c.out])
        for sub in subs:
            n = self.sname(sub)
            if sub in self.need_q and f"Qs{n}" not in done:
                if len(sub) == 1:
                    t = self._qterm(sub[0], w, ind)
                    w(f"{ind}const vec<T> Qs{n} = tv<T>({t});")
                else:
                    if f"qs{n}" not in done:
                        done.add(f"qs{n}")
                        t = [self._qterm(x, w, ind) for x in sub]
                        w(f"{ind}const mom qs{n} = {' + '.join(t)};")
                    w(f"{ind}const vec<T> Qs{n} = tv<T>(qs{n});")
                done.add(f"Qs{n}")
        if c.op not in AMP_OPS and c.op not in LINEAR_OPS:
            sub, pid = self.subset[c.out], c.prop
            n = self.sname(sub)
            if f"d{n}_{pid}" not in done:
                if f"qs{n}" not in done:
                    done.add(f"qs{n}")
                    t = [self._qterm(x, w, ind) for x in sub]
                    w(f"{ind}const mom qs{n} = {' + '.join(t)};")
                w(f"{ind}const cx<T> d{n}_{pid} = cvt<T>(inv_denominator(qs{n}, "
                  f"cx<double>{{pe{pid}.pole_r, pe{pid}.pole_i}}));")
                done.add(f"d{n}_{pid}")

    def _fixed_vector_positions(self):
        """positions that hold the same massless vector leg in every ordering"""
        p = self.p
        out = {}
        for k in range(self.nl):
            cand = {o[k] for o in p.orderings}
            if len(cand) == 1:
                L = cand.pop()
                if p.legs[L].kind == V and p.legs[L].particle == P_ZERO:
                    out[k] = L
        return out

    def _position_external(self, k, nest=False):
        """the external state at position k; in the helicity nest (helicities
        +-1) a position that always holds the same massless vector leg uses the
        event's precomputed polarisation factors"""
        p = self.p
        leg = p.legs[p.orderings[0][k]]
        if leg.kind == V:
            if nest and k in self._fixed_vector_positions():
                return f"const wf<T> w{k} = vxxxxx0<T>(VP{k}, hp{k}, {self._pos_nsv[k]});"
            return (f"const wf<T> w{k} = vxxxxx<T>(tv<T>({self._physical(k, self._w, self._ind)}), T(pe{leg.particle}.m), "
                    f"hp{k}, {self._pos_nsv[k]});")
        return f"const cx<T> w{k} = sxxxxx<T>();"

    def _template_stash_plan(self):
        """Which currents of the template nest wait in LDS: a current formed in
        one loop and read in deeper loops is written once where it is formed
        and read back at the top of every deeper loop that uses it, so it does
        not occupy registers across the loops in between.  Outer currents
        first, up to TEMPLATE_STASH_WORDS words per lane."""
        import re
        self._tstash_loads, self._tstash_puts, self._tstash_words = {}, {}, 0
        rec = []
        self._bind_positions(lambda line: None, "")
        self._emit_template_nest(lambda line: None, "", record=rec)
        items = {}
        for lvl, idx, line in rec:
            items.setdefault((lvl, idx), []).append(line)
        defs, uses = {}, {}
        for (lvl, idx), lines in sorted(items.items()):
            code = "\n".join(lines)
            for nm in re.findall(r"const wf<T> (\w+) =", code):
                defs[nm] = (lvl, idx)
            for t in set(re.findall(r"[A-Za-z_]\w*", code)):
                uses.setdefault(t, set()).add(lvl)
        cand = []
        for nm, (lvl, idx) in defs.items():
            deeper = sorted(l for l in uses.get(nm, ()) if l > lvl)
            if deeper:
                cand.append((lvl, -len(deeper), nm, idx, deeper))
        off = 0
        for lvl, _, nm, idx, deeper in sorted(cand):
            if off + 8 > TEMPLATE_STASH_WORDS:
                break
            self._tstash_puts.setdefault((lvl, idx), []).append((nm, off))
            for l in deeper:
                self._tstash_loads.setdefault(l, []).append((nm, off))
            off += 8
        self._tstash_words = off

    def _emit_template_nest(self, w, ind, record=None, use_stash=True):
        """one ordering's helicity sum as a loop nest over the positions
        (nest.template_schedule); the row of the workspace is the helicity
        combination's index in the canonical table of the legs"""
        p = self.p
        stash = record is None and use_stash
        loads = getattr(self, "_tstash_loads", {}) if stash else {}
        puts = getattr(self, "_tstash_puts", {}) if stash else {}
        nl = self.nl
        sc = nest.template_schedule(p)
        by_level = {}
        for it in sc.items:
            by_level.setdefault(it.level, []).append(it)
        # the running sum of the vertex vectors lives in the loop of the last one
        rs = next(it for it in sc.items if it.kind == "rsum")
        self._rt_level = rs.level
        outer = [(a, cf) for a, cf in rs.data if self._r_level(sc, a) < rs.level]
        if TEMPLATE_EARLY_CURRENT_SUMS or TEMPLATE_EARLY_VERTEX_SUM:
            for lvl in list(by_level):
                by_level[lvl] = self._early_consumers(by_level[lvl], lvl == rs.level)
        lst = by_level[rs.level]
        first = next(i for i, it in enumerate(lst) if it.kind in ("rvec", "rsum"))
        lst.insert(first, nest.Item("rstart", rs.level, tuple(outer), 0))
        by_level[rs.level] = [it for it in lst if it.kind != "rsum"]
        w(f"{ind}// helicity loop nest over positions, outermost first: {sc.order}")
        prev = "0"
        self._done = set()
        self._opaque = set()
        for lvl, k in enumerate(sc.order):
            ch = sc.choices[k]
            if ch != (-1, 1):
                raise NotImplementedError("template nests need two-state positions")
            unrolled = lvl >= len(sc.order) - p.template_unroll
            w(f"{ind}#pragma unroll{'' if unrolled else ' 1'}")
            w(f"{ind}for (int c{k} = 0; c{k} < 2; ++c{k}) {{")
            ind += "  "
            w(f"{ind}const int hp{k} = 2 * c{k} - 1;")
            w(f"{ind}const int r{lvl} = {prev} + (c{k} << ({nl - 1} - lk{k}));")
            prev = f"r{lvl}"
            self._scope = lvl
            if TEMPLATE_KIN_PER_LEVEL:
                self._done = set()
            for nm, off in loads.get(lvl, []):
                w(f"{ind}const wf<T> {nm} = stash_get<wf<T>>(lds_rows, {off});")
            for idx, it in enumerate(by_level.get(lvl, [])):
                if record is not None:
                    self._template_item(lambda line, lvl=lvl, idx=idx: record.append((lvl, idx, line)), it, ind, prev)
                    continue
                self._template_item(w, it, ind, prev)
                for nm, off in puts.get((lvl, idx), []):
                    w(f"{ind}stash_put(lds_rows, {off}, {nm});")
        for _ in sc.order:
            ind = ind[:-2]
            w(f"{ind}}}")
        self._scope = None

    def _early_consumers(self, lst, rt_loop):
        """one loop's items with every consumer that shrinks the live set (a
        vertex vector of the running sum in the sum's loop, a sum of partial
        currents) moved to just after the item that forms the last of its
        operands in this loop, or to the front when none does; movers with the
        same anchor keep their order, every other item keeps its order"""
        p = self.p

        def movable(it):
            if it.kind == "rvec":
                return rt_loop and TEMPLATE_EARLY_VERTEX_SUM
            return (it.kind == "call" and TEMPLATE_EARLY_CURRENT_SUMS
                    and p.calls[it.data[0]].op in ir.LINEAR_OPS)

        def outs(it):
            if it.kind == "ext":
                return (it.data[0],)
            if it.kind == "call":
                return (p.calls[it.data[0]].out,)
            return ()

        out, moved = [], set()
        for it in lst:
            if not movable(it):
                out.append(it)
                continue
            ins = set(p.calls[it.data[0]].ins)
            at = max((i for i, o in enumerate(out) if ins & set(outs(o))), default=-1) + 1
            while at < len(out) and id(out[at]) in moved:
                at += 1
            out.insert(at, it)
            moved.add(id(it))
        rs = [it for it in out if it.kind == "rsum"]
        out = [it for it in out if it.kind != "rsum"] + rs
        assert sorted(map(id, out)) == sorted(map(id, lst))
        return out

    def _r_level(self, sc, amp):
        for it in sc.items:
            if it.kind == "rvec" and self.p.calls[it.data[0]].out == amp:
                return it.level
        raise KeyError(amp)

    def _template_item(self, w, it, ind, row):
        p = self.p
        if it.kind == "ext":
            (k,) = it.data
            self._w, self._ind = w, ind
            w(ind + self._position_external(k, nest=True))
        elif it.kind == "call":
            k, _ = it.data
            self._lazy_kinematics(w, ind, p.calls[k], self._done)
            self._call(w, p.calls[k], ind)
        elif it.kind == "rvec":
            k, sp = it.data
            c = p.calls[k]
            coef = dict(p.jamp[0]).get(c.out, 0.0)
            self._lazy_kinematics(w, ind, c, self._done)
            a = [f"w{x}" for x in c.ins]
            Q = lambda x: f"Qs{self.sname(self.subset[x])}"
            gr = f"g{c.cpl}_0.r"
            fn = nest.ROOT_SPLIT[(c.op, sp)]
            if fn == "vvv_r3":
                rhs = f"vvv_r3<T>({a[0]}, {Q(c.ins[0])}, {a[1]}, {Q(c.ins[1])}, {Q(c.ins[2])}, {gr})"
            elif fn == "gggg_r4":
                rhs = f"gggg_r4<T>({a[0]}, {a[1]}, {a[2]}, {gr})"
            else:
                rhs = f"gggg_r2<T>({a[0]}, {a[2]}, {a[3]}, {gr})"
            if it.level == self._rt_level:
                # accumulate at once, so that only the running sum stays live
                w(f"{ind}Rt = waxpy<T>(T({_c(coef)}), {rhs}, Rt);")
            else:
                w(f"{ind}const wf<T> R{c.out} = {rhs};")
        elif it.kind == "rstart":
            terms = [(a, cf) for a, cf in it.data]
            if terms:
                comps = [" + ".join(f"T({_c(cf)}) * R{a}.c[{m}]" for a, cf in terms) for m in range(4)]
                w(f"{ind}wf<T> Rt = {{{{{', '.join(comps)}}}}};")
            else:
                w(f"{ind}wf<T> Rt = {{}};")
        elif it.kind == "adot":
            w(f"{ind}{self._work_store(row, 'dot(w0, Rt)')}")
        else:
            raise ValueError(it.kind)

    # ------------------------------------------------------------------ calls
    def _call(self, w, c, ind, args=None):
        op, ins, o = c.op, c.ins, c.out
        g0, g1 = f"g{c.cpl}_0", f"g{c.cpl}_1"
        gr = f"g{c.cpl}_0.r"
        pid = c.prop
        mass = f"T(pe{pid}.m)"
        inum = f"mk<T>(T(pe{pid}.inum_r), T(pe{pid}.inum_i))"
        massive = "true" if pid in MASSIVE_VECTORS else "false"
        a = args if args is not None else [f"w{x}" for x in ins]
        Q = lambda x: f"Qs{self.sname(self.subset[x])}"
        if op in AMP_OPS:
            lhs = f"{ind}const cx<T> amp{o} = "
        elif ir.OUT_KIND[op] == S:
            lhs = f"{ind}const cx<T> w{o} = "
        else:
            lhs = f"{ind}const wf<T> w{o} = "
        d = f"d{self.sname(self.subset[o])}_{pid}" if op not in AMP_OPS and op not in LINEAR_OPS else ""
        if op == "iov":
            rhs = f"iovxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {g1})"
        elif op == "fvi":
            rhs = f"fvixxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {Q(o)}, {mass}, {d})"
        elif op == "fvo":
            rhs = f"fvoxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {Q(o)}, {mass}, {d})"
        elif op == "jio":
            rhs = f"jioxxx<T, {massive}>({a[0]}, {a[1]}, {g0}, {g1}, {Q(o)}, {inum}, {d})"
        elif op == "ios":
            rhs = f"iosxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0}, {g1})"
        elif op == "fsi":
            rhs = f"fsixxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {Q(o)}, {mass}, {d})"
        elif op == "fso":
            rhs = f"fsoxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {Q(o)}, {mass}, {d})"
        elif op == "hio":
            rhs = f"hioxxx<T>({a[0]}, {a[1]}, {g0}, {g1}, {d})"
        elif op == "vvv":
            rhs = f"vvvxxx<T>({a[0]}, {Q(ins[0])}, {a[1]}, {Q(ins[1])}, {a[2]}, {Q(ins[2])}, {gr})"
        elif op == "jvv":
            rhs = f"jvvxxx<T, {massive}>({a[0]}, {Q(ins[0])}, {a[1]}, {Q(ins[1])}, {gr}, {inum}, {d})"
        elif op == "gggg":
            rhs = f"ggggxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {gr})"
        elif op == "jggg":
            rhs = f"jgggxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {gr}, {Q(o)}, {inum}, {d})"
        elif op == "wwww":
            rhs = f"wwwwxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {gr})"
        elif op == "jwww":
            rhs = f"jwwwxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {gr}, {Q(o)}, {inum}, {d})"
        elif op == "vvs":
            rhs = f"vvsxxx<T>({a[0]}, {a[1]}, {a[2]}, {g0})"
        elif op == "jvs":
            rhs = f"jvsxxx<T, {massive}>({a[0]}, {a[1]}, {g0}, {Q(o)}, {inum}, {d})"
        elif op == "hvv":
            rhs = f"hvvxxx<T>({a[0]}, {a[1]}, {g0}, {d})"
        elif op == "vvss":
            rhs = f"vvssxx<T>({a[0]}, {a[1]}, {a[2]}, {a[3]}, {g0})"
        elif op == "jvss":
            rhs = f"jvssxx<T, {massive}>({a[0]}, {a[1]}, {a[2]}, {g0}, {Q(o)}, {inum}, {d})"
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
        elif op == "vadd":
            rhs = f"vadd<T>({a[0]}, {a[1]})"
        elif op == "vsub":
            rhs = f"vsub<T>({a[0]}, {a[1]})"
        else:
            raise ValueError(op)
        w(lhs + rhs + ";")

    def _colour(self, w, J, ind="      "):
        """me2 += Re(J^dagger C J) with the constant colour matrix C = num / den"""
        p = self.p
        den = p.colour_denominator()
        n = p.n_flows
        w(f"{ind}T cs = T(0);")
        for f in range(n):
            w(f"{ind}{{")
            w(f"{ind}  const cx<T> jf = {J(f)};")
            w(f"{ind}  T r = T({_c(Fraction(p.colour[f][f]) * den)}) * norm2(jf);")
            for g in range(f + 1, n):
                cfg = Fraction(p.colour[f][g]) * den
                if cfg != 0:
                    w(f"{ind}  {{ const cx<T> jg = {J(g)}; r += T({_c(2 * cfg)}) * (jf.r * jg.r + jf.i * jg.i); }}")
            w(f"{ind}  cs += r;")
            w(f"{ind}}}")
        w(f"{ind}me2 += double(cs) * {_c(Fraction(1, den))};")


    def _colour_compressed(self, w, J, ind="      "):
        """me2 += Re(J^dagger C J) with the rows of C decomposed into their
        distinct colour factors (the paper's Sec. 5.4): row f sums the flows
        g >= f that share a factor first, then multiplies each such sum once,
        T_f = sum_k c_k (sum over g >= f with C'_fg = c_k of J_g), where C' is C
        on the diagonal and 2 C above it; |M|^2 = sum_f Re(J_f^* T_f)."""
        p = self.p
        den = p.colour_denominator()
        n = p.n_flows
        w(f"{ind}T cs = T(0);")
        for f in range(n):
            groups = {}
            for g in range(f, n):
                v = Fraction(p.colour[f][g]) * den * (1 if g == f else 2)
                if v != 0:
                    groups.setdefault(v, []).append(g)
            if not groups:
                continue
            w(f"{ind}{{")
            w(f"{ind}  cx<T> t = {{T(0), T(0)}};")
            for v, gs in groups.items():
                w(f"{ind}  t = t + T({_c(v)}) * ({' + '.join(J(g) for g in gs)});")
            w(f"{ind}  cs += {J(f)}.r * t.r + {J(f)}.i * t.i;")
            w(f"{ind}}}")
        w(f"{ind}me2 += double(cs) * {_c(Fraction(1, den))};")

    def _colour_form(self, w, J, ind="      "):
        """the IR's colour form on VALU"""
        if self.p.colour_form == "compressed":
            self._colour_compressed(w, J, ind)
        else:
            self._colour(w, J, ind)


_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
_DEVICE_HEADERS = ("generated_common.hpp", "heget_device.hpp", "kernel_args.hpp", "phase_space.hpp",
                   "colour_mfma.hpp")


def source_digest(proc):
    """SHA-256 over a process kernel's generated source and the device headers
    it includes: it changes whenever the compiled kernel can change, so a
    measurement tied to one kernel can tell that it has gone stale."""
    import hashlib
    from . import build
    h = hashlib.sha256(Gen(proc).emit().encode())
    flags = [f for k, f in enumerate(build.FLAGS) if f != "-I" and (k == 0 or build.FLAGS[k - 1] != "-I")]
    h.update(" ".join(flags + build.GEN_FLAGS).encode())   # the compile flags, less include paths
    for name in _DEVICE_HEADERS:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def generate(proc, out_dir):
    src = Gen(proc).emit()
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
    from .build import PROCESSES
    for name in PROCESSES:
        print(generate(processes.by_name(name), out))


if __name__ == "__main__":
    main(sys.argv)
