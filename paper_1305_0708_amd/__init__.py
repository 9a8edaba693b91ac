"""heget on MI355X: per-event tree-level SM helicity amplitudes (HEGET-style)
as hand-written HIP for gfx950 behind the C ABI of include/heget.h.

Python is argument marshalling only: ``Process`` turns an ``ir.Process`` into
the C IR structs, and ``eval`` / ``integrate`` pass device pointers and the
current HIP stream to libheget.so.  PyTorch provides device memory and
streams.  Every step of the amplitude path runs in the library's kernels; if
libheget.so is missing the calls raise.
"""
import ctypes

from . import _lib, ir
from ._lib import HEGET_FP64, HEGET_MIXED, HegetError, check

__all__ = ["Process", "default_sm", "HegetError", "ir"]


def default_sm(**kw):
    """SM inputs of the benchmark workloads (overridable by keyword)."""
    d = dict(alpha=1.0 / 128.0, sw2=0.2222, mz=91.1876, wz=2.4952, mw=80.4, ww=2.085,
             mt=175.0, wt=1.55, mh=125.0, wh=0.00407, alpha_s=0.118, mb_yuk=4.7, complex_mass=0)
    d.update(kw)
    return d


class _IRBuffers:
    """C structs for one ir.Process, kept alive while the library reads them."""

    def __init__(self, proc, sm, helicities=None):
        L = _lib
        self.legs = (L.heget_leg * proc.n_legs)(*[
            L.heget_leg(l.kind, int(l.incoming), l.flow, l.particle, l.colour) for l in proc.legs])
        self.cpl = (L.heget_coupling * len(proc.couplings))(*[
            L.heget_coupling(ir.CPL[c.kind], c.particle, c.charge, c.t3) for c in proc.couplings])
        calls = []
        for c in proc.calls:
            ins = list(c.ins) + [-1] * (4 - len(c.ins))
            calls.append(L.heget_call(ir.OP[c.op], (ctypes.c_int32 * 4)(*ins), c.out, c.cpl, c.prop))
        self.calls = (L.heget_call * len(calls))(*calls)
        dense = [0.0] * (len(proc.jamp) * proc.n_amps * 2)
        for f, terms in enumerate(proc.jamp):
            for a, coef in terms:
                k = (f * proc.n_amps + a) * 2
                dense[k] += complex(coef).real
                dense[k + 1] += complex(coef).imag
        self.jamp = (ctypes.c_double * len(dense))(*dense)
        den = proc.colour_denominator()
        num = [float(x * den) for row in proc.colour for x in row]
        self.colour = (ctypes.c_double * len(num))(*num)
        hels = helicities if helicities is not None else proc.helicities
        flat = [int(h) for row in hels for h in row]
        self.hel = (ctypes.c_int8 * len(flat))(*flat)
        self.sm = L.heget_sm(**sm)
        orders = proc.orderings or []
        flat_o = [int(x) for o in orders for x in o]
        self.orders = (ctypes.c_int8 * max(len(flat_o), 1))(*flat_o)
        flat_m = [int(x) for r in (proc.flow_map or []) for x in r]
        self.flow_map = (ctypes.c_int8 * max(len(flat_m), 1))(*flat_m)
        tree = proc.ps_tree or []
        self.ps_nodes = (L.heget_ps_node * max(len(tree), 1))(*[
            L.heget_ps_node(part, mapping, (ctypes.c_int32 * 2)(d0, d1)) for part, mapping, d0, d1 in tree])
        self.ir = L.heget_process_ir(
            proc.n_legs, self.legs, self.sm, len(proc.couplings), self.cpl, len(calls), self.calls,
            proc.n_amps, proc.n_flows, self.jamp, self.colour, float(den), len(hels), self.hel,
            proc.n_a_n_b, proc.symmetry, int(proc.cut_enabled), proc.cut_pt, proc.cut_dr,
            len(orders), self.orders if orders else None, self.flow_map if flat_m else None,
            len(tree), self.ps_nodes if tree else None, float(proc.ps_window),
            float(proc.ps_hadronic[0]) if proc.ps_hadronic else 0.0,
            float(proc.ps_hadronic[1]) if proc.ps_hadronic else 0.0,
            ir.COLOUR_FORMS[proc.colour_form], ir.DIVISIONS[proc.division])


def uniforms(n, n_u, seed=0, counter_offset=0, stream=None):
    """The Philox step alone: uniforms of events counter_offset .. + n - 1 as a
    float64 CUDA tensor [n_u][n] (heget_uniforms)."""
    import torch
    out = torch.empty((n_u, max(n, 0)), dtype=torch.float64, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    check(_lib.load().heget_uniforms(seed, counter_offset, n, n_u, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(s.cuda_stream)))
    return out


def result_from_sums(sums, n, lib=None):
    """The heget_integrate result of n events from the three sums (sum w,
    sum w^2, accepted) that heget_integrate_async writes (heget_result_from_sums)."""
    L = lib or _lib.load()
    h = (ctypes.c_double * 3)(*[float(x) for x in list(sums)[:3]])
    r = _lib.heget_result()
    check(L.heget_result_from_sums(h, n, ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in r._fields_}


class Process:
    """A created process handle (heget_process_create)."""

    def __init__(self, proc, precision="fp64", sm=None, helicities=None):
        self.ir = proc
        s = default_sm(**proc.sm_overrides)
        if sm:
            s.update(sm)
        self._buf = _IRBuffers(proc, s, helicities)
        self._lib = _lib.load()
        self.precision = precision
        prec = HEGET_FP64 if precision == "fp64" else HEGET_MIXED
        h = ctypes.c_void_p()
        check(self._lib.heget_process_create(ctypes.byref(self._buf.ir), prec, ctypes.byref(h)))
        self._h = h

    @property
    def n_legs(self):
        return self.ir.n_legs

    @property
    def n_helicities(self):
        return self._lib.heget_process_n_helicities(self._h)

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def eval(self, n=None, momenta=None, seed=0, counter_offset=0, sqrt_s=None, me2_out=None,
             momenta_out=None, want_momenta=False, stream=None):
        """|M|^2 summed over helicities and colours for n events.  momenta: a
        float64 CUDA tensor [n_legs][4][n] (SoA) or None to generate them from
        (seed, counter_offset, sqrt_s).  Returns me2 (and momenta if requested)."""
        import torch
        if momenta is not None:
            if momenta.dtype != torch.float64 or not momenta.is_cuda or not momenta.is_contiguous():
                raise ValueError("momenta must be a contiguous float64 CUDA tensor")
            if momenta.dim() != 3 or momenta.shape[0] != self.n_legs or momenta.shape[1] != 4:
                raise ValueError(f"momenta must have shape [{self.n_legs}][4][n]")
            n = momenta.shape[2] if n is None else n
            if n != momenta.shape[2]:
                raise ValueError("n does not match momenta")
        if n is None:
            raise ValueError("n is required when momenta are generated")
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        dev = momenta.device if momenta is not None else torch.device("cuda")
        if n < 0:
            # let the library report the invalid size
            check(self._lib.heget_eval(self._h, n, None, seed, counter_offset, float(sqrt_s), None, None,
                                       self._stream(stream)))
        if me2_out is None:
            me2_out = torch.empty(n, dtype=torch.float64, device=dev)
        if want_momenta and momenta_out is None:
            momenta_out = torch.empty((self.n_legs, 4, n), dtype=torch.float64, device=dev)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        check(self._lib.heget_eval(self._h, n, ptr(momenta), seed, counter_offset, float(sqrt_s),
                                   ptr(me2_out), ptr(momenta_out), self._stream(stream)))
        return (me2_out, momenta_out) if want_momenta else me2_out

    def generate(self, n, seed=0, counter_offset=0, sqrt_s=None, momenta_out=None, want_weights=False,
                 stream=None):
        """The momenta heget_eval generates (Philox -> the process's phase
        space), as a float64 CUDA tensor [n_legs][4][n], without evaluating
        |M|^2; with want_weights also each event's phase-space weight [n]."""
        import torch
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        if momenta_out is None:
            momenta_out = torch.empty((self.n_legs, 4, max(n, 0)), dtype=torch.float64, device="cuda")
        weights = torch.empty(max(n, 0), dtype=torch.float64, device="cuda") if want_weights else None
        check(self._lib.heget_generate(self._h, n, seed, counter_offset, float(sqrt_s),
                                       ctypes.c_void_p(momenta_out.data_ptr()),
                                       ctypes.c_void_p(weights.data_ptr()) if weights is not None else None,
                                       self._stream(stream)))
        return (momenta_out, weights) if want_weights else momenta_out

    def integrate(self, n, seed=0, sqrt_s=None, stream=None):
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        r = _lib.heget_result()
        check(self._lib.heget_integrate(self._h, n, float(sqrt_s), seed, ctypes.byref(r), self._stream(stream)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    def integrate_async(self, n, sums_out, seed=0, sqrt_s=None, stream=None):
        """heget_integrate_async: enqueue one integrate step and return at
        once; sums_out (a float64 CUDA tensor, 3 contiguous values) receives
        (sum w, sum w^2, accepted) when the stream gets there."""
        import torch
        if sums_out.dtype != torch.float64 or not sums_out.is_cuda or not sums_out.is_contiguous() \
                or sums_out.numel() < 3:
            raise ValueError("sums_out must be a contiguous float64 CUDA tensor of at least 3 values")
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        check(self._lib.heget_integrate_async(self._h, n, float(sqrt_s), seed, ctypes.c_void_p(sums_out.data_ptr()),
                                              self._stream(stream)))
        return sums_out

    def result_from_sums(self, sums, n):
        """heget_result_from_sums: the heget_integrate result of n events from
        the three sums of integrate_async (a sequence of 3 floats)"""
        return result_from_sums(sums, n, self._lib)

    def integrate_noalloc(self, n, seed=0, sqrt_s=None, stream=None):
        """heget_integrate_noalloc: heget_integrate with no allocation in the
        call (the library's fixed scratch; n <= HEGET_NOALLOC_MAX_EVENTS)"""
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        r = _lib.heget_result()
        check(self._lib.heget_integrate_noalloc(self._h, n, float(sqrt_s), seed, ctypes.byref(r),
                                                self._stream(stream)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    @property
    def grid_dims(self):
        """uniforms per event that an adaptive grid maps (0 for RAMBO processes)"""
        return self._lib.heget_process_grid_dims(self._h)

    def integrate_adaptive(self, n, iterations=5, bins=16, seed=0, sqrt_s=None, stream=None):
        """heget_integrate_adaptive: (per-pass results, combined result, chi^2
        per degree of freedom, final grid [dims][bins + 1] as numpy)"""
        import numpy as np
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        per = (_lib.heget_result * iterations)()
        comb = _lib.heget_result()
        chi2 = ctypes.c_double()
        dims = max(self.grid_dims, 0)
        grid = np.zeros((dims, bins + 1))
        gp = grid.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if dims else None
        check(self._lib.heget_integrate_adaptive(self._h, n, iterations, bins, float(sqrt_s), seed, per,
                                                 ctypes.byref(comb), ctypes.byref(chi2), gp,
                                                 self._stream(stream)))
        as_dict = lambda r: {k: getattr(r, k) for k, _ in r._fields_}
        return [as_dict(r) for r in per], as_dict(comb), chi2.value, grid

    def filter_helicities(self, n_probe=64, seed=12345, sqrt_s=None, rel_threshold=1e-20):
        sqrt_s = self.ir.sqrt_s if sqrt_s is None else sqrt_s
        kept = ctypes.c_int32()
        check(self._lib.heget_filter_helicities(self._h, n_probe, seed, float(sqrt_s), rel_threshold,
                                                ctypes.byref(kept)))
        return kept.value

    def close(self):
        if getattr(self, "_h", None):
            check(self._lib.heget_process_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The serving engine (heget_server_*): requests heget_integrate(process,
    n, sqrt_s, seed) submitted at any time run as fused launches over the
    resident processes; results are bit-identical to Process.integrate."""

    def __init__(self, processes, arena_bytes=1 << 30, slots_per_process=2, max_batch_blocks=4096,
                 max_chunk_blocks=1024):
        self._lib = _lib.load()
        self._procs = list(processes)               # keep the handles alive
        arr = (ctypes.c_void_p * len(self._procs))(*[p._h.value for p in self._procs])
        self._arr = arr
        cfg = _lib.heget_server_config(len(self._procs), ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)),
                                       int(arena_bytes), int(slots_per_process), int(max_batch_blocks),
                                       int(max_chunk_blocks))
        h = ctypes.c_void_p()
        check(self._lib.heget_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._me2 = {}

    def submit(self, process, n, seed, sqrt_s, want_me2=False):
        """Queue a request for self.processes[process]; returns its ticket."""
        import numpy as np
        buf = np.empty(n, dtype=np.float64) if want_me2 else None
        t = ctypes.c_uint64()
        ptr = ctypes.c_void_p(buf.ctypes.data) if buf is not None else None
        check(self._lib.heget_server_submit(self._h, int(process), int(n), int(seed), float(sqrt_s), ptr,
                                            ctypes.byref(t)))
        if buf is not None:
            self._me2[t.value] = buf
        return t.value

    def poll(self, ticket, wait=True):
        """None if not done (wait=False), else (result dict, latency in s[, |M|^2 array])."""
        r = _lib.heget_result()
        lat = ctypes.c_double()
        done = ctypes.c_int32()
        try:
            check(self._lib.heget_server_poll(self._h, int(ticket), 1 if wait else 0, ctypes.byref(r),
                                              ctypes.byref(lat), ctypes.byref(done)))
        except Exception:
            self._me2.pop(ticket, None)
            raise
        if not done.value:
            return None
        res = {k: getattr(r, k) for k, _ in r._fields_}
        me2 = self._me2.pop(ticket, None)
        return (res, lat.value) if me2 is None else (res, lat.value, me2)

    def stats(self):
        st = _lib.heget_server_stats()
        check(self._lib.heget_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            check(self._lib.heget_server_destroy(self._h))
            self._h = None
            self._me2.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
