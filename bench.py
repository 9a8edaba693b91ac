"""Benchmark: helicity- and colour-summed |M|^2 events/s on one GPU.

Workload: g g -> t tbar -> (b e+ nu_e)(bbar mu- nu_mu~) at sqrt(s_hat) = 1 TeV,
2^20 RAMBO events per step from a Philox seed, all 256 helicity combinations,
two colour flows.  One step = the whole hot path over one batch: Philox ->
RAMBO -> external wavefunctions -> vertex/propagator chain -> jamps ->
colour form -> helicity sum -> weights -> deterministic cross-section
reduction (heget_integrate).  The FP64 path is the headline; the mixed
path, and both with exactly-vanishing helicities filtered out, are reported
beside it.

Prints ONE JSON line (rank 0).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "helicity+colour-summed |M|^2 events/s, FP64 vs mixed; p50/p99 serve latency"
N_EVENTS = 1 << 20
SQRT_S = 1000.0
SEED = 0x48454746
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector (packed)

# Counter measurements of one amplitude-kernel launch in the integrate step
# (FP64, 2^20 events), tied to the kernel source they were taken on (a
# different digest reports them as null / falls back to the flop model):
#  * HBM traffic from two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE;
#    KiB per dispatch, steady-state launches), scaled by what the same counters
#    read for a plain 1 GiB device copy in the same runs (FETCH_SIZE read
#    524,299.5 KiB for 1,048,576 KiB fetched -> x2.0; WRITE_SIZE read
#    1,048,576 KiB -> x1.0);
#  * FP64 flops executed per event, 2 FMA + MUL + ADD + TRANS from the
#    SQ_INSTS_VALU_*_F64 counters per wave (one event per lane): the arithmetic
#    the compiled kernel does, after the compiler has dropped the operations on
#    the structural zeros of fixed-helicity massless spinors that the IR flop
#    model still counts; the same from SQ_INSTS_VALU_*_F32 for the mixed kernel.
# All were re-taken on the kernel with the bra sums accumulated bra by bra
# (the same values as on the kernel before it).
COUNTERS_FP64 = {"source_digest": "a6d472db08ef9e1a5f8d879906a6034d4bcf3e5b4b04639feffeaf8ecf2bc8bf",
                 "fetch_kib": 832.5625, "fetch_scale": 2.0, "write_kib": 63189.25, "write_scale": 1.0,
                 "flop_per_event": 3990, "flop_per_event_mixed": 2331}


# Counter measurements of further kernels, (process, precision) -> figures per
# event from rocprofv3 --pmc runs of `bench.py --profile-leg <prec>
# --profile-proc <process>` (the summaries under profiles/), tied to the kernel
# source they were taken on: executed VALU flops (2 FMA + MUL + ADD + TRANS of
# the precision's SQ_INSTS_VALU_* counters x 64 lanes, per event) and, for the
# MFMA colour form, MFMA flops (SQ_INSTS_VALU_MFMA_MOPS_* x 512 per event).
KERNEL_COUNTERS = {
    # u d -> u d H H -> 4b, 2^21 events per launch (profiles/amp_ud_udhh_4b_2p21ev.md)
    ("ud_udhh_4b", "mixed"): {
        "source_digest": "b9b1fce845d836bd1039eff40ff5ebbfd9d44327065d42117192dcaadc27c0c8",
        "valu_flop_per_event": 3004, "fp64_flop_per_event": 2219, "events": 1 << 21, "kernel_s": 0.2567e-3,
        "source": "executed FP32 flops from SQ_INSTS_VALU_*_F32 (FP64 denominators and reductions beside)"},
    ("ud_udhh_4b", "fp64"): {
        "source_digest": "b9b1fce845d836bd1039eff40ff5ebbfd9d44327065d42117192dcaadc27c0c8",
        "valu_flop_per_event": 5223, "events": 1 << 21, "kernel_s": 0.3522e-3,
        "source": "executed FP64 flops from SQ_INSTS_VALU_*_F64"},
    # u ubar -> t tbar g g g, 2^18 events per launch (profiles/amp_uu_ttggg_2p18ev.md)
    ("uu_ttggg", "fp64"): {
        "source_digest": "403c91b4612e1d795cd305f62fcab31dc1c0cf2a6a88f44eeb8ce20437242777",
        "valu_flop_per_event": 28103623, "events": 1 << 18, "kernel_s": 239.8e-3,
        "source": "executed FP64 flops from SQ_INSTS_VALU_*_F64"},
    ("uu_ttggg", "mixed"): {
        "source_digest": "403c91b4612e1d795cd305f62fcab31dc1c0cf2a6a88f44eeb8ce20437242777",
        "valu_flop_per_event": 20706944, "fp64_flop_per_event": 909127, "events": 1 << 18, "kernel_s": 145.6e-3,
        "source": "executed FP32 flops from SQ_INSTS_VALU_*_F32 (FP64 momenta and denominators beside)"},
    # g g -> g g g g, 2^20 events per launch (profiles/amp_gg_4g_mfma_2p20ev.md)
    ("gg_4g", "fp64"): {
        "source_digest": "5b85ba6f8532ce81d46e3714da91ba4bec0c80b05b387f10be4666f477c1b3bd",
        "valu_flop_per_event": 3613187, "mfma_flop_per_event": 2097152, "events": 1 << 20, "kernel_s": 174.6e-3,
        "source": "executed FP64 flops from SQ_INSTS_VALU_*_F64; MFMA flops from SQ_INSTS_VALU_MFMA_MOPS_F64"},
    ("gg_4g_ddm", "fp64"): {
        "source_digest": "24d9abe3bc7ecc28d42dbbe3825031185b1e9827b5ad7a5d64b8ce331e623c95",
        "valu_flop_per_event": 3556867, "events": 1 << 20, "kernel_s": 93.6e-3,
        "source": "executed FP64 flops from SQ_INSTS_VALU_*_F64"},
    ("gg_4g_ddm", "mixed"): {
        "source_digest": "24d9abe3bc7ecc28d42dbbe3825031185b1e9827b5ad7a5d64b8ce331e623c95",
        "valu_flop_per_event": 2810735, "fp64_flop_per_event": 125396, "events": 1 << 20, "kernel_s": 62.6e-3,
        "source": "executed FP32 flops from SQ_INSTS_VALU_*_F32 (FP64 kinematics beside)"},
    ("gg_4g_cf", "mixed"): {
        "source_digest": "b22b89d2ceeced9ef238bf79b940b1d4c77e76fdb346325a6d7b8b5c41311eec",
        "valu_flop_per_event": 3790063, "fp64_flop_per_event": 125396, "events": 1 << 20, "kernel_s": 87.7e-3,
        "source": "executed FP32 flops from SQ_INSTS_VALU_*_F32 (FP64 kinematics beside)"},
}


def counters_valid(proc_ir):
    from paper_1305_0708_amd import codegen
    return codegen.source_digest(proc_ir) == COUNTERS_FP64["source_digest"]


def measured_traffic(proc_ir):
    t = COUNTERS_FP64
    if not counters_valid(proc_ir):
        return None
    return 1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def time_path(torch, proc, steps, warmup, n=N_EVENTS, sqrt_s=SQRT_S, seed=SEED, synchronous_too=False):
    """Per step: one integrate step of n events (Philox, phase space, the
    amplitude kernel with its per-block partial sums, the fixed-order
    reduction) queued with heget_integrate_async, its three sums into a row of
    a device buffer; the steps run back to back and the host waits once, after
    the last.  Every step's result is read back and turned into a cross
    section after the timed region.  With synchronous_too also the
    heget_integrate call, which waits for each step's result.  Also times the
    amplitude kernel alone with HIP events on the launch stream.
    Returns (seconds per step, kernel seconds, last step's result, seconds per
    synchronous step or None)."""
    sums = torch.empty((max(steps, warmup, 1), 3), dtype=torch.float64, device="cuda")
    rows = [sums[k] for k in range(sums.shape[0])]
    stream = torch.cuda.current_stream()
    for k in range(warmup):
        proc.integrate_async(n, rows[k], seed=seed, sqrt_s=sqrt_s, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        proc.integrate_async(n, rows[k], seed=seed + k, sqrt_s=sqrt_s, stream=stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    res = [proc.result_from_sums(row, n) for row in sums[:steps].cpu().tolist()]
    r = res[-1]
    wall_sync = None
    if synchronous_too:
        t0 = time.perf_counter()
        for k in range(steps):
            rs = proc.integrate(n, seed=seed + k, sqrt_s=sqrt_s, stream=stream)
        torch.cuda.synchronize()
        wall_sync = (time.perf_counter() - t0) / steps
        assert rs == r, "the synchronous call must give the queued step's result"
    # amplitude kernel alone: eval with |M|^2 written, timed with events on the stream it runs on
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    proc.eval(n=n, seed=seed, sqrt_s=sqrt_s, me2_out=out)
    ev0.record(stream)
    for k in range(steps):
        proc.eval(n=n, seed=seed + k, sqrt_s=sqrt_s, me2_out=out)
    ev1.record(stream)
    ev1.synchronize()
    kern = ev0.elapsed_time(ev1) / 1e3 / steps
    return wall, kern, r, wall_sync


def settle_clocks(torch, proc, seconds=0.5, n=N_EVENTS, sqrt_s=SQRT_S):
    """untimed launches of the kernel about to be timed for about half a
    second before the warm-up steps, so that the GPU has left its idle clocks
    when timing starts (the first timed steps of a fresh box otherwise run
    slow)"""
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        proc.eval(n=n, seed=SEED, sqrt_s=sqrt_s, me2_out=out)
        torch.cuda.synchronize()


def cpu_baseline(oracle, target_seconds=12.0):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    mom = oracle.generate(SEED, 256, 6, SQRT_S)
    t0 = time.perf_counter()
    oracle.me2(oracle.GG_TT_6F, mom, oracle.params(), threads=cores)
    rate = 256 / (time.perf_counter() - t0)
    n = int(min(max(rate * target_seconds, 512), 200000))
    mom = oracle.generate(SEED, n, 6, SQRT_S)
    t0 = time.perf_counter()
    f = oracle.me2(oracle.GG_TT_6F, mom, oracle.params(), threads=cores)
    dt = time.perf_counter() - t0
    assert np.all(f > 0)
    # the same oracle on one core, on a smaller sample (about 3 s)
    n1 = int(min(max(n / dt / cores * 3.0, 64), n))
    t0 = time.perf_counter()
    oracle.me2(oracle.GG_TT_6F, mom[:n1], oracle.params(), threads=1)
    dt1 = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": n / dt, "unit": "events/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} events of the same workload (first {n} Philox counters), {dt:.1f} s",
            "value_1core": n1 / dt1, "sample_1core": f"first {n1} of those events, {dt1:.1f} s",
            "cpu": cpu}


HBM_PEAK_GBS = 8000.0       # MI355X HBM3E


def resonance_leg(torch, H, processes, steps, warmup, r_rambo):
    """C1 with the paper's resonance phase space (Appendix A: tops and W's
    Breit-Wigner mapped within min(20, m/Gamma) widths) in place of RAMBO:
    integrate steps of 2^20 events in FP64, and the Monte Carlo error of sigma
    against RAMBO's.  The tree's sigma is the rate inside the resonance windows,
    RAMBO's the whole phase space."""
    proc = H.Process(processes.gg_ttbar_6f_bw(), precision="fp64")
    wall, kern, r, _ = time_path(torch, proc, steps, warmup)
    return {"workload": "gg->ttbar->6f as configured, events from the resonance tree "
                        "(t, tbar, W+, W- Breit-Wigner mapped) instead of RAMBO",
            "events_per_s": N_EVENTS / wall, "ms_per_step": wall * 1e3, "kernel_ms": kern * 1e3,
            "sigma_pb": r["sigma_pb"], "sigma_err_pb": r["err_pb"],
            "rel_err": r["err_pb"] / r["sigma_pb"],
            "rambo_rel_err": r_rambo["err_pb"] / r_rambo["sigma_pb"]}


def adaptive_leg(torch, H, processes, passes=6, bins=32):
    """heget_integrate_adaptive on the resonance-tree C1: passes of 2^20 FP64
    events through a VEGAS grid refined after each (the BASES role of the
    paper's Sec. 1 and 6).  Wall time per pass includes the per-pass bin sums
    and grid refinement on the device and the call's final synchronisation
    (the handle's buffers are allocated by the warm-up call)."""
    import time
    proc = H.Process(processes.gg_ttbar_6f_bw(), precision="fp64")
    proc.integrate_adaptive(N_EVENTS, iterations=2, bins=bins, seed=SEED, sqrt_s=SQRT_S)   # warm-up, buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per, comb, chi2, _ = proc.integrate_adaptive(N_EVENTS, iterations=passes, bins=bins, seed=SEED, sqrt_s=SQRT_S)
    wall = time.perf_counter() - t0
    rel = [p["err_pb"] / p["sigma_pb"] for p in per]
    return {"workload": f"gg->ttbar->6f, resonance tree, {passes} passes of 2^20 events, {bins} bins x "
                        f"{proc.grid_dims} dims",
            "events_per_s": passes * N_EVENTS / wall, "ms_per_pass": wall / passes * 1e3,
            "rel_err_per_pass": [round(x, 6) for x in rel],
            "sigma_pb": comb["sigma_pb"], "sigma_err_pb": comb["err_pb"], "chi2_per_dof": chi2}


def counter_figures(pir, prec, kern_s, n):
    """executed TFLOP/s of a kernel from counters taken on the same kernel
    source (None when no counters match it)"""
    from paper_1305_0708_amd import codegen
    c = KERNEL_COUNTERS.get((pir.name, prec))
    if c is None or codegen.source_digest(pir) != c["source_digest"]:
        return None
    out = {"flop_per_event": c["valu_flop_per_event"], "source": c["source"],
           "valu_tflops": c["valu_flop_per_event"] * n / kern_s / 1e12,
           "valu_peak": FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS}
    if "mfma_flop_per_event" in c:
        out["mfma_tflops"] = c["mfma_flop_per_event"] * n / kern_s / 1e12
        out["mfma_peak"] = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
    return out


def config_leg(torch, H, pir, workload, steps, warmup, n=N_EVENTS, precisions=("fp64", "mixed"), seed=SEED):
    """integrate steps of n events of one more configuration, per precision; a
    precision the library refuses for this process is reported as refused"""
    out = {"workload": workload, "events_per_step": n}
    for prec in precisions:
        try:
            proc = H.Process(pir, precision=prec)
        except H.HegetError as e:
            out[prec] = {"refused": str(e)}
            continue
        settle_clocks(torch, proc, n=n, sqrt_s=pir.sqrt_s)
        wall, kern, r, _ = time_path(torch, proc, steps, warmup, n=n, sqrt_s=pir.sqrt_s, seed=seed)
        out[prec] = {"events_per_s": n / wall, "ms_per_step": wall * 1e3, "kernel_ms": kern * 1e3,
                     "sigma_pb": r["sigma_pb"], "sigma_err_pb": r["err_pb"], "n_accepted": r["n_accepted"]}
        cf = counter_figures(pir, prec, kern, n)
        if cf:
            out[prec]["counters"] = cf
        proc.close()
    return out


def oracle_leg(torch, H, oracle, pir, oracle_proc, oracle_kw, nout, seed, cut=None, target_seconds=3.0,
               precisions=("fp64", "mixed"), extended=False):
    """The oracle beside the GPU on a bounded sample of the same workload:
    its events/s on every host core, and the GPU's error against it on the
    sample's events (the oracle's momenta fed to heget_eval): max and median
    relative error of |M|^2 per precision, and the relative error of sigma over
    the sample (the same RAMBO weight on both sides)."""
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    pid, prm = getattr(oracle, oracle_proc), oracle.params(**oracle_kw)
    probe = oracle.generate(seed, 64, nout, pir.sqrt_s)
    t0 = time.perf_counter()
    oracle.me2(pid, probe, prm, threads=cores)
    rate = 64 / (time.perf_counter() - t0)
    n = int(min(max(rate * target_seconds, 256), 1 << 18))
    mom = oracle.generate(seed, n, nout, pir.sqrt_s)
    t0 = time.perf_counter()
    f = oracle.me2(pid, mom, prm, threads=cores)
    dt = time.perf_counter() - t0
    passed = oracle.cut_gluons(mom, *cut) if cut else np.ones(n, dtype=np.int32)
    f = f * passed
    out = {"value": n / dt, "unit": "events/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} events of the same workload (first {n} Philox counters), {dt:.1f} s"}
    if extended:
        t0 = time.perf_counter()
        f = oracle.me2(pid, mom, prm, threads=cores, extended=True) * passed
        out["reference"] = f"long-double oracle on the sample ({time.perf_counter() - t0:.1f} s)"
    vol = oracle.phase_space_volume(pir.sqrt_s, nout)
    sig_ref = oracle.cross_section(f, vol, pir.sqrt_s, pir.n_a_n_b, pir.symmetry, passed=passed)[0]
    soa = torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()
    nz = f != 0
    for prec in precisions:
        try:
            proc = H.Process(pir, precision=prec)
        except H.HegetError as e:
            out[f"{prec}_error"] = {"refused": str(e)}
            continue
        got = proc.eval(momenta=soa).cpu().numpy()
        proc.close()
        err = np.abs(got[nz] - f[nz]) / np.abs(f[nz])
        sig = oracle.cross_section(got, vol, pir.sqrt_s, pir.n_a_n_b, pir.symmetry, passed=passed)[0]
        out[f"{prec}_error"] = {"me2_max_rel": float(err.max()), "me2_median_rel": float(np.median(err)),
                                "sigma_rel": sig / sig_ref - 1.0, "events": int(nz.sum()),
                                "cut_events_exactly_zero": bool(np.all(got[~nz] == 0.0))}
    return out


def tree_oracle_leg(torch, H, oracle, pir, oracle_proc, seed, target_seconds=3.0, precisions=("fp64", "mixed")):
    """oracle_leg for a process whose phase space is a tree of flat two-body
    steps with massive final legs: the oracle's own tree generator gives the
    sample's momenta and weights"""
    import numpy as np
    from oracle import phase_space_tree as T
    from paper_1305_0708_amd import ir as IR
    assert all(node[1] == IR.PS_FLAT and node[0] == IR.P_ZERO for node in pir.ps_tree)
    nodes = [(0.0, 0.0, None if k == 0 else "flat", d0, d1, None) for k, (_, _, d0, d1) in enumerate(pir.ps_tree)]
    prm = oracle.params()
    masses = [prm.mt if leg.particle == IR.P_TOP else 0.0 for leg in pir.legs]
    cores = len(os.sched_getaffinity(0))
    pid, nl = getattr(oracle, oracle_proc), pir.n_legs
    probe, _ = T.generate(seed, 32, pir.sqrt_s, nodes, nl, leg_mass=masses)
    oracle.me2(pid, probe[:1], prm, threads=cores)    # builds the diagrams and the colour matrix
    t0 = time.perf_counter()
    oracle.me2(pid, probe, prm, threads=cores)
    rate = 32 / (time.perf_counter() - t0)
    n = int(min(max(rate * target_seconds, 256), 1 << 16))
    mom, w = T.generate(seed, n, pir.sqrt_s, nodes, nl, leg_mass=masses)
    t0 = time.perf_counter()
    f = oracle.me2(pid, mom, prm, threads=cores)
    dt = time.perf_counter() - t0
    passed = oracle.cut_gluons(mom, pir.cut_pt, pir.cut_dr) if pir.cut_enabled else np.ones(n, dtype=np.int32)
    passed = passed * (w > 0)
    f = f * passed
    out = {"value": n / dt, "unit": "events/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} events of the same workload (first {n} Philox counters of the tree), {dt:.1f} s"}
    sig_ref = oracle.cross_section(f, w, pir.sqrt_s, pir.n_a_n_b, pir.symmetry, passed=passed)[0]
    soa = torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()
    nz = f != 0
    for prec in precisions:
        proc = H.Process(pir, precision=prec)
        got = proc.eval(momenta=soa).cpu().numpy()
        proc.close()
        err = np.abs(got[nz] - f[nz]) / np.abs(f[nz])
        sig = oracle.cross_section(got, w, pir.sqrt_s, pir.n_a_n_b, pir.symmetry, passed=passed)[0]
        out[f"{prec}_error"] = {"me2_max_rel": float(err.max()), "me2_median_rel": float(np.median(err)),
                                "sigma_rel": sig / sig_ref - 1.0, "events": int(nz.sum()),
                                "cut_events_exactly_zero": bool(np.all(got[~nz] == 0.0))}
    return out


def compression_text(pir):
    c = pir.colour_compression()
    return (f"the {c['flows']} x {c['flows']} colour matrix compressed to its {c['distinct_factors']} distinct "
            f"factors ({c['compressed_multiplications']:,} multiplications per form instead of "
            f"{c['dense_multiply_adds']:,} multiply-adds)")


def phase_space_leg(torch, proc, steps, warmup):
    """heget_generate alone (Philox -> RAMBO -> SoA momenta), the HBM-bound
    kernel of the path: 32 bytes per leg per event written."""
    n = N_EVENTS
    out = torch.empty((proc.n_legs, 4, n), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        proc.generate(n, seed=SEED, sqrt_s=SQRT_S, momenta_out=out)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for k in range(steps):
        proc.generate(n, seed=SEED + k, sqrt_s=SQRT_S, momenta_out=out)
    ev1.record(stream)
    ev1.synchronize()
    t = ev0.elapsed_time(ev1) / 1e3 / steps
    nbytes = n * proc.n_legs * 4 * 8
    return {"kernel": "generate_momenta<6>", "events": n, "bytes_written": nbytes, "kernel_ms": t * 1e3,
            "achieved_gbs": nbytes / t / 1e9, "peak_gbs": HBM_PEAK_GBS, "frac": nbytes / t / 1e9 / HBM_PEAK_GBS}


SERVE_SEED = 0x48454749
# the four configurations; the engine runs mixed precision, where C2 keeps its
# 120-flow trace basis with the colour matrix compressed to its distinct
# factors (FP32 on VALU); the unbatched FP64 baseline runs the 120-flow dense
# form on MFMA
SERVE_PROCESSES = ("ee_mumu", "gg_ttbar_6f", "gg_4g_cf", "ud_udhh_4b")
SERVE_BASELINE_PROCESSES = ("ee_mumu", "gg_ttbar_6f", "gg_4g", "ud_udhh_4b")
SERVE_WEIGHTS = (40, 30, 20, 10)
SERVE_SQRT_S = (200.0, 1000.0, 1000.0, 2000.0)


def serve_leg(n_requests, rate=200.0):
    """Poisson request stream over the four configurations, served by the
    engine in mixed precision, against one-at-a-time FP64 heget_integrate."""
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes, serve
    reqs = serve.poisson_mix(SERVE_SEED, n_requests, rate, SERVE_WEIGHTS, SERVE_SQRT_S)
    mixed = [H.Process(processes.by_name(n), precision="mixed") for n in SERVE_PROCESSES]
    fp64 = [H.Process(processes.by_name(n), precision="fp64") for n in SERVE_BASELINE_PROCESSES]
    warm = [serve.Request(0.0, k, 4096, 1, SERVE_SQRT_S[k]) for k in range(4)]
    srv = H.Server(mixed, arena_bytes=1 << 30, slots_per_process=2, max_batch_blocks=4096, max_chunk_blocks=1024)
    serve.replay_engine(srv, warm)
    serve.replay_unbatched(fp64, warm)
    _, eng = serve.replay_engine(srv, reqs)
    st = srv.stats()
    # capacity: the same requests all at once (an arrival rate above any
    # capacity), so the engine is never idle; the offered stream's utilisation
    # is its event rate over that capacity
    burst = [serve.Request(0.0, r.process, r.n, r.seed, r.sqrt_s) for r in reqs]
    _, cap = serve.replay_engine(srv, burst)
    srv.close()
    offered = sum(r.n for r in reqs) / reqs[-1].t_arrival
    _, base = serve.replay_unbatched(fp64, reqs)
    eng.update({"precision": "mixed", "launches": st["launches"], "segments": st["segments"],
                "max_busy_slots": st["max_busy_slots"], "arena_high_water_bytes": st["arena_high_water"],
                "offered_events_per_s": offered,
                "capacity": {"events_per_s": cap["events_per_s"], "wall_s": cap["wall_s"], "p50_s": cap["p50_s"],
                             "p99_s": cap["p99_s"], "kind": "every request submitted at t = 0"},
                "utilisation": offered / cap["events_per_s"]})
    base.update({"precision": "fp64", "kind": "unbatched: one heget_integrate at a time in arrival order"})
    return {"workload": f"{n_requests} Poisson requests at {rate:g}/s over "
                        f"{'/'.join(SERVE_PROCESSES)} (baseline {'/'.join(SERVE_BASELINE_PROCESSES)}) "
                        f"in proportions {'/'.join(map(str, SERVE_WEIGHTS))}, "
                        "n log-uniform in [2^10, 2^20), sqrt_s = nominal x 2^U(-1/2,1/2)",
            "engine": eng, "baseline": base}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 50 steps of C1 time about 6 ms: long enough that one host stall does not move the average
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the serving replay (0: skip it)")
    ap.add_argument("--profile-leg", choices=["fp64", "mixed"], default=None,
                    help="run only this precision's steps (for rocprofv3 of the dominant kernel)")
    ap.add_argument("--profile-proc", default="gg_ttbar_6f",
                    help="process of --profile-leg: gg_ttbar_6f (default), gg_4g, gg_4g_ddm, ud_udhh_4b, ud_udhhh, "
                         "ww_ww, gg_5g_ddm (2^16 events per launch), ee_mumu, "
                         "'generate' for the phase-space kernel of gg_ttbar_6f alone, or 'adaptive' for the "
                         "adaptive integration of its resonance-tree form (FP64)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 1 GiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.profile_leg == "mixed" and args.profile_proc in ("gg_4g", "gg_5g_ddm"):
        print("bench.py: the mixed-precision 120-flow MFMA kernel is switched off on the GPU "
              "(an unexplained fault); profile gg_4g_ddm in mixed precision", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 "
              "(more GPUs would each take a range of Philox counters)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes, codegen, flops

    proc_ir = processes.gg_ttbar_6f()
    if args.profile_leg:
        if args.profile_proc == "generate":
            proc = H.Process(proc_ir, precision=args.profile_leg)
            out = phase_space_leg(torch, proc, args.steps, args.warmup)
            print(json.dumps(out), flush=True)
            return
        if args.profile_proc == "adaptive":
            print(json.dumps(adaptive_leg(torch, H, processes)), flush=True)
            return
        pir = processes.by_name(args.profile_proc)
        proc = H.Process(pir, precision=args.profile_leg)
        n = {"gg_5g_ddm": 1 << 16, "gg_5g_cf": 1 << 16, "gg_5g_split": 1 << 16, "ud_udhh_4b": 1 << 21, "ee_mumu": 65536,
             "uu_ttggg": 1 << 18, "uu_ttggg_cf": 1 << 18}.get(args.profile_proc, N_EVENTS)
        settle_clocks(torch, proc, n=n, sqrt_s=pir.sqrt_s)
        wall, kern, r, _ = time_path(torch, proc, args.steps, args.warmup, n=n, sqrt_s=pir.sqrt_s)
        out = {"proc": args.profile_proc, "leg": args.profile_leg, "ms_per_step": wall * 1e3,
               "kernel_ms": kern * 1e3, "events_per_launch": n, "events_per_s": n / wall,
               "n_accepted": r["n_accepted"], "source_digest": codegen.source_digest(pir)}
        if args.copy_calibration:
            src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
            dst = torch.empty_like(src)
            src.fill_(1.0)
            torch.cuda.synchronize()
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            out["copy_bytes_each_way"] = src.numel() * 8
        print(json.dumps(out), flush=True)
        return
    fp64 = H.Process(proc_ir, precision="fp64")
    mixed = H.Process(proc_ir, precision="mixed")

    settle_clocks(torch, fp64)
    wall64, kern64, r64, sync64 = time_path(torch, fp64, args.steps, args.warmup, synchronous_too=True)
    wallmx, kernmx, rmx, syncmx = time_path(torch, mixed, args.steps, args.warmup, synchronous_too=True)

    # with the exactly-vanishing helicity combinations dropped (4 of 256 survive)
    fp64f = H.Process(proc_ir, precision="fp64")
    nk = fp64f.filter_helicities(n_probe=64, seed=99, sqrt_s=SQRT_S, rel_threshold=1e-20)
    mixedf = H.Process(proc_ir, precision="mixed")
    mixedf.filter_helicities(n_probe=64, seed=99, sqrt_s=SQRT_S, rel_threshold=1e-20)
    wall64f, kern64f, _, _ = time_path(torch, fp64f, args.steps, args.warmup)
    wallmxf, kernmxf, _, _ = time_path(torch, mixedf, args.steps, args.warmup)

    model_flop_event = flops.per_event(proc_ir)
    if counters_valid(proc_ir):
        flop_event, flop_source = COUNTERS_FP64["flop_per_event"], "executed FP64 flops from SQ_INSTS_VALU_*_F64"
        mixed_flop_event = COUNTERS_FP64["flop_per_event_mixed"]
        mixed_flop_source = "executed FP32 flops from SQ_INSTS_VALU_*_F32"
    else:
        # counters taken on another kernel source: no executed-flop figure
        flop_event, flop_source = None, "none: the counters were taken on another kernel source"
        mixed_flop_event, mixed_flop_source = None, flop_source
    achieved = flop_event * N_EVENTS / kern64 / 1e12 if flop_event else None
    value = N_EVENTS / wall64
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall64 * 1e3,
        "synchronous": {"events_per_s": N_EVENTS / sync64, "ms_per_step": sync64 * 1e3,
                        "how": "heget_integrate, the host waiting for every step's sigma"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gg->ttbar->(b e+ nu_e)(bbar mu- nu_mu~), sqrt_s_hat=1 TeV, 2^20 RAMBO events "
                               "per step, 256 helicity combinations, 2 colour flows",
                   "events_per_step": N_EVENTS, "helicities": 256},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "traffic": measured_traffic(proc_ir),
                     "traffic_unit": "bytes per launch",
                     "kernel": "amp_gg_ttbar_6f<double>", "kernel_ms": kern64 * 1e3,
                     "flop_per_event": flop_event, "flop_source": flop_source,
                     "model_flop_per_event": model_flop_event},
        "mixed": {"value": N_EVENTS / wallmx, "ms_per_step": wallmx * 1e3, "kernel_ms": kernmx * 1e3,
                  "synchronous_ms_per_step": syncmx * 1e3,
                  "tflops": mixed_flop_event * N_EVENTS / kernmx / 1e12 if mixed_flop_event else None, "peak": FP32_PEAK_TFLOPS,
                  "flop_per_event": mixed_flop_event, "flop_source": mixed_flop_source,
                  "sigma_pb": rmx["sigma_pb"]},
        "helicity_filtered": {"helicities": nk, "fp64_value": N_EVENTS / wall64f,
                              "mixed_value": N_EVENTS / wallmxf, "fp64_kernel_ms": kern64f * 1e3,
                              "mixed_kernel_ms": kernmxf * 1e3},
        "sigma_pb": r64["sigma_pb"], "sigma_err_pb": r64["err_pb"],
    }
    line["phase_space"] = phase_space_leg(torch, fp64, args.steps, args.warmup)
    line["resonance_phase_space"] = resonance_leg(torch, H, processes, args.steps, args.warmup, r64)
    line["adaptive_integration"] = adaptive_leg(torch, H, processes)
    line["triple_higgs"] = config_leg(
        torch, H, processes.ud_udhhh(), "u d -> u d H H H by W W and Z Z fusion (quartic scalar vertex), "
        "sqrt_s_hat = 2 TeV, 2^20 events per step, 16 helicity combinations, 2 colour flows",
        args.steps, args.warmup)
    line["w_scattering"] = config_leg(
        torch, H, processes.ww_ww(), "W- W+ -> W- W+ (massive external W, weak quartic vertex), "
        "sqrt_s_hat = 1 TeV, 2^20 events per step, 81 helicity combinations", args.steps, args.warmup)
    line["hadronic_collision"] = config_leg(
        torch, H, processes.gg_ttbar_6f_had(), "gg -> t tbar -> 6f at a 14 TeV hadron collider (parton densities "
        "1), tops in |y| < 2.5 by rapidity, ln(m^2 + pT^2) and azimuth, x_a, x_b from momentum conservation, "
        "resonance-tree decays, 2^20 events per step", args.steps, args.warmup)
    # seven gluons: 120 DDM orderings x 128 helicities per event
    line["seven_gluons"] = config_leg(
        torch, H, processes.by_name("gg_5g_ddm"), "g g -> g g g g g, sqrt_s_hat = 1 TeV, pT > 20 GeV, "
        "Delta R > 0.4, 2^16 events per step, 128 helicity combinations, 120 DDM colour flows on MFMA",
        3, 1, n=1 << 16, precisions=("fp64",))
    line["seven_gluons"]["split"] = config_leg(
        torch, H, processes.by_name("gg_5g_split"), "the same FP64 program divided into two kernels (the orderings' "
        "amplitudes to the workspace, then the colour form), launched per round of resident blocks", 3, 1,
        n=1 << 16, precisions=("fp64",))
    line["seven_gluons"]["compressed"] = config_leg(
        torch, H, processes.by_name("gg_5g_cf"), f"the same, {compression_text(processes.by_name('gg_5g_cf'))}; "
        "mixed precision on VALU", 3, 1, n=1 << 16, precisions=("mixed",))
    # u ubar -> t tbar g g g: the paper's long amplitude (Sec. 5.3-5.5) from its Feynman diagrams
    ql = processes.by_name("uu_ttggg")
    ncur = sum(1 for c in ql.calls if c.op not in ("iov",))
    line["long_amplitude"] = config_leg(
        torch, H, ql, f"u ubar -> t tbar g g g, sqrt_s_hat = 1 TeV, stable tops, pT > 20 GeV and Delta R > 0.4 "
        f"on every final leg, flat two-body tree phase space, 2^18 events per step, 128 helicity combinations; "
        f"{ql.n_amps} Feynman diagrams as {ncur} current calls and {ql.n_amps} amplitude calls, {ql.n_flows} "
        f"colour flows, dense colour form; the program divided into {ql.row_parts} device functions, helicity "
        f"rows one at a time", 3, 1, n=1 << 18, seed=0x54544703)
    line["long_amplitude"]["colour"] = ql.colour_compression()
    line["long_amplitude"]["compressed"] = config_leg(
        torch, H, processes.by_name("uu_ttggg_cf"), f"the same with {compression_text(ql)}", 3, 1, n=1 << 18,
        seed=0x54544703)
    # the other configured workloads, each with the oracle timed beside it on a
    # sample of its events and the GPU's error against the oracle on that sample
    import oracle as O
    legs = {}
    c0 = processes.ee_mumu()
    legs["c0"] = config_leg(
        torch, H, c0, "e+ e- -> mu+ mu- via photon and Z, sqrt_s = 200 GeV, 65,536 RAMBO events per step, "
        "16 helicity combinations", args.steps, args.warmup, n=65536, seed=0x48454745)
    if not args.no_cpu_baseline:
        legs["c0"]["oracle"] = oracle_leg(torch, H, O, c0, "EE_MUMU", {}, 2, 0x48454745, target_seconds=1.0,
                                          extended=True)
    c2 = processes.by_name("gg_4g")
    c2d = processes.by_name("gg_4g_ddm")
    # C2 launches take 60-180 ms each: at most 10 timed steps per leg
    c2_steps, c2_warmup = min(args.steps, 10), min(args.warmup, 2)
    legs["c2"] = config_leg(
        torch, H, c2, "g g -> g g g g, sqrt_s_hat = 1 TeV, pT > 20 GeV and Delta R > 0.4 by rejection, 2^20 RAMBO "
        "events per step, 64 helicity combinations, 120 trace-basis flows, dense 120 x 120 colour form on MFMA",
        c2_steps, c2_warmup, seed=0x48454747)
    legs["c2"]["compressed"] = config_leg(
        torch, H, processes.by_name("gg_4g_cf"), f"the same events through the same 120 trace-basis flows, "
        f"{compression_text(processes.by_name('gg_4g_cf'))}; mixed precision runs it on VALU, FP64 keeps the dense "
        "MFMA form", c2_steps, c2_warmup, precisions=("mixed",), seed=0x48454747)
    legs["c2"]["ddm_basis"] = config_leg(
        torch, H, c2d, "the same events and |M|^2 through the 24-flow DDM basis, colour form on VALU",
        c2_steps, c2_warmup, seed=0x48454747)
    if not args.no_cpu_baseline:
        legs["c2"]["oracle"] = oracle_leg(torch, H, O, c2, "GG_4G", {}, 4, 0x48454747, cut=(20.0, 0.4))
        legs["c2"]["ddm_basis"]["oracle"] = oracle_leg(torch, H, O, c2d, "GG_4G", {}, 4, 0x48454747,
                                                       cut=(20.0, 0.4), target_seconds=1.0)
        legs["c2"]["compressed"]["oracle"] = oracle_leg(torch, H, O, processes.by_name("gg_4g_cf"), "GG_4G", {}, 4,
                                                        0x48454747, cut=(20.0, 0.4), target_seconds=1.0,
                                                        precisions=("mixed",))
    c3 = processes.ud_udhh_4b()
    legs["c3"] = config_leg(
        torch, H, c3, "u d -> u d H H (W W and Z Z fusion), H -> b bbar, sqrt_s_hat = 2 TeV, 2^21 RAMBO events "
        "per step, 256 helicity combinations, complex-mass W and Z; mixed precision keeps the propagator "
        "denominators in FP64", args.steps, args.warmup, n=1 << 21, precisions=("mixed", "fp64"), seed=0x48454748)
    if not args.no_cpu_baseline:
        legs["c3"]["oracle"] = oracle_leg(torch, H, O, c3, "UD_UDHH_4B", {"cms": 1}, 6, 0x48454748,
                                          precisions=("mixed", "fp64"))
    if not args.no_cpu_baseline:
        line["long_amplitude"]["oracle"] = tree_oracle_leg(torch, H, O, ql, "UU_TTGGG", 0x54544703)
    line["configs"] = legs
    if args.serve_requests > 0:
        line["serve"] = serve_leg(args.serve_requests)
    if not args.no_cpu_baseline:
        import oracle
        line["cpu_baseline"] = cpu_baseline(oracle)
        line["mixed"]["error_vs_oracle"] = oracle_leg(torch, H, oracle, proc_ir, "GG_TT_6F", {}, 6, SEED,
                                                      target_seconds=2.0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
