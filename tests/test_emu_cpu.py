"""The MFMA colour-form kernels on the CPU lane emulator (tests/emu): the
library's generated kernels and host code built for x86-64 with
AddressSanitizer on every access, one fiber per lane, the wave operations and
the two MFMA lane layouts emulated.  Ragged launches (n = 45: one block of 45
lanes; n = 300: two blocks, the second with 44 active lanes and three waves
with none) must make no invalid access, give the same bits with the lanes run
in ascending and in descending order (no lane reads what another wrote without
a barrier), and match the FP64 oracle: within 1e-12 in FP64, at FP32's scale in
mixed precision.  The emulated library lifts the create-time refusal of mixed
precision for these kernels (its copy of heget_abi.hip only), so that the FP32
MFMA path the GPU does not run is still checked on the CPU."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
OUT = os.path.join(EMU, "_build", "mixed_allowed")
LIFT = [("if (prec == HEGET_MIXED && entry->colour_mfma_mixed)\n    return fail(", "if (false)\n    return fail(")]


@pytest.fixture(scope="module")
def emu_lib():
    sys.path.insert(0, EMU)
    import build_emu
    if not os.path.exists(build_emu.CXX) or not build_emu.asan_runtime():
        pytest.skip("host clang++ with the AddressSanitizer runtime not available")
    lib = build_emu.build(processes=("gg_4g", "gg_5g_ddm", "gg_4g_cf"), abi_edits=LIFT, out=OUT)
    return lib, build_emu.asan_runtime()


def run(emu_lib, name, prec, n, seed, order, cus):
    lib, asan = emu_lib
    out = os.path.join(OUT, f"run_{name}_{prec}_{n}_{order}.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               EMU_LANE_ORDER=str(order), EMU_CUS=str(cus))
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_emu.py"), lib, name, prec, str(n), hex(seed), out],
                       env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, f"emulated {name} {prec} n={n}: rc {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    d = np.load(out)
    return d["me2"], d["mom"]


@pytest.mark.parametrize("name,prec,n,cus", [
    ("gg_4g", "fp64", 300, 1),      # one persistent block walks both 256-event blocks
    ("gg_4g", "mixed", 300, 2),
    ("gg_4g", "mixed", 45, 1),
    ("gg_5g_ddm", "mixed", 45, 1),
    ("gg_4g_cf", "mixed", 300, 2),  # the colour form compressed to its distinct factors, FP32 on VALU
])
def test_mfma_colour_form_on_ragged_launches(emu_lib, oracle, name, prec, n, cus):
    seed, nout, pid = {"gg_4g": (0x48454747, 4, oracle.GG_4G), "gg_4g_cf": (0x48454747, 4, oracle.GG_4G),
                       "gg_5g_ddm": (0x47474735, 5, oracle.GG_5G)}[name]
    me2, mom = run(emu_lib, name, prec, n, seed, 0, cus)
    if name != "gg_5g_ddm":
        me2_rev, _ = run(emu_lib, name, prec, n, seed, 1, cus)
        assert np.array_equal(me2, me2_rev), "results depend on the order the lanes run in"
    ref_mom = oracle.generate(seed, n, nout, 1000.0)
    assert np.abs(np.transpose(mom, (2, 0, 1)) - ref_mom).max() < 1e-13 * 1000.0
    ref = oracle.me2(pid, ref_mom) * oracle.cut_gluons(ref_mom, 20.0, 0.4)
    nz = ref != 0
    assert np.all(me2[~nz] == 0.0)
    err = np.abs(me2[nz] - ref[nz]) / ref[nz]
    print(f"emulated {name} {prec} n={n}: max rel err {err.max():.2e}, median {np.median(err):.2e}")
    if prec == "fp64":
        assert err.max() <= 1e-12
    else:
        assert np.median(err) < 1e-5 and err.max() < 1e-4


# ---------------------------------------------------- diagram call lists (quark lines)
QL_OUT = os.path.join(EMU, "_build", "quark_lines")


@pytest.fixture(scope="module")
def emu_ql():
    sys.path.insert(0, EMU)
    import build_emu
    if not os.path.exists(build_emu.CXX) or not build_emu.asan_runtime():
        pytest.skip("host clang++ with the AddressSanitizer runtime not available")
    lib = build_emu.build(processes=("uu_ttg", "uu_ttgg"), out=QL_OUT)
    return lib, build_emu.asan_runtime()


@pytest.mark.parametrize("name,prec", [("uu_ttg", "fp64"), ("uu_ttgg", "fp64"), ("uu_ttgg", "mixed")])
def test_quark_line_kernels(emu_ql, oracle, name, prec):
    """u ubar -> t tbar + 1 gluon (the helicity loop nest) and + 2 gluons (the
    helicity rows one at a time, the program divided into two device
    functions) on the oracle's momenta: no invalid access, events failing the
    cut exactly 0, the rest within 1e-12 of the oracle in FP64 (FP32's scale
    in mixed precision)"""
    import fp64_bounds as B
    lib, asan = emu_ql
    mom = B.tree_events(oracle, name)[0][:45]
    path = os.path.join(QL_OUT, f"mom_{name}.npy")
    np.save(path, np.ascontiguousarray(np.transpose(mom, (1, 2, 0))))
    out = os.path.join(QL_OUT, f"run_{name}_{prec}.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", EMU_LANE_ORDER="0",
               EMU_CUS="1")
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_emu.py"), lib, name, prec, str(len(mom)), "0x1", out,
                        path], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, f"emulated {name} {prec}: rc {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    me2 = np.load(out)["me2"]
    ref = B.reference(oracle, name, mom, extended=False)
    nz = ref != 0
    assert np.all(me2[~nz] == 0.0)
    err = np.abs(me2[nz] - ref[nz]) / ref[nz]
    print(f"emulated {name} {prec}: max rel err {err.max():.2e}, median {np.median(err):.2e}")
    assert err.max() <= (1e-12 if prec == "fp64" else 1e-5)


# ------------------------------------------------- the integrate entry points
FR_OUT = os.path.join(EMU, "_build", "integrate")


@pytest.fixture(scope="module")
def emu_int():
    sys.path.insert(0, EMU)
    import build_emu
    if not os.path.exists(build_emu.CXX) or not build_emu.asan_runtime():
        pytest.skip("host clang++ with the AddressSanitizer runtime not available")
    lib = build_emu.build(processes=("ee_mumu",), out=FR_OUT)
    return lib, build_emu.asan_runtime()


@pytest.mark.parametrize("n,cus", [(45, 1), (300, 2), (2000, 3)])
def test_integrate_entry_points_agree(emu_int, n, cus):
    """heget_integrate (twice in a row), heget_integrate_noalloc (the
    library's scratch) and heget_integrate_async (sums into caller memory) on
    ragged launches: the same three sums bit for bit, every event accepted,
    no invalid access"""
    lib, asan = emu_int
    out = os.path.join(FR_OUT, f"sums_{n}_{cus}.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", EMU_LANE_ORDER="0",
               EMU_CUS=str(cus))
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_emu.py"), lib, "ee_mumu", "fp64", str(n), "0x2F",
                        out, "--integrate"], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, f"emulated integrate n={n}: rc {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    s = np.load(out)["sums"]
    assert s[0, 2] == n and s[0, 0] > 0
    for k in (1, 2, 3):
        assert np.array_equal(s[k], s[0]), (k, s)
