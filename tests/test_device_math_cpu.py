"""The device code's own integer and floating-point primitives, compiled from
the device headers for the CPU (the emulator's host stand-in of the HIP
runtime): the device Philox4x32-10, written with the three-input bit
instruction, against the known-answer vectors of its defining publication;
the uniforms built from the words' bits against their definition; the log of
the RAMBO energies, the kinematics' square root, reciprocal and quotient
against long double.  (On the CPU the hardware estimates that the square root
and reciprocal start from are exact; the GPU parity tests cover the device's.)"""
import os
import re
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(EMU, "_build", "device_math")


@pytest.fixture(scope="module")
def checker():
    sys.path.insert(0, EMU)
    import build_emu
    if not os.path.exists(build_emu.CXX):
        pytest.skip("host clang++ not available")
    os.makedirs(OUT, exist_ok=True)
    # the device headers as the emulator takes them (empty register-class asm barriers dropped)
    src = os.path.join(OUT, "src")
    for name in os.listdir(build_emu.CSRC):
        if name.endswith(".hpp"):
            build_emu._copy(name, src)
    exe = os.path.join(OUT, "device_math_check")
    cmd = [build_emu.CXX, "-std=c++17", "-O2", "-w", "-I", EMU, "-I", src, "-I", os.path.join(ROOT, "include"),
           os.path.join(EMU, "device_math_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_device_philox_matches_the_known_answers(checker):
    r = subprocess.run([checker, "philox", os.path.join(HERE, "golden", "philox4x32_10_kat.txt")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout
    assert re.search(r"rows (\d+) mismatches 0", r.stdout) and int(re.search(r"rows (\d+)", r.stdout).group(1)) >= 3


def test_device_log_within_two_ulp(checker):
    """2,000,000 inputs: RAMBO's u u' (three in four), single u, and x just below 1"""
    r = subprocess.run([checker, "log", "2000000", "0x10C"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    ulp = float(re.search(r"max_ulp ([0-9.]+)", r.stdout).group(1))
    print(r.stdout.strip())
    assert ulp <= 2.0


def test_device_uniforms_bit_for_bit(checker):
    r = subprocess.run([checker, "unit", "5000000", "0x55"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    assert re.search(r"mismatches 0", r.stdout)


def test_device_sqrt_reciprocal_quotient(checker):
    """1,000,000 inputs over 2^-60 .. 2^60: the square root correctly rounded,
    the reciprocal and quotient within one unit in the last place; sqrt_pos
    maps zero and negative rounding residues to 0"""
    r = subprocess.run([checker, "roots", "1000000", "0x77"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    print(r.stdout.strip())
    v = {k: float(x) for k, x in re.findall(r"(\w+) (-?[0-9.e+-]+)", r.stdout)}
    assert v["sqrt_ulp"] <= 0.5 and v["recip_ulp"] <= 1.0 and v["quot_ulp"] <= 1.0
    assert v["sqrt0"] == 0.0 and v["sqrtneg"] == 0.0
