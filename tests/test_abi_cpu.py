"""CPU checks of the C ABI library: it loads, exports every symbol that
include/heget.h declares, rejects malformed IRs before touching the device,
and its IR fingerprint agrees with the code generator's."""
import dataclasses
import os
import re
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "heget.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(heget_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1305_0708_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "heget_eval" in names and "heget_process_create" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_1305_0708_amd import _lib
    assert sorted(_lib.EXPORTED) == names


def _create(proc):
    import paper_1305_0708_amd as H
    return H.Process(proc)


def _status(fn):
    import paper_1305_0708_amd as H
    try:
        fn()
    except H.HegetError as e:
        return e.status
    return 0


@pytest.mark.parametrize("name", ["ee_mumu", "gg_ttbar_6f", "gg_ttbar_6f_bw", "gg_ttbar_6f_had", "ud_udhh_4b", "ud_udhhh", "ww_ww", "gg_4g", "gg_4g_ddm", "gg_5g_ddm"])
def test_fingerprint_matches_compiled_kernel(name):
    # a valid IR passes validation and the kernel lookup; without a GPU the
    # first device allocation then fails with HEGET_E_OOM (on a GPU: success)
    from paper_1305_0708_amd import processes
    import torch
    st = _status(lambda: _create(processes.by_name(name)))
    if torch.cuda.is_available():
        assert st == 0
    else:
        assert st == -3


def test_structural_change_is_unsupported():
    from paper_1305_0708_amd import processes
    q = processes.gg_ttbar_6f()
    q.colour[0][0] = Fraction(17, 3)
    assert _status(lambda: _create(q)) == -5


@pytest.mark.parametrize("mutate,expect", [
    (lambda q: q.calls.__setitem__(0, dataclasses.replace(q.calls[0], ins=(3, 99))), -2),   # undefined slot
    (lambda q: q.calls.__setitem__(0, dataclasses.replace(q.calls[0], ins=(0, 4))), -2),    # wrong kind
    (lambda q: q.calls.__setitem__(5, dataclasses.replace(q.calls[5], out=2)), -2),         # amplitude reused
    (lambda q: q.calls.__setitem__(0, dataclasses.replace(q.calls[0], cpl=9)), -2),         # bad coupling
    (lambda q: q.colour[0].__setitem__(1, Fraction(1)), -2),                               # not symmetric
    (lambda q: setattr(q, "helicities", [(2,) * 8]), -2),                                   # bad helicity
])
def test_malformed_ir_rejected(mutate, expect):
    from paper_1305_0708_amd import processes
    q = processes.gg_ttbar_6f()
    mutate(q)
    assert _status(lambda: _create(q)) == expect


def test_python_validation_agrees():
    from paper_1305_0708_amd import processes
    for name in ("ee_mumu", "gg_ttbar_6f", "gg_ttbar_6f_bw", "ud_udhh_4b"):
        processes.by_name(name).validate()


@pytest.mark.parametrize("tree", [
    [(0, 0, -2, -3), (3, 1, 2, -4), (3, 1, 5, -5), (1, 1, 3, 4), (1, 1, 6, 6)],     # leg 6 twice, 7 never
    [(0, 0, -2, -3), (3, 1, 2, -4), (3, 1, 5, -5), (1, 1, 3, 4), (1, 1, 6, 1)],     # a beam as daughter
    [(0, 0, -2, -3), (3, 1, 2, -1), (3, 1, 5, -5), (1, 1, 3, 4), (1, 1, 6, 7)],     # node before its parent
    [(0, 0, -2, -3), (3, 2, 2, -4), (3, 1, 5, -5), (1, 1, 3, 4), (1, 1, 6, 7)],     # unknown mapping
    [(0, 0, -2, -3), (0, 1, 2, -4), (3, 1, 5, -5), (1, 1, 3, 4), (1, 1, 6, 7)],     # Breit-Wigner without mass
])
def test_malformed_phase_space_tree_rejected(tree):
    """the library rejects a bad resonance tree (HEGET_E_IR) and so does the
    Python IR; the fingerprint is taken from a valid tree"""
    from paper_1305_0708_amd import processes
    q = processes.gg_ttbar_6f_bw()
    q.ps_tree = tree
    assert _status(lambda: _create(q)) == -2
    if tree[1][0] != 0:
        with pytest.raises(ValueError):
            q.validate()


def test_colour_matrices_are_exact_fierz():
    # the product IR's colour matrices, checked against the SU(3) Fierz identity
    from paper_1305_0708_amd import processes
    from test_oracle_amplitudes import fierz_trace_product
    c1 = processes.gg_ttbar_6f().colour
    # flows (T^a T^b)_ij and (T^b T^a)_ij: sum_col |(ab)_ij|^2 = Tr(a b b a)
    assert c1[0][0] == fierz_trace_product([[1, 2, 2, 1]])
    assert c1[0][1] == fierz_trace_product([[1, 2, 1, 2]])


def test_adaptive_entry_points_reject_a_null_handle(lib):
    """argument errors come back before any device call"""
    from paper_1305_0708_amd import _lib
    comb = _lib.heget_result()
    assert lib.heget_integrate_adaptive(None, 1024, 2, 8, 1000.0, 1, None, comb, None, None, None) \
        == _lib.HEGET_E_INVALID
    assert lib.heget_process_grid_dims(None) == -1


@pytest.mark.parametrize("name,expect", [("gg_4g", -5), ("gg_5g_ddm", -5), ("gg_4g_ddm", None), ("gg_4g_cf", None),
                                         ("gg_5g_cf", None)])
def test_mixed_precision_on_the_mfma_colour_form_is_refused(name, expect):
    """the mixed kernels of processes whose FP32 colour form runs on MFMA are
    refused at create, before any allocation (HEGET_E_UNSUPPORTED); a process
    whose FP32 colour form runs on VALU (a small basis, or the compressed form
    of a large one) gets past the check (then, without a GPU, HEGET_E_OOM at the
    first device allocation)"""
    import paper_1305_0708_amd as H
    import torch
    from paper_1305_0708_amd import processes
    st = _status(lambda: H.Process(processes.by_name(name), precision="mixed"))
    if expect is None:
        expect = 0 if torch.cuda.is_available() else -3
    assert st == expect


@pytest.mark.parametrize("name", ["gg_4g_cf", "gg_5g_cf"])
def test_compressed_form_keeps_mfma_out_of_the_fp32_kernel(name):
    """the generated source of a compressed colour form: the FP32 branch calls
    no MFMA colour form (the FP64 branch keeps the dense one), and the kernel's
    registry entry says so"""
    from paper_1305_0708_amd import codegen, processes
    pir = processes.by_name(name)
    assert pir.uses_colour_mfma() and not pir.mixed_uses_mfma()
    src = codegen.Gen(pir).emit()
    a = src.index("if constexpr (sizeof(T) == 4) {")
    b = src.index("} else {", a)
    fp32 = src[a:b]
    assert "colour_form_" not in fp32 and "Mfma" not in fp32 and "cs += " in fp32
    assert "colour_form_resident" in src[b:] or "colour_form_mfma" in src[b:]
    entry = next(l for l in src.splitlines() if l.startswith("static const GenEntry entry"))
    assert entry.endswith(", 0, nullptr, nullptr, nullptr, nullptr};")   # colour_mfma_mixed = 0, fused


def test_integrate_async_rejects_bad_arguments(lib):
    """heget_integrate_async and heget_result_from_sums check their arguments
    before any device call"""
    import ctypes
    from paper_1305_0708_amd import _lib
    sums = (ctypes.c_double * 3)()
    r = _lib.heget_result()
    assert lib.heget_integrate_async(None, 1024, 1000.0, 1, ctypes.cast(sums, ctypes.c_void_p), None) \
        == _lib.HEGET_E_INVALID
    assert lib.heget_result_from_sums(None, 1024, ctypes.byref(r)) == _lib.HEGET_E_INVALID
    assert lib.heget_result_from_sums(sums, 1, ctypes.byref(r)) == _lib.HEGET_E_INVALID


def test_result_from_sums_is_the_monte_carlo_estimate():
    """sigma = sum w / n and its error sqrt((sum w^2 / n - sigma^2) / (n - 1)),
    worked by hand for w = (1, 2, 3, 4): sigma 2.5, variance 7.5 - 6.25 = 1.25"""
    import math
    import paper_1305_0708_amd as H
    r = H.result_from_sums([10.0, 30.0, 4.0], 4)
    assert r["sigma_gev2"] == 2.5 and r["n_accepted"] == 4 and r["n_generated"] == 4
    assert abs(r["err_gev2"] - math.sqrt(1.25 / 3)) < 1e-15
    assert abs(r["sigma_pb"] / r["sigma_gev2"] - 0.3893793721e9) < 1e-3
