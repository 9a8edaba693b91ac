"""Child-process entry of the CPU lane emulator (tests only): create a process
handle through the emulated library's C ABI and evaluate n events, writing
|M|^2 and the momenta used to an .npz file.

    python run_emu.py LIB NAME PRECISION N SEED OUT [MOMENTA.npy]
    python run_emu.py LIB NAME PRECISION N SEED OUT --integrate

The second form writes the three reduced sums of heget_integrate (twice in a
row), heget_integrate_async and heget_integrate_noalloc instead.

Run with the sanitizer runtime preloaded (LD_PRELOAD) and ASAN_OPTIONS
detect_leaks=0; any invalid access aborts the child with a report.
"""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.environ.get("EMU_ROOT") or os.path.dirname(os.path.dirname(HERE))   # the source tree built
sys.path.insert(0, ROOT)
sys.modules["torch"] = None      # the emulated library takes host pointers


def main(argv):
    lib_path, name, prec, n, seed, out = argv[:6]
    n, seed = int(n), int(seed, 0)
    from paper_1305_0708_amd import _lib, processes
    import paper_1305_0708_amd as H
    L = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    L.heget_process_create.argtypes = [ctypes.POINTER(_lib.heget_process_ir), ctypes.c_int, ctypes.POINTER(vp)]
    L.heget_eval.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, vp, vp, vp]
    L.heget_process_destroy.argtypes = [vp]
    L.heget_last_error.restype = ctypes.c_char_p
    pir = processes.by_name(name)
    buf = H._IRBuffers(pir, H.default_sm(**pir.sm_overrides))
    h = ctypes.c_void_p()
    st = L.heget_process_create(ctypes.byref(buf.ir), _lib.HEGET_FP64 if prec == "fp64" else _lib.HEGET_MIXED,
                                ctypes.byref(h))
    if st != 0:
        print("create:", st, L.heget_last_error().decode(), flush=True)
        return 3
    if len(argv) > 6 and argv[6] == "--integrate":
        return integrate(L, h, pir, n, seed, out)
    me2 = np.zeros(n)
    if len(argv) > 6:
        mom = np.ascontiguousarray(np.load(argv[6]), dtype=np.float64)   # [legs][4][n]
        mom_in, mom_out = mom, None
    else:
        mom_in, mom_out = None, np.zeros((pir.n_legs, 4, n))
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
    st = L.heget_eval(h, n, ptr(mom_in), seed, 0, float(pir.sqrt_s), ptr(me2), ptr(mom_out), None)
    if st != 0:
        print("eval:", st, L.heget_last_error().decode(), flush=True)
        return 4
    np.savez(out, me2=me2, mom=mom_in if mom_in is not None else mom_out)
    L.heget_process_destroy(h)
    return 0


def integrate(L, h, pir, n, seed, out):
    from paper_1305_0708_amd import _lib
    vp = ctypes.c_void_p
    res = ctypes.POINTER(_lib.heget_result)
    L.heget_integrate.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, res, vp]
    L.heget_integrate_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, res, vp]
    L.heget_integrate_async.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, vp, vp]
    rows = []
    for fn in (L.heget_integrate, L.heget_integrate, L.heget_integrate_noalloc):
        r = _lib.heget_result()
        st = fn(h, n, float(pir.sqrt_s), seed, ctypes.byref(r), None)
        if st != 0:
            print("integrate:", st, L.heget_last_error().decode(), flush=True)
            return 5
        rows.append([r.sum_w, r.sum_w2, float(r.n_accepted)])
    sums = np.zeros(3)
    st = L.heget_integrate_async(h, n, float(pir.sqrt_s), seed, ctypes.c_void_p(sums.ctypes.data), None)
    if st != 0:
        print("integrate_async:", st, L.heget_last_error().decode(), flush=True)
        return 6
    rows.append(list(sums))
    np.savez(out, sums=np.array(rows))
    L.heget_process_destroy(h)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
