"""heget_integrate_async against heget_integrate: the same sums bit for bit,
for steps queued back to back on one stream with no wait between them, the
partials buffer grown in the middle of the queue and a smaller step after it."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,prec", [("gg_ttbar_6f", "fp64"), ("gg_ttbar_6f", "mixed"), ("ud_udhh_4b", "fp64")])
def test_queued_steps_equal_synchronous_ones(name, prec):
    import torch
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    print(f"integrate_async {name} {prec}", flush=True)
    p = H.Process(processes.by_name(name), precision=prec)
    steps = [(5000, 11), (5000, 12), (70001, 13), (300, 14), (70001, 15)]
    sums = torch.full((len(steps), 3), float("nan"), dtype=torch.float64, device="cuda")
    for k, (n, seed) in enumerate(steps):
        p.integrate_async(n, sums[k], seed=seed)
    torch.cuda.synchronize()
    got = sums.cpu().tolist()
    for k, (n, seed) in enumerate(steps):
        ref = p.integrate(n, seed=seed)
        assert got[k] == [ref["sum_w"], ref["sum_w2"], float(ref["n_accepted"])], (k, n, seed)
        assert p.result_from_sums(got[k], n) == ref


def test_pageable_host_sums_are_refused():
    """sums_out in pageable host memory is refused with HEGET_E_INVALID before
    any launch.  The test asks HIP itself first and calls the library only when
    HIP reports the pointer unregistered, the case the library refuses, so no
    kernel can be launched at pageable memory."""
    import ctypes
    import numpy as np
    import torch
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import _lib, processes

    class Attr(ctypes.Structure):
        _fields_ = [("type", ctypes.c_int), ("device", ctypes.c_int), ("devicePointer", ctypes.c_void_p),
                    ("hostPointer", ctypes.c_void_p), ("isManaged", ctypes.c_int), ("allocationFlags", ctypes.c_uint)]
    print("integrate_async pageable sums", flush=True)
    p = H.Process(processes.by_name("ee_mumu"), precision="fp64")
    host = np.zeros(3)
    hip = ctypes.CDLL("libamdhip64.so")
    a = Attr()
    st = hip.hipPointerGetAttributes(ctypes.byref(a), ctypes.c_void_p(host.ctypes.data))
    hip.hipGetLastError()
    if st == 0 and a.type != 0:
        pytest.skip(f"HIP reports this host array as memory type {a.type}")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = p._lib.heget_integrate_async(p._h, 4096, 200.0, 1, ctypes.c_void_p(host.ctypes.data), stream)
    assert rc == _lib.HEGET_E_INVALID
    # pinned host memory is accepted, and gives the same sums as device memory
    pinned = torch.zeros(3, dtype=torch.float64, pin_memory=True)
    dev = torch.zeros(3, dtype=torch.float64, device="cuda")
    assert p._lib.heget_integrate_async(p._h, 4096, 200.0, 1, ctypes.c_void_p(pinned.data_ptr()), stream) == 0
    p.integrate_async(4096, dev, seed=1, sqrt_s=200.0)
    torch.cuda.synchronize()
    assert pinned.tolist() == dev.cpu().tolist() and pinned[2].item() == 4096
