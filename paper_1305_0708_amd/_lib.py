"""ctypes declarations of include/heget.h (argument marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheget.so")

HEGET_OK, HEGET_E_INVALID, HEGET_E_IR, HEGET_E_OOM, HEGET_E_HIP, HEGET_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
HEGET_FP64, HEGET_MIXED = 0, 1
HEGET_NOALLOC_MAX_EVENTS = 1 << 26     # include/heget.h

EXPORTED = ["heget_process_create", "heget_process_destroy", "heget_eval", "heget_integrate",
            "heget_process_n_helicities", "heget_filter_helicities", "heget_last_error", "heget_generate",
            "heget_uniforms",
            "heget_integrate_adaptive", "heget_process_grid_dims", "heget_integrate_noalloc",
            "heget_integrate_async", "heget_result_from_sums",
            "heget_server_create", "heget_server_submit", "heget_server_poll", "heget_server_stats_get",
            "heget_server_destroy"]


class heget_sm(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("sw2", ctypes.c_double),
                ("mz", ctypes.c_double), ("wz", ctypes.c_double),
                ("mw", ctypes.c_double), ("ww", ctypes.c_double),
                ("mt", ctypes.c_double), ("wt", ctypes.c_double),
                ("mh", ctypes.c_double), ("wh", ctypes.c_double),
                ("alpha_s", ctypes.c_double), ("mb_yuk", ctypes.c_double),
                ("complex_mass", ctypes.c_int32)]


class heget_leg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("incoming", ctypes.c_int32), ("flow", ctypes.c_int32),
                ("particle", ctypes.c_int32), ("colour", ctypes.c_int32)]


class heget_coupling(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("particle", ctypes.c_int32),
                ("charge", ctypes.c_double), ("t3", ctypes.c_double)]


class heget_call(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("in_", ctypes.c_int32 * 4), ("out", ctypes.c_int32),
                ("coupling", ctypes.c_int32), ("prop", ctypes.c_int32)]


class heget_ps_node(ctypes.Structure):
    _fields_ = [("particle", ctypes.c_int32), ("mapping", ctypes.c_int32), ("daughter", ctypes.c_int32 * 2)]


class heget_process_ir(ctypes.Structure):
    _fields_ = [("n_legs", ctypes.c_int32), ("legs", ctypes.POINTER(heget_leg)),
                ("sm", heget_sm),
                ("n_couplings", ctypes.c_int32), ("couplings", ctypes.POINTER(heget_coupling)),
                ("n_calls", ctypes.c_int32), ("calls", ctypes.POINTER(heget_call)),
                ("n_amps", ctypes.c_int32), ("n_flows", ctypes.c_int32),
                ("jamp", ctypes.POINTER(ctypes.c_double)),
                ("colour_num", ctypes.POINTER(ctypes.c_double)), ("colour_den", ctypes.c_double),
                ("n_hel", ctypes.c_int32), ("helicities", ctypes.POINTER(ctypes.c_int8)),
                ("n_a_n_b", ctypes.c_int32), ("symmetry", ctypes.c_int32),
                ("cut_enabled", ctypes.c_int32), ("cut_pt", ctypes.c_double), ("cut_dr", ctypes.c_double),
                ("n_orderings", ctypes.c_int32), ("orderings", ctypes.POINTER(ctypes.c_int8)),
                ("flow_map", ctypes.POINTER(ctypes.c_int8)),
                ("n_ps_nodes", ctypes.c_int32), ("ps_nodes", ctypes.POINTER(heget_ps_node)),
                ("ps_window", ctypes.c_double), ("ps_hadron_ymax", ctypes.c_double),
                ("ps_hadron_ptmin", ctypes.c_double), ("colour_form", ctypes.c_int32),
                ("division", ctypes.c_int32)]


class heget_result(ctypes.Structure):
    _fields_ = [("sigma_gev2", ctypes.c_double), ("err_gev2", ctypes.c_double),
                ("sigma_pb", ctypes.c_double), ("err_pb", ctypes.c_double),
                ("sum_w", ctypes.c_double), ("sum_w2", ctypes.c_double),
                ("n_generated", ctypes.c_int64), ("n_accepted", ctypes.c_int64)]


class heget_server_config(ctypes.Structure):
    _fields_ = [("n_processes", ctypes.c_int32), ("processes", ctypes.POINTER(ctypes.c_void_p)),
                ("arena_bytes", ctypes.c_int64), ("slots_per_process", ctypes.c_int32),
                ("max_batch_blocks", ctypes.c_int32), ("max_chunk_blocks", ctypes.c_int32)]


class heget_server_stats(ctypes.Structure):
    _fields_ = [("requests_submitted", ctypes.c_int64), ("requests_done", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("segments", ctypes.c_int64), ("events", ctypes.c_int64),
                ("arena_high_water", ctypes.c_int64), ("max_busy_slots", ctypes.c_int32)]


_lib = None


def load(path=None):
    """Load the in-tree libheget.so.  Raises if it has not been built: there is
    no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # load PyTorch's HIP runtime first so that libheget.so binds to the same one
        import torch  # noqa: F401
    except ImportError:
        pass
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libheget.so not built ({path}); run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.heget_process_create.argtypes = [ctypes.POINTER(heget_process_ir), ctypes.c_int, ctypes.POINTER(vp)]
    L.heget_process_create.restype = ctypes.c_int
    L.heget_process_destroy.argtypes = [vp]
    L.heget_process_destroy.restype = ctypes.c_int
    L.heget_eval.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, vp, vp, vp]
    L.heget_eval.restype = ctypes.c_int
    L.heget_generate.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, vp, vp, vp]
    L.heget_generate.restype = ctypes.c_int
    L.heget_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, vp, vp]
    L.heget_uniforms.restype = ctypes.c_int
    L.heget_integrate.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.POINTER(heget_result), vp]
    L.heget_integrate.restype = ctypes.c_int
    L.heget_integrate_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                          ctypes.POINTER(heget_result), vp]
    L.heget_integrate_noalloc.restype = ctypes.c_int
    L.heget_integrate_async.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, vp, vp]
    L.heget_integrate_async.restype = ctypes.c_int
    L.heget_result_from_sums.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                         ctypes.POINTER(heget_result)]
    L.heget_result_from_sums.restype = ctypes.c_int
    L.heget_integrate_adaptive.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_uint64, ctypes.POINTER(heget_result),
                                           ctypes.POINTER(heget_result), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), vp]
    L.heget_integrate_adaptive.restype = ctypes.c_int
    L.heget_process_grid_dims.argtypes = [vp]
    L.heget_process_grid_dims.restype = ctypes.c_int32
    L.heget_process_n_helicities.argtypes = [vp]
    L.heget_process_n_helicities.restype = ctypes.c_int32
    L.heget_filter_helicities.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_int32)]
    L.heget_filter_helicities.restype = ctypes.c_int
    L.heget_server_create.argtypes = [ctypes.POINTER(heget_server_config), ctypes.POINTER(vp)]
    L.heget_server_create.restype = ctypes.c_int
    L.heget_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, vp,
                                      ctypes.POINTER(ctypes.c_uint64)]
    L.heget_server_submit.restype = ctypes.c_int
    L.heget_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(heget_result),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    L.heget_server_poll.restype = ctypes.c_int
    L.heget_server_stats_get.argtypes = [vp, ctypes.POINTER(heget_server_stats)]
    L.heget_server_stats_get.restype = ctypes.c_int
    L.heget_server_destroy.argtypes = [vp]
    L.heget_server_destroy.restype = ctypes.c_int
    L.heget_last_error.argtypes = []
    L.heget_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


class HegetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"heget status {status}: {msg}")
        self.status = status


def check(status):
    if status != HEGET_OK:
        raise HegetError(status, load().heget_last_error().decode())
