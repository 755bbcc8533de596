"""ctypes declarations of the libhamlet C ABI (include/hamlet.h).

Argument marshalling only: no step of the computation runs here.  Loading
fails loudly when the shared library has not been built.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# HAMLET_LIB names another build of the library (the autotuner's candidates)
LIB_PATH = os.environ.get("HAMLET_LIB") or os.path.join(_PKG, "libhamlet.so")

HAMLET_OK = 0
HAMLET_FP64 = 0
HAMLET_FP32_FP64E = 1

_STATUS = {0: "HAMLET_OK", -1: "HAMLET_EINVAL", -2: "HAMLET_ENOMEM", -3: "HAMLET_EDEVICE",
           -4: "HAMLET_EUNSUPPORTED"}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_void_pp = ctypes.POINTER(ctypes.c_void_p)
c_double_pp = ctypes.POINTER(c_double_p)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n_grid", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("omega_m", ctypes.c_double),
        ("h", ctypes.c_double),
        ("f_growth", ctypes.c_double),
        ("sigma_v", ctypes.c_double),
        ("pk_n2", c_double_p),
        ("n_pk", ctypes.c_int32),
        ("hist_width", ctypes.c_double),
        ("sample_distances", ctypes.c_int32),
        ("sample_sigma_nl", ctypes.c_int32),
        ("sample_cosmology", ctypes.c_int32),
    ]


class Catalog(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("rhat", c_double_p),
        ("mu", c_double_p),
        ("sigma_mu", c_double_p),
        ("cz", c_double_p),
        ("sigma_cz", c_double_p),
    ]


class HmcOpts(ctypes.Structure):
    _fields_ = [
        ("n_iter", ctypes.c_int32),
        ("n_leapfrog", ctypes.c_int32),
        ("warmup", ctypes.c_int32),
        ("jitter_eps", ctypes.c_int32),
        ("eps0", ctypes.c_double),
        ("target_accept", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("resume", ctypes.c_int32),
        ("seeds", ctypes.POINTER(ctypes.c_uint64)),
    ]


class Schedule(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "threads_xy", "threads_x", "threads_gather", "threads_scatter", "tile_width", "pencils_scatter",
        "pencils_gather", "radix_plan")] + [("radix", ctypes.c_int32 * 3)]


class NutsOpts(ctypes.Structure):
    _fields_ = [
        ("n_iter", ctypes.c_int32),
        ("warmup", ctypes.c_int32),
        ("max_depth", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("eps0", ctypes.c_double),
        ("target_accept", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("seeds", ctypes.POINTER(ctypes.c_uint64)),
    ]


class ServerDesc(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("max_running", ctypes.c_int32),
        ("ticks_ahead", ctypes.c_int32),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("queued", ctypes.c_int32),
        ("running", ctypes.c_int32),
        ("finished", ctypes.c_int32),
        ("ticks", ctypes.c_int64),
        ("bytes_in_use", ctypes.c_size_t),
    ]


# Every function the header declares, with its ctypes signature.
SIGNATURES = {
    "hamlet_plan_create": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.POINTER(Catalog), ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "hamlet_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "hamlet_plan_footprint_bytes": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.c_int64,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "hamlet_logpost_grad": (ctypes.c_int, [c_void_pp, ctypes.c_int32, c_void_pp, c_double_pp, c_double_pp,
                                           c_void_pp, c_double_pp, c_double_pp, c_double_pp]),
    "hamlet_logpost_grad_entries": (ctypes.c_int, [c_void_pp, ctypes.c_int32, c_void_pp, c_double_pp, c_double_pp,
                                                   c_void_pp, c_double_pp, c_double_pp, c_double_pp]),
    "hamlet_leapfrog": (ctypes.c_int, [c_void_pp, ctypes.c_int32, c_double_p, c_int32_p, c_void_pp, c_double_pp,
                                       c_double_pp, c_void_pp, c_double_pp, c_double_pp, c_double_pp]),
    "hamlet_hmc_run": (ctypes.c_int, [c_void_pp, ctypes.c_int32, ctypes.POINTER(HmcOpts), c_void_pp, c_double_pp,
                                      c_double_pp, c_void_pp, c_double_pp, ctypes.POINTER(c_int32_p), c_double_p]),
    "hamlet_nuts_run": (ctypes.c_int, [c_void_pp, ctypes.c_int32, ctypes.POINTER(NutsOpts), c_void_pp, c_double_pp,
                                       c_double_pp, c_void_pp, ctypes.POINTER(c_int32_p), ctypes.POINTER(c_int32_p),
                                       ctypes.POINTER(c_int32_p), c_double_pp, c_double_p]),
    "hamlet_flat_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "hamlet_pack_flat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_double_p, c_double_p, c_double_p]),
    "hamlet_unpack_flat": (ctypes.c_int, [ctypes.c_void_p, c_double_p, ctypes.c_void_p, c_double_p, c_double_p]),
    "hamlet_sphere_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_double_p, ctypes.c_int32,
                                             c_double_p]),
    "hamlet_velocity_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hamlet_density_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hamlet_field_stats_accumulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hamlet_shell_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_void_p]),
    "hamlet_shell_stats_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                                 ctypes.c_int32, ctypes.c_void_p]),
    "hamlet_server_create": (ctypes.c_int, [ctypes.POINTER(ServerDesc), ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "hamlet_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "hamlet_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanDesc), ctypes.POINTER(Catalog),
                                            ctypes.POINTER(HmcOpts), c_double_p, c_double_p, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_int64)]),
    "hamlet_server_tick": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "hamlet_server_job_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, c_int32_p]),
    "hamlet_server_take": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, c_double_p, c_double_p, c_double_p,
                                          c_double_p, c_double_p, c_int32_p, c_double_p]),
    "hamlet_profile_start": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "hamlet_profile_stop": (ctypes.c_int, [ctypes.c_void_p, c_double_p, ctypes.POINTER(ctypes.c_int64)]),
    "hamlet_schedule_get": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule)]),
    "hamlet_last_error": (ctypes.c_char_p, []),
}

_lib = None


class HamletError(RuntimeError):
    pass


def load(path=LIB_PATH):
    """Load libhamlet.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhamlet.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2203_02369_amd.build" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != HAMLET_OK:
        msg = load().hamlet_last_error().decode(errors="replace")
        raise HamletError("%s: %s" % (_STATUS.get(status, str(status)), msg))


def ptr_array(ctype, values):
    arr = (ctype * len(values))()
    for i, v in enumerate(values):
        arr[i] = ctypes.cast(ctypes.c_void_p(v), ctype) if v is not None else None
    return arr


def double_ptr(addr):
    return ctypes.cast(ctypes.c_void_p(addr), c_double_p) if addr else None
