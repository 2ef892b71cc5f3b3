"""ctypes binding of libcola (include/cola.h): argument marshalling only.

Every computation runs in the HIP library; this module only converts torch tensors to device
pointers, passes torch's current HIP stream, and raises on a non-zero status.  If libcola.so is
missing the import fails loudly -- there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcola.so")

COLA_OK = 0
STATUS_NAMES = {0: "COLA_OK", -1: "COLA_ERR_INVALID_ARG", -2: "COLA_ERR_UNSUPPORTED_SIZE",
                -3: "COLA_ERR_WORKSPACE_TOO_SMALL", -4: "COLA_ERR_HIP", -5: "COLA_ERR_STATE",
                -6: "COLA_ERR_NONFINITE"}

# every exported symbol of include/cola.h
EXPORTS = ("cola_workspace_bytes", "cola_ic_2lpt", "cola_pm_force", "cola_step",
           "cola_power_spectrum", "cola_power_spectrum_jing", "cola_cic_density", "cola_cic_workspace_bytes",
           "cola_fft_workspace_bytes", "cola_fft_r2c", "cola_fft_c2r", "cola_schedule_table",
           "cola_linear_power", "cola_status_string", "cola_version", "cola_profiler_enable",
           "cola_profiler_num_kinds", "cola_profiler_kind_name", "cola_profiler_read", "cola_copy",
           "cola_last_error", "cola_autotune", "cola_ensemble_run", "cola_ensemble_release",
           "cola_lc_param_count", "cola_lc_packed_bytes", "cola_lc_workspace_bytes", "cola_lc_pack",
           "cola_lc_forward", "cola_lc_backward", "cola_lc_loss", "cola_lc_adam", "cola_step_lc",
           "cola_pm_fields_workspace_bytes", "cola_pm_fields", "cola_positions", "cola_mfma_selftest",
           "cola_profiler_read_groups", "cola_fof_workspace_bytes", "cola_fof", "cola_fof_catalogue",
           "cola_fof_mass_histogram", "cola_particle_mass", "cola_power_multipoles", "cola_pm_force_lc",
           "cola_mesh_force", "cola_fft_set_shape", "cola_pm_force_noalloc")


class ColaError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.cola_status_string(status).decode() if _lib is not None else "?"
        if status == -4 and _lib is not None:
            msg += "; " + _lib.cola_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({msg})")


class Cosmology(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("omega_b", ctypes.c_double), ("h", ctypes.c_double),
                ("n_s", ctypes.c_double), ("sigma_8", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double), ("n_part", ctypes.c_int32), ("pm_factor", ctypes.c_int32),
                ("z_init", ctypes.c_double), ("a_final", ctypes.c_double),
                ("n_steps", ctypes.c_int32), ("sampling", ctypes.c_int32),
                ("n_real", ctypes.c_int32), ("frame", ctypes.c_int32), ("sampling_power", ctypes.c_double)]


_F3 = ctypes.c_void_p * 3


class Particles(ctypes.Structure):
    _fields_ = [("x", _F3), ("p", _F3), ("psi1", _F3), ("psi2", _F3),
                ("node", ctypes.c_int32), ("force_node", ctypes.c_int32),
                ("force_ws", ctypes.c_void_p)]


class EnsembleClass(ctypes.Structure):
    _fields_ = [("prob", Problem), ("seeds", ctypes.POINTER(ctypes.c_uint64)),
                ("parts", ctypes.POINTER(Particles)), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("n_out", ctypes.c_int32), ("a_out", ctypes.POINTER(ctypes.c_double)),
                ("n_pk", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("k_mean", ctypes.c_void_p), ("pk", ctypes.c_void_p), ("n_modes", ctypes.c_void_p),
                ("net", ctypes.c_void_p), ("lc_ws", ctypes.c_void_p), ("lc_ws_bytes", ctypes.c_size_t)]


class LcNet(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("in_scale", ctypes.c_float * 4), ("out_scale", ctypes.c_float),
                ("out_scale_slope", ctypes.c_float), ("out_band", ctypes.c_float),
                ("n_knots", ctypes.c_int32), ("knot_a", ctypes.c_float * 8), ("knot_v", ctypes.c_float * 8),
                ("n_gknots", ctypes.c_int32), ("gknot_u", ctypes.c_float * 10), ("gknot_t", (ctypes.c_float * 10) * 8),
                ("params", ctypes.c_void_p), ("grads", ctypes.c_void_p), ("adam_m", ctypes.c_void_p),
                ("adam_v", ctypes.c_void_p), ("packed", ctypes.c_void_p)]


def _load():
    # torch bundles its own HIP runtime under the same soname (libamdhip64.so.7).  Whichever is
    # loaded first serves the whole process, and the streams and device pointers this binding
    # passes in come from torch's instance, so torch must be loaded before libcola.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcola.so not built at {LIB_PATH}; run python -m paper_1509_04685_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P, C, PP = ctypes.POINTER(Problem), ctypes.POINTER(Cosmology), ctypes.POINTER(Particles)
    N = ctypes.POINTER(LcNet)
    sig = {
        "cola_workspace_bytes": (sz, [P, i32]),
        "cola_ic_2lpt": (ctypes.c_int, [P, C, ctypes.POINTER(ctypes.c_uint64), PP, vp, sz, vp]),
        "cola_pm_force": (ctypes.c_int, [P, PP, ctypes.POINTER(vp), vp, sz, vp]),
        "cola_step": (ctypes.c_int, [P, C, i32, i32, PP, vp, sz, vp]),
        "cola_power_spectrum": (ctypes.c_int, [P, C, PP, dbl, i32, i32, vp, vp, vp, vp, sz, vp]),
        "cola_power_spectrum_jing": (ctypes.c_int, [P, C, PP, dbl, i32, i32, i32, vp, vp, vp, vp, sz, vp]),
        "cola_cic_density": (ctypes.c_int, [ctypes.POINTER(vp), i64, i32, dbl, vp, vp, sz, vp]),
        "cola_cic_workspace_bytes": (sz, [i64, i32]),
        "cola_fft_workspace_bytes": (sz, [i32]),
        "cola_fft_r2c": (ctypes.c_int, [i32, vp, vp, vp, sz, vp]),
        "cola_fft_c2r": (ctypes.c_int, [i32, vp, vp, vp, sz, vp]),
        "cola_schedule_table": (ctypes.c_int, [P, C, ctypes.POINTER(dbl)]),
        "cola_linear_power": (dbl, [C, dbl]),
        "cola_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "cola_version": (ctypes.c_char_p, []),
        "cola_profiler_enable": (ctypes.c_int, [ctypes.c_int]),
        "cola_profiler_num_kinds": (ctypes.c_int, []),
        "cola_profiler_kind_name": (ctypes.c_char_p, [ctypes.c_int]),
        "cola_profiler_read": (ctypes.c_int, [i32, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64)]),
        "cola_copy": (ctypes.c_int, [vp, vp, sz, vp]),
        "cola_last_error": (ctypes.c_char_p, []),
        "cola_autotune": (ctypes.c_int, [P, i32, vp, sz, vp, ctypes.c_char_p, sz]),
        "cola_ensemble_run": (ctypes.c_int, [i32, ctypes.POINTER(EnsembleClass), C, i32, vp]),
        "cola_ensemble_release": (ctypes.c_int, []),
        "cola_lc_param_count": (i64, [i32]),
        "cola_lc_packed_bytes": (sz, [i32]),
        "cola_lc_workspace_bytes": (sz, [i32, i32, i32, i32]),
        "cola_lc_pack": (ctypes.c_int, [N, vp]),
        "cola_lc_forward": (ctypes.c_int, [N, i32, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, i32, vp, sz, vp]),
        "cola_lc_backward": (ctypes.c_int, [N, i32, vp, vp, sz, vp]),
        "cola_lc_loss": (ctypes.c_int, [i32, dbl, ctypes.POINTER(vp), i64, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), vp, vp, vp]),
        "cola_lc_adam": (ctypes.c_int, [N, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
        "cola_step_lc": (ctypes.c_int, [P, C, i32, i32, PP, N, vp, sz, vp, sz, vp]),
        "cola_pm_fields_workspace_bytes": (sz, [i32]),
        "cola_pm_fields": (ctypes.c_int, [i32, dbl, ctypes.POINTER(vp), i64, vp, ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), vp, sz, vp]),
        "cola_positions": (ctypes.c_int, [P, PP, ctypes.POINTER(vp), vp]),
        "cola_mfma_selftest": (ctypes.c_int, [vp, vp, vp, vp]),
        "cola_profiler_read_groups": (ctypes.c_int, [i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                                     ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "cola_fof_workspace_bytes": (sz, [i64, dbl, dbl]),
        "cola_fof": (ctypes.c_int, [ctypes.POINTER(vp), i64, dbl, dbl, vp, vp, vp, sz, vp]),
        "cola_fof_catalogue": (ctypes.c_int, [ctypes.POINTER(vp), i64, dbl, vp, vp, i32, dbl, i64, vp, vp, vp,
                                              ctypes.POINTER(vp), vp, vp, sz, vp]),
        "cola_fof_mass_histogram": (ctypes.c_int, [vp, i64, i32, dbl, ctypes.POINTER(dbl), i32, vp, vp]),
        "cola_particle_mass": (dbl, [C, dbl, i32]),
        "cola_pm_force_lc": (ctypes.c_int, [P, PP, N, dbl, vp, sz, ctypes.POINTER(vp), vp, sz, vp]),
        "cola_pm_force_noalloc": (ctypes.c_int, [P, PP, ctypes.POINTER(vp), vp]),
        "cola_mesh_force": (ctypes.c_int, [i32, dbl, vp, ctypes.POINTER(vp), vp, sz, vp]),
        "cola_fft_set_shape": (ctypes.c_int, [i32, ctypes.c_char_p, i32, i32, i32]),
        "cola_power_multipoles": (ctypes.c_int, [P, C, PP, dbl, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def check(status, where):
    if status != COLA_OK:
        raise ColaError(status, where)
