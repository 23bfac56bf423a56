"""ctypes declarations of the C ABI in include/lp.h (argument marshalling only).

Importing this module loads the in-tree HIP library ``_lp_hip.so``; it raises
ImportError if the library has not been built.  There is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "_lp_hip.so")

LP_OK, LP_EINVAL, LP_ENOMEM, LP_EDEVICE, LP_ETIME, LP_ESTATE = 0, -1, -2, -3, -4, -5
LP_MESH_FLAT, LP_MESH_SPHERICAL = 0, 1
LP_F64, LP_F32, LP_BF16, LP_F16_SCALED = 0, 1, 2, 3
LP_DELETE, LP_FREEZE = 0, 1
LP_ST_OOB, LP_ST_LAND, LP_ST_DELETED, LP_ST_AGED = 1, 2, 4, 8
LP_KERNEL_RK4 = 0
LP_KERNEL_EULER = 1
LP_KERNEL_RKF45 = 2
LP_INTERP_LINEAR, LP_INTERP_NEAREST = 0, 1

# every function declared in include/lp.h
EXPORTS = (
    "fieldset_create", "fieldset_push_snapshot", "fieldset_push_snapshot_f64",
    "fieldset_push_snapshot_device", "fieldset_get_snapshot", "fieldset_resident",
    "fieldset_destroy", "lp_philox_normals",
    "pset_create", "pset_create_device", "pset_execute", "pset_status", "pset_get",
    "pset_get_noalloc",
    "pset_get_step_exponents", "pset_get_behaviour", "pset_records_behaviour",
    "fieldset_push_tracer", "fieldset_push_tracer_device",
    "pset_records", "pset_timing", "pset_destroy", "lp_last_error", "lp_version",
    "pset_execute_batch", "pset_autotune_batch",
    "surrogate_param_count", "surrogate_create", "surrogate_get_params", "surrogate_set_params",
    "surrogate_forward", "surrogate_gradients", "surrogate_train_step", "surrogate_destroy",
    "surrogate_train", "pset_execute_surrogate", "surrogate_features", "surrogate_check",
)


class lp_grid_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lon", C.c_void_p), ("lat", C.c_void_p), ("depth", C.c_void_p),
                ("mesh", C.c_int32), ("dtype", C.c_int32), ("capacity", C.c_int32),
                ("time_period", C.c_double), ("land", C.c_void_p)]


class lp_exec_opts(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("recovery", C.c_int32), ("Kh", C.c_double),
                ("run_id", C.c_uint32), ("seed", C.c_uint32), ("output_stride", C.c_int32),
                ("sort_every", C.c_int32), ("profile", C.c_int32),
                ("stencil_cache", C.c_int32), ("interp", C.c_int32),
                ("rkf_tol", C.c_double), ("rkf_min_exp", C.c_int32), ("rkf_max_exp", C.c_int32),
                ("sink_speed", C.c_double), ("dwell_depth", C.c_double), ("maxage", C.c_double),
                ("sample_tracer", C.c_int32), ("graph", C.c_int32), ("sort_steps", C.c_int32)]


class lp_counts(C.Structure):
    _fields_ = [("n", C.c_int64), ("active", C.c_int64), ("oob", C.c_int64),
                ("land", C.c_int64), ("deleted", C.c_int64), ("particle_steps", C.c_int64),
                ("time", C.c_double), ("step", C.c_int64), ("rejected_steps", C.c_int64)]


class lp_tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("stencil_cache", C.c_int32), ("sort_every", C.c_int32),
                ("sort_steps", C.c_int32), ("ms", C.c_double)]


class lp_surrogate_cfg(C.Structure):
    _fields_ = [("n_segments", C.c_int64), ("steps_per_segment", C.c_int32), ("dt", C.c_double),
                ("round_size", C.c_int32), ("batch", C.c_int32), ("iterations", C.c_int64),
                ("lr", C.c_double), ("seed", C.c_uint32)]


class lp_train_stats(C.Structure):
    _fields_ = [("segments_kept", C.c_int64), ("segments_dropped", C.c_int64),
                ("iterations", C.c_int64), ("first_loss", C.c_double),
                ("final_loss", C.c_double), ("gen_ms", C.c_double), ("train_ms", C.c_double)]


class lp_surrogate_stats(C.Structure):
    _fields_ = [("segments", C.c_int64), ("evaluated", C.c_int64), ("accepted", C.c_int64),
                ("fallback", C.c_int64), ("mlp_ms", C.c_double), ("coarse_ms", C.c_double),
                ("fine_ms", C.c_double), ("total_ms", C.c_double), ("sort_ms", C.c_double)]


class LPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lp error {code}: {msg}")
        self.code = code


def _declare(L):
    P = C.c_void_p
    I = C.c_int
    pp = C.POINTER(C.c_void_p)
    sig = {
        "fieldset_create": ([C.POINTER(lp_grid_desc), pp], I),
        "fieldset_push_snapshot": ([P, C.c_double, P, P, P, P], I),
        "fieldset_push_snapshot_f64": ([P, C.c_double, P, P, P, P], I),
        "fieldset_push_snapshot_device": ([P, C.c_double, P, P, P, P], I),
        "fieldset_get_snapshot": ([P, C.c_double, P, P, P], I),
        "lp_philox_normals": ([C.c_uint32, C.c_uint32, C.c_int64, P, P, P, P], I),
        "fieldset_resident": ([P, C.POINTER(C.c_int32), P], I),
        "fieldset_destroy": ([P], None),
        "pset_create": ([P, C.c_int64, P, P, P, C.c_double, C.c_int64, pp], I),
        "pset_create_device": ([P, C.c_int64, P, P, P, C.c_double, C.c_int64, P, pp], I),
        "pset_execute": ([P, C.c_double, C.c_double, C.c_double, C.POINTER(lp_exec_opts), P], I),
        "pset_status": ([P, C.POINTER(lp_counts), P], I),
        "pset_get": ([P, P, P, P, P, P, P], I),
        "pset_get_noalloc": ([P, P, P, P, P, P, P], I),
        "pset_get_step_exponents": ([P, P], I),
        "pset_get_behaviour": ([P, P, P], I),
        "pset_records_behaviour": ([P, P, P], I),
        "fieldset_push_tracer": ([P, C.c_double, P, P], I),
        "fieldset_push_tracer_device": ([P, C.c_double, P, P], I),
        "pset_records": ([P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), P, P, P, P, P, P, P], I),
        "pset_timing": ([P, C.POINTER(C.c_double), C.POINTER(C.c_int64)], I),
        "pset_execute_batch": ([C.POINTER(C.c_void_p), C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.POINTER(lp_exec_opts), C.c_int32, P], I),
        "pset_autotune_batch": ([C.POINTER(C.c_void_p), C.c_int32, C.c_double, C.c_int32,
                                 C.POINTER(lp_exec_opts), C.c_char_p, C.POINTER(lp_tune)], I),
        "pset_destroy": ([P], None),
        "surrogate_param_count": ([], C.c_int64),
        "surrogate_create": ([C.c_uint32, pp], I),
        "surrogate_get_params": ([P, P], I),
        "surrogate_set_params": ([P, P], I),
        "surrogate_forward": ([P, C.c_int64, P, P], I),
        "surrogate_gradients": ([P, C.c_int64, P, P, P, P], I),
        "surrogate_train_step": ([P, C.c_int64, P, P, C.c_double, P], I),
        "surrogate_destroy": ([P], None),
        "surrogate_train": ([P, P, C.POINTER(lp_surrogate_cfg), C.POINTER(lp_train_stats), P], I),
        "pset_execute_surrogate": ([P, P, C.c_double, C.c_double, C.c_int32, C.c_double,
                                    C.POINTER(lp_surrogate_stats), P], I),
        "surrogate_features": ([P, C.c_int64, P, P, C.c_double, P], I),
        "surrogate_check": ([P, C.c_int64, P, P, P, P, P, P, C.c_double, P, P, P], I),
        "lp_last_error": ([], C.c_char_p),
        "lp_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def load():
    # torch carries its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes this library bind to that same runtime instance, so the stream
    # handles and device pointers torch hands over are valid here; loading the
    # library first would put a second HIP runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIBPATH):
        raise ImportError(f"HIP library not built: {LIBPATH} is missing "
                          "(run __graft_entry__.build())")
    return _declare(C.CDLL(LIBPATH))


lib = load()


def check(rc: int):
    if rc != LP_OK:
        raise LPError(rc, lib.lp_last_error().decode())
    return rc
