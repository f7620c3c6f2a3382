"""Loader of the HIP library and ctypes signatures of its C ABI
(include/mi355lbm.h).  There is no fallback: a missing library raises."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355lbm.so")

_lib = None


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("u_in", ctypes.c_double), ("nu", ctypes.c_double), ("omega2", ctypes.c_double),
        ("mode", ctypes.c_int32), ("galilean", ctypes.c_int32),
        ("lam", ctypes.c_double),
        ("obstacle_bc", ctypes.c_int32),
        ("body_force", ctypes.c_double * 3),
        ("avg_start", ctypes.c_int64),
        ("snap_every", ctypes.c_int32), ("snap_count", ctypes.c_int32),
        ("snap_start", ctypes.c_int64),
        ("force_every", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
        ("perturb_seed", ctypes.c_uint64), ("perturb_amp", ctypes.c_double),
        ("re", ctypes.c_double), ("l_ref", ctypes.c_double),
        ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("force_capacity", ctypes.c_int64),
    ]


class FnoParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nx", "ny", "nz", "cin", "cout", "width", "layers", "mx", "my", "mz", "proj_hidden", "max_batch",
                 "proj_act")] + [("proj_w0", ctypes.c_float), ("arch", ctypes.c_int32),
                                 ("ff_hidden", ctypes.c_int32)]


class UnetParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("nx", "ny", "nz", "cin", "cout")] + \
               [("widths", ctypes.c_int32 * 4), ("bottleneck", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


def _sig(L):
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.lbm_default_params.argtypes = [P(LbmParams), i32, i32, i32]
    L.lbm_create.argtypes = [P(LbmParams), vp, i64, vp, vp, vp, vp, vp, P(vp)]
    L.lbm_workspace_size.argtypes = [P(LbmParams), vp, P(ctypes.c_size_t)]
    L.lbm_create_in.argtypes = [P(LbmParams), vp, i64, vp, vp, vp, vp, vp, ctypes.c_size_t, vp, P(vp)]
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_mean_fields.argtypes = [vp, vp, ctypes.c_int, P(i64)]
    L.lbm_mean_fields_pooled.argtypes = [vp, i32, i32, vp]
    L.lbm_snapshots.argtypes = [vp, vp, ctypes.c_int, P(i32), vp]
    L.lbm_forces.argtypes = [vp, vp, i64, P(i64), vp]
    L.lbm_moments.argtypes = [vp, vp, ctypes.c_int]
    L.lbm_get_populations.argtypes = [vp, vp]
    L.lbm_set_populations.argtypes = [vp, vp]
    L.lbm_get_populations_box.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp]
    L.lbm_mass.argtypes = [vp, P(dbl)]
    L.lbm_export_state.argtypes = [vp, vp, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.lbm_import_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_info.argtypes = [vp, P(i64), P(dbl), P(i32)]
    L.lbm_profile.argtypes = [vp, ctypes.c_int]
    L.lbm_profile_read.argtypes = [vp, P(dbl), P(i64)]
    L.lbm_bandwidth_probe.argtypes = [vp, i32, P(dbl)]
    L.lbm_copy_bandwidth.argtypes = [i64, i32, vp, P(dbl)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    if hasattr(L, "fno_create"):
        L.fno_param_count.argtypes = [P(FnoParams)]
        L.fno_param_count.restype = i64
        L.fno_create.argtypes = [P(FnoParams), ctypes.c_uint64, vp, P(vp)]
        L.fno_set_params.argtypes = [vp, vp, i64]
        L.fno_get_params.argtypes = [vp, vp, i64]
        L.fno_forward.argtypes = [vp, vp, i32, vp]
        L.fno_loss_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.fno_adam_step.argtypes = [vp, ctypes.c_float]
        L.fno_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
        L.fno_destroy.argtypes = [vp]
        L.fno_destroy.restype = None
        L.fno_last_error.argtypes = [vp]
        L.fno_field_minmax.argtypes = [vp, i64, i32, i64, vp, vp, vp]
        L.fno_field_minmax_noalloc.argtypes = [vp, i64, i32, i64, vp, vp, vp]
        L.fno_field_scale.argtypes = [vp, i64, i32, i64, vp, vp, i32, vp]
        L.fno_last_error.restype = ctypes.c_char_p
    if hasattr(L, "unet_create"):
        L.unet_param_count.argtypes = [P(UnetParams)]
        L.unet_param_count.restype = i64
        L.unet_create.argtypes = [P(UnetParams), ctypes.c_uint64, vp, P(vp)]
        L.unet_set_params.argtypes = [vp, vp, i64]
        L.unet_get_params.argtypes = [vp, vp, i64]
        L.unet_bn_stats.argtypes = [vp, vp, i64]
        L.unet_forward.argtypes = [vp, vp, i32, i32, vp]
        L.unet_loss_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.unet_adam_step.argtypes = [vp, ctypes.c_float]
        L.unet_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
        L.unet_destroy.argtypes = [vp]
        L.unet_destroy.restype = None
        L.unet_last_error.argtypes = [vp]
        L.unet_last_error.restype = ctypes.c_char_p


def load():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run python -m paper_2606_16765_amd.build)")
        # torch bundles its own HIP runtime (same SONAME, different file
        # name in its NEEDED entries); loading torch first makes this
        # library bind to that runtime, so device pointers and streams are
        # shared with torch instead of living in a second runtime instance
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        _sig(L)
        _lib = L
    return _lib


class HipError(RuntimeError):
    pass


CODES = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSTABLE", 5: "ESTATE"}


def check(rc, obj=None, what=""):
    if rc != 0:
        L = load()
        msg = L.lbm_last_error(obj)
        msg = msg.decode() if msg else ""
        err = HipError(f"{what} failed: {CODES.get(rc, rc)}: {msg}")
        err.code = rc
        raise err
