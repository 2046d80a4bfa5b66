"""ctypes binding of libmmx.so: argument marshalling only.

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, passes raw device pointers and the current torch stream,
and turns status codes into exceptions.  There is no CPU fallback: if the
library is missing, importing this module raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmmx.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EHIP, MM_ESTATE, MM_ENOTSUP, MM_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MM_F32, MM_F64 = 1, 2
MM_DEMAG, MM_EXCHANGE = 1, 2
MM_NO_RENORM, MM_NO_GRAPH = 1, 2

# Exported names (kept in sync with include/mmx.h; a CPU test checks both).
EXPORTS = [
    "mm_plan_opts_default", "demag_tensor_init", "mm_plan_destroy", "mm_plan_set_stream", "mm_plan_info",
    "mm_plan_bytes", "mm_plan_attach_memory", "mm_plan_scratch_bytes", "mm_plan_attach_scratch", "mm_plan_set_dmi", "mm_plan_set_anisotropy",
    "mm_plan_set_stt",
    "h_eff", "llg_step", "llg_rkf45_step", "mm_minimize_bb", "h_eff_adjoint", "llg_step_adjoint",
    "llg_step_adjoint_noalloc",
    "mm_demag_tensor_get", "mm_demag_tensor_set", "mm_demag_spectrum_get",
    "mm_batch_create", "mm_batch_h_eff", "mm_batch_llg_step", "mm_batch_tensor_set", "mm_batch_info",
    "mm_batch_schedule", "mm_batch_destroy", "mm_plan_schedule",
    "mm_plan_time_passes", "mm_device_copy", "mm_llg_stability",
    "mm_strerror", "mm_last_error",
]


class MMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (msg, code, _lib.mm_last_error().decode() if _lib else ""))
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [("far_radius", ctypes.c_double), ("L", ctypes.c_int64 * 3),
                ("autotune", ctypes.c_int), ("pow2_padding", ctypes.c_int)]


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError("libmmx.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2606_01114_amd/build.py" % LIBPATH)
    # The library and torch must share one HIP runtime (device pointers and
    # streams cross between them): load torch's first so that the library's
    # libamdhip64 dependency resolves to it.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIBPATH)
    vp, i64p, dp, ci, cu, cd = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                ctypes.c_int, ctypes.c_uint, ctypes.c_double)
    sig = {
        "mm_plan_opts_default": [ctypes.POINTER(PlanOpts)],
        "demag_tensor_init": [ctypes.POINTER(vp), i64p, dp, ci, vp, ctypes.POINTER(PlanOpts)],
        "mm_plan_destroy": [vp],
        "mm_plan_bytes": [i64p, ci, ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_size_t),
                          ctypes.POINTER(ctypes.c_size_t)],
        "mm_plan_attach_memory": [vp, vp, vp],
        "mm_plan_scratch_bytes": [i64p, ci, ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_size_t)],
        "mm_plan_attach_scratch": [vp, vp, ctypes.c_size_t],
        "mm_plan_set_dmi": [vp, ci, cd],
        "mm_plan_set_anisotropy": [vp, cd, dp],
        "mm_plan_set_stt": [vp, cd, cd, cd, cd, cd, dp],
        "mm_plan_set_stream": [vp, vp],
        "mm_plan_info": [vp, i64p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)],
        "h_eff": [vp, vp, vp, cd, cd, vp, cu, dp],
        "llg_step": [vp, vp, vp, cd, cd, cd, cd, cd, ci, dp, cu],
        "llg_rkf45_step": [vp, vp, vp, cd, cd, cd, cd, dp, cd, dp, cu, dp, ctypes.POINTER(ci)],
        "mm_minimize_bb": [vp, vp, vp, cd, cd, dp, cd, ci, ctypes.POINTER(ci), dp],
        "h_eff_adjoint": [vp, vp, vp, cd, cd, vp, vp, vp, cu],
        "llg_step_adjoint": [vp, vp, vp, cd, cd, cd, cd, cd, dp, cu, vp, vp],
        "llg_step_adjoint_noalloc": [vp, vp, vp, cd, cd, cd, cd, cd, dp, cu, vp, vp],
        "mm_demag_tensor_get": [vp, dp],
        "mm_demag_tensor_set": [vp, dp],
        "mm_demag_spectrum_get": [vp, dp],
        "mm_batch_create": [ctypes.POINTER(vp), ci, i64p, dp, ci, vp, ctypes.POINTER(PlanOpts)],
        "mm_batch_h_eff": [vp, ctypes.POINTER(vp), dp, cd, ctypes.POINTER(vp), cu],
        "mm_batch_llg_step": [vp, ctypes.POINTER(vp), dp, cd, cd, cd, cd, ci, cu],
        "mm_batch_tensor_set": [vp, ci, dp],
        "mm_batch_info": [vp, i64p, ctypes.POINTER(ctypes.c_size_t)],
        "mm_batch_destroy": [vp],
        "mm_batch_schedule": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "mm_plan_schedule": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "mm_plan_time_passes": [vp, ci, dp],
        "mm_device_copy": [vp, vp, ctypes.c_size_t, vp],
        "mm_llg_stability": [dp, cd, cd, cd, cd, dp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.mm_strerror.argtypes = [ctypes.c_int]
    L.mm_strerror.restype = ctypes.c_char_p
    L.mm_last_error.argtypes = []
    L.mm_last_error.restype = ctypes.c_char_p
    return L


_lib = None
_lib = _load()


def lib():
    return _lib


def check(rc):
    if rc != MM_OK:
        raise MMError(rc, _lib.mm_strerror(rc).decode())
    return rc
