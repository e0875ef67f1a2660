"""ctypes view of the C ABI in include/swarmsf.h (argument marshalling only)."""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libswarmsf.so")

SF_OK, SF_EINVAL, SF_ENOMEM, SF_EDEVICE, SF_EUNSUPPORTED = range(5)
SF_FP64, SF_FP32, SF_BF16, SF_FP16 = range(4)
SF_RESID_HISTORY = 1
SF_GENERIC_KERNEL = 2
SF_USE_GRAPH = 4
SF_AUTOTUNE = 8
SF_PERSISTENT = 16
SF_FP_RESIDUAL = 32
SF_SAMPLE_NONFINITE_INPUT, SF_SAMPLE_NONFINITE, SF_SAMPLE_NOT_CONVERGED = 1, 2, 4
SF_CONV_TOL = 1e-3
PRECISIONS = {"fp64": SF_FP64, "fp32": SF_FP32, "bf16": SF_BF16, "fp16": SF_FP16}

EXPORTED = ["sf_setup", "sf_destroy", "sf_project", "sf_project_backward", "sf_feasibility",
            "sf_qp_equality", "sf_qp_equality_backward", "sf_qp_equality_backward_noalloc", "sf_factor_table",
            "sf_last_error"]


class SfConfig(ctypes.Structure):
    _fields_ = [("n_robots", c_int32), ("dims", c_int32), ("degree", c_int32), ("horizon", c_int32),
                ("t_final", c_double), ("safety_a", c_double), ("safety_b", c_double),
                ("vmax", c_double), ("amax", c_double),
                ("rho_coll", c_double), ("rho_vel", c_double), ("rho_acc", c_double),
                ("ws_a", c_double), ("ws_b", c_double), ("rho_ws", c_double),
                ("ws_x", c_double), ("ws_y", c_double), ("ws_z", c_double)]


class SfBatch(ctypes.Structure):
    _fields_ = [("n_problems", c_int32), ("cfg_slot", POINTER(c_int32)), ("sample_count", POINTER(c_int32))]


class SfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"swarmsf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libswarmsf.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.sf_setup.argtypes = [POINTER(SfConfig), c_int32, POINTER(vp)]
    L.sf_setup.restype = c_int32
    L.sf_destroy.argtypes = [vp]
    L.sf_destroy.restype = None
    L.sf_project.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, vp, vp, c_int32, vp, vp, vp, vp, c_int32,
                             vp, c_int32, vp]
    L.sf_project.restype = c_int32
    L.sf_project_backward.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, c_int32, vp, c_int32,
                                      vp, vp, vp, vp, vp, vp, vp, vp]
    L.sf_project_backward.restype = c_int32
    L.sf_feasibility.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, vp, vp]
    L.sf_feasibility.restype = c_int32
    L.sf_qp_equality.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, vp, vp]
    L.sf_qp_equality.restype = c_int32
    L.sf_qp_equality_backward.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, vp, vp]
    L.sf_qp_equality_backward.restype = c_int32
    L.sf_qp_equality_backward_noalloc.argtypes = [vp, POINTER(SfBatch), c_int32, vp, vp, vp, vp]
    L.sf_qp_equality_backward_noalloc.restype = c_int32
    L.sf_factor_table.argtypes = [POINTER(SfConfig), POINTER(c_double), c_int64, POINTER(c_int64)]
    L.sf_factor_table.restype = c_int32
    L.sf_last_error.argtypes = []
    L.sf_last_error.restype = c_char_p
    _lib = L
    return L


def check(code):
    if code != SF_OK:
        raise SfError(code, lib().sf_last_error().decode())


def make_config(c) -> SfConfig:
    return SfConfig(int(c.n_robots), int(c.dims), int(c.degree), int(c.horizon), float(c.t_final),
                    float(c.safety_a), float(c.safety_b), float(c.vmax), float(c.amax),
                    float(getattr(c, "rho_coll", 1.0)), float(getattr(c, "rho_vel", 1.0)),
                    float(getattr(c, "rho_acc", 1.0)),
                    float(getattr(c, "ws_a", 0.0)), float(getattr(c, "ws_b", 0.0)),
                    float(getattr(c, "rho_ws", 1.0)), float(getattr(c, "ws_x", 0.0)),
                    float(getattr(c, "ws_y", 0.0)), float(getattr(c, "ws_z", 0.0)))
