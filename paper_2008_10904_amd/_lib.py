"""ctypes binding of libresolvent.so (argument marshalling only; every step of the method runs in the HIP
library).  The structures mirror include/resolvent.h field for field."""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libresolvent.so")

RES_OK, RES_EINVAL, RES_EGRID, RES_ESTEP, RES_EUNSTABLE, RES_ENONFINITE, RES_ENOMEM, RES_EHIP, RES_ENOTSUP = range(9)
RES_OP_TRIDIAG, RES_OP_ADR2D, RES_OP_ADR3D3C = 1, 2, 3
RES_FP64, RES_MIXED = 0, 1
RES_TRANSIENT, RES_PERIODIC = 0, 1
RES_TIMING_STEPPER, RES_TIMING_SYNTHESIS, RES_TIMING_PROJECTION, RES_TIMING_QR = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 256 << 20  # RESOLVENT_NOALLOC_SCRATCH_BYTES: the no-allocation apply's fixed workspace

_dp = POINTER(c_double)


class OpDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("precision", c_int32), ("h", c_double), ("ninst", c_int32),
                ("inst_offsets", POINTER(c_int64)), ("lower", _dp), ("diag", _dp), ("upper", _dp),
                ("nx", c_int64), ("ny", c_int64), ("nz", c_int64),
                ("cxm", _dp), ("cxp", _dp), ("cym", _dp), ("cyp", _dp), ("czm", _dp), ("czp", _dp),
                ("dfield", _dp), ("coupling", _dp),
                ("probe", c_int32), ("probe_tol", c_double), ("probe_tmax", c_double), ("probe_seed", c_uint64)]


class Grid(ctypes.Structure):
    _fields_ = [("omega0", c_double), ("domega", c_double), ("n_omega", c_int32)]


class Run(ctypes.Structure):
    _fields_ = [("method", c_int32), ("tail", c_int64), ("periods", c_int32), ("stride", c_int64)]


# Every symbol include/resolvent.h declares, with its ctypes signature.
SIGNATURES = {
    "resolvent_op_create": (c_int32, [POINTER(OpDesc), c_void_p, POINTER(c_void_p)]),
    "resolvent_op_destroy": (None, [c_void_p]),
    "resolvent_op_size": (c_int64, [c_void_p]),
    "resolvent_op_decay_time": (c_double, [c_void_p]),
    "resolvent_op_set_diagonal": (c_int32, [c_void_p, _dp, c_int32, c_void_p]),
    "resolvent_apply": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_void_p, c_void_p, c_void_p]),
    "resolvent_apply_noalloc": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_void_p, c_void_p,
                                          c_void_p]),
    "resolvent_workspace_size": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, POINTER(c_size_t)]),
    "resolvent_grid_from_omegas": (c_int32, [_dp, c_int32, c_double, c_int64, POINTER(Grid), POINTER(c_int64)]),
    "resolvent_adjoint_apply": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_void_p, c_void_p,
                                          c_void_p]),
    "resolvent_modes": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_int32, c_void_p, _dp,
                                  c_void_p, c_void_p, _dp, c_void_p]),
    "resolvent_krylov": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_int32, c_void_p, _dp,
                                   c_void_p, c_void_p, _dp, c_void_p]),
    "resolvent_apply_backward": (c_int32, [c_void_p, POINTER(Grid), POINTER(Run), c_int32, c_void_p, c_void_p,
                                           c_void_p, _dp, c_int32, c_void_p]),
    "resolvent_op_check": (c_int32, [c_void_p, c_void_p]),
    "resolvent_op_set_graphs": (c_int32, [c_void_p, c_int32]),
    "resolvent_op_set_backward_rows": (c_int32, [c_void_p, c_int32]),
    "resolvent_op_get_plan": (c_int32, [c_void_p, POINTER(c_int32)]),
    "resolvent_op_set_plan": (c_int32, [c_void_p, POINTER(c_int32)]),
    "resolvent_op_set_step_power": (c_int32, [c_void_p, c_int32]),
    "resolvent_op_set_weights": (c_int32, [c_void_p, _dp, _dp, _dp, _dp]),
    "resolvent_op_get_step_power": (c_int32, [c_void_p, POINTER(c_int32)]),
    "resolvent_op_tune": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), _dp, c_void_p]),
    "resolvent_op_set_timing": (c_int32, [c_void_p, c_int32]),
    "resolvent_op_get_timing": (c_int32, [c_void_p, c_int32, _dp, POINTER(c_int64)]),
    "resolvent_signal_run": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                       c_void_p]),
    "resolvent_fir_design": (c_int32, [c_int32, c_int32, _dp, _dp, _dp]),
    "resolvent_fir_apply": (c_int32, [c_int32, c_int64, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "resolvent_trm_modes": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_int32, c_void_p, c_int32, _dp, c_int32,
                                      c_int32, c_int32, c_int64, c_int64, c_double, _dp, _dp, c_void_p, c_void_p,
                                      c_void_p, c_void_p]),
    "resolvent_strerror": (ctypes.c_char_p, [c_int32]),
    "resolvent_last_error": (ctypes.c_char_p, []),
}

_lib = None


class ResolventError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (status %d)" % (message, code))
        self.code = code


def load():
    """Load the HIP library; raises ImportError if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libresolvent.so is not built: run `python -m paper_2008_10904_amd.build` "
                          "(the resolvent path has no CPU fallback)")
    # PyTorch ships its own HIP runtime.  Importing it first makes the loader resolve the library's
    # libamdhip64.so.7 to that same, already loaded runtime; loaded the other way round the process would hold
    # two HIP runtimes, and the one not initialised by torch reports no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code):
    if code != RES_OK:
        lib = load()
        detail = lib.resolvent_last_error().decode()
        msg = lib.resolvent_strerror(code).decode()
        raise ResolventError(code, msg + (": " + detail if detail else ""))
