"""ctypes declarations of the dbq C ABI (include/dbq.h).  Loading fails loudly when the HIP
library has not been built: there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DBQ_LIBRARY selects another build of the same library (e.g. a variant compiled with different
# kernel tuning flags); by default the in-tree libdbq.so next to this file is loaded.
LIB_PATH = os.environ.get("DBQ_LIBRARY") or os.path.join(HERE, "libdbq.so")

DBQ_OK, DBQ_NOT_CONVERGED = 0, 1
DBQ_EINVAL, DBQ_EBREAKDOWN, DBQ_ESINGULAR, DBQ_EHIP, DBQ_ENOMEM = -1, -2, -3, -4, -5
DBQ_FP64, DBQ_MIXED = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EBREAKDOWN", -3: "ESINGULAR",
                -4: "EHIP", -5: "ENOMEM"}

EXPORTED = ["dbq_create", "dbq_destroy", "dbq_last_error", "dbq_set_stream", "dbq_geometry",
            "dbq_geometry_host", "dbq_site_tile", "wilson_apply", "gmresdr_first_rhs", "dbicgstab_solve",
            "project_shifts", "gmres_proj_solve", "link_force", "kappa_critical",
            "kappa_critical_ritz", "dbq_set_timing",
            "dbq_kernel_time",
            "dbq_reset_timing", "dbq_version", "dbq_tile_schedule_host", "dbq_stream_probe",
            "wilson_apply_noalloc"]


class Operator(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("links", ctypes.c_void_p),
                ("kappa", ctypes.c_double), ("mu", ctypes.c_double),
                ("schur", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("matvecs", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("restarts", ctypes.c_int64), ("reliable_updates", ctypes.c_int64),
                ("rel_true_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int32), ("fp64_continued", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"} | {
            "status_name": STATUS_NAMES.get(self.status, str(self.status))}


_lib = None


def load():
    """Load libdbq.so (built by ``python -m paper_0710_1988_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_0710_1988_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PI32 = ctypes.POINTER(ctypes.c_int32)
    PD = ctypes.POINTER(ctypes.c_double)
    POP = ctypes.POINTER(Operator)
    PST = ctypes.POINTER(Stats)
    sig = {
        "dbq_create": ([ctypes.POINTER(P), P], ctypes.c_int),
        "dbq_destroy": ([P], ctypes.c_int),
        "dbq_last_error": ([P], ctypes.c_char_p),
        "dbq_set_stream": ([P, P], ctypes.c_int),
        "dbq_geometry": ([P, PI32, P, P], ctypes.c_int),
        "dbq_geometry_host": ([PI32, PI32, PI32], ctypes.c_int),
        "dbq_site_tile": ([PI32, PI32], ctypes.c_int),
        "wilson_apply": ([P, POP, P, P, I32, I32, I32], ctypes.c_int),
        "wilson_apply_noalloc": ([P, POP, P, P, I32, I32, I32], ctypes.c_int),
        "gmresdr_first_rhs": ([P, POP, P, P, I32, I32, D, I64, P, PD, PI32, PST], ctypes.c_int),
        "dbicgstab_solve": ([P, POP, I32, ctypes.POINTER(P), PI32, ctypes.POINTER(P),
                             ctypes.POINTER(P), PI32, D, I64, I32, I32, PST], ctypes.c_int),
        "project_shifts": ([P, POP, P, I32, P, P, I32, PD], ctypes.c_int),
        "gmres_proj_solve": ([P, POP, P, I32, P, P, I32, I32, D, I64, PST], ctypes.c_int),
        "link_force": ([P, POP, P, P, I32, I32, P], ctypes.c_int),
        "kappa_critical": ([P, PI32, P, I32, I32, D, I64, PD, PD, PD], ctypes.c_int),
        "kappa_critical_ritz": ([P, PI32, P, I32, I32, D, I64, PD, PD, PD, I32, PD], ctypes.c_int),
        "dbq_set_timing": ([P, I32], ctypes.c_int),
        "dbq_kernel_time": ([P, I32, PD, ctypes.POINTER(I64), PD], ctypes.c_int),
        "dbq_reset_timing": ([P], ctypes.c_int),
        "dbq_version": ([], ctypes.c_char_p),
        "dbq_tile_schedule_host": ([PI32, I32, I32, PI32, PI32], ctypes.c_int),
        "dbq_stream_probe": ([P, P, P, I64, I32, I32, PD], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib
