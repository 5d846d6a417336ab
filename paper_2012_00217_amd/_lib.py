"""ctypes loader and prototypes for libmbl.so (declared in include/mbl.h).

The library is loaded from this package directory only.  There is no
fallback: if it is missing, importing the solver API raises.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MBL_LIBRARY") or os.path.join(HERE, "libmbl.so")

MBL_OK, MBL_EINVAL, MBL_ENOMEM, MBL_EDEVICE, MBL_ENOCONV, MBL_EBREAKDOWN, MBL_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -8)
MBL_F64, MBL_F32, MBL_MIXED, MBL_PCG32 = 0, 1, 2, 3

STATUS_NAMES = {0: "MBL_OK", -1: "MBL_EINVAL", -2: "MBL_ENOMEM", -3: "MBL_EDEVICE",
                -4: "MBL_ENOCONV", -5: "MBL_EBREAKDOWN", -8: "MBL_EINTERNAL"}


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("pcg_iters", C.c_int), ("precision", C.c_int),
                ("verbose", C.c_int), ("timing", C.c_int), ("seed", C.c_uint64)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("iters_fp64", C.c_int), ("nconv", C.c_int),
                ("applies", C.c_int64), ("pcg_steps", C.c_int64), ("seconds", C.c_double),
                ("t_pcg", C.c_double), ("t_rr", C.c_double), ("max_resid", C.c_double),
                ("cg_apply1_launches", C.c_int64 * 2), ("cg_apply2_launches", C.c_int64 * 2),
                ("cg_apply1_ms", C.c_double * 2), ("cg_apply2_ms", C.c_double * 2)]


vp, i64, dbl, cint = C.c_void_p, C.c_int64, C.c_double, C.c_int
dptr = C.POINTER(C.c_double)
u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)

PROTOTYPES = {
    "mbl_last_error": (C.c_char_p, []),
    "mbl_version": (cint, []),
    "mbl_set_allocator": (cint, [vp, vp, vp]),
    "mbl_hamiltonian_create": (cint, [cint, dbl, dbl, dbl, dptr, vp, C.POINTER(vp)]),
    "mbl_hamiltonian_destroy": (cint, [vp]),
    "mbl_hamiltonian_dim": (cint, [vp, i64p]),
    "mbl_sector_states": (cint, [vp, u64p]),
    "mbl_rank": (cint, [vp, u64p, i64, i64p]),
    "mbl_diagonal": (cint, [vp, dbl, vp, vp, vp]),
    "mbl_apply_block": (cint, [vp, dbl, cint, vp, i64, vp, i64, cint, vp]),
    "mbl_fold_apply": (cint, [vp, dbl, cint, vp, i64, vp, i64, vp, i64, cint, vp]),
    "mbl_pcg": (cint, [vp, dbl, cint, vp, i64, vp, i64, cint, cint, vp]),
    "mbl_gram": (cint, [cint, i64, vp, i64, cint, vp, i64, cint, vp, i64, vp]),
    "mbl_block_combine": (cint, [cint, i64, vp, i64, cint, vp, i64, vp, i64, cint, vp]),
    "mbl_small_eigh": (cint, [cint, vp, i64, vp, vp, i64, vp]),
    "mbl_spectrum_bounds": (cint, [vp, dbl, dptr, dptr, vp]),
    "mbl_solve_opts_default": (cint, [C.POINTER(SolveOpts)]),
    "mbl_lobpcg_solve": (cint, [vp, dbl, cint, cint, dbl, C.POINTER(SolveOpts), dptr, vp, i64,
                                dptr, C.POINTER(SolveInfo), vp]),
}

_lib = None


def load():
    """The loaded library (ctypes.CDLL); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2012_00217_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MblError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, allow=()):
    if status != MBL_OK and status not in allow:
        raise MblError(status, load().mbl_last_error().decode(errors="replace"))
    return status
