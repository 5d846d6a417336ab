"""ctypes loader and prototypes for libmbl.so (declared in include/mbl.h).

The library is loaded from this package directory only.  There is no
fallback: if it is missing, importing the solver API raises.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MBL_LIBRARY") or os.path.join(HERE, "libmbl.so")

MBL_OK, MBL_EINVAL, MBL_ENOMEM, MBL_EDEVICE, MBL_ENOCONV, MBL_EBREAKDOWN, MBL_ETIMEOUT = (
    0, -1, -2, -3, -4, -5, -6)
MBL_ECANCELLED, MBL_EINTERNAL = -7, -8
MBL_F64, MBL_F32, MBL_MIXED, MBL_PCG32 = 0, 1, 2, 3

STATUS_NAMES = {0: "MBL_OK", -1: "MBL_EINVAL", -2: "MBL_ENOMEM", -3: "MBL_EDEVICE",
                -4: "MBL_ENOCONV", -5: "MBL_EBREAKDOWN", -6: "MBL_ETIMEOUT", -7: "MBL_ECANCELLED",
                -8: "MBL_EINTERNAL"}


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("pcg_iters", C.c_int), ("precision", C.c_int),
                ("verbose", C.c_int), ("timing", C.c_int), ("seed", C.c_uint64),
                ("lock", C.c_int), ("max_seconds", C.c_double), ("cancel", C.POINTER(C.c_int)),
                ("guard_cg", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("iters_fp64", C.c_int), ("nconv", C.c_int),
                ("applies", C.c_int64), ("pcg_steps", C.c_int64), ("seconds", C.c_double),
                ("t_pcg", C.c_double), ("t_rr", C.c_double), ("max_resid", C.c_double),
                ("cg_apply1_launches", C.c_int64 * 2), ("cg_apply2_launches", C.c_int64 * 2),
                ("cg_apply1_ms", C.c_double * 2), ("cg_apply2_ms", C.c_double * 2),
                ("cg_apply1_bytes", C.c_double * 2), ("cg_apply2_bytes", C.c_double * 2),
                ("pcg_columns", C.c_int64), ("t_apply", C.c_double), ("t_gram", C.c_double),
                ("t_small", C.c_double), ("cg_split", C.c_int),
                ("cg_launches_all", C.c_int64 * 2),
                ("cg_apply1_ms_all", C.c_double * 2), ("cg_apply2_ms_all", C.c_double * 2),
                ("cg_apply1_bytes_all", C.c_double * 2), ("cg_apply2_bytes_all", C.c_double * 2)]


class Problem(C.Structure):
    _fields_ = [("L", C.c_int), ("Sz", C.c_double), ("J", C.c_double), ("Delta", C.c_double),
                ("h_host", C.POINTER(C.c_double)), ("sigma", C.c_double), ("eps", C.c_double),
                ("nev", C.c_int), ("block", C.c_int), ("tol", C.c_double),
                ("precision", C.c_int), ("max_iter", C.c_int), ("pcg_iters", C.c_int),
                ("seed", C.c_uint64), ("want_vectors", C.c_int)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("sigma", C.c_double), ("nconv", C.c_int),
                ("iters", C.c_int), ("applies", C.c_int64), ("max_resid", C.c_double),
                ("seconds", C.c_double), ("latency", C.c_double),
                ("evals_host", C.POINTER(C.c_double)), ("resid_host", C.POINTER(C.c_double)),
                ("evecs_dev", C.c_void_p), ("ldv", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("in_flight", C.c_int64), ("p50_latency", C.c_double),
                ("p99_latency", C.c_double), ("throughput_pairs", C.c_double),
                ("budget_bytes", C.c_size_t), ("peak_bytes", C.c_size_t)]


vp, i64, dbl, cint = C.c_void_p, C.c_int64, C.c_double, C.c_int

# mbl_alloc_fn / mbl_free_fn
AllocFn = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FreeFn = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
dptr = C.POINTER(C.c_double)
u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)

PROTOTYPES = {
    "mbl_last_error": (C.c_char_p, []),
    "mbl_version": (cint, []),
    "mbl_set_allocator": (cint, [AllocFn, FreeFn, vp]),
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
    "mbl_gram_noalloc": (cint, [cint, i64, vp, i64, cint, vp, i64, cint, vp, i64, vp]),
    "mbl_block_combine": (cint, [cint, i64, vp, i64, cint, vp, i64, vp, i64, cint, vp]),
    "mbl_small_eigh": (cint, [cint, vp, i64, vp, vp, i64, vp]),
    "mbl_spectrum_bounds": (cint, [vp, dbl, dptr, dptr, vp]),
    "mbl_solve_opts_default": (cint, [C.POINTER(SolveOpts)]),
    "mbl_lobpcg_solve": (cint, [vp, dbl, cint, cint, dbl, C.POINTER(SolveOpts), dptr, vp, i64,
                                dptr, C.POINTER(SolveInfo), vp]),
    "mbl_footprint_bytes": (cint, [cint, dbl, cint, cint, C.POINTER(C.c_size_t)]),
    "mbl_entanglement_entropy": (cint, [vp, vp, i64, cint, cint, dptr, vp]),
    "mbl_gap_ratio": (cint, [dptr, cint, dptr]),
    "mbl_slices_solve": (cint, [vp, cint, dptr, cint, cint, dbl, C.POINTER(SolveOpts), dptr, dptr,
                                cint]),
    "mbl_batch_solve": (cint, [cint, C.POINTER(Problem), C.POINTER(Result), cint]),
    "mbl_server_create": (cint, [cint, C.c_size_t, cint, C.POINTER(vp)]),
    "mbl_server_cancel": (cint, [vp, C.c_uint64]),
    "mbl_server_submit": (cint, [vp, C.POINTER(Problem), C.POINTER(C.c_uint64)]),
    "mbl_server_wait": (cint, [vp, C.c_uint64, dbl, C.POINTER(Result)]),
    "mbl_server_stats_get": (cint, [vp, C.POINTER(ServerStats)]),
    "mbl_server_destroy": (cint, [vp]),
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
