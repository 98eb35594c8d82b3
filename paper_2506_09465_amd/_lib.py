"""ctypes declarations of the C ABI in include/iugkp.h (argument marshalling only)."""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiugkp.so")

OK = 0
W_NOT_CONVERGED = 1
E_INVALID_ARG = -1
E_NOMEM = -2
E_DEVICE = -3
E_FIXED_OVERFLOW = -4
E_NONFINITE = -5
E_CG_BREAKDOWN = -6
E_CG_NOT_CONVERGED = -7
E_DIVERGED = -8

MEM_HOST, MEM_DEVICE = 0, 1
RNG_FRESH, RNG_CRN = 0, 1
FACES_OFF, FACES_EVERY, FACES_FINAL = 0, 1, 2
SCHEME_EMITTERS, SCHEME_PERSISTENT = 0, 1
EST_ANALOG, EST_EXPECTED = 0, 1
PRECOND_NONE, PRECOND_MG = 0, 1


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double),
                ("dy", C.c_double), ("t_ref", C.c_double), ("cv", C.c_double),
                ("vg", C.c_double), ("tau", C.c_void_p), ("wall_T", C.c_void_p),
                ("T_init", C.c_void_p), ("diff_x", C.c_void_p), ("diff_y", C.c_void_p),
                ("mem_kind", C.c_int), ("source", C.c_void_p), ("n_bands", C.c_int),
                ("band_C", C.c_void_p), ("band_vg", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("particles_per_iter", C.c_uint64),
                ("rng_mode", C.c_int), ("rng_epoch", C.c_uint32), ("max_iters", C.c_int),
                ("res_tol", C.c_double), ("newton", C.c_int), ("cg_tol", C.c_double),
                ("cg_max_iters", C.c_int), ("tally_faces", C.c_int), ("avg_iters", C.c_int),
                ("block_size", C.c_int), ("march", C.c_int), ("cg_waves", C.c_int),
                ("scheme", C.c_int), ("estimator", C.c_int), ("own_stream", C.c_int),
                ("cg_precond", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("res", C.c_double), ("flights", C.c_uint64),
                ("segments", C.c_uint64), ("crossings", C.c_uint64),
                ("tot_flights", C.c_uint64), ("tot_segments", C.c_uint64),
                ("tot_crossings", C.c_uint64), ("ms_march", C.c_double),
                ("ms_update", C.c_double), ("ms_cg", C.c_double), ("cg_iters_last", C.c_int),
                ("cg_iters_total", C.c_int), ("fixed_point_F", C.c_int),
                ("n_per_emitter", C.c_uint64), ("n_emitters", C.c_int), ("status", C.c_int)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


# (name, restype, argtypes) of every exported entry point
P = C.c_void_p
SIGNATURES = [
    ("iugkp_create", C.c_int, [C.POINTER(Problem), C.POINTER(Options), P, C.POINTER(P)]),
    ("iugkp_destroy", None, [P]),
    ("iugkp_step", C.c_int, [P, C.c_int]),
    ("iugkp_step_group", C.c_int, [P, C.c_int, C.c_int]),
    ("iugkp_step_faces", C.c_int, [P, C.c_int, C.c_int]),
    ("iugkp_solve", C.c_int, [P, P, P, P, C.POINTER(Stats)]),
    ("iugkp_get_tallies", C.c_int, [P, P, P, P, P, P]),
    ("iugkp_get_state", C.c_int, [P, P, P, P, P]),
    ("iugkp_set_state", C.c_int, [P, C.c_uint32, C.c_double, P, P]),
    ("iugkp_get_residuals", C.c_int, [P, P, C.c_int]),
    ("iugkp_get_stats", C.c_int, [P, C.POINTER(Stats)]),
    ("iugkp_march_tuning", C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_float)]),
    ("iugkp_get_particles", C.c_int, [P, P, P, P, P, P, P, P]),
    ("iugkp_get_shares", C.c_int, [P, P, P, P, P, P, P]),
    ("iugkp_d_eff", C.c_double, [C.c_double, C.c_double]),
    ("iugkp_adjoint", C.c_int, [P, P, P, P, C.c_int, C.c_double, P]),
    ("iugkp_batch_create", C.c_int, [P, P, C.c_int, P, C.POINTER(P)]),
    ("iugkp_batch_solve", C.c_int, [P, P, P, P, P]),
    ("iugkp_batch_destroy", None, [P]),
    ("iugkp_strerror", C.c_char_p, [C.c_int]),
    ("iugkp_last_error", C.c_char_p, []),
    ("iugkp_dev_philox", C.c_int, [P, C.c_uint32, C.c_uint32, P, C.c_int64, P]),
    ("iugkp_dev_math", C.c_int, [C.c_int, P, P, P, C.c_int64, P]),
    ("iugkp_batch_tuning", C.c_int, [P, P, P, P]),
    ("iugkp_batch_tiles", C.c_int, [P, P]),
    ("iugkp_diffusion_solve", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_double, P, P, P, P, P, C.c_double, C.c_int, P, P]),
    ("iugkp_diffusion_solve_noalloc", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double,
                                                C.c_double, C.c_double, P, P, P, P, P,
                                                C.c_double, C.c_int, P, P]),
    ("iugkp_dev_atomics", C.c_int, [C.c_int, C.c_int64, C.c_int64, C.c_int64, P, P]),
    ("iugkp_dev_segments", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, P,
                                     C.c_int64, P, P]),
]

_lib = None


def lib():
    """Load libiugkp.so (built in-tree); fails loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2506_09465_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# Live solver and batch objects.  They are closed by an exit hook that runs at
# the start of interpreter shutdown, while torch and the HIP runtime are still
# up; a handle reached only by the garbage collector later in the shutdown is
# left to the process exit instead of being destroyed then (its streams,
# events and device memory would be released after the runtime, or a
# profiler attached to it, may already have shut down).
_live = weakref.WeakSet()


def register(obj) -> None:
    """Track an object with a close() method until it is closed or collected."""
    _live.add(obj)


def _close_all() -> None:
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


atexit.register(_close_all)


def finalizing(_is_finalizing=sys.is_finalizing) -> bool:
    return _is_finalizing()


class IugkpError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().iugkp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().iugkp_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code: int, where: str, allow_warning: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_warning):
        raise IugkpError(code, where)
    return code
