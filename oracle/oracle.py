"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iugkp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wno-unused-function"]

FRESH, CRN = 0, 1
FACES_OFF, FACES_EVERY, FACES_FINAL = 0, 1, 2
ANALOG, EXPECTED = 0, 1
PRECOND_NONE, PRECOND_MG = 0, 1

OK = 0
W_NOT_CONVERGED = 1
E_INVALID_ARG = -1
E_FIXED_OVERFLOW = -4
E_NONFINITE = -5
E_CG_BREAKDOWN = -6
E_CG_NOT_CONVERGED = -7
E_DIVERGED = -8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", *GCC_FLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double),
                ("dy", C.c_double), ("t_ref", C.c_double), ("cv", C.c_double),
                ("vg", C.c_double), ("tau", C.c_void_p), ("wall_T", C.c_void_p),
                ("T_init", C.c_void_p), ("diff_x", C.c_void_p), ("diff_y", C.c_void_p),
                ("source", C.c_void_p), ("n_bands", C.c_int), ("band_C", C.c_void_p),
                ("band_vg", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("particles_per_iter", C.c_uint64),
                ("rng_mode", C.c_int), ("rng_epoch", C.c_uint32), ("max_iters", C.c_int),
                ("res_tol", C.c_double), ("newton", C.c_int), ("cg_tol", C.c_double),
                ("cg_max_iters", C.c_int), ("tally_faces", C.c_int), ("avg_iters", C.c_int),
                ("estimator", C.c_int), ("cg_precond", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iter", C.c_uint32), ("F", C.c_int), ("n_per_emitter", C.c_uint64),
                ("n_cells", C.c_int), ("n_bfaces", C.c_int), ("n_emitters", C.c_int),
                ("tau_min", C.c_double), ("lam_min", C.c_double), ("d0", C.c_double),
                ("res", C.c_double), ("flights", C.c_uint64), ("segments", C.c_uint64),
                ("crossings", C.c_uint64), ("tot_flights", C.c_uint64),
                ("tot_segments", C.c_uint64), ("tot_crossings", C.c_uint64),
                ("cg_iters_last", C.c_int), ("cg_iters_total", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_log.argtypes = [C.c_double]
        L.orc_log.restype = C.c_double
        L.orc_cos2pi.argtypes = [C.c_double]
        L.orc_cos2pi.restype = C.c_double
        L.orc_expm.argtypes = [C.c_double]
        L.orc_expm.restype = C.c_double
        L.orc_philox_batch.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P]
        L.orc_math_batch.argtypes = [C.c_int, P, P, P, C.c_uint64]
        L.orc_split_weight.argtypes = [C.c_int64, C.c_uint64, C.c_uint64]
        L.orc_split_weight.restype = C.c_int64
        L.orc_tree_sum.argtypes = [P, C.c_uint64]
        L.orc_tree_sum.restype = C.c_double
        L.orc_fixed_exponent.argtypes = [C.POINTER(_Problem), P]
        L.orc_fixed_exponent.restype = C.c_int
        L.orc_trace_ray.argtypes = [C.POINTER(_Problem), C.c_double, C.c_double, C.c_int,
                                    C.c_int, C.c_double, C.c_double, C.c_double, P, C.c_int,
                                    P, P]
        L.orc_trace_ray.restype = C.c_int
        L.orc_newton_operator.argtypes = [C.POINTER(_Problem), P, P, P]
        L.orc_cg.argtypes = [C.POINTER(_Problem), P, P, P, P, P, C.c_double, C.c_int, P]
        L.orc_pcg_mg.argtypes = [C.POINTER(_Problem), P, P, P, P, P, C.c_double, C.c_int, P]
        L.orc_mg_precondition.argtypes = [C.POINTER(_Problem), P, P, P, P, P]
        L.orc_mg_levels.argtypes = [C.POINTER(_Problem), P, P, C.c_int]
        L.orc_create.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(P)]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int, C.c_int]
        L.orc_solve.argtypes = [P, P, P, P]
        L.orc_get_info.argtypes = [P, C.POINTER(_Info)]
        L.orc_get_tallies.argtypes = [P, P, P, P, P, P]
        L.orc_get_E.argtypes = [P, P]
        L.orc_get_G.argtypes = [P, P]
        L.orc_get_residuals.argtypes = [P, P, C.c_int]
        L.orc_set_state.argtypes = [P, C.c_uint32, C.c_double, P, P]
        L.orc_adjoint.argtypes = [P, P, P, P, C.c_int, C.c_double, P]
        L.orc_bands_create.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(P)]
        L.orc_bands_destroy.argtypes = [P]
        L.orc_bands_step.argtypes = [P, C.c_int, C.c_int]
        L.orc_bands_solve.argtypes = [P, P, P, P]
        L.orc_bands_get_info.argtypes = [P, C.POINTER(_Info)]
        L.orc_bands_get_E.argtypes = [P, P]
        L.orc_bands_get_band.argtypes = [P, C.c_int, P, P, P, P, P, P]
        L.orc_persist_create.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(P)]
        L.orc_persist_destroy.argtypes = [P]
        L.orc_persist_step.argtypes = [P, C.c_int, C.c_int]
        L.orc_persist_solve.argtypes = [P, P, P, P]
        L.orc_persist_get_info.argtypes = [P, C.POINTER(_Info)]
        L.orc_persist_get_E.argtypes = [P, P]
        L.orc_persist_count.argtypes = [P]
        L.orc_persist_count.restype = C.c_uint64
        L.orc_persist_get_particles.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_persist_get_tallies.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_persist_get_shares.argtypes = [P, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- building blocks
def philox(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 of each row of ctr (n,4) uint32 under key (k0, k1)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.array(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    L = lib()
    for i in range(ctr.shape[0]):
        L.orc_philox4x32_10(ctr[i].ctypes.data, k.ctypes.data, out[i].ctypes.data)
    return out


def philox_batch(ctr: np.ndarray, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.ctypes.data, ctr.shape[0], int(key[0]), int(key[1]), out.ctypes.data)
    return out


def math_batch(op: int, x: np.ndarray, y: Optional[np.ndarray] = None) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_math_batch(op, x.ctypes.data, _ptr(y), out.ctypes.data, x.size)
    return out


def u53(hi: int, lo: int) -> float:
    return lib().orc_u53(hi, lo)


def log(x: float) -> float:
    return lib().orc_log(x)


def cos2pi(u: float) -> float:
    return lib().orc_cos2pi(u)


def expm(T: float) -> float:
    return lib().orc_expm(T)


def split_weight(G: int, n: int, k: int) -> int:
    return lib().orc_split_weight(G, n, k)


def tree_sum(v: np.ndarray) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_tree_sum(v.ctypes.data, v.size)


# ---------------------------------------------------------------- problem marshalling
class _Keep:
    """Holds the numpy arrays a _Problem points into."""

    def __init__(self, w, diff_x=None, diff_y=None, T_init=None):
        self.tau = np.ascontiguousarray(w.tau, dtype=np.float64)
        self.wall = np.ascontiguousarray(w.wall_T, dtype=np.float64)
        Ti = T_init if T_init is not None else w.T_init
        self.T_init = None if Ti is None else np.ascontiguousarray(Ti, dtype=np.float64)
        self.dxa = None if diff_x is None else np.ascontiguousarray(diff_x, dtype=np.float64)
        self.dya = None if diff_y is None else np.ascontiguousarray(diff_y, dtype=np.float64)
        S = getattr(w, "source", None)
        self.src = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        K = int(getattr(w, "n_bands", 1) or 1)
        self.bC = None if K < 2 else np.ascontiguousarray(w.band_C, dtype=np.float64)
        self.bv = None if K < 2 else np.ascontiguousarray(w.band_vg, dtype=np.float64)
        self.p = _Problem(w.dim, w.nx, w.ny, w.dx, w.dy, w.t_ref, w.cv, w.vg,
                          self.tau.ctypes.data, self.wall.ctypes.data, _ptr(self.T_init),
                          _ptr(self.dxa), _ptr(self.dya), _ptr(self.src), K if K > 1 else 0,
                          _ptr(self.bC), _ptr(self.bv))


def fixed_exponent(w) -> int:
    k = _Keep(w)
    return lib().orc_fixed_exponent(C.byref(k.p), None)


def trace_ray(w, x0, y0, ix, iy, sx, sy, ell, max_events=100000):
    k = _Keep(w)
    ev = np.zeros(3 * max_events, dtype=np.int32)
    kind = C.c_int(0)
    cell = C.c_int(0)
    n = lib().orc_trace_ray(C.byref(k.p), x0, y0, ix, iy, sx, sy, ell, ev.ctypes.data,
                            max_events, C.addressof(kind), C.addressof(cell))
    return ev[:3 * n].reshape(-1, 3), kind.value, cell.value


def newton_operator(w, diff_x, diff_y=None):
    k = _Keep(w, diff_x, diff_y)
    gx = np.zeros(w.ny * (w.nx + 1))
    gy = np.zeros(max(1, (w.ny + 1) * w.nx if w.dim == 2 else 1))
    dg = np.zeros(w.nx * w.ny)
    lib().orc_newton_operator(C.byref(k.p), gx.ctypes.data, gy.ctypes.data, dg.ctypes.data)
    return gx, gy, dg


def cg(w, diff_x, diff_y, b, tol=1e-10, max_iters=100000, precond=PRECOND_NONE):
    k = _Keep(w, diff_x, diff_y)
    gx, gy, dg = newton_operator(w, diff_x, diff_y)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    its = C.c_int(0)
    f = lib().orc_pcg_mg if precond == PRECOND_MG else lib().orc_cg
    rc = f(C.byref(k.p), gx.ctypes.data, gy.ctypes.data, dg.ctypes.data,
           b.ctypes.data, x.ctypes.data, tol, max_iters, C.addressof(its))
    return rc, x, its.value


def mg_precondition(w, diff_x, diff_y, b):
    """x = M b: one V-cycle of the multigrid preconditioner."""
    k = _Keep(w, diff_x, diff_y)
    gx, gy, dg = newton_operator(w, diff_x, diff_y)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    lib().orc_mg_precondition(C.byref(k.p), gx.ctypes.data, gy.ctypes.data, dg.ctypes.data,
                              b.ctypes.data, x.ctypes.data)
    return x


def mg_levels(w):
    """(nx, ny) of every level of the multigrid hierarchy."""
    k = _Keep(w, None, None)
    nx = np.zeros(64, dtype=np.int32)
    ny = np.zeros(64, dtype=np.int32)
    L = lib().orc_mg_levels(C.byref(k.p), nx.ctypes.data, ny.ctypes.data, 64)
    return list(zip(nx[:L].tolist(), ny[:L].tolist()))


# ---------------------------------------------------------------- the iteration
@dataclass
class Info:
    iter: int
    F: int
    n_per_emitter: int
    n_cells: int
    n_bfaces: int
    n_emitters: int
    tau_min: float
    lam_min: float
    d0: float
    res: float
    flights: int
    segments: int
    crossings: int
    tot_flights: int
    tot_segments: int
    tot_crossings: int
    cg_iters_last: int
    cg_iters_total: int


class OracleError(RuntimeError):
    def __init__(self, rc: int, where: str):
        super().__init__(f"oracle {where} failed with code {rc}")
        self.rc = rc


class Oracle:
    """One oracle solve: create from a Workload, step, read tallies/state, solve."""

    def __init__(self, w, *, seed=None, particles=None, rng_mode=FRESH, epoch=0,
                 max_iters=None, res_tol=None, newton=None, diff_x=None, diff_y=None,
                 cg_tol=None, cg_max_iters=200000, tally_faces=FACES_EVERY, avg_iters=0,
                 T_init=None, estimator=0, cg_precond=0):
        self.w = w
        newton = w.newton if newton is None else newton
        self._keep = _Keep(w, diff_x, diff_y, T_init)
        self.opts = _Options(w.seed if seed is None else seed,
                             w.particles_per_iter if particles is None else particles,
                             rng_mode, epoch, w.max_iters if max_iters is None else max_iters,
                             w.res_tol if res_tol is None else res_tol, int(bool(newton)),
                             w.cg_tol if cg_tol is None else cg_tol, cg_max_iters, tally_faces,
                             avg_iters, int(estimator), int(cg_precond))
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(self._keep.p), C.byref(self.opts), C.byref(h))
        if rc != OK:
            raise OracleError(rc, "create")
        self.h = h
        info = self.info()
        self.nc, self.nb, self.ne = info.n_cells, info.n_bfaces, info.n_emitters
        self.nfx = w.ny * (w.nx + 1)
        self.nfy = (w.ny + 1) * w.nx if w.dim == 2 else 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def info(self) -> Info:
        i = _Info()
        lib().orc_get_info(self.h, C.byref(i))
        return Info(*[getattr(i, f[0]) for f in _Info._fields_])

    def step(self, n=1, faces=True) -> int:
        return lib().orc_step(self.h, n, int(bool(faces)))

    def tallies(self):
        D = np.zeros(self.nc, np.int64)
        W = np.zeros(self.nc, np.int64)
        Px = np.zeros(self.nfx, np.int64)
        Py = np.zeros(max(self.nfy, 1), np.int64)
        B = np.zeros(self.nb, np.int64)
        lib().orc_get_tallies(self.h, D.ctypes.data, W.ctypes.data, Px.ctypes.data,
                              Py.ctypes.data, B.ctypes.data)
        return {"D": D, "W": W, "Phix": Px, "Phiy": Py[:self.nfy], "B": B}

    def E(self) -> np.ndarray:
        E = np.zeros(self.nc)
        lib().orc_get_E(self.h, E.ctypes.data)
        return E

    def G(self) -> np.ndarray:
        G = np.zeros(self.ne, np.int64)
        lib().orc_get_G(self.h, G.ctypes.data)
        return G

    def residuals(self, n) -> np.ndarray:
        r = np.zeros(n)
        lib().orc_get_residuals(self.h, r.ctypes.data, n)
        return r

    def set_state(self, it, d0, E, G) -> int:
        E = np.ascontiguousarray(E, dtype=np.float64)
        G = np.ascontiguousarray(G, dtype=np.int64)
        return lib().orc_set_state(self.h, it, d0, E.ctypes.data, G.ctypes.data)

    def adjoint(self, dLdT, max_iters=200, tol=1e-10):
        """Gradient of L with respect to every wall face temperature and every
        cell source, given dL/dT per cell (steady state, CRN paths)."""
        g = np.ascontiguousarray(dLdT, dtype=np.float64)
        gw = np.zeros(self.nb)
        gs = np.zeros(self.nc)
        its = C.c_int(0)
        rc = lib().orc_adjoint(self.h, g.ctypes.data, gw.ctypes.data, gs.ctypes.data,
                               int(max_iters), float(tol), C.addressof(its))
        return rc, gw, gs, its.value

    def solve(self):
        T = np.zeros(self.nc)
        qx = np.zeros(self.nfx)
        qy = np.zeros(max(self.nfy, 1))
        rc = lib().orc_solve(self.h, T.ctypes.data, qx.ctypes.data, qy.ctypes.data)
        return rc, T, qx, qy[:self.nfy]


class Bands:
    """The multi-band oracle (problem with n_bands >= 2): create, step, read."""

    def __init__(self, w, *, seed=None, particles=None, rng_mode=FRESH, epoch=0, max_iters=None,
                 res_tol=None, tally_faces=FACES_EVERY):
        self.w = w
        self._keep = _Keep(w)
        self.opts = _Options(w.seed if seed is None else seed,
                             w.particles_per_iter if particles is None else particles,
                             rng_mode, epoch, w.max_iters if max_iters is None else max_iters,
                             w.res_tol if res_tol is None else res_tol, 0, 1e-10, 1, tally_faces, 0)
        h = C.c_void_p()
        rc = lib().orc_bands_create(C.byref(self._keep.p), C.byref(self.opts), C.byref(h))
        if rc != OK:
            raise OracleError(rc, "bands_create")
        self.h = h
        self.K = int(w.n_bands)
        self.nc = w.nx * w.ny
        self.nb = w.n_bfaces
        self.ne = self.nc + self.nb
        self.nfx = w.ny * (w.nx + 1)
        self.nfy = (w.ny + 1) * w.nx if w.dim == 2 else 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_bands_destroy(h)
            self.h = None

    def info(self) -> Info:
        i = _Info()
        lib().orc_bands_get_info(self.h, C.byref(i))
        return Info(*[getattr(i, f[0]) for f in _Info._fields_])

    def step(self, n=1, faces=True) -> int:
        return lib().orc_bands_step(self.h, n, int(bool(faces)))

    def E(self) -> np.ndarray:
        E = np.zeros(self.nc)
        lib().orc_bands_get_E(self.h, E.ctypes.data)
        return E

    def band(self, k):
        D = np.zeros(self.nc, np.int64)
        W = np.zeros(self.nc, np.int64)
        Px = np.zeros(self.nfx, np.int64)
        Py = np.zeros(max(self.nfy, 1), np.int64)
        B = np.zeros(self.nb, np.int64)
        G = np.zeros(self.ne, np.int64)
        lib().orc_bands_get_band(self.h, int(k), D.ctypes.data, W.ctypes.data, Px.ctypes.data,
                                 Py.ctypes.data, B.ctypes.data, G.ctypes.data)
        return {"D": D, "W": W, "Phix": Px, "Phiy": Py[:self.nfy], "B": B, "G": G}

    def solve(self):
        T = np.zeros(self.nc)
        qx = np.zeros(self.nfx)
        qy = np.zeros(max(self.nfy, 1))
        rc = lib().orc_bands_solve(self.h, T.ctypes.data, qx.ctypes.data, qy.ctypes.data)
        return rc, T, qx, qy[:self.nfy]


class Persist:
    """The persistent-particle oracle (Sec. 3.2 steps (1)-(6) with a fixed
    population): create, step, read particles, tallies and shares."""

    def __init__(self, w, *, seed=None, particles=None, rng_mode=FRESH, epoch=0, max_iters=None,
                 res_tol=None, tally_faces=FACES_EVERY, avg_iters=0):
        self.w = w
        self._keep = _Keep(w)
        self.opts = _Options(w.seed if seed is None else seed,
                             w.particles_per_iter if particles is None else particles,
                             rng_mode, epoch, w.max_iters if max_iters is None else max_iters,
                             w.res_tol if res_tol is None else res_tol, 0, 1e-10, 1, tally_faces,
                             avg_iters)
        h = C.c_void_p()
        rc = lib().orc_persist_create(C.byref(self._keep.p), C.byref(self.opts), C.byref(h))
        if rc != OK:
            raise OracleError(rc, "persist_create")
        self.h = h
        self.nc = w.nx * w.ny
        self.nb = w.n_bfaces
        self.nfx = w.ny * (w.nx + 1)
        self.nfy = (w.ny + 1) * w.nx if w.dim == 2 else 0
        self.n = int(lib().orc_persist_count(h))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_persist_destroy(h)
            self.h = None

    def info(self) -> Info:
        i = _Info()
        lib().orc_persist_get_info(self.h, C.byref(i))
        return Info(*[getattr(i, f[0]) for f in _Info._fields_])

    def step(self, n=1, faces=True) -> int:
        return lib().orc_persist_step(self.h, n, int(bool(faces)))

    def E(self) -> np.ndarray:
        E = np.zeros(self.nc)
        lib().orc_persist_get_E(self.h, E.ctypes.data)
        return E

    def particles(self):
        n = self.n
        d = {k: np.zeros(n) for k in ("x", "y", "sx", "sy")}
        d["q"] = np.zeros(n, np.int64)
        d["kind"] = np.zeros(n, np.int32)
        d["loc"] = np.zeros(n, np.int32)
        lib().orc_persist_get_particles(self.h, *[d[k].ctypes.data for k in
                                                  ("x", "y", "sx", "sy", "q", "kind", "loc")])
        return d

    def tallies(self):
        d = {"W": np.zeros(self.nc, np.int64), "Wh": np.zeros(self.nc, np.int64),
             "Nrc": np.zeros(self.nc, np.uint32), "Phix": np.zeros(self.nfx, np.int64),
             "Phiy": np.zeros(max(self.nfy, 1), np.int64), "B": np.zeros(self.nb, np.int64),
             "Nb": np.zeros(self.nb, np.uint32)}
        lib().orc_persist_get_tallies(self.h, *[d[k].ctypes.data for k in
                                                ("W", "Wh", "Nrc", "Phix", "Phiy", "B", "Nb")])
        d["Phiy"] = d["Phiy"][:self.nfy]
        return d

    def shares(self):
        d = {"wc": np.zeros(self.nc, np.int64), "rc": np.zeros(self.nc, np.int64),
             "wb": np.zeros(self.nb, np.int64), "rb": np.zeros(self.nb, np.int64)}
        lib().orc_persist_get_shares(self.h, *[d[k].ctypes.data for k in ("wc", "rc", "wb", "rb")])
        return d

    def solve(self):
        T = np.zeros(self.nc)
        qx = np.zeros(self.nfx)
        qy = np.zeros(max(self.nfy, 1))
        rc = lib().orc_persist_solve(self.h, T.ctypes.data, qx.ctypes.data, qy.ctypes.data)
        return rc, T, qx, qy[:self.nfy]
