"""Python front end of the gfx950 IUGKP library.

torch provides device memory and the current HIP stream; every step of the
method runs in the library's kernels.  A problem is any object with the
attributes dim, nx, ny, dx, dy, t_ref, cv, vg, tau, wall_T and optionally
T_init, source and the frequency bands n_bands, band_C, band_vg (tau then
[n_bands][n_cells]) (for example a `synth.Workload`).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _dev_f64(a, device) -> Optional[torch.Tensor]:
    if a is None:
        return None
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64) if not torch.is_tensor(a) else a)
    return t.to(device=device, dtype=torch.float64).contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class _Marshal:
    """Device copies of a problem's arrays plus the Problem/Options structs."""

    def __init__(self, w, device, *, seed, particles, rng_mode, epoch, max_iters, res_tol,
                 newton, diff_x, diff_y, cg_tol, cg_max_iters, tally_faces, avg_iters,
                 block_size, march=0, cg_waves=0, scheme=0, estimator=0, own_stream=False,
                 cg_precond=0, T_init=None):
        self.tau = _dev_f64(w.tau, device)
        self.wall = _dev_f64(w.wall_T, device)
        Ti = T_init if T_init is not None else getattr(w, "T_init", None)
        self.T_init = _dev_f64(Ti, device)
        self.dx_arr = _dev_f64(diff_x, device)
        self.dy_arr = _dev_f64(diff_y, device)
        self.src = _dev_f64(getattr(w, "source", None), device)
        K = int(getattr(w, "n_bands", 1) or 1)
        self.bC = _dev_f64(getattr(w, "band_C", None), device) if K > 1 else None
        self.bv = _dev_f64(getattr(w, "band_vg", None), device) if K > 1 else None
        self.problem = L.Problem(int(w.dim), int(w.nx), int(w.ny), float(w.dx), float(w.dy),
                                 float(w.t_ref), float(w.cv), float(w.vg), _ptr(self.tau),
                                 _ptr(self.wall), _ptr(self.T_init), _ptr(self.dx_arr),
                                 _ptr(self.dy_arr), L.MEM_DEVICE, _ptr(self.src), K,
                                 _ptr(self.bC), _ptr(self.bv))
        self.options = L.Options(int(seed), int(particles), int(rng_mode), int(epoch),
                                 int(max_iters), float(res_tol), int(bool(newton)),
                                 float(cg_tol), int(cg_max_iters), int(tally_faces),
                                 int(avg_iters), int(block_size), int(march), int(cg_waves),
                                 int(scheme), int(estimator), int(bool(own_stream)),
                                 int(cg_precond))


def _defaults(w, kw):
    return dict(seed=kw.pop("seed", getattr(w, "seed", 0)),
                particles=kw.pop("particles", getattr(w, "particles_per_iter", 100_000)),
                rng_mode=kw.pop("rng_mode", L.RNG_FRESH), epoch=kw.pop("epoch", 0),
                max_iters=kw.pop("max_iters", getattr(w, "max_iters", 200)),
                res_tol=kw.pop("res_tol", getattr(w, "res_tol", 1e-6)),
                newton=kw.pop("newton", getattr(w, "newton", False)),
                diff_x=kw.pop("diff_x", None), diff_y=kw.pop("diff_y", None),
                cg_tol=kw.pop("cg_tol", getattr(w, "cg_tol", 1e-10)),
                cg_max_iters=kw.pop("cg_max_iters", 200_000),
                tally_faces=kw.pop("tally_faces", L.FACES_EVERY),
                avg_iters=kw.pop("avg_iters", 0), block_size=kw.pop("block_size", 0),
                march=kw.pop("march", 0), cg_waves=kw.pop("cg_waves", 0),
                scheme=kw.pop("scheme", 0), estimator=kw.pop("estimator", 0),
                own_stream=kw.pop("own_stream", False),
                cg_precond=kw.pop("cg_precond", L.PRECOND_NONE),
                T_init=kw.pop("T_init", None))


class Solver:
    """One problem on one GPU: create, step, read tallies/state, solve."""

    def __init__(self, w, device="cuda", **kw):
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the IUGKP library needs a ROCm GPU (torch.cuda) device")
        opts = _defaults(w, kw)
        if kw:
            raise TypeError(f"unknown options {sorted(kw)}")
        self.w = w
        # the stream the library issues on stays referenced while the solver lives
        self._stream = torch.cuda.current_stream(self.device)
        self.K = int(getattr(w, "n_bands", 1) or 1)
        self.nc = int(w.nx * w.ny)
        self.nb = 2 * int(w.ny) + (2 * int(w.nx) if w.dim == 2 else 0)
        self.ne = self.nc + self.nb
        self.nfx = int(w.ny) * (int(w.nx) + 1)
        self.nfy = (int(w.ny) + 1) * int(w.nx) if w.dim == 2 else 0
        with torch.cuda.device(self.device):
            self._m = _Marshal(w, self.device, **opts)
            h = C.c_void_p()
            L.check(L.lib().iugkp_create(C.byref(self._m.problem), C.byref(self._m.options),
                                         C.c_void_p(_stream_handle(self.device)), C.byref(h)),
                    "iugkp_create")
        self.h = h
        L.register(self)

    def close(self):
        if getattr(self, "h", None):
            L.lib().iugkp_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=L.finalizing):
        # (module globals may already be gone when the collector runs at shutdown)
        try:
            if _finalizing():
                return
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ stepping
    def step(self, n: int = 1, faces: Optional[bool] = None) -> int:
        with torch.cuda.device(self.device):
            if faces is None:
                rc = L.lib().iugkp_step(self.h, int(n))
            else:
                rc = L.lib().iugkp_step_faces(self.h, int(n), int(bool(faces)))
        return rc

    def solve(self):
        T = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        qx = torch.empty(self.nfx, dtype=torch.float64, device=self.device)
        qy = torch.empty(max(self.nfy, 1), dtype=torch.float64, device=self.device)
        st = L.Stats()
        with torch.cuda.device(self.device):
            rc = L.lib().iugkp_solve(self.h, T.data_ptr(), qx.data_ptr(), qy.data_ptr(),
                                     C.byref(st))
        L.check(rc, "iugkp_solve", allow_warning=True)
        return rc, T, qx, qy[:self.nfy], st.as_dict()

    # ------------------------------------------------------------------ readers
    def tallies(self):
        """Tallies of the last iteration; (K, n) per-band blocks for K frequency bands."""
        K = self.K
        z = lambda n: torch.empty(max(K * n, 1), dtype=torch.int64, device=self.device)
        D, W, Px, Py, B = z(self.nc), z(self.nc), z(self.nfx), z(self.nfy), z(self.nb)
        with torch.cuda.device(self.device):
            L.check(L.lib().iugkp_get_tallies(self.h, D.data_ptr(), W.data_ptr(), Px.data_ptr(),
                                              Py.data_ptr(), B.data_ptr()), "iugkp_get_tallies")
        out = {"D": D, "W": W, "Phix": Px, "Phiy": Py[:K * self.nfy], "B": B}
        if K > 1:
            out = {k: v.view(K, -1) for k, v in out.items()}
        return out

    def state(self):
        it = C.c_uint32(0)
        d0 = C.c_double(0.0)
        E = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        G = torch.empty(self.K * self.ne, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.lib().iugkp_get_state(self.h, C.addressof(it), C.addressof(d0),
                                            E.data_ptr(), G.data_ptr()), "iugkp_get_state")
        return it.value, d0.value, E, G

    def set_state(self, it: int, d0: float, E, G) -> int:
        E = _dev_f64(E, self.device)
        G = torch.as_tensor(G).to(device=self.device, dtype=torch.int64).contiguous()
        with torch.cuda.device(self.device):
            return L.lib().iugkp_set_state(self.h, int(it), float(d0), E.data_ptr(), G.data_ptr())

    def particles(self):
        """Persistent population (scheme 1): x, y, sx, sy, q, kind, loc."""
        st = self.stats()
        n = int(st["n_per_emitter"]) * self.ne
        f = lambda: torch.empty(n, dtype=torch.float64, device=self.device)
        x, y, sx, sy = f(), f(), f(), f()
        q = torch.empty(n, dtype=torch.int64, device=self.device)
        kind = torch.empty(n, dtype=torch.int32, device=self.device)
        loc = torch.empty(n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.lib().iugkp_get_particles(self.h, x.data_ptr(), y.data_ptr(), sx.data_ptr(),
                                                sy.data_ptr(), q.data_ptr(), kind.data_ptr(),
                                                loc.data_ptr()), "iugkp_get_particles")
        return {"x": x, "y": y, "sx": sx, "sy": sy, "q": q, "kind": kind, "loc": loc}

    def shares(self):
        """Persistent population: N_rc, N_b of the last iteration, next shares and
        carried remainders (w_c, r_c per cell, w_b, r_b per wall face)."""
        u = lambda n: torch.empty(n, dtype=torch.int32, device=self.device)
        i = lambda n: torch.empty(n, dtype=torch.int64, device=self.device)
        d = {"Nrc": u(self.nc), "Nb": u(self.nb), "wc": i(self.nc), "rc": i(self.nc),
             "wb": i(self.nb), "rb": i(self.nb)}
        with torch.cuda.device(self.device):
            L.check(L.lib().iugkp_get_shares(self.h, *[d[k].data_ptr() for k in
                                                       ("Nrc", "Nb", "wc", "rc", "wb", "rb")]),
                    "iugkp_get_shares")
        return d

    def adjoint(self, dLdT, max_iters: int = 200, tol: float = 1e-10):
        """Gradients of a loss L(T) of the steady state reached by this solver
        (CRN, uniform tau) with respect to every wall face temperature and every
        cell source, given dL/dT per cell.  Returns (rc, grad_wall, grad_source,
        passes); rc is 0 or the not-converged warning."""
        g = _dev_f64(dLdT, self.device)
        gw = torch.empty(self.nb, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        its = C.c_int(0)
        with torch.cuda.device(self.device):
            rc = L.lib().iugkp_adjoint(self.h, g.data_ptr(), gw.data_ptr(), gs.data_ptr(),
                                       int(max_iters), float(tol), C.addressof(its))
        L.check(rc, "iugkp_adjoint", allow_warning=True)
        return rc, gw, gs, its.value

    def stats(self) -> dict:
        st = L.Stats()
        L.check(L.lib().iugkp_get_stats(self.h, C.byref(st)), "iugkp_get_stats")
        return st.as_dict()

    def march_tuning(self):
        """(form, ms): the particle step's form for face-tallied iterations
        ("tiles256", "tiles512", "stripes", "stripes_pieces", or None while the
        handle still measures them) and the measured milliseconds per form
        (None where not measured)."""
        form = C.c_int(0)
        ms = (C.c_float * 4)()
        L.check(L.lib().iugkp_march_tuning(self.h, C.byref(form), ms), "iugkp_march_tuning")
        names = ("tiles256", "tiles512", "stripes", "stripes_pieces")
        return (names[form.value] if form.value >= 0 else None,
                {n: (float(v) if v >= 0 else None) for n, v in zip(names, ms)})

    def residuals(self) -> np.ndarray:
        n = self.stats()["iters"]
        r = np.zeros(max(n, 1))
        k = L.lib().iugkp_get_residuals(self.h, r.ctypes.data, n)
        return r[:max(k, 0)]


def diffusion_solve(problem, D_x, D_y, b, tol: float = 1e-10, max_iters: int = 200_000,
                    device="cuda", no_alloc: bool = False):
    """x with A x = b for the Newton operator of `problem` (its mesh, tau and
    vg) with the diffusion coefficients D_x, D_y per cell (D_y unused in 1D):
    (rc, x, cg_iterations); rc is 0, or the library's error code when the CG
    broke down or did not converge (x then holds the last iterate).  With
    no_alloc the library's no-allocation entry point runs the solve (this
    wrapper still allocates x with torch)."""
    dev = torch.device(device)
    tau = _dev_f64(problem.tau, dev)
    dx_ = _dev_f64(D_x, dev)
    dy_ = _dev_f64(D_y, dev) if int(problem.dim) == 2 else None
    bb = _dev_f64(b, dev)
    x = torch.empty_like(bb)
    its = C.c_int(0)
    with torch.cuda.device(dev):
        fn = L.lib().iugkp_diffusion_solve_noalloc if no_alloc else L.lib().iugkp_diffusion_solve
        rc = fn(int(problem.dim), int(problem.nx), int(problem.ny),
                float(problem.dx), float(problem.dy), float(problem.vg), tau.data_ptr(),
                dx_.data_ptr(), _ptr(dy_), bb.data_ptr(), x.data_ptr(), float(tol),
                int(max_iters), C.addressof(its), C.c_void_p(_stream_handle(dev)))
    if rc not in (L.OK, L.E_CG_NOT_CONVERGED, L.E_CG_BREAKDOWN):
        L.check(rc, "iugkp_diffusion_solve")
    return rc, x, its.value


def solve(problem, device="cuda", **opts):
    """Steady state of one problem: (T, (q_x, q_y), stats, status) with T per
    cell and the heat flux on the x and y faces (device tensors); status is 0
    or the not-converged warning.  Options as Solver."""
    s = Solver(problem, device=device, **opts)
    try:
        rc, T, qx, qy, st = s.solve()
    finally:
        s.close()
    return T, (qx, qy), st, rc


def step_group(solvers: Sequence["Solver"], n: int = 1) -> int:
    """n iterations of several independent solvers, each iteration enqueued on
    all of them before any is waited for; with own_stream=True solvers their
    kernels overlap on the GPU.  Results equal per-solver step()."""
    hs = (C.c_void_p * len(solvers))(*[s.h for s in solvers])
    return L.lib().iugkp_step_group(C.cast(hs, C.c_void_p), len(solvers), int(n))


def d_eff(lam: float, delta: float) -> float:
    return L.lib().iugkp_d_eff(float(lam), float(delta))


def dev_philox(ctr: torch.Tensor, key0: int, key1: int) -> torch.Tensor:
    """Philox4x32-10 blocks for an (n, 4) int32-bit-pattern counter tensor on the GPU."""
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    L.check(L.lib().iugkp_dev_philox(ctr.data_ptr(), int(key0) & 0xFFFFFFFF,
                                     int(key1) & 0xFFFFFFFF, out.data_ptr(), ctr.shape[0],
                                     C.c_void_p(_stream_handle(ctr.device))), "iugkp_dev_philox")
    return out


def dev_atomics(lds: bool, n_words: int = 262144, per_thread: int = 64,
                n_threads: int = 256 * 8192, device="cuda") -> float:
    """Tally-throughput ceiling: int64 atomic adds per second to random words
    of a global array of n_words, or of a workgroup's LDS array."""
    ms = C.c_double(0.0)
    dev = torch.device(device)
    with torch.cuda.device(dev):
        L.check(L.lib().iugkp_dev_atomics(int(bool(lds)), int(n_words), int(per_thread),
                                          int(n_threads), C.addressof(ms),
                                          C.c_void_p(_stream_handle(dev))), "iugkp_dev_atomics")
    return n_threads * per_thread / (ms.value / 1e3)


def dev_segments(dim: int, nx: int, ny: int, dx: float, dy: float,
                 rays: torch.Tensor) -> torch.Tensor:
    """Closed-form segment walks on the device: rays (n, 7) float64 rows
    (x0, y0, ix, iy, sx, sy, ell) -> (n, 3) int64 (absorbed, cell or face, crossings)."""
    rays = rays.to(torch.float64).contiguous()
    out = torch.empty((rays.shape[0], 3), dtype=torch.int64, device=rays.device)
    L.check(L.lib().iugkp_dev_segments(int(dim), int(nx), int(ny), float(dx), float(dy),
                                       rays.data_ptr(), rays.shape[0], out.data_ptr(),
                                       C.c_void_p(_stream_handle(rays.device))),
            "iugkp_dev_segments")
    return out


def dev_math(op: int, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
    x = x.contiguous()
    out = torch.empty_like(x)
    L.check(L.lib().iugkp_dev_math(int(op), x.data_ptr(), None if y is None else y.contiguous().data_ptr(),
                                   out.data_ptr(), x.numel(),
                                   C.c_void_p(_stream_handle(x.device))), "iugkp_dev_math")
    return out
