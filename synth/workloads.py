"""Seeded synthetic problem definitions for the steady gray phonon BTE solver.

This module only *describes* problems: mesh sizes, relaxation-time fields,
wall temperatures, particle budgets and seeds.  It holds none of the solver's
arithmetic, so that both the CPU oracle and the HIP library can be driven
from the same inputs without sharing any computation.

Geometries follow the paper's numerical tests (Section 4):
  * 1D film of thickness L between isothermal walls T_H / T_L (Sec. 4.1),
    100 uniform cells, |V_g| = C = 1;
  * 1D film with piecewise-constant relaxation time split at L/2 (Sec. 4.2);
  * 1D film with tau(x) = 10^(|A1 sin(2 pi x / L)| - A2) (Sec. 4.3);
  * 2D square cavity, hot top wall, other walls cold (Sec. 4.4);
  * uniform-field consistency example with two Kn regions (Sec. 3.2).
The larger sizes (256^2 cavity, 512^2 two-material domain, a batch of 256
uneven cavities) are the benchmark workloads of this project; they keep the
paper's structure and scale it up.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    """A problem instance plus the run options that go with it."""

    name: str
    dim: int
    nx: int
    ny: int
    dx: float
    dy: float
    t_ref: float
    cv: float
    vg: float
    tau: np.ndarray            # (ny*nx,) float64, cell c = ix + nx*iy
    wall_T: np.ndarray         # (n_bfaces,) float64: left rows, right rows, bottom cols, top cols
    T_init: Optional[np.ndarray] = None   # (ny*nx,) or None -> t_ref everywhere
    source: Optional[np.ndarray] = None   # (ny*nx,) volumetric heat source or None
    # frequency bands (n_bands >= 2): tau is then (n_bands*ny*nx,) band-major, and
    # band_C / band_vg replace cv / vg
    n_bands: int = 1
    band_C: Optional[np.ndarray] = None
    band_vg: Optional[np.ndarray] = None
    # run options
    seed: int = 0
    particles_per_iter: int = 100_000
    newton: bool = False
    cg_tol: float = 1e-10
    res_tol: float = 1e-6
    max_iters: int = 200

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny

    @property
    def n_bfaces(self) -> int:
        return 2 * self.ny + (2 * self.nx if self.dim == 2 else 0)

    @property
    def n_emitters(self) -> int:
        return self.n_cells + self.n_bfaces

    def n_per_emitter(self) -> int:
        """Particles per emitter: an equal share of the budget, at least one."""
        return max(1, self.particles_per_iter // self.n_emitters)


def _walls_1d(t_left: float, t_right: float) -> np.ndarray:
    return np.array([t_left, t_right], dtype=np.float64)


def _walls_2d(nx: int, ny: int, left: float, right: float, bottom: float, top: float) -> np.ndarray:
    return np.concatenate([
        np.full(ny, left), np.full(ny, right), np.full(nx, bottom), np.full(nx, top)
    ]).astype(np.float64)


def slab_1d(n: int = 100, kn: float = 1.0, length: float = 1.0, t_hot: float = 1.01,
            t_cold: float = 0.99, t_ref: float = 1.0, particles: int = 100_000,
            seed: int = 0, newton: bool = False, name: str = "slab1d") -> Workload:
    """1D film between a hot left wall and a cold right wall (Sec. 4.1).

    Constant relaxation time with Kn = |V_g| tau / L; C = |V_g| = 1.
    """
    vg = 1.0
    tau = np.full(n, kn * length / vg, dtype=np.float64)
    return Workload(name=name, dim=1, nx=n, ny=1, dx=length / n, dy=1.0, t_ref=t_ref,
                    cv=1.0, vg=vg, tau=tau, wall_T=_walls_1d(t_hot, t_cold), seed=seed,
                    particles_per_iter=particles, newton=newton)


def slab_1d_two_tau(n: int = 100, tau_left: float = 10.0, tau_right: float = 0.1,
                    particles: int = 100_000, seed: int = 0,
                    name: str = "slab1d_discontinuous") -> Workload:
    """1D film with tau = tau_left for x < L/2 and tau_right for x > L/2 (Sec. 4.2)."""
    w = slab_1d(n=n, kn=1.0, particles=particles, seed=seed, name=name)
    xc = (np.arange(n) + 0.5) / n
    w.tau = np.where(xc < 0.5, tau_left, tau_right).astype(np.float64)
    return w


def slab_1d_multiscale(n: int = 100, a1: float = 2.0, a2: float = 1.0,
                       particles: int = 100_000, seed: int = 0) -> Workload:
    """1D film with tau(x) = 10^(|a1 sin(2 pi x/L)| - a2) at cell centres (Sec. 4.3).

    a2 = +1 is the sign for which tau spans [1e-1, 1e1] as the paper states.
    """
    w = slab_1d(n=n, kn=1.0, particles=particles, seed=seed, name="slab1d_multiscale")
    xc = (np.arange(n) + 0.5) / n
    w.tau = np.power(10.0, np.abs(a1 * np.sin(2.0 * math.pi * xc)) - a2).astype(np.float64)
    return w


def uniform_field_1d(n: int = 20, dx: float = 0.1, tau_left: float = 0.1,
                     tau_right: float = 1e-4, particles: int = 20_000, seed: int = 0) -> Workload:
    """Uniform-field consistency example (Sec. 3.2): T = 1 everywhere, walls at 1,
    two regions of very different Kn.  Temperatures are measured from t_ref = 0.5
    so that the equilibrium energy is non-zero."""
    vg = 1.0
    xc = (np.arange(n) + 0.5)
    tau = np.where(xc < n / 2, tau_left, tau_right).astype(np.float64)
    w = Workload(name="uniform1d", dim=1, nx=n, ny=1, dx=dx, dy=1.0, t_ref=0.5, cv=1.0,
                 vg=vg, tau=tau, wall_T=_walls_1d(1.0, 1.0), seed=seed,
                 particles_per_iter=particles)
    w.T_init = np.ones(n, dtype=np.float64)
    return w


def cavity_2d(n: int = 256, kn: float = 1.0, ny: Optional[int] = None, t_hot: float = 1.01,
              t_cold: float = 0.99, t_ref: float = 1.0, particles: int = 10_000_000,
              seed: int = 0, newton: bool = True, name: str = "cavity2d") -> Workload:
    """2D square cavity, top wall hot, the other three cold (Sec. 4.4).

    Side length L = 1 along x; the y extent is ny*dy with dy = dx (ny defaults to n).
    """
    ny = n if ny is None else ny
    vg = 1.0
    d = 1.0 / n
    tau = np.full(n * ny, kn / vg, dtype=np.float64)
    return Workload(name=name, dim=2, nx=n, ny=ny, dx=d, dy=d, t_ref=t_ref, cv=1.0, vg=vg,
                    tau=tau, wall_T=_walls_2d(n, ny, t_cold, t_cold, t_cold, t_hot),
                    seed=seed, particles_per_iter=particles, newton=newton)


def two_material_2d(n: int = 512, kn_right: float = 0.01, ratio: float = 100.0,
                    particles: int = 50_000_000, seed: int = 0, newton: bool = False,
                    name: str = "two_material2d") -> Workload:
    """Gray 2D square whose left half has a relaxation time `ratio` times the right
    half's (null-collision stress case); hot top wall, cold others."""
    w = cavity_2d(n=n, kn=kn_right, particles=particles, seed=seed, newton=newton, name=name)
    ix = np.tile(np.arange(n), n)
    w.tau = np.where(ix < n // 2, kn_right * ratio, kn_right).astype(np.float64)
    return w


@dataclasses.dataclass
class BatchInstance:
    n: int
    kn: float
    walls: tuple          # (left, right, bottom, top) temperatures
    particles: int
    seed: int


def batch_instances(count: int = 256, seed: int = 2506) -> List[BatchInstance]:
    """Uneven batch of independent 2D gray cavities.

    Side n ~ U{32..256}, Kn ~ log-uniform[1e-3, 10], four wall temperatures
    ~ U[0.98, 1.02], particle budget growing linearly with cell count from 1e4
    (32^2) to 1e6 (256^2); instance b uses Philox seed b.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(32, 257))
        kn = float(10.0 ** rng.uniform(-3.0, 1.0))
        walls = tuple(float(x) for x in rng.uniform(0.98, 1.02, size=4))
        particles = int(round(1e4 + (1e6 - 1e4) * (n * n - 1024) / (65536 - 1024)))
        out.append(BatchInstance(n=n, kn=kn, walls=walls, particles=particles, seed=b))
    return out


def batch_workloads(count: int = 256, seed: int = 2506, newton: bool = True) -> List[Workload]:
    ws = []
    for b, inst in enumerate(batch_instances(count, seed)):
        w = cavity_2d(n=inst.n, kn=inst.kn, particles=inst.particles, seed=inst.seed,
                      newton=newton, name=f"batch{b}")
        w.wall_T = _walls_2d(inst.n, inst.n, *inst.walls)
        ws.append(w)
    return ws


def gaussian_source(nx: int, ny: int, dx: float, dy: float, amp: float,
                    width: float) -> np.ndarray:
    """amp * exp(-r^2 / (2 width^2)) at the cell centres, r from the domain centre."""
    x = (np.arange(nx) + 0.5) * dx - 0.5 * nx * dx
    y = (np.arange(ny) + 0.5) * dy - 0.5 * ny * dy
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    return (amp * np.exp(-r2 / (2.0 * width * width))).reshape(-1).astype(np.float64)


@dataclasses.dataclass
class AdjointCase:
    """Probe-misfit problem: a cavity with a Gaussian source, probe cells and
    the target temperatures there; loss = sum over probes (T_p - target_p)^2."""

    workload: Workload
    probes: np.ndarray          # (n_probes,) int64 cell indices, distinct
    target: np.ndarray          # (n_probes,) float64
    walls4: np.ndarray          # (4,) left, right, bottom, top wall temperatures


def adjoint_case(n: int = 256, kn: float = 0.1, n_probes: int = 64, particles: int = 10_000_000,
                 amp: float = 0.01, width: float = 0.05, seed: int = 0) -> AdjointCase:
    """The 2D cavity (top 1.01, others 0.99) with a Gaussian source of width
    0.05 L at the centre, n_probes distinct random probe cells and target
    temperatures drawn uniformly in [0.99, 1.01] (numpy default_rng(seed))."""
    w = cavity_2d(n=n, kn=kn, particles=particles, seed=seed, newton=True,
                  name=f"adjoint{n}_kn{kn}")
    w.source = gaussian_source(n, n, w.dx, w.dy, amp, width * n * w.dx)
    rng = np.random.default_rng(seed)
    probes = np.sort(rng.choice(n * n, size=n_probes, replace=False)).astype(np.int64)
    target = rng.uniform(0.99, 1.01, size=n_probes)
    return AdjointCase(w, probes, target, np.array([0.99, 0.99, 0.99, 1.01]))


def slab_1d_bands(n: int = 20, C=(0.5, 0.3, 0.2), vg=(1.0, 0.7, 0.4), kn=(2.0, 0.3, 0.05),
                  kn_left_factor: float = 1.0, t_hot: float = 1.01, t_cold: float = 0.99,
                  particles: int = 200_000, seed: int = 0, name: str = "slab1d_bands") -> Workload:
    """1D film with a few frequency bands: band k has heat capacity C[k], group
    speed vg[k] and Kn[k] = vg tau / L; the left half's tau is kn_left_factor
    times the right half's (null collisions when != 1)."""
    K = len(C)
    L, d = 1.0, 1.0 / n
    x = (np.arange(n) + 0.5) * d
    tau = np.zeros(K * n)
    for k in range(K):
        t = kn[k] * L / vg[k]
        tau[k * n:(k + 1) * n] = np.where(x < 0.5, t * kn_left_factor, t)
    return Workload(name=name, dim=1, nx=n, ny=1, dx=d, dy=1.0, t_ref=1.0,
                    cv=float(sum(C)), vg=float(vg[0]), tau=tau,
                    wall_T=_walls_1d(t_hot, t_cold), seed=seed, particles_per_iter=particles,
                    n_bands=K, band_C=np.array(C, dtype=np.float64),
                    band_vg=np.array(vg, dtype=np.float64))


def sine_dispersion_bands(K: int = 40, omega_cut: float = 0.57819, kn_max: float = 10.0,
                          length: float = 1.0, v0: float = 1.0):
    """K midpoint bands over (0, omega_cut omega_max] of the dispersion with group
    speed v(w) = v0 cos(pi w / 2 w_max): C_k proportional to k(w)^2 / v(w) with
    k(w) the wavenumber (the integral of dw / v), normalised to sum 1;
    tau_k proportional to w^-2, scaled so the lowest band has Kn = kn_max
    (the cut makes the Kn span 1e4).  Returns (C, vg, tau_right)."""
    w = (np.arange(K) + 0.5) / K * omega_cut          # in units of w_max
    v = v0 * np.cos(0.5 * np.pi * w)
    kw = (2.0 / (np.pi * v0)) * np.arctanh(np.sin(0.5 * np.pi * w))
    C = kw ** 2 / v
    C = C / C.sum()
    tau = (w[0] / w) ** 2
    tau = tau * (kn_max * length / (v[0] * tau[0]))
    return C.astype(np.float64), v.astype(np.float64), tau.astype(np.float64)


def nongray_two_material_2d(n: int = 512, K: int = 40, ratio: float = 100.0,
                            particles: int = 50_000_000, amp: float = 0.01, width: float = 0.05,
                            seed: int = 0, name: str = "nongray2d") -> Workload:
    """2D non-gray two-material square: the left half's relaxation times are
    `ratio` times the right half's for every band (null collisions), K bands of
    the sine dispersion (Kn 1e-3 .. 10 in the right half), hot top wall 1.01,
    others 0.99, Gaussian source of width `width` L at the centre."""
    C, v, tau_r = sine_dispersion_bands(K)
    d = 1.0 / n
    ix = np.tile(np.arange(n), n)
    left = ix < n // 2
    tau = np.concatenate([np.where(left, t * ratio, t) for t in tau_r]).astype(np.float64)
    w = Workload(name=name, dim=2, nx=n, ny=n, dx=d, dy=d, t_ref=1.0, cv=1.0, vg=float(v[0]),
                 tau=tau, wall_T=_walls_2d(n, n, 0.99, 0.99, 0.99, 1.01), seed=seed,
                 particles_per_iter=particles, n_bands=K, band_C=C, band_vg=v)
    w.source = gaussian_source(n, n, d, d, amp, width)
    return w


def seeded_temperature(n_cells: int, seed: int = 512, t_ref: float = 1.0,
                       amp: float = 0.01) -> np.ndarray:
    """Initial temperature field t_ref + amp * U(-1, 1) per cell
    (numpy default_rng(seed)): every cell emits from the first iteration on."""
    rng = np.random.default_rng(seed)
    return t_ref + amp * rng.uniform(-1.0, 1.0, size=n_cells)
