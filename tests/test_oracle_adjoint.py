"""Oracle: volumetric heat source and the adjoint of the steady state.

Pins (none of them re-types the oracle's arithmetic):
  * source: FRESH iterations averaged vs the collision-probability fixed point
    with the source (exact E3 integral kernel), and the steady-state energy
    balance  sum(source emission) = sum(wall absorption)  with cold walls;
  * adjoint: the exact gradient from a dense transfer matrix assembled
    independently (unit-impulse iterations of the oracle, dense numpy solves),
    central finite differences of the forward solve with common random
    numbers, and the reciprocity of the transfer matrix on a uniform mesh.
"""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import cavity_2d, slab_1d, gaussian_source


def _src_1d(w, amp=0.02):
    x = (np.arange(w.nx) + 0.5) / w.nx
    return amp * (1.0 + np.sin(np.pi * x))


def test_source_fixed_point_matches_cp_1d(oracle_mod):
    """Source emission S V tau_min per cell and iteration: FRESH iterations
    averaged after burn-in against the CP fixed point with the source."""
    w = slab_1d(n=20, kn=0.5, particles=200_000)
    w.source = _src_1d(w)
    s = cp.Slab(w)
    E_star, _ = s.fixed_point(source=w.source)
    E_nosrc, _ = s.fixed_point()
    assert np.min(E_star - E_nosrc) > 1e-3      # the source is visible
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_OFF)
    o.step(25)
    Es = []
    for _ in range(60):
        o.step(1, faces=False)
        Es.append(o.E())
    Es = np.array(Es)
    bm = Es.reshape(6, 10, -1).mean(axis=1)
    se = bm.std(axis=0, ddof=1) / math.sqrt(6)
    z = (Es.mean(axis=0) - E_star) / np.maximum(se, 1e-7)
    assert np.abs(z).max() < 6.0


def test_source_energy_balance_cold_walls(oracle_mod):
    """Walls at t_ref emit nothing: at the CRN steady state every unit of source
    energy leaves through the walls, sum(B) = sum(G_src), up to the residual."""
    w = cavity_2d(n=12, kn=0.3, particles=60_000, newton=False, t_hot=1.0, t_cold=1.0)
    w.source = gaussian_source(12, 12, w.dx, w.dy, 0.05, 0.2)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, max_iters=400, res_tol=1e-11,
                          tally_faces=oracle_mod.FACES_OFF)
    rc, T, _, _ = o.solve()
    assert rc == 0
    info = o.info()
    Gs = np.rint(np.ldexp(w.source * (w.dx * w.dy) * info.tau_min, info.F))
    B = o.tallies()["B"]
    assert B.sum() == pytest.approx(Gs.sum(), rel=1e-8)
    assert np.all(T > 1.0)                       # heated everywhere, walls colder


def _dense_transfer(oracle_mod, w, epoch=0):
    """T[:, e] = fraction of emitter e's N particles ending in each cell, from
    one oracle iteration per emitter with only that emitter emitting."""
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, epoch=epoch, newton=False,
                          tally_faces=oracle_mod.FACES_OFF)
    N = o.info().n_per_emitter
    nc, ne = o.nc, o.ne
    q = 1 << 20
    T = np.zeros((nc, ne))
    for e in range(ne):
        G = np.zeros(ne, np.int64)
        G[e] = q * N
        assert o.set_state(0, 0.0, np.zeros(nc), G) == 0
        assert o.step(1, faces=False) == 0
        T[:, e] = o.tallies()["D"] / float(q * N)
    return T, o.info()


def _dense_gradient(w, info, Tm, probes, target, src):
    """Steady state and exact gradient of L = sum (T_p - target)^2 from the dense
    transfer matrix: D* = (I - Tcc)^-1 (Tcc Gs + Tcw Gw)."""
    nc = w.n_cells
    V = w.dx * w.dy
    F, tmin, lam = info.F, info.tau_min, info.lam_min
    Tcc, Tcw = Tm[:, :nc], Tm[:, nc:]
    A_f = np.where(np.arange(w.n_bfaces) < 2 * w.ny, w.dy, w.dx)
    Gw = np.ldexp(w.cv * (w.wall_T - w.t_ref) * lam * A_f / 4.0, F)
    Gs = np.ldexp(src * V * tmin, F)
    Dst = np.linalg.solve(np.eye(nc) - Tcc, Tcc @ Gs + Tcw @ Gw)
    Tst = w.t_ref + np.ldexp(Dst, -F) / V / w.cv
    dLdT = np.zeros(nc)
    dLdT[probes] = 2.0 * (Tst[probes] - target)
    u = np.ldexp(dLdT / w.cv / V, -F)
    psi = np.linalg.solve((np.eye(nc) - Tcc).T, u)
    g_src = (Tcc.T @ psi) * np.ldexp(V * tmin, F)
    g_wall = (Tcw.T @ psi) * np.ldexp(w.cv * lam * A_f / 4.0, F)
    return Tst, dLdT, g_wall, g_src


@pytest.mark.parametrize("newton", [False, True])
def test_adjoint_matches_dense_transfer_matrix(oracle_mod, newton):
    w = cavity_2d(n=6, ny=5, kn=0.4, particles=30_000, newton=False)
    w.source = gaussian_source(6, 5, w.dx, w.dy, 0.03, 0.2)
    Tm, info = _dense_transfer(oracle_mod, w)
    rng = np.random.default_rng(3)
    probes = rng.choice(w.n_cells, size=7, replace=False)
    target = rng.uniform(0.99, 1.01, size=7)
    Tst, dLdT, g_wall, g_src = _dense_gradient(w, info, Tm, probes, target, w.source)
    kw = {}
    if newton:
        lam = w.vg * w.tau
        D = np.full(w.n_cells, cp.d_eff(float(lam[0]), w.dx))
        kw = dict(newton=True, diff_x=D, diff_y=D)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, max_iters=2000, res_tol=1e-13,
                          tally_faces=oracle_mod.FACES_OFF, **kw)
    rc, T, _, _ = o.solve()
    assert rc == 0
    # the forward CRN solve reaches the dense steady state
    assert np.max(np.abs(T - Tst)) < 1e-12
    rc, gw, gs, its = o.adjoint(dLdT, max_iters=2000, tol=1e-13)
    assert rc == 0 and its > 1
    scale_s = np.max(np.abs(g_src))
    scale_w = np.max(np.abs(g_wall))
    assert np.max(np.abs(gs - g_src)) < 1e-9 * scale_s
    assert np.max(np.abs(gw - g_wall)) < 1e-9 * scale_w


def test_adjoint_vs_central_differences(oracle_mod):
    """Central differences (h = 1e-4) of the CRN steady state with respect to the
    four wall temperatures and three source cells."""
    n = 8
    base = cavity_2d(n=n, kn=0.1, particles=40_000, newton=False)
    base.source = gaussian_source(n, n, base.dx, base.dy, 0.02, 0.1)
    rng = np.random.default_rng(5)
    probes = rng.choice(n * n, size=6, replace=False)
    target = rng.uniform(0.99, 1.01, size=6)
    lam = base.vg * base.tau
    D = np.full(n * n, cp.d_eff(float(lam[0]), base.dx))

    def solve(wall, src):
        w = cavity_2d(n=n, kn=0.1, particles=40_000, newton=False)
        w.wall_T = wall
        w.source = src
        o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, max_iters=3000, res_tol=1e-12,
                              tally_faces=oracle_mod.FACES_OFF, newton=True, diff_x=D, diff_y=D)
        rc, T, _, _ = o.solve()
        assert rc == 0
        return o, T

    def loss(T):
        return float(np.sum((T[probes] - target) ** 2))

    o, T0 = solve(base.wall_T, base.source)
    dLdT = np.zeros(n * n)
    dLdT[probes] = 2.0 * (T0[probes] - target)
    rc, gw, gs, _ = o.adjoint(dLdT, max_iters=3000, tol=1e-12)
    assert rc == 0
    walls = [np.arange(0, n), np.arange(n, 2 * n), np.arange(2 * n, 3 * n), np.arange(3 * n, 4 * n)]
    h = 1e-4
    for faces in walls:
        wp, wm = base.wall_T.copy(), base.wall_T.copy()
        wp[faces] += h
        wm[faces] -= h
        fd = (loss(solve(wp, base.source)[1]) - loss(solve(wm, base.source)[1])) / (2 * h)
        ad = gs.dtype.type(gw[faces].sum())
        # the stated target is 1e-3; the adjoint is the exact transpose of the CRN map
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-14, (faces[0], ad, fd)
    hs = 1e-4
    for c in (int(probes[0]), 27, 36):
        sp, sm = base.source.copy(), base.source.copy()
        sp[c] += hs
        sm[c] -= hs
        fd = (loss(solve(base.wall_T, sp)[1]) - loss(solve(base.wall_T, sm)[1])) / (2 * hs)
        assert abs(gs[c] - fd) <= 1e-6 * abs(fd) + 1e-14, (c, gs[c], fd)


def test_transfer_reciprocity_uniform_mesh(oracle_mod):
    """Reciprocity of the linearised transport: on a uniform mesh with one
    relaxation time the cell-to-cell transfer is symmetric in expectation,
    so T_cc - T_cc^T is pure Monte Carlo noise."""
    w = cavity_2d(n=5, kn=0.5, particles=200_000, newton=False)
    Tm, info = _dense_transfer(oracle_mod, w)
    nc = w.n_cells
    N = info.n_per_emitter
    Tcc = Tm[:, :nc]
    var = (Tcc * (1 - Tcc) + Tcc.T * (1 - Tcc.T)) / N
    z = (Tcc - Tcc.T) / np.sqrt(np.maximum(var, 1e-12))
    assert np.abs(z).max() < 5.5
    # and not trivially: the transfer is far from diagonal
    assert np.sum(Tcc) - np.trace(Tcc) > 0.3 * np.sum(Tcc)


def test_adjoint_rejects_unsupported(oracle_mod):
    w = cavity_2d(n=4, kn=0.5, particles=2_000, newton=False)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.FRESH)
    rc, *_ = o.adjoint(np.ones(16))
    assert rc == oracle_mod.E_INVALID_ARG
    w.tau[3] *= 2.0
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN)
    rc, *_ = o.adjoint(np.ones(16))
    assert rc == oracle_mod.E_INVALID_ARG
