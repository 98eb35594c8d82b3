"""Pins of the oracle's inexact-Newton (diffusion) correction, Sec. 3.3."""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, cavity_2d


def test_d_eff_definition_and_limits():
    for lam, d in [(0.5, 0.1), (0.05, 0.1), (2.0, 0.1), (0.013, 0.01)]:
        assert cp.d_eff(lam, d) == pytest.approx(cp.d_eff_second_moment(lam, d), rel=1e-11)
    # lam >> delta: lam^2 / 3 ; lam << delta: lam delta / 4
    assert cp.d_eff(10.0, 1e-3) == pytest.approx(100.0 / 3.0, rel=1e-4)
    assert cp.d_eff(1e-4, 1.0) == pytest.approx(1e-4 / 4.0, rel=1e-6)


@pytest.mark.parametrize("kn", [1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0])
def test_dsa_factor_below_half(kn):
    """The accelerated deterministic iteration E -> E_half + A^-1 (E_half - E) on
    the exact 1D kernel contracts by less than 1/2 per iteration at every Kn."""
    w = slab_1d(n=100, kn=kn)
    rho = cp.dsa_spectral_radius(w)
    assert rho < 0.5


def _dense_2d(w, Dx, Dy):
    nx, ny = w.nx, w.ny
    n = nx * ny
    A = np.zeros((n, n))
    lam = w.vg * w.tau

    def add(c1, c2, g):
        A[c1, c1] += g
        if c2 is not None:
            A[c2, c2] += g
            A[c1, c2] -= g
            A[c2, c1] -= g

    for iy in range(ny):
        for k in range(nx + 1):
            if k in (0, nx):
                c = iy * nx + (0 if k == 0 else nx - 1)
                add(c, None, Dx[c] / (w.dx * (w.dx / 2 + 2 * lam[c] / 3)))
            else:
                a, b = Dx[iy * nx + k - 1], Dx[iy * nx + k]
                add(iy * nx + k - 1, iy * nx + k, 2 * a * b / (a + b) / w.dx ** 2)
    if w.dim == 2:
        for k in range(ny + 1):
            for ix in range(nx):
                if k in (0, ny):
                    c = (0 if k == 0 else ny - 1) * nx + ix
                    add(c, None, Dy[c] / (w.dy * (w.dy / 2 + 2 * lam[c] / 3)))
                else:
                    a, b = Dy[(k - 1) * nx + ix], Dy[k * nx + ix]
                    add((k - 1) * nx + ix, k * nx + ix, 2 * a * b / (a + b) / w.dy ** 2)
    return A


@pytest.mark.parametrize("dim", [1, 2])
def test_cg_solves_the_operator(oracle_mod, dim):
    rng = np.random.default_rng(2)
    if dim == 1:
        w = slab_1d(n=37, kn=0.01)
    else:
        w = cavity_2d(n=9, ny=7, kn=0.05)
    w.tau = w.tau * rng.uniform(0.5, 2.0, size=w.tau.size)
    Dx = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-3
    Dy = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-3
    A = _dense_2d(w, Dx, Dy)
    assert np.allclose(A, A.T)
    assert np.all(np.linalg.eigvalsh(A) > 0)
    b = rng.normal(size=w.tau.size)
    rc, x, its = oracle_mod.cg(w, Dx, Dy if dim == 2 else None, b, tol=1e-12)
    assert rc == 0
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    assert its <= 4 * w.tau.size
    # stopping rule: one iteration short of convergence fails with CG_NOT_CONVERGED
    rc2, _, its2 = oracle_mod.cg(w, Dx, Dy if dim == 2 else None, b, tol=1e-12, max_iters=its - 1)
    assert rc2 == oracle_mod.E_CG_NOT_CONVERGED and its2 == its - 1
    # zero right-hand side: x = 0, no iteration
    rc3, x3, its3 = oracle_mod.cg(w, Dx, Dy if dim == 2 else None, np.zeros_like(b))
    assert rc3 == 0 and its3 == 0 and not x3.any()


def _deff_arrays(w):
    lam = w.vg * w.tau
    Dx = np.array([cp.d_eff(l, w.dx) for l in lam])
    Dy = np.array([cp.d_eff(l, w.dy) for l in lam]) if w.dim == 2 else None
    return Dx, Dy


def test_newton_keeps_the_crn_fixed_point(oracle_mod):
    """With common random numbers the iteration is a fixed affine map; the Newton
    correction only accelerates it: both converge to the same fixed point."""
    w = slab_1d(n=20, kn=0.1, particles=40_000)
    Dx, _ = _deff_arrays(w)
    plain = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=False, res_tol=1e-11,
                              max_iters=3000, tally_faces=oracle_mod.FACES_OFF)
    rc, T_plain, _, _ = plain.solve()
    assert rc == 0
    newt = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx,
                             res_tol=1e-11, max_iters=200, tally_faces=oracle_mod.FACES_OFF)
    rc, T_newt, _, _ = newt.solve()
    assert rc == 0
    dT = T_plain - w.t_ref
    assert np.abs(T_newt - T_plain).max() <= 1e-8 * np.abs(dT).max()
    assert newt.info().iter * 5 < plain.info().iter


def test_newton_accelerates_small_kn(oracle_mod):
    """Kn = 0.01, 100 cells: without acceleration ~3.6e4 iterations would be needed
    (spectral radius 0.9996 of the exact kernel); with it, a few tens."""
    w = slab_1d(n=100, kn=0.01, particles=400_000)
    s = cp.Slab(w)
    rho_plain = np.max(np.abs(np.linalg.eigvals(s.K)))
    assert rho_plain > 0.999
    Dx, _ = _deff_arrays(w)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx, res_tol=1e-6,
                          max_iters=60, tally_faces=oracle_mod.FACES_OFF)
    rc, T, _, _ = o.solve()
    assert rc == 0
    assert o.info().iter <= 30
    # diffusive limit: an almost linear profile between the wall values (the CRN
    # fixed point of one random map carries noise amplified by 1/(1 - rho), so
    # the check is on the shape, not on a tight band)
    E_star, _ = s.fixed_point()
    x = (np.arange(w.nx) + 0.5) / w.nx
    slope, icpt = np.polyfit(x, T - w.t_ref, 1)
    assert slope == pytest.approx(np.polyfit(x, E_star, 1)[0], rel=0.25)
    resid = (T - w.t_ref) - (slope * x + icpt)
    assert np.std(resid) < 0.2 * np.std(T - w.t_ref)


def test_newton_2d_runs_and_conserves(oracle_mod):
    w = cavity_2d(n=16, kn=0.02, particles=1_000_000)
    Dx, Dy = _deff_arrays(w)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx, diff_y=Dy,
                          res_tol=1e-6, max_iters=60, tally_faces=oracle_mod.FACES_FINAL)
    rc, T, qx, qy = o.solve()
    assert rc == 0 and o.info().iter <= 40
    assert np.all(T > 0.99 - 2e-3) and np.all(T < 1.01 + 2e-3)
    # hot top wall: net flux enters through the top and leaves through the others
    n = w.nx
    top_in = -qy.reshape(n + 1, n)[n].sum()
    assert top_in > 0


# ------------------------------------------------------------------ 2D reading
def test_2d_transfer_kernel_constructions():
    """The 2D flat-cell kernel (quadrature of the Bickley radial density, and its
    Fourier form) against what fixes it independently: its x marginal is the
    exact 1D flat-cell kernel (E_3 form), it sums to one, and the two
    constructions agree where both are accurate."""
    for lam in (0.03, 0.3, 1.0, 3.0, 10.0):
        R = 40 if lam <= 1.0 else 127
        P = cp.transfer_2d(lam, R)
        full_rows = P[:, 0] + 2.0 * P[:, 1:].sum(axis=1)      # sum over n of P(m, n)
        tol = 2e-5 if lam <= 1.0 else 1e-4      # Fourier form: truncated alias sum
        for m in range(4):
            assert full_rows[m] == pytest.approx(cp.flat_cell_jump_1d(lam, m), rel=tol, abs=1e-9)
        total = full_rows[0] + 2.0 * full_rows[1:].sum()
        assert total == pytest.approx(1.0, abs=2e-5 if lam <= 3.0 else 2e-3)
    a = cp.transfer_2d_real(1.0, 6)
    b = cp.transfer_2d_fourier(1.0, 6)
    assert np.abs(a - b).max() < 1e-4      # the Fourier form's alias tail


def _oracle_dense_operator(oracle_mod, w, D):
    gx, gy, dg = oracle_mod.newton_operator(w, D, D)
    nx, ny = w.nx, w.ny
    A = np.diag(dg.copy())
    for iy in range(ny):
        for k in range(1, nx):
            g = gx[iy * (nx + 1) + k]
            a, b = iy * nx + k - 1, iy * nx + k
            A[a, b] -= g
            A[b, a] -= g
    for k in range(1, ny):
        for ix in range(nx):
            g = gy[k * nx + ix]
            a, b = (k - 1) * nx + ix, k * nx + ix
            A[a, b] -= g
            A[b, a] -= g
    return A


@pytest.mark.parametrize("lam_cells", [0.03, 0.3, 1.0, 10.0])
def test_dsa_2d_expected_contraction(oracle_mod, lam_cells):
    """Reading R6 in 2D: on a 32 x 32 cavity the accelerated map
    E -> E_half + A^-1 (E_half - E) of the exact expected flat-cell kernel, with
    the operator the oracle assembles, contracts by less than 1/2 per iteration
    (the survey's 1D bound carried to 2D with walls)."""
    M = 32
    w = cavity_2d(n=M, kn=lam_cells / M, particles=1000)
    D = np.full(M * M, cp.d_eff(lam_cells / M, w.dx))
    A = _oracle_dense_operator(oracle_mod, w, D)
    K = cp.dense_transfer_2d(M, M, lam_cells)
    I = np.eye(M * M)
    T = K + np.linalg.solve(A, K - I)
    rho = float(np.max(np.abs(np.linalg.eigvals(T))))
    assert rho < 0.5, rho


# ------------------------------------------------------------------ sampled map
@pytest.mark.parametrize("lam_dx", [0.03, 0.1, 0.3, 1.0])
@pytest.mark.parametrize("n_per", [10, 100])
def test_crn_newton_converges_or_reports_divergence(oracle_mod, lam_dx, n_per):
    """Under common random numbers the Newton iteration iterates one sampled map.
    Where few particles leave each cell that map is far from its expectation
    and the correction can amplify the difference; the solve must then stop
    with DIVERGED within 10 iterations (growth rule of reading R6), never run
    into the fixed-point budget, and converge otherwise."""
    n = 100
    w = slab_1d(n=n, kn=lam_dx / n, particles=n_per * (n + 2), newton=True)
    Dx, _ = _deff_arrays(w)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx, res_tol=1e-6,
                          max_iters=80, tally_faces=oracle_mod.FACES_OFF)
    rc, _, _, _ = o.solve()
    it = o.info().iter
    r = o.residuals(it)
    assert rc in (oracle_mod.OK, oracle_mod.E_DIVERGED), rc
    if rc == oracle_mod.E_DIVERGED:
        assert it <= 10
        assert r[-1] > 1.0 and r[-1] > r[-2]
    else:
        assert r[-1] < 1e-6
    if lam_dx == 1.0 and n_per == 100:
        assert rc == oracle_mod.OK


def test_growth_rule_precedes_budget(oracle_mod):
    """A diverging Newton iteration whose next emission also leaves the
    fixed-point range reports DIVERGED, and the plain iteration on the same
    sampled map (a sub-stochastic map: it cannot grow) is not stopped by it."""
    n = 100
    w = slab_1d(n=n, kn=0.03 / n, particles=10 * (n + 2), newton=True)
    Dx, _ = _deff_arrays(w)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx, max_iters=80,
                          tally_faces=oracle_mod.FACES_OFF)
    rc, _, _, _ = o.solve()
    assert rc == oracle_mod.E_DIVERGED
    # the same iterate with the budget check alone would have overflowed
    G = o.G()
    assert np.abs(G.astype(np.float64)).sum() > 2.0 ** 62
    p = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=False, max_iters=40,
                          tally_faces=oracle_mod.FACES_OFF)
    rc, _, _, _ = p.solve()
    assert rc == oracle_mod.W_NOT_CONVERGED
