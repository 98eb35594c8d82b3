"""Pins of the oracle's multigrid-preconditioned CG for the Newton system of
Sec. 3.3 (the paper leaves the linear solver open): the V-cycle against its
definition in dense matrix form (Galerkin coarse operators P^T A P, damped
Jacobi smoothing, scaled coarse correction), its symmetry and positivity,
and the solve against a direct solve."""
import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, cavity_2d, two_material_2d

from test_oracle_newton import _dense_2d

OMEGA, SCALE = 0.8, 1.8


def _random_problem(w, seed):
    rng = np.random.default_rng(seed)
    w.tau = w.tau * rng.uniform(0.5, 2.0, size=w.tau.size)
    Dx = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-3
    Dy = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-3 if w.dim == 2 else None
    return Dx, Dy


def _prolongation(nx, ny):
    """Piecewise-constant P: fine cell (ix, iy) takes aggregate (ix // 2, iy // 2)."""
    NX, NY = (nx + 1) // 2, (ny + 1) // 2
    P = np.zeros((nx * ny, NX * NY))
    for iy in range(ny):
        for ix in range(nx):
            P[iy * nx + ix, (iy // 2) * NX + ix // 2] = 1.0
    return P, NX, NY


def _vcycle_dense(A, nx, ny):
    """The V-cycle as a matrix, from its definition: with S = I - omega D^-1 A
    two sweeps from zero give (I - S^2) A^-1 b, the coarse correction adds
    s P M_c P^T (b - A x), two more sweeps follow; one cell: 1 / a."""
    n = nx * ny
    if n == 1:
        return np.array([[1.0 / A[0, 0]]])
    P, NX, NY = _prolongation(nx, ny)
    Mc = _vcycle_dense(P.T @ A @ P, NX, NY)
    I = np.eye(n)
    S = I - OMEGA * np.diag(1.0 / np.diag(A)) @ A
    S2 = S @ S
    Ainv = np.linalg.inv(A)
    X2 = (I - S2) @ Ainv                            # after the pre-sweeps
    X3 = X2 + SCALE * P @ Mc @ P.T @ (I - A @ X2)   # after the correction
    return S2 @ X3 + (I - S2) @ Ainv                # after the post-sweeps


def test_levels_halve_to_one_cell(oracle_mod):
    assert oracle_mod.mg_levels(slab_1d(n=100)) == [(100, 1), (50, 1), (25, 1), (13, 1), (7, 1),
                                                    (4, 1), (2, 1), (1, 1)]
    assert oracle_mod.mg_levels(cavity_2d(n=37, ny=6)) == [(37, 6), (19, 3), (10, 2), (5, 1),
                                                          (3, 1), (2, 1), (1, 1)]
    assert oracle_mod.mg_levels(cavity_2d(n=1, ny=1)) == [(1, 1)]


@pytest.mark.parametrize("shape", [(1, 13), (2, 9), (5, 3), (7, 6), (4, 4)])
def test_vcycle_matches_dense_definition(oracle_mod, shape):
    """M applied to every unit vector equals the dense V-cycle built from the
    Galerkin products P^T A P of the assembled operator; M is symmetric and
    positive definite (a valid CG preconditioner)."""
    if shape[0] == 1:
        w = slab_1d(n=shape[1], kn=0.05)
    else:
        w = cavity_2d(n=shape[0], ny=shape[1], kn=0.05)
    Dx, Dy = _random_problem(w, 3)
    A = _dense_2d(w, Dx, Dy)
    n = w.nx * w.ny
    M = np.column_stack([oracle_mod.mg_precondition(w, Dx, Dy, e) for e in np.eye(n)])
    ref = _vcycle_dense(A, w.nx, w.ny)
    assert np.abs(M - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0


@pytest.mark.parametrize("dim", [1, 2])
def test_pcg_mg_solves_the_operator(oracle_mod, dim):
    w = slab_1d(n=37, kn=0.01) if dim == 1 else cavity_2d(n=9, ny=7, kn=0.05)
    Dx, Dy = _random_problem(w, 2)
    A = _dense_2d(w, Dx, Dy)
    rng = np.random.default_rng(5)
    b = rng.normal(size=w.tau.size)
    rc, x, its = oracle_mod.cg(w, Dx, Dy, b, tol=1e-12, precond=oracle_mod.PRECOND_MG)
    assert rc == 0
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    rc_p, _, its_p = oracle_mod.cg(w, Dx, Dy, b, tol=1e-12)
    assert rc_p == 0 and its < its_p
    rc2, _, its2 = oracle_mod.cg(w, Dx, Dy, b, tol=1e-12, max_iters=its - 1,
                                 precond=oracle_mod.PRECOND_MG)
    assert rc2 == oracle_mod.E_CG_NOT_CONVERGED and its2 == its - 1
    rc3, x3, its3 = oracle_mod.cg(w, Dx, Dy, np.zeros_like(b), precond=oracle_mod.PRECOND_MG)
    assert rc3 == 0 and its3 == 0 and not x3.any()


def _deff(w):
    lam = w.vg * np.asarray(w.tau)
    u, inv = np.unique(lam, return_inverse=True)
    Dx = np.array([cp.d_eff(l, w.dx) for l in u])[inv]
    Dy = np.array([cp.d_eff(l, w.dy) for l in u])[inv] if w.dim == 2 else None
    return Dx, Dy


@pytest.mark.parametrize("case", ["kn0.01", "kn1", "kn10", "two_material", "slab"])
def test_pcg_mg_iterations_independent_of_size(oracle_mod, case):
    """The DSA systems of the benchmark problems at 64^2 (and a 1000-cell slab):
    the V-cycle keeps the count a small constant where plain CG needs hundreds,
    and the solution meets the stopping rule."""
    if case == "two_material":
        w = two_material_2d(n=64, kn_right=0.01, ratio=100.0)
    elif case == "slab":
        w = slab_1d(n=1000, kn=0.003)
    else:
        w = cavity_2d(n=64, kn=float(case[2:]))
    Dx, Dy = _deff(w)
    A = _dense_2d(w, Dx, Dy) if w.nx * w.ny <= 1000 else None
    b = np.random.default_rng(7).normal(size=w.nx * w.ny)
    rc, x, its = oracle_mod.cg(w, Dx, Dy, b, tol=1e-10, precond=oracle_mod.PRECOND_MG)
    assert rc == 0 and its <= 30, its
    rc_p, xp, its_p = oracle_mod.cg(w, Dx, Dy, b, tol=1e-10, max_iters=200_000)
    assert its_p > 5 * its
    if A is not None:
        assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert np.abs(x - xp).max() <= 1e-6 * np.abs(xp).max()


def test_newton_with_mg_reaches_the_same_fixed_point(oracle_mod):
    """CRN Newton iterations with either linear solver converge to the same
    fixed point (the solver changes only how A^-1 r is computed)."""
    w = cavity_2d(n=12, kn=0.02, particles=200_000)
    Dx, Dy = _deff(w)
    out = []
    for pc in (oracle_mod.PRECOND_NONE, oracle_mod.PRECOND_MG):
        o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, newton=True, diff_x=Dx, diff_y=Dy,
                              res_tol=1e-10, max_iters=200, tally_faces=oracle_mod.FACES_OFF,
                              cg_precond=pc)
        rc, T, _, _ = o.solve()
        assert rc == 0
        out.append((T, o.info()))
    (Ta, ia), (Tb, ib) = out
    assert np.abs(Ta - Tb).max() <= 1e-7 * np.abs(Ta - w.t_ref).max()
    assert ib.cg_iters_total * 3 < ia.cg_iters_total


def test_precond_option_checked(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(slab_1d(n=8), cg_precond=2)
