"""The oracle's whole-solve behaviour: convergence rate, checkpoint/resume,
determinism, output modes and error paths."""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, cavity_2d, two_material_2d


def test_c0_crn_converges_at_the_kernel_rate(oracle_mod):
    """1D slab, Kn = 1, 1e5 particles: with common random numbers the iteration is
    a fixed linear map whose contraction is close to the exact kernel's spectral
    radius 0.619, i.e. about 29 iterations to a relative change of 1e-6."""
    w = slab_1d(kn=1.0, particles=100_000)
    rho = np.max(np.abs(np.linalg.eigvals(cp.Slab(w).K)))
    assert rho == pytest.approx(0.619, abs=2e-3)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, tally_faces=oracle_mod.FACES_FINAL)
    rc, T, qx, _ = o.solve()
    assert rc == 0
    n = o.info().iter - 1           # the last one is the extra face-tally iteration
    assert 22 <= n <= 36
    res = o.residuals(n)
    rate = (res[n - 1] / res[5]) ** (1.0 / (n - 6))
    assert rate == pytest.approx(rho, abs=0.08)
    # heat flux is divergence free across the slab (1D: same on every face) in steady state
    q = qx / ((0.01 - (-0.01)) / 4.0)
    assert np.ptp(q) < 0.05
    assert q.mean() == pytest.approx(cp.Slab(w).psi(), abs=0.03)


def test_checkpoint_resume_is_bitwise(oracle_mod):
    w = cavity_2d(n=12, ny=9, kn=0.3, particles=60_000, newton=False)
    a = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    a.step(7)
    ref_E, ref_G, ref_t = a.E(), a.G(), a.tallies()
    b = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    b.step(4)
    it, d0, E, G = b.info().iter, b.info().d0, b.E(), b.G()
    c = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    assert c.set_state(it, d0, E, G) == 0
    c.step(3)
    assert np.array_equal(c.E(), ref_E) and np.array_equal(c.G(), ref_G)
    for k in ref_t:
        assert np.array_equal(c.tallies()[k], ref_t[k])
    assert c.info().res == a.info().res


def test_seed_determinism_and_sensitivity(oracle_mod):
    w = two_material_2d(n=16, kn_right=0.05, ratio=10.0, particles=50_000)
    r = []
    for seed in (0, 0, 1):
        o = oracle_mod.Oracle(w, seed=seed)
        o.step(2)
        r.append(o.tallies()["W"])
    assert np.array_equal(r[0], r[1])
    assert not np.array_equal(r[0], r[2])


def test_crn_slot_is_fixed_fresh_slot_moves(oracle_mod):
    """CRN: the Philox slot is the epoch, so the same state gives the same tallies
    at any iteration index; FRESH: the slot is the iteration index."""
    w = slab_1d(n=30, kn=0.5, particles=20_000)
    for mode, same in ((oracle_mod.CRN, True), (oracle_mod.FRESH, False)):
        o = oracle_mod.Oracle(w, rng_mode=mode, epoch=5)
        o.step(1)
        d0, E1, G1 = o.info().d0, o.E(), o.G()
        o.set_state(1, d0, E1, G1)
        o.step(1)
        ta = o.tallies()["D"]
        o.set_state(7, d0, E1, G1)
        o.step(1)
        tb = o.tallies()["D"]
        assert np.array_equal(ta, tb) == same


def test_final_face_mode_equals_every_mode_last_iteration(oracle_mod):
    w = slab_1d(n=40, kn=0.7, particles=40_000)
    a = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, tally_faces=oracle_mod.FACES_FINAL,
                          res_tol=1e-4)
    rc, Ta, qa, _ = a.solve()
    n = a.info().iter
    b = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, tally_faces=oracle_mod.FACES_EVERY)
    b.step(n)
    F, tm = b.info().F, b.info().tau_min
    assert np.array_equal(Ta, w.t_ref + b.E() / w.cv)
    assert np.array_equal(qa, np.ldexp(b.tallies()["Phix"].astype(np.float64), -F) / (1.0 * tm))
    # tallies without faces are identical to tallies with faces
    c = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, tally_faces=oracle_mod.FACES_OFF)
    c.step(n)
    assert np.array_equal(c.E(), b.E())


def test_averaging_mode(oracle_mod):
    w = slab_1d(n=20, kn=1.0, particles=20_000, seed=3)
    a = oracle_mod.Oracle(w, avg_iters=5, max_iters=4, res_tol=1e-12)
    rc, T, q, _ = a.solve()
    assert rc == oracle_mod.W_NOT_CONVERGED and a.info().iter == 9
    b = oracle_mod.Oracle(w, max_iters=4, res_tol=1e-12)
    b.step(4)
    acc = np.zeros(w.nx)
    for _ in range(5):
        b.step(1)
        acc = acc + b.E()
    assert np.array_equal(T, w.t_ref + (acc / 5.0) / w.cv)


def test_error_paths(oracle_mod):
    w = slab_1d(n=10)
    w.tau[3] = float("nan")
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(w)
    assert e.value.rc == oracle_mod.E_INVALID_ARG
    w = slab_1d(n=10)
    w.tau[3] = 1e-9          # ratio > 1e6
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(w)
    w = slab_1d(n=10)
    w.ny = 2
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(w)
    w = slab_1d(n=10)
    with pytest.raises(oracle_mod.OracleError):       # Newton without coefficients
        oracle_mod.Oracle(w, newton=True)
    # not converged within max_iters: positive warning, outputs written
    o = oracle_mod.Oracle(slab_1d(n=10, particles=5000), max_iters=2, res_tol=1e-9)
    rc, T, _, _ = o.solve()
    assert rc == oracle_mod.W_NOT_CONVERGED and np.all(np.isfinite(T))
    # CG iteration cap
    w = slab_1d(n=30, kn=0.01, particles=5000)
    Dx = np.full(30, cp.d_eff(0.01, w.dx))
    o = oracle_mod.Oracle(w, newton=True, diff_x=Dx, cg_max_iters=1)
    assert o.step(1) == oracle_mod.E_CG_NOT_CONVERGED
    # fixed-point budget overflow on a restored state
    o = oracle_mod.Oracle(slab_1d(n=10, particles=5000))
    G = o.G()
    G[0] = 2 ** 62 + 10
    assert o.set_state(0, 0.0, o.E(), G) == oracle_mod.E_FIXED_OVERFLOW
