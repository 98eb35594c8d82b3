"""Oracle: the expected-value estimator (variance reduction: the collision
probability of every cell along a ray deposited instead of one sampled
collision point, the particle form of the CDF-weighted sum of Sec. 2).

Pins: exact conservation (sum D + sum B = sum G per iteration, per-cell face
balance net inflow = D - G), the one-iteration expectation of D, W and B
against the exact collision-probability model of a film with constant and
discontinuous tau, a smaller spread than the analog estimator at the same
particle count, and the steady state against the CP fixed point."""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_two_tau, two_material_2d


def _one_iteration(oracle_mod, w, estimator, seeds, particles):
    """D, W, B (float energy units) of the first iteration for several seeds."""
    out = {"D": [], "W": [], "B": []}
    for s in seeds:
        o = oracle_mod.Oracle(w, seed=s, particles=particles, estimator=estimator,
                              tally_faces=oracle_mod.FACES_OFF, newton=False)
        assert o.step(1, faces=False) == 0
        F = o.info().F
        t = o.tallies()
        for k in out:
            out[k].append(np.ldexp(t[k].astype(np.float64), -F))
    return {k: np.array(v) for k, v in out.items()}


@pytest.mark.parametrize("case", ["kn1", "two_tau"])
def test_expected_one_iteration_matches_cp(oracle_mod, case):
    if case == "kn1":
        w = slab_1d(n=16, kn=1.0, t_hot=1.01, t_cold=0.99)
        w.T_init = np.linspace(1.008, 0.992, 16)
    else:
        w = slab_1d_two_tau(n=16, tau_left=4.0, tau_right=0.5)
        w.T_init = np.linspace(1.008, 0.992, 16)
    s = cp.Slab(w)
    Gc = s.cell_emission(w.cv * (np.asarray(w.T_init) - w.t_ref))
    want = {"D": s.expected_D(Gc), "W": s.expected_W(Gc), "B": s.expected_B(Gc)}
    r = _one_iteration(oracle_mod, w, oracle_mod.EXPECTED, range(8), 20_000)
    for k in ("D", "W", "B"):
        m = r[k].mean(axis=0)
        se = r[k].std(axis=0, ddof=1) / math.sqrt(r[k].shape[0])
        z = (m - want[k]) / np.maximum(se, 1e-15)
        assert np.abs(z).max() < 6.0, (k, np.abs(z).max())


def test_expected_spread_below_analog(oracle_mod):
    w = slab_1d(n=16, kn=1.0)
    w.T_init = np.linspace(1.008, 0.992, 16)
    ev = _one_iteration(oracle_mod, w, oracle_mod.EXPECTED, range(8), 20_000)["D"]
    an = _one_iteration(oracle_mod, w, oracle_mod.ANALOG, range(8), 20_000)["D"]
    sd_ev = np.sqrt((ev.std(axis=0, ddof=1) ** 2).sum())
    sd_an = np.sqrt((an.std(axis=0, ddof=1) ** 2).sum())
    assert sd_ev < 0.5 * sd_an, (sd_ev, sd_an)


@pytest.mark.parametrize("case", ["slab", "two_tau", "square"])
def test_expected_conservation_exact(oracle_mod, case):
    if case == "slab":
        w = slab_1d(n=12, kn=0.3, particles=5000)
    elif case == "two_tau":
        w = slab_1d_two_tau(n=12, tau_left=2.0, tau_right=0.05, particles=5000)
    else:
        w = two_material_2d(n=10, kn_right=0.05, ratio=10.0, particles=20_000)
    o = oracle_mod.Oracle(w, estimator=oracle_mod.EXPECTED, tally_faces=oracle_mod.FACES_EVERY,
                          newton=False)
    nc = w.nx * w.ny
    for _ in range(3):
        G = o.G().astype(object)
        assert o.step(1, faces=True) == 0
        t = o.tallies()
        assert sum(int(v) for v in t["D"]) + sum(int(v) for v in t["B"]) == sum(G)
        # per-cell balance: net inflow through the faces = D - G
        Px = t["Phix"].astype(object).reshape(w.ny, w.nx + 1)
        inflow = (Px[:, :-1] - Px[:, 1:]).reshape(-1)
        if w.dim == 2:
            Py = t["Phiy"].astype(object).reshape(w.ny + 1, w.nx)
            inflow = inflow + (Py[:-1, :] - Py[1:, :]).reshape(-1)
        assert np.array_equal(inflow, t["D"].astype(object) - G[:nc])


def test_expected_steady_state_matches_cp(oracle_mod):
    """CRN iterations of the expected-value estimator converge to a fixed point
    whose mean over independent epochs matches the CP steady state."""
    w = slab_1d_two_tau(n=16, tau_left=4.0, tau_right=1.0)
    s = cp.Slab(w)
    E_star, _ = s.fixed_point()
    Es = []
    for ep in range(8):
        o = oracle_mod.Oracle(w, particles=20_000, rng_mode=oracle_mod.CRN, epoch=ep,
                              estimator=oracle_mod.EXPECTED, max_iters=300, res_tol=1e-10,
                              tally_faces=oracle_mod.FACES_OFF, newton=False)
        rc, T, _, _ = o.solve()
        assert rc == 0
        Es.append(o.E())
    Es = np.array(Es)
    z = (Es.mean(axis=0) - E_star) / np.maximum(Es.std(axis=0, ddof=1) / math.sqrt(8), 1e-15)
    assert np.abs(z).max() < 6.0


def test_expected_rejected_where_undefined(oracle_mod):
    """The adjoint traces analog paths and the persistent population moves one
    candidate path at a time: neither takes the expected-value estimator."""
    import ctypes as C
    w = slab_1d(n=8)
    o = oracle_mod.Oracle(w, rng_mode=oracle_mod.CRN, estimator=oracle_mod.EXPECTED, newton=False)
    o.step(1)
    assert o.adjoint(np.ones(8))[0] == oracle_mod.E_INVALID_ARG
    p = oracle_mod.Persist(w)
    p.opts.estimator = oracle_mod.EXPECTED
    h = C.c_void_p()
    assert oracle_mod.lib().orc_persist_create(C.byref(p._keep.p), C.byref(p.opts),
                                               C.byref(h)) == oracle_mod.E_INVALID_ARG
