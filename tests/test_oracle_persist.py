"""Oracle: persistent particles, the paper's variable-tau iteration (Sec. 3.2
steps (1)-(6)) with a fixed population kept between iterations.

Pins: exact integer bookkeeping of one iteration recomputed from the particle
arrays (every particle ends in exactly one cell or wall face; null particles
keep their weight, real and wall particles take their cell's or face's share;
the shares split the available energy exactly; positions stay inside their
cells; E = W / V), the equilibrium and the uniform-field example of Sec. 3.2
staying uniform, and the steady state and heat flux of films with constant
and discontinuous tau against the exact collision-probability model."""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_two_tau, uniform_field_1d, two_material_2d


def _moved_weights(before, shares):
    """Weight each particle flies with in the next iteration."""
    q = before["q"].astype(object)
    k, loc = before["kind"], before["loc"]
    out = np.array(q, dtype=object)
    real, wall = k == 1, k == 2
    out[real] = shares["wc"][loc[real]].astype(object)
    out[wall] = shares["wb"][loc[wall]].astype(object)
    return out


def _check_face_balance(w, before, after, qm, tal):
    """Net inflow through each cell's faces = weight ending its path in the
    cell - weight starting from it (wall re-emissions enter through their
    wall face, absorptions leave through theirs): exact integers."""
    nx, ny = w.nx, w.ny
    net = np.zeros(nx * ny, dtype=object)
    for i in range(len(qm)):
        if after["kind"][i] != 2:
            net[after["loc"][i]] += qm[i]
        if before["kind"][i] != 2:
            net[before["loc"][i]] -= qm[i]
    Px = tal["Phix"].astype(object).reshape(ny, nx + 1)
    inflow = (Px[:, :-1] - Px[:, 1:]).reshape(-1)
    if w.dim == 2:
        Py = tal["Phiy"].astype(object).reshape(ny + 1, nx)
        inflow = inflow + (Py[:-1, :] - Py[1:, :]).reshape(-1)
    assert np.array_equal(inflow, net)


def _check_iteration(o, w, before, sh0, after, sh1, tal, Gw, Gs, faces=False):
    nc, nb = o.nc, o.nb
    qm = _moved_weights(before, sh0)
    assert np.array_equal(after["q"].astype(object), qm), "moved weights"
    # every particle ends in exactly one cell or wall face
    assert sum(int(v) for v in tal["W"]) + sum(int(v) for v in tal["B"]) == sum(qm)
    k, loc = after["kind"], after["loc"]
    W = np.zeros(nc, dtype=object); Wh = np.zeros(nc, dtype=object)
    B = np.zeros(nb, dtype=object)
    for i in range(len(qm)):
        if k[i] == 2:
            B[loc[i]] += qm[i]
        else:
            W[loc[i]] += qm[i]
            if k[i] == 1:
                Wh[loc[i]] += qm[i]
    assert np.array_equal(W, tal["W"].astype(object))
    assert np.array_equal(Wh, tal["Wh"].astype(object))
    assert np.array_equal(B, tal["B"].astype(object))
    assert np.array_equal(np.bincount(loc[k == 1], minlength=nc), tal["Nrc"])
    assert np.array_equal(np.bincount(loc[k == 2], minlength=nb), tal["Nb"])
    # the shares split the available energy exactly
    for c in range(nc):
        avail = int(tal["Wh"][c]) + int(Gs[c]) + int(sh0["rc"][c])
        n = int(tal["Nrc"][c])
        if n:
            assert n * int(sh1["wc"][c]) + int(sh1["rc"][c]) == avail
            assert 0 <= int(sh1["rc"][c]) < n
        else:
            assert int(sh1["wc"][c]) == 0 and int(sh1["rc"][c]) == avail
    for b in range(nb):
        avail = int(Gw[b]) + int(sh0["rb"][b])
        n = int(tal["Nb"][b])
        if n:
            assert n * int(sh1["wb"][b]) + int(sh1["rb"][b]) == avail
            assert 0 <= int(sh1["rb"][b]) < n
        else:
            assert int(sh1["wb"][b]) == 0 and int(sh1["rb"][b]) == avail
    # positions inside their cells
    cell = k != 2
    ix = loc[cell] % w.nx
    x = after["x"][cell]
    assert np.all(x >= ix * w.dx) and np.all(x <= (ix + 1) * w.dx)
    if w.dim == 2:
        iy = loc[cell] // w.nx
        y = after["y"][cell]
        assert np.all(y >= iy * w.dy) and np.all(y <= (iy + 1) * w.dy)
    F = o.info().F
    assert np.array_equal(o.E(), np.ldexp(tal["W"].astype(np.float64), -F) / (w.dx * w.dy))
    if faces:
        _check_face_balance(w, before, after, qm, tal)


@pytest.mark.parametrize("case", ["slab", "two_tau", "square"])
def test_persist_bookkeeping_exact(oracle_mod, case):
    if case == "slab":
        w = slab_1d(n=12, kn=0.5, particles=3000, seed=3)
    elif case == "two_tau":
        w = slab_1d_two_tau(n=12, tau_left=2.0, tau_right=0.05, particles=3000, seed=4)
    else:
        w = two_material_2d(n=10, kn_right=0.05, ratio=10.0, particles=6000, seed=5)
    o = oracle_mod.Persist(w, tally_faces=oracle_mod.FACES_EVERY)
    N = o.info().n_per_emitter
    sh = o.shares()
    # creation: N particles per wall face carry the face's emission
    Gw = [N * int(sh["wb"][b]) + int(sh["rb"][b]) for b in range(o.nb)]
    Gs = np.zeros(o.nc, dtype=np.int64)
    p = o.particles()
    assert o.n == N * (o.nc + o.nb)
    assert np.all(p["kind"][: N * o.nc] == 0) and np.all(p["kind"][N * o.nc:] == 2)
    for it in range(4):
        assert o.step(1, faces=(it % 2 == 0)) == 0
        p1, sh1, tal = o.particles(), o.shares(), o.tallies()
        _check_iteration(o, w, p, sh, p1, sh1, tal, Gw, Gs, faces=(it % 2 == 0))
        p, sh = p1, sh1


def test_persist_source_share(oracle_mod):
    """With a source every cell's share gains the same S V tau_min each iteration."""
    w = slab_1d(n=10, kn=0.5, particles=2000, t_hot=1.0, t_cold=1.0)
    w.source = np.linspace(0.0, 0.1, 10)
    o = oracle_mod.Persist(w, tally_faces=oracle_mod.FACES_OFF)
    gs = []
    sh = o.shares()
    for _ in range(3):
        o.step(1, faces=False)
        sh1, tal = o.shares(), o.tallies()
        n = tal["Nrc"].astype(object)
        total = n * sh1["wc"].astype(object) + sh1["rc"].astype(object)
        gs.append(total - tal["Wh"].astype(object) - sh["rc"].astype(object))
        sh = sh1
    assert all(np.array_equal(gs[0], g) for g in gs[1:])
    F = o.info().F
    tau_min = float(np.min(w.tau))
    want = [round(math.ldexp(s * (w.dx * w.dy) * tau_min, F)) for s in w.source]
    assert [int(v) for v in gs[0]] == want


def _replicas(oracle_mod, w, R, burn, n, faces=False):
    """Time averages of E (and of the left wall face's flux tally) over n
    iterations after burn, for R independent seeds; the mean over replicas and
    its standard error (a persistent population is correlated from one
    iteration to the next, so the replicas, not the iterations, are the
    independent samples)."""
    Es, fl = [], []
    for r in range(R):
        o = oracle_mod.Persist(w, seed=1000 + r,
                               tally_faces=oracle_mod.FACES_EVERY if faces else oracle_mod.FACES_OFF)
        assert o.step(burn, faces=faces) == 0
        acc = np.zeros(o.nc)
        f = 0.0
        for _ in range(n):
            assert o.step(1, faces=faces) == 0
            acc += o.E()
            if faces:
                f += math.ldexp(float(o.tallies()["Phix"][0]), -o.info().F)
        Es.append(acc / n)
        fl.append(f / n)
    Es, fl = np.array(Es), np.array(fl)
    return (Es.mean(axis=0), Es.std(axis=0, ddof=1) / math.sqrt(R), fl.mean(),
            fl.std(ddof=1) / math.sqrt(R))


def test_persist_equilibrium_stays(oracle_mod):
    w = slab_1d(n=12, kn=0.3, particles=30_000, t_hot=1.02, t_cold=1.02)
    w.T_init = np.full(12, 1.02)
    Em, se, _, _ = _replicas(oracle_mod, w, 8, 5, 30)
    z = (Em - 0.02) / np.maximum(se, 1e-9)
    assert np.abs(z).max() < 6.0


def test_persist_uniform_field_sec32(oracle_mod):
    """Kn 0.1 | 1e-4 on a 0.1 grid, T = 1 everywhere and at the walls: with the
    common time scale and null collisions the field stays uniform."""
    w = uniform_field_1d(particles=30_000)
    E0 = oracle_mod.Persist(w).E()
    Em, se, _, _ = _replicas(oracle_mod, w, 8, 5, 30)
    z = (Em - E0) / np.maximum(se, 1e-12)
    assert np.abs(z).max() < 6.0


@pytest.mark.parametrize("case", ["kn1", "two_tau"])
def test_persist_steady_state_matches_cp(oracle_mod, case):
    if case == "kn1":
        w = slab_1d(n=16, kn=1.0, particles=60_000, seed=1)
    else:
        w = slab_1d_two_tau(n=16, tau_left=4.0, tau_right=1.0, particles=60_000, seed=2)
    s = cp.Slab(w)
    E_star, G = s.fixed_point()
    Em, se, f, se_f = _replicas(oracle_mod, w, 8, 25, 50, faces=True)
    z = (Em - E_star) / np.maximum(se, 1e-9)
    assert np.abs(z).max() < 6.0, (np.abs(z).max(), Em - E_star)
    # heat flux through the left wall face
    q, se_q = f / (w.dy * s.tau_min), se_f / (w.dy * s.tau_min)
    assert abs(q - s.heat_flux_left(G)) < 6.0 * se_q, (q, s.heat_flux_left(G), se_q)


def test_persist_rejects(oracle_mod):
    w = slab_1d(n=8)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Persist(w, particles=0)
