"""Pins of the oracle's particle transport against geometry, the exact 1D
collision-probability model, 2D marginals/symmetries, conservation and the
paper's uniform-field consistency example (Sec. 3.2)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_two_tau, cavity_2d, two_material_2d, uniform_field_1d


# ------------------------------------------------------------------ ray geometry
def _grid(nx, ny, d=1.0):
    w = cavity_2d(n=nx, ny=ny, kn=1.0, particles=10)
    w.dx = w.dy = d
    return w


def test_ray_simple_1d(oracle_mod):
    w = slab_1d(n=4, kn=1.0)
    w.dx = 1.0
    ev, kind, cell = oracle_mod.trace_ray(w, 0.25, 0.5, 0, 0, 1.0, 0.0, 2.0)
    assert kind == 0 and cell == 2
    assert ev.tolist() == [[0, 1, 1], [0, 2, 1]]
    # strict crossing rule: t == ell does not cross
    ev, kind, cell = oracle_mod.trace_ray(w, 0.5, 0.5, 0, 0, 1.0, 0.0, 0.5)
    assert len(ev) == 0 and kind == 0 and cell == 0
    # zero length and zero direction never cross
    assert len(oracle_mod.trace_ray(w, 0.5, 0.5, 0, 0, 1.0, 0.0, 0.0)[0]) == 0
    assert len(oracle_mod.trace_ray(w, 0.5, 0.5, 0, 0, 0.0, 0.0, 5.0)[0]) == 0
    # leftward exit through the left wall: boundary face 0, absorbed at wall 0
    ev, kind, cell = oracle_mod.trace_ray(w, 1.5, 0.5, 1, 0, -1.0, 0.0, 3.0)
    assert ev.tolist() == [[0, 1, -1], [0, 0, -1]] and kind == 1 and cell == 0
    # rightward exit through the right wall: boundary index ny + row = 1
    ev, kind, cell = oracle_mod.trace_ray(w, 3.5, 0.5, 3, 0, 1.0, 0.0, 1.0)
    assert ev.tolist() == [[0, 4, 1]] and kind == 1 and cell == 1


def test_ray_vertex_tie_x_first(oracle_mod):
    w = _grid(3, 3)
    s = 1.0 / math.sqrt(2.0)
    ev, kind, cell = oracle_mod.trace_ray(w, 0.5, 0.5, 0, 0, s, s, 1.0)
    # t_x == t_y exactly: x-face (row 0, k=1 -> index 1) before y-face (k=1, col 1 -> 4)
    assert ev.tolist() == [[0, 1, 1], [1, 1 * 3 + 1, 1]]
    assert kind == 0 and cell == 1 + 3 * 1


def test_ray_along_face_and_corner(oracle_mod):
    w = _grid(3, 3)
    # moving along the y = 1 face line with sy = 0: only x crossings, stays in row 0
    ev, kind, cell = oracle_mod.trace_ray(w, 0.2, 1.0, 0, 0, 1.0, 0.0, 2.5)
    assert ev.tolist() == [[0, 1, 1], [0, 2, 1]] and cell == 2
    # exact diagonal into the top-right corner: the x boundary face absorbs first
    s = 1.0 / math.sqrt(2.0)
    ev, kind, cell = oracle_mod.trace_ray(w, 2.5, 2.5, 2, 2, s, s, 5.0)
    assert ev.tolist() == [[0, 2 * 4 + 3, 1]] and kind == 1 and cell == 3 + 2


def test_ray_against_exact_rational_geometry(oracle_mod):
    """Random rays: the crossing sequence equals the faces sorted by the exact
    rational crossing distance, up to the end (no near-ties drawn)."""
    rng = np.random.default_rng(11)
    nx, ny, d = 7, 5, 0.37
    w = _grid(nx, ny, d)
    checked = 0
    while checked < 300:
        ix, iy = int(rng.integers(nx)), int(rng.integers(ny))
        x0 = (ix + rng.uniform()) * d
        y0 = (iy + rng.uniform()) * d
        th = rng.uniform(0, 2 * math.pi)
        sx, sy = math.cos(th), math.sin(th)
        ell = rng.exponential(4 * d)
        ev, kind, cell = oracle_mod.trace_ray(w, x0, y0, ix, iy, sx, sy, ell)
        X0, Y0, SX, SY, L, D = map(Fraction, (x0, y0, sx, sy, ell, d))
        events = []
        for k in range(nx + 1):
            t = (k * D - X0) / SX if sx != 0 else None
            if t is not None and t > 0:
                events.append((t, 0, k))
        for k in range(ny + 1):
            t = (k * D - Y0) / SY if sy != 0 else None
            if t is not None and t > 0:
                events.append((t, 1, k))
        events.sort()
        ts = [e[0] for e in events] + [L]
        gaps = [abs(a - b) for a, b in zip(sorted(ts), sorted(ts)[1:])]
        if gaps and min(gaps) < Fraction(1, 10**9):
            continue
        want = []
        cx, cy = ix, iy
        for t, axis, k in events:
            if t >= L:
                break
            if axis == 0:
                want.append([0, cy * (nx + 1) + k, 1 if sx > 0 else -1])
                if k in (0, nx):
                    break
                cx += 1 if sx > 0 else -1
            else:
                want.append([1, k * nx + cx, 1 if sy > 0 else -1])
                if k in (0, ny):
                    break
                cy += 1 if sy > 0 else -1
        assert ev.tolist() == want
        checked += 1


# ------------------------------------------------------------------ 1D CP model
def _one_iteration(O, w, **kw):
    o = O.Oracle(w, tally_faces=O.FACES_EVERY, **kw)
    info = o.info()
    G0 = o.G()
    assert o.step(1) == 0
    return o, info, G0, o.tallies()


@pytest.mark.parametrize("case", ["kn0.05", "kn1", "two_tau"])
def test_one_iteration_expectation_1d(oracle_mod, case):
    if case == "kn0.05":
        w = slab_1d(n=20, kn=0.05, particles=1_000_000)
    elif case == "kn1":
        w = slab_1d(n=20, kn=1.0, particles=1_000_000)
    else:
        w = slab_1d_two_tau(n=20, tau_left=0.5, tau_right=0.02, particles=1_000_000)
    rng = np.random.default_rng(1)
    w.T_init = 1 + 0.01 * rng.uniform(-1, 1, size=w.nx)
    o, info, G0, t = _one_iteration(oracle_mod, w)
    F, N = info.F, info.n_per_emitter
    s = cp.Slab(w)
    Gc = G0[:w.nx] * 2.0 ** -F
    zD = (t["D"] * 2.0 ** -F - s.expected_D(Gc)) / np.sqrt(s.variance_D(Gc, N))
    assert np.abs(zD).max() < 5.0
    EB = s.expected_B(Gc)
    B = t["B"] * 2.0 ** -F
    sdB = np.sqrt(np.abs(EB) * np.abs(Gc).max() / N) + 1e-12
    assert np.all(np.abs(B - EB) < 6 * sdB)
    # candidate (null + real) events: W = D / r in expectation
    EW = s.expected_W(Gc)
    assert np.all(np.abs(t["W"] * 2.0 ** -F - EW) < 6 * np.sqrt(s.variance_W(Gc, N)))
    # the heat flux through the left wall face in this iteration
    q0 = t["Phix"][0] * 2.0 ** -F
    assert q0 == pytest.approx(s.Gw[0] - EB[0], abs=6 * sdB[0])


def test_fixed_point_matches_cp_1d(oracle_mod):
    """FRESH iterations averaged after burn-in vs the CP fixed point (I - K)^-1 b,
    including the face-tally heat flux (heat-flux ratio Psi)."""
    w = slab_1d(n=20, kn=1.0, particles=200_000)
    s = cp.Slab(w)
    E_star, G_star = s.fixed_point()
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    o.step(15)
    F = o.info().F
    Es, qs = [], []
    for _ in range(60):
        o.step(1)
        Es.append(o.E())
        qs.append(o.tallies()["Phix"][0] * 2.0 ** -F / s.tau_min)
    Es = np.array(Es)
    # batch means over 6 batches of 10 (iterations are correlated)
    bm = Es.reshape(6, 10, -1).mean(axis=1)
    se = bm.std(axis=0, ddof=1) / math.sqrt(6)
    z = (Es.mean(axis=0) - E_star) / np.maximum(se, 1e-7)
    assert np.abs(z).max() < 6.0
    qb = np.array(qs).reshape(6, 10).mean(axis=1)
    psi = qb.mean() / (w.vg * (s.Ew[0] - s.Ew[1]) / 4.0)
    psi_se = qb.std(ddof=1) / math.sqrt(6) / (w.vg * (s.Ew[0] - s.Ew[1]) / 4.0)
    assert abs(psi - s.psi()) < 6 * psi_se + 1e-3


# ------------------------------------------------------------------ 2D
def _single_emitter(n_side, lam_over_d, particles, emit_cell=True):
    w = cavity_2d(n=n_side, kn=1.0, particles=particles, newton=False)
    d = 1.0 / n_side
    w.tau[:] = lam_over_d * d
    w.wall_T[:] = w.t_ref
    w.T_init = np.full(n_side * n_side, w.t_ref)
    return w


def test_2d_marginals_match_1d_kernel(oracle_mod):
    """One emitting cell at the centre of a 25x25 mesh, lambda = dx: both the
    column sums and the row sums of D equal the 1D flat-cell kernel row
    (the x and y marginals of the projected 3D isotropic flight)."""
    n = 25
    w = _single_emitter(n, 1.0, particles=(n * n + 4 * n) * 200_000)
    c = n // 2
    w.T_init[c + n * c] = w.t_ref + 0.5
    o, info, G0, t = _one_iteration(oracle_mod, w)
    F, N = info.F, info.n_per_emitter
    G = G0[c + n * c] * 2.0 ** -F
    D = t["D"].reshape(n, n) * 2.0 ** -F
    assert abs(t["B"].sum() * 2.0 ** -F) < 1e-4 * G
    K, _, _, _ = cp.cp_1d(np.full(n, 1.0), 1.0)
    p = K[c]
    sd = np.sqrt(N * (G / N) ** 2 * p * (1 - p))
    use = N * p > 20
    assert use.sum() >= 9
    for marg in (D.sum(axis=0), D.sum(axis=1)):
        z = (marg - G * p) / sd
        assert np.abs(z[use]).max() < 5.0
    # 90-degree rotation symmetry in expectation
    cnt = np.abs(D) / (G / N)
    both = (cnt + np.rot90(cnt)) > 20
    diff = (D - np.rot90(D)) / (G / N)
    z = diff[both] / np.sqrt(cnt + np.rot90(cnt))[both]
    assert np.abs(z).max() < 6.0


def test_2d_wall_emission_depth_law(oracle_mod):
    """A single left-wall row emits; column sums of D follow the cosine-law depth
    distribution 2[E3(t1) - E3(t2)] of the 1D wall kernel."""
    nx, ny = 10, 121
    w = cavity_2d(n=nx, ny=ny, kn=1.0, particles=(nx * ny + 2 * (nx + ny)) * 4000, newton=False)
    w.tau[:] = 2.0 * w.dx
    w.wall_T[:] = w.t_ref
    row = ny // 2
    w.wall_T[row] = w.t_ref + 0.3
    o, info, G0, t = _one_iteration(oracle_mod, w)
    F, N = info.F, info.n_per_emitter
    Gw = G0[nx * ny + row] * 2.0 ** -F
    D = t["D"].reshape(ny, nx) * 2.0 ** -F
    _, Pw, _, Pww = cp.cp_1d(np.full(nx, 2.0), 1.0)
    p = Pw[0]
    sd = np.sqrt(N * (Gw / N) ** 2 * p * (1 - p))
    z = (D.sum(axis=0) - Gw * p) / sd
    assert np.abs(z).max() < 5.0
    Bright = t["B"][ny:2 * ny].sum() * 2.0 ** -F
    pr = Pww[0, 1]
    assert abs(Bright - Gw * pr) < 5 * math.sqrt(N * (Gw / N) ** 2 * pr * (1 - pr))


def _face_divergence_identity(w, t, G):
    nx, ny = w.nx, w.ny
    Px = t["Phix"].reshape(ny, nx + 1)
    net = Px[:, :-1] - Px[:, 1:]
    if w.dim == 2:
        Py = t["Phiy"].reshape(ny + 1, nx)
        net = net + Py[:-1, :] - Py[1:, :]
    return net.reshape(-1), (t["D"] - G[:nx * ny])


@pytest.mark.parametrize("kind", ["1d", "2d", "2d_null"])
def test_exact_integer_conservation(oracle_mod, kind):
    if kind == "1d":
        w = slab_1d(n=50, kn=0.3, particles=200_000)
    elif kind == "2d":
        w = cavity_2d(n=24, ny=17, kn=0.2, particles=300_000, newton=False)
    else:
        w = two_material_2d(n=24, kn_right=0.05, ratio=20.0, particles=300_000)
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    for _ in range(3):
        G = o.G()
        o.step(1)
        t = o.tallies()
        # every emitted unit ends in a real collision or a wall
        assert int(G.sum()) == int(t["D"].sum()) + int(t["B"].sum())
        # per cell: net face inflow = deposit - emission (heat-flux divergence, Sec. 3.3)
        net, dd = _face_divergence_identity(w, t, G)
        assert np.array_equal(net, dd)
        # candidate events include the real ones
        if kind != "2d_null":
            assert np.array_equal(t["W"], t["D"])


def test_uniform_field_invariance_1d(oracle_mod):
    """Sec. 3.2 consistency example: T = 1 everywhere and at the walls, Kn 0.1 | 1e-4
    on a 0.1 grid.  With the common time scale tau_min and null collisions the
    field stays uniform in expectation."""
    w = uniform_field_1d(particles=150_000)
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    info = o.info()
    E0 = o.E()
    s = cp.Slab(w)
    # the exact expectation is the identity on a uniform field
    assert np.allclose(s.step(E0), E0, rtol=1e-10)
    o.step(1)
    E1 = o.E()
    G = s.cell_emission(E0)
    sd = np.sqrt(s.variance_W(G, info.n_per_emitter)) / s.V
    assert np.abs((E1 - E0) / sd).max() < 6.0


def test_uniform_field_invariance_2d_two_material(oracle_mod):
    w = two_material_2d(n=16, kn_right=0.02, ratio=10.0, particles=400_000)
    w.t_ref = 0.5
    w.wall_T[:] = 1.0
    w.T_init = np.ones(w.n_cells)
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_EVERY)
    E0 = o.E()
    Es = []
    for _ in range(4):
        o.step(1)
        Es.append(o.E())
    m = np.mean(Es, axis=0)
    # relative deviation of the mean field, coarse band from the emitted particle count
    rel = (m - E0) / E0
    assert abs(rel.mean()) < 3e-3
    assert np.abs(rel).max() < 0.1


def _ballistic_fraction(x, y, L):
    """Fraction of directions (3D isotropic, z infinite) from (x, y) in [0,L]^2 that
    end on the top wall: the planar angle it subtends over 2 pi."""
    a1 = math.atan2(L - y, L - x)
    a2 = math.atan2(L - y, -x)
    return (a2 - a1) / (2 * math.pi)


def test_2d_ballistic_limit(oracle_mod):
    """Kn = 100 in the square cavity: E(x) -> sum_w E_w (planar angle of w) / 2 pi
    up to O(1/Kn); checked cell by cell against the per-iteration noise."""
    n = 12
    w = cavity_2d(n=n, kn=100.0, particles=3_000_000, newton=False)
    o = oracle_mod.Oracle(w, tally_faces=oracle_mod.FACES_OFF)
    o.step(2)
    Es = []
    for _ in range(10):
        o.step(1)
        Es.append(o.E())
    Es = np.array(Es)
    E = Es.mean(axis=0).reshape(n, n)
    se = (Es.std(axis=0, ddof=1) / math.sqrt(len(Es))).reshape(n, n)
    Eh, Ec = 0.01, -0.01
    z = []
    for iy in range(1, n - 1):
        for ix in range(1, n - 1):
            f = _ballistic_fraction((ix + 0.5) / n, (iy + 0.5) / n, 1.0)
            ref = Eh * f + Ec * (1 - f)
            z.append((E[iy, ix] - ref) / (se[iy, ix] + 2e-4))
    z = np.array(z)
    assert np.abs(z).max() < 5.0
    assert abs(z.mean()) < 1.0
