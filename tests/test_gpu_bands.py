"""GPU parity of frequency-band problems (an extension of the paper's gray
model): the HIP path through the C ABI against the oracle's band solver,
element by element on the same seeded inputs.  Tallies, emission and the
fixed-point state agree bit for bit per band; E, the residual and the outputs
too (same IEEE operations in the same order on both sides)."""
import numpy as np
import pytest

from synth import slab_1d_bands, nongray_two_material_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _np(t):
    return t.detach().cpu().numpy()


_ORACLE_KEYS = ("seed", "particles", "rng_mode", "epoch", "max_iters", "res_tol", "tally_faces")


def _pair(oracle_mod, gpu, w, **kw):
    o = oracle_mod.Bands(w, **{k: v for k, v in kw.items() if k in _ORACLE_KEYS})
    s = gpu.Solver(w, **kw)
    return o, s


def _same_state(o, s, tag=""):
    K = o.K
    it, d0, E, G = s.state()
    G = _np(G).reshape(K, -1)
    ts = {k: _np(v) for k, v in s.tallies().items()}
    for k in range(K):
        ob = o.band(k)
        assert np.array_equal(ob["G"], G[k]), f"{tag} band {k} G differs"
        for key in ("D", "W", "Phix", "Phiy", "B"):
            assert np.array_equal(ob[key], ts[key][k]), f"{tag} band {k} tally {key} differs"
    assert np.array_equal(o.E(), _np(E)), f"{tag} E differs"
    oi, st = o.info(), s.stats()
    assert (oi.flights, oi.segments, oi.crossings) == (st["flights"], st["segments"], st["crossings"])
    assert oi.res == st["res"] and oi.d0 == d0 and oi.iter == it


def _mixed_2d(n=40, K=4, particles=120_000, seed=3):
    """Two-material bands, band 0 with one relaxation time everywhere (no null
    collisions, a smaller LDS window than the others)."""
    w = nongray_two_material_2d(n=n, K=K, particles=particles, seed=seed)
    nc = n * n
    w.tau = np.array(w.tau)
    w.tau[:nc] = w.tau[:nc].min()
    return w


CASES = {
    "slab_uniform": lambda: slab_1d_bands(n=20, particles=60_000),
    "slab_two_tau_src": lambda: _with_source(slab_1d_bands(n=23, kn_left_factor=4.0,
                                                           particles=70_000, seed=5)),
    "nongray_24": lambda: nongray_two_material_2d(n=24, K=6, particles=150_000, seed=1),
    "mixed_40": lambda: _mixed_2d(),
    "ragged_37x21": lambda: _ragged(),
}


def _with_source(w):
    w.source = 0.05 * np.linspace(0.0, 1.0, w.nx * w.ny)
    return w


def _ragged():
    """Non-square two-material mesh with ragged tiles and a window smaller
    than the domain."""
    w = nongray_two_material_2d(n=8, K=3, particles=100_000, seed=7)
    nx, ny = 53, 37
    C, v = w.band_C, w.band_vg
    ix = np.tile(np.arange(nx), ny)
    tau_r = np.array([0.02, 0.2, 2.0])
    w.nx, w.ny, w.dx, w.dy = nx, ny, 1.0 / nx, 0.7 / ny
    w.tau = np.concatenate([np.where(ix < nx // 3, t * 10.0, t) for t in tau_r])
    w.wall_T = np.full(2 * ny + 2 * nx, 0.99)
    w.wall_T[2 * ny + nx:] = 1.01
    w.source = None
    w.band_C, w.band_vg = C[:3] / C[:3].sum(), v[:3]
    return w


# march 0: bands whose free paths reach half the domain's height run their
# face-tallied iterations by row stripes (in the 2D cases here: the first two;
# band 0 of mixed_40 without null collisions); march 1: every band on tiles
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("rng", ["fresh", "crn"])
@pytest.mark.parametrize("march", [0, 1])
def test_band_iterations_bitwise(oracle_mod, gpu, name, rng, march):
    w = CASES[name]()
    kw = dict(rng_mode=oracle_mod.CRN if rng == "crn" else oracle_mod.FRESH, epoch=9)
    o, s = _pair(oracle_mod, gpu, w, march=march, **kw)
    _same_state(o, s, "initial")
    for i, faces in enumerate([True, False, True]):
        assert o.step(1, faces=faces) == 0
        assert s.step(1, faces=faces) == 0
        _same_state(o, s, f"{name} iteration {i}")


@pytest.mark.parametrize("faces", ["every", "final", "off"])
def test_band_solve_bitwise(oracle_mod, gpu, faces):
    mode = {"every": oracle_mod.FACES_EVERY, "final": oracle_mod.FACES_FINAL,
            "off": oracle_mod.FACES_OFF}[faces]
    w = nongray_two_material_2d(n=24, K=5, particles=100_000, seed=2)
    o, s = _pair(oracle_mod, gpu, w, max_iters=6, res_tol=1e-12, tally_faces=mode)
    rco, To, qxo, qyo = o.solve()
    rcs, Ts, qxs, qys, st = s.solve()
    assert rco == rcs == 1          # not converged within 6 iterations, on both sides
    assert np.array_equal(To, _np(Ts))
    assert np.array_equal(qxo, _np(qxs)) and np.array_equal(qyo, _np(qys))
    assert o.info().iter == st["iters"]
    if faces == "off":
        assert not np.any(_np(qxs))


def test_band_solve_converges_bitwise(oracle_mod, gpu):
    """CRN iterations to a fixed point (slab, three bands, two materials, source)."""
    w = _with_source(slab_1d_bands(n=16, kn_left_factor=4.0, particles=40_000, seed=4))
    o, s = _pair(oracle_mod, gpu, w, rng_mode=oracle_mod.CRN, max_iters=400, res_tol=1e-9)
    rco, To, qxo, _ = o.solve()
    rcs, Ts, qxs, _, st = s.solve()
    assert rco == rcs == 0
    assert np.array_equal(To, _np(Ts)) and np.array_equal(qxo, _np(qxs))
    assert o.info().iter == st["iters"]


def test_band_resume_bitwise(gpu):
    w = nongray_two_material_2d(n=24, K=4, particles=80_000, seed=6)
    a = gpu.Solver(w)
    a.step(2)
    it, d0, E, G = a.state()
    a.step(2)
    b = gpu.Solver(w)
    assert b.set_state(it, d0, E, G) == 0
    b.step(2)
    _, _, Ea, Ga = a.state()
    _, _, Eb, Gb = b.state()
    assert torch.equal(Ea, Eb) and torch.equal(Ga, Gb)
    ta, tb = a.tallies(), b.tallies()
    assert all(torch.equal(ta[k], tb[k]) for k in ta)


def test_band_problem_rejections(gpu):
    from paper_2506_09465_amd import _lib as L
    w = slab_1d_bands(n=10, particles=10_000)
    for bad in (dict(newton=True), dict(avg_iters=2)):
        with pytest.raises(L.IugkpError) as e:
            gpu.Solver(w, **bad)
        assert e.value.code == L.E_INVALID_ARG
    s = gpu.Solver(w, rng_mode=L.RNG_CRN)
    s.step(1)
    with pytest.raises(L.IugkpError) as e:
        s.adjoint(np.ones(w.nx))
    assert e.value.code == L.E_INVALID_ARG
    w.band_C = np.array([0.5, -0.3, 0.2])
    with pytest.raises(L.IugkpError):
        gpu.Solver(w)


def test_band_full_size_properties(gpu):
    """The 512^2, 40-band two-material problem with its source at the full
    particle count, in the benchmark's launch configuration: every band's
    energy is conserved exactly (absorbed in cells + absorbed by walls =
    emitted), and E and T follow from the band tallies."""
    w = nongray_two_material_2d()
    s = gpu.Solver(w, tally_faces=gpu.FACES_OFF)
    K, nc = w.n_bands, w.nx * w.ny
    for _ in range(2):
        _, _, _, G0 = s.state()
        assert s.step(1) == 0
        t = s.tallies()
        G0 = G0.view(K, -1).cpu()
        absorbed = t["D"].cpu().sum(dim=1) + t["B"].cpu().sum(dim=1)
        assert torch.equal(absorbed, G0.sum(dim=1))
    st = s.stats()
    # zero-weight particles are not flown (cells still near t_ref early on)
    assert 0 < st["flights"] <= st["n_per_emitter"] * st["n_emitters"] <= w.particles_per_iter
    F = st["fixed_point_F"]
    W = t["W"].cpu().numpy()
    V = w.dx * w.dy
    Wsum = np.zeros(nc)
    for k in range(K):
        Wsum = Wsum + np.ldexp(W[k].astype(np.float64), -F)
    _, _, E, _ = s.state()
    assert np.array_equal(Wsum / V, _np(E))


def test_band_full_size_stripes_equal_tiles(gpu):
    """The 512^2, 40-band problem with face tallies in the benchmark's launch
    configuration: its two long-path bands by row stripes (march 0) give the
    tallies of every band on emitter tiles (march 1) bit for bit."""
    w = nongray_two_material_2d()
    a = gpu.Solver(w, tally_faces=gpu.FACES_EVERY)
    b = gpu.Solver(w, tally_faces=gpu.FACES_EVERY, march=1)
    for it in range(2):
        assert a.step(1, faces=True) == 0 and b.step(1, faces=True) == 0
        ta, tb = a.tallies(), b.tallies()
        for k in ta:
            assert torch.equal(ta[k], tb[k]), (it, k)
        assert torch.equal(a.state()[2], b.state()[2])
    sa, sb = a.stats(), b.stats()
    assert (sa["flights"], sa["segments"], sa["crossings"]) == (sb["flights"], sb["segments"],
                                                              sb["crossings"])
    a.close()
    b.close()
