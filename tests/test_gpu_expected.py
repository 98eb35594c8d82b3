"""GPU parity of the expected-value estimator (deposits of every cell's
collision probability along each ray): the HIP path through the C ABI
against the oracle on the same seeded inputs, tallies, emission, E and the
outputs bit for bit (own exp on both sides, checked bitwise on its own)."""
import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_two_tau, cavity_2d, two_material_2d

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


_LAUNCH_KEYS = ("cg_waves", "block_size", "march")


def _pair(oracle_mod, gpu, w, **kw):
    o = oracle_mod.Oracle(w, estimator=oracle_mod.EXPECTED,
                          **{k: v for k, v in kw.items() if k not in _LAUNCH_KEYS})
    s = gpu.Solver(w, estimator=gpu.EST_EXPECTED, **kw)
    return o, s


def _same_iteration(o, s, tag=""):
    to = o.tallies()
    ts = {k: _np(v) for k, v in s.tallies().items()}
    for k in ("D", "W", "Phix", "Phiy", "B"):
        assert np.array_equal(to[k], ts[k]), f"{tag} tally {k} differs"
    it, d0, E, G = s.state()
    assert np.array_equal(o.E(), _np(E)), f"{tag} E differs"
    assert np.array_equal(o.G(), _np(G)), f"{tag} G differs"
    oi, st = o.info(), s.stats()
    assert (oi.flights, oi.segments, oi.crossings) == (st["flights"], st["segments"], st["crossings"])
    assert oi.res == st["res"] and oi.d0 == d0 and oi.iter == it


def test_expm_bitwise(oracle_mod, gpu):
    rng = np.random.default_rng(21)
    n = 1_000_000
    x = np.concatenate([rng.uniform(0.0, 1.0, n // 2), rng.uniform(0.0, 720.0, n // 2)])
    x[:5] = [0.0, 700.0, 700.5, 0.34657359027997264, 1e-300]
    ref = oracle_mod.math_batch(6, x)
    got = gpu.dev_math(6, torch.from_numpy(x).cuda(), None).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def _diff(w):
    lam = w.vg * np.asarray(w.tau)
    Dx = np.array([cp.d_eff(l, w.dx) for l in lam])
    Dy = np.array([cp.d_eff(l, w.dy) for l in lam]) if w.dim == 2 else None
    return Dx, Dy


def _src(w):
    w.source = 0.1 * np.linspace(0.0, 1.0, w.nx * w.ny)
    return w


CASES = {
    "slab_kn1": lambda: slab_1d(n=40, kn=1.0, particles=40_000),
    "slab_kn0.02": lambda: slab_1d(n=40, kn=0.02, particles=40_000),
    "slab_two_tau_src": lambda: _src(slab_1d_two_tau(n=30, tau_left=3.0, tau_right=0.05,
                                                     particles=40_000)),
    "cavity_ragged": lambda: cavity_2d(n=37, ny=23, kn=0.1, particles=60_000, newton=False),
    "two_material_window": lambda: two_material_2d(n=48, kn_right=0.05, ratio=20.0,
                                                   particles=120_000),
    # rows too long for one stripe: several row stripes
    "wide_600x40": lambda: cavity_2d(n=600, ny=40, kn=0.05, particles=150_000, newton=False),
    "wide_null_400x60": lambda: _two_material_wide(),
}


def _two_material_wide():
    w = cavity_2d(n=400, ny=60, kn=0.02, particles=150_000, newton=False)
    ix = np.tile(np.arange(400), 60)
    w.tau = np.where(ix < 150, 20.0 * np.asarray(w.tau), np.asarray(w.tau))
    return w


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("rng", ["fresh", "crn"])
@pytest.mark.parametrize("march", [1, 2])
def test_expected_iterations_bitwise(oracle_mod, gpu, name, rng, march):
    """march 1: emitter tiles (the default); march 2: row stripes on 2D meshes."""
    w = CASES[name]()
    o, s = _pair(oracle_mod, gpu, w, newton=False, march=march,
                 rng_mode=oracle_mod.CRN if rng == "crn" else oracle_mod.FRESH, epoch=3)
    for i, faces in enumerate([True, False, True]):
        assert o.step(1, faces=faces) == 0
        assert s.step(1, faces=faces) == 0
        _same_iteration(o, s, f"{name} iteration {i}")


@pytest.mark.parametrize("kind", ["1d", "2d"])
def test_expected_newton_bitwise(oracle_mod, gpu, kind):
    w = slab_1d(n=60, kn=0.02, particles=30_000) if kind == "1d" else \
        cavity_2d(n=24, ny=19, kn=0.05, particles=60_000)
    Dx, Dy = _diff(w)
    o, s = _pair(oracle_mod, gpu, w, newton=True, diff_x=Dx, diff_y=Dy,
                 tally_faces=oracle_mod.FACES_EVERY)
    for i in range(3):
        assert o.step(1) == 0 and s.step(1) == 0
        _same_iteration(o, s, f"newton {kind} {i}")


def test_expected_solve_bitwise(oracle_mod, gpu):
    w = cavity_2d(n=20, kn=0.3, particles=30_000, newton=False)
    o, s = _pair(oracle_mod, gpu, w, newton=False, rng_mode=oracle_mod.CRN, max_iters=60,
                 res_tol=1e-8, tally_faces=oracle_mod.FACES_FINAL)
    rco, To, qxo, qyo = o.solve()
    rcs, Ts, qxs, qys, st = s.solve()
    assert rco == rcs
    assert np.array_equal(To, _np(Ts))
    assert np.array_equal(qxo, _np(qxs)) and np.array_equal(qyo, _np(qys))


def test_expected_rejections(gpu):
    from paper_2506_09465_amd import _lib as L
    from synth import slab_1d_bands
    w = slab_1d(n=10, particles=5000)
    with pytest.raises(L.IugkpError):
        gpu.Solver(w, estimator=gpu.EST_EXPECTED, scheme=gpu.SCHEME_PERSISTENT)
    with pytest.raises(L.IugkpError):
        gpu.Solver(slab_1d_bands(n=10, particles=5000), estimator=gpu.EST_EXPECTED)
    s = gpu.Solver(w, estimator=gpu.EST_EXPECTED, rng_mode=gpu.RNG_CRN)
    s.step(1)
    with pytest.raises(L.IugkpError):
        s.adjoint(np.ones(10))


def test_expected_full_size_conservation(gpu):
    """256^2 cavity at Kn 0.1 with 1e7 particles and face tallies (the
    benchmark's launch shape): every iteration deposits exactly the emitted
    energy (sum D + sum B = sum G)."""
    w = cavity_2d(n=256, kn=0.1, particles=10_000_000, newton=False)
    s = gpu.Solver(w, estimator=gpu.EST_EXPECTED, tally_faces=gpu.FACES_EVERY)
    for _ in range(2):
        G = s.state()[3]
        assert s.step(1) == 0
        t = s.tallies()
        assert int(t["D"].sum()) + int(t["B"].sum()) == int(G.sum())
