"""GPU parity of the persistent-particle scheme (Sec. 3.2 steps (1)-(6) with a
fixed population): the HIP path through the C ABI against the oracle's
persistent solver on the same seeded inputs.  The whole population (position,
direction, weight, kind, location), the tallies, the counts, the shares and
carried remainders, E, the residual and the outputs agree bit for bit."""
import numpy as np
import pytest

from synth import slab_1d, slab_1d_two_tau, two_material_2d, cavity_2d

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


_ORACLE_KEYS = ("seed", "particles", "rng_mode", "epoch", "max_iters", "res_tol", "tally_faces",
                "avg_iters")


def _pair(oracle_mod, gpu, w, **kw):
    o = oracle_mod.Persist(w, **{k: v for k, v in kw.items() if k in _ORACLE_KEYS})
    s = gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, **kw)
    return o, s


def _same(o, s, tag, tallies=True):
    po, ps = o.particles(), {k: _np(v) for k, v in s.particles().items()}
    for k in ("x", "y", "sx", "sy", "q", "kind", "loc"):
        assert np.array_equal(po[k], ps[k]), f"{tag}: particle {k} differs"
    sho, shs = o.shares(), {k: _np(v) for k, v in s.shares().items()}
    for k in ("wc", "rc", "wb", "rb"):
        assert np.array_equal(sho[k], shs[k]), f"{tag}: share {k} differs"
    assert np.array_equal(o.E(), _np(s.state()[2])), f"{tag}: E differs"
    if tallies:
        to = o.tallies()
        ts = {k: _np(v) for k, v in s.tallies().items()}
        for ko, ks in (("W", "W"), ("Wh", "D"), ("Phix", "Phix"), ("Phiy", "Phiy"), ("B", "B")):
            assert np.array_equal(to[ko], ts[ks]), f"{tag}: tally {ko} differs"
        assert np.array_equal(to["Nrc"], shs["Nrc"].view(np.uint32)), f"{tag}: N_rc differs"
        assert np.array_equal(to["Nb"], shs["Nb"].view(np.uint32)), f"{tag}: N_b differs"
        oi, st = o.info(), s.stats()
        assert (oi.flights, oi.segments, oi.crossings) == (st["flights"], st["segments"],
                                                           st["crossings"]), tag
        assert oi.res == st["res"] and oi.iter == st["iters"], tag


def _source(w):
    w.source = 0.2 * np.linspace(0.0, 1.0, w.nx * w.ny)
    return w


CASES = {
    "slab_kn05": lambda: slab_1d(n=24, kn=0.5, particles=30_000, seed=1),
    "slab_two_tau_src": lambda: _source(slab_1d_two_tau(n=21, tau_left=2.0, tau_right=0.02,
                                                        particles=30_000, seed=2)),
    "square_two_material": lambda: two_material_2d(n=24, kn_right=0.02, ratio=20.0,
                                                   particles=80_000, seed=3),
    "cavity_long_paths": lambda: cavity_2d(n=20, kn=3.0, particles=40_000, newton=False, seed=4),
    "ragged_rect_src": lambda: _source(cavity_2d(n=37, ny=13, kn=0.1, particles=50_000,
                                                 newton=False, seed=5)),
    # tall cells crossed by long paths: many columns with runs of three or more y faces
    "tall_long_paths": lambda: cavity_2d(n=11, ny=41, kn=2.0, particles=40_000, newton=False,
                                         seed=8),
    # 4000 columns: the row-stripe face pass holds four rows of faces per
    # workgroup, so 25 rows make seven stripes (the last one short)
    "wide_many_stripes": lambda: cavity_2d(n=4000, ny=25, kn=0.002, particles=120_000,
                                           newton=False, seed=9),
    # degenerate 2D meshes: one column (every y face in it), one row (only
    # the two y walls)
    "column_1x9": lambda: cavity_2d(n=1, ny=9, kn=3.0, particles=20_000, newton=False, seed=10),
    "row_40x1": lambda: cavity_2d(n=40, ny=1, kn=0.5, particles=20_000, newton=False, seed=11),
}


# march 2: y faces of face-tallied moves by the row-stripe pass (2D);
# march 1: as global atomics in the move
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("rng", ["fresh", "crn"])
@pytest.mark.parametrize("march", [1, 2])
def test_persist_iterations_bitwise(oracle_mod, gpu, name, rng, march):
    w = CASES[name]()
    o, s = _pair(oracle_mod, gpu, w, rng_mode=oracle_mod.CRN if rng == "crn" else oracle_mod.FRESH,
                 epoch=7, march=march)
    _same(o, s, f"{name} creation", tallies=False)
    for i, faces in enumerate([True, False, True, False]):
        assert o.step(1, faces=faces) == 0
        assert s.step(1, faces=faces) == 0
        _same(o, s, f"{name} iteration {i}")


@pytest.mark.parametrize("mode", ["every", "final", "off", "avg"])
def test_persist_solve_bitwise(oracle_mod, gpu, mode):
    faces = {"every": oracle_mod.FACES_EVERY, "final": oracle_mod.FACES_FINAL,
             "off": oracle_mod.FACES_OFF, "avg": oracle_mod.FACES_EVERY}[mode]
    w = two_material_2d(n=16, kn_right=0.05, ratio=10.0, particles=40_000, seed=6)
    kw = dict(max_iters=8, res_tol=1e-12, tally_faces=faces, avg_iters=3 if mode == "avg" else 0)
    o, s = _pair(oracle_mod, gpu, w, **kw)
    rco, To, qxo, qyo = o.solve()
    rcs, Ts, qxs, qys, st = s.solve()
    assert rco == rcs == 1
    assert np.array_equal(To, _np(Ts))
    assert np.array_equal(qxo, _np(qxs)) and np.array_equal(qyo, _np(qys))
    assert o.info().iter == st["iters"]


def test_persist_rejections(gpu):
    from paper_2506_09465_amd import _lib as L
    w = slab_1d(n=10, particles=5000)
    with pytest.raises(L.IugkpError) as e:
        gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, newton=True, diff_x=np.ones(10))
    assert e.value.code == L.E_INVALID_ARG
    s = gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, rng_mode=gpu.RNG_CRN)
    s.step(2)
    it, d0, E, G = s.state()
    assert s.set_state(it, d0, E, G) == L.E_INVALID_ARG
    with pytest.raises(L.IugkpError):
        s.adjoint(np.ones(10))
    g = gpu.Solver(w)
    with pytest.raises(L.IugkpError):
        g.particles()
    with pytest.raises(L.IugkpError):
        gpu.BatchSolver([w, w], scheme=gpu.SCHEME_PERSISTENT)


def test_persist_full_size_bookkeeping(gpu):
    """The 256^2 cavity at Kn 0.1 with 1e7 particles (the benchmark's launch
    shape): every particle ends in one cell or wall face, the moved weights
    are the previous iteration's shares, and the shares split the available
    energy exactly, checked with exact integer sums on the device."""
    w = cavity_2d(n=256, kn=0.1, particles=10_000_000, newton=False)
    s = gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, tally_faces=gpu.FACES_EVERY)
    nc, nb = w.nx * w.ny, w.n_bfaces
    for it in range(3):
        p0, sh0 = s.particles(), s.shares()
        assert s.step(1, faces=(it != 1)) == 0
        p1, sh1, t = s.particles(), s.shares(), s.tallies()
        k0, l0 = p0["kind"].long(), p0["loc"].long()
        moved = torch.where(k0 == 1, sh0["wc"][l0.clamp(max=nc - 1)],
                            torch.where(k0 == 2, sh0["wb"][l0.clamp(max=nb - 1)], p0["q"]))
        assert torch.equal(moved, p1["q"])
        assert int(t["W"].sum()) + int(t["B"].sum()) == int(moved.sum())
        k1, l1 = p1["kind"].long(), p1["loc"].long()
        assert int((k1 == 1).sum()) == int(sh1["Nrc"].sum())
        assert int((k1 == 2).sum()) == int(sh1["Nb"].sum())
        avail_c = t["D"] + sh0["rc"]
        n = sh1["Nrc"].long()
        assert torch.equal(n * sh1["wc"] + sh1["rc"], avail_c)
        nbw = sh1["Nb"].long()
        assert bool(((sh1["rc"] >= 0) & ((sh1["rc"] < n) | (n == 0))).all())
        assert bool(((sh1["rb"] >= 0) & ((sh1["rb"] < nbw) | (nbw == 0))).all())
        cell = k1 != 2
        ix = (l1[cell] % w.nx).double()
        x = p1["x"][cell]
        assert bool(((x >= ix * w.dx) & (x <= (ix + 1) * w.dx)).all())
    st = s.stats()
    assert st["segments"] == st["n_per_emitter"] * (nc + nb)


@pytest.mark.parametrize("kn", [0.1, 10.0])
def test_persist_full_size_stripes_equal_atomics(gpu, kn):
    """The benchmark's persistent configuration (256^2 cavity, 1e7 particles,
    faces every iteration): the row-stripe face pass and the move's global
    atomics give the same population and tallies bit for bit."""
    w = cavity_2d(n=256, kn=kn, particles=10_000_000, newton=False)
    a = gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, tally_faces=gpu.FACES_EVERY)
    b = gpu.Solver(w, scheme=gpu.SCHEME_PERSISTENT, tally_faces=gpu.FACES_EVERY, march=1)
    for it in range(2):
        assert a.step(1) == 0 and b.step(1) == 0
        ta, tb = a.tallies(), b.tallies()
        for k in ta:
            assert torch.equal(ta[k], tb[k]), f"iteration {it}: tally {k} differs"
        pa, pb = a.particles(), b.particles()
        for k in pa:
            assert torch.equal(pa[k], pb[k]), f"iteration {it}: particle {k} differs"
    assert a.stats()["tot_crossings"] == b.stats()["tot_crossings"]
    a.close()
    b.close()
