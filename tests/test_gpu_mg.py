"""GPU parity of the multigrid-preconditioned CG of the Newton step: the HIP
path through the C ABI against the oracle on the same seeded inputs, CG
iteration counts, E and G bit for bit, for every split of the hierarchy
between group-wide levels and the levels each workgroup keeps in LDS, for
several workgroup shapes, and at the benchmark's full mesh size."""
import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, cavity_2d, two_material_2d

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


def _diff(w):
    lam = w.vg * np.asarray(w.tau)
    u, inv = np.unique(lam, return_inverse=True)
    Dx = np.array([cp.d_eff(l, w.dx) for l in u])[inv]
    Dy = np.array([cp.d_eff(l, w.dy) for l in u])[inv] if w.dim == 2 else None
    return Dx, Dy


# (workload, cg_waves); the comment gives the levels kept by the whole group
CASES = {
    "one_cell": (lambda: cavity_2d(n=1, ny=1, kn=0.1, particles=2000), 0),        # none
    "strip_1x9": (lambda: cavity_2d(n=1, ny=9, kn=0.05, particles=5000), 0),      # none
    "slab_1000": (lambda: slab_1d(n=1000, kn=0.003, particles=50_000), 0),        # none
    "slab_3000": (lambda: slab_1d(n=3000, kn=0.001, particles=60_000), 0),        # 3000, 1500
    "slab_3000_w1": (lambda: slab_1d(n=3000, kn=0.001, particles=60_000), 1),
    "ragged_37x23": (lambda: cavity_2d(n=37, ny=23, kn=0.01, particles=50_000), 0),
    "cavity_64": (lambda: cavity_2d(n=64, kn=0.01, particles=100_000), 0),        # 4096
    "rect_100x77": (lambda: cavity_2d(n=100, ny=77, kn=0.01, particles=100_000), 3),
    "wide_300x50": (lambda: cavity_2d(n=300, ny=50, kn=0.01, particles=100_000), 0),
    "two_material_96": (lambda: two_material_2d(n=96, kn_right=0.01, ratio=100.0,
                                                particles=100_000), 12),
    "groups_512": (lambda: cavity_2d(n=512, kn=0.005, particles=300_000), 0),    # 4 levels
}


@pytest.mark.parametrize("name", list(CASES))
def test_mg_newton_bitwise(oracle_mod, gpu, name):
    make, waves = CASES[name]
    w = make()
    Dx, Dy = _diff(w)
    kw = dict(newton=True, diff_x=Dx, diff_y=Dy, tally_faces=oracle_mod.FACES_EVERY,
              cg_precond=oracle_mod.PRECOND_MG)
    o = oracle_mod.Oracle(w, **kw)
    s = gpu.Solver(w, cg_waves=waves, **kw)
    for i in range(2):
        assert o.step(1) == 0 and s.step(1) == 0
        _, _, E, G = s.state()
        assert np.array_equal(o.E(), _np(E)), f"{name} iteration {i}: E differs"
        assert np.array_equal(o.G(), _np(G)), f"{name} iteration {i}: G differs"
        assert o.info().cg_iters_last == s.stats()["cg_iters_last"], name


def test_mg_full_mesh_bitwise(oracle_mod, gpu):
    """The 256^2 cavity of the benchmark (its CG launch shape depends on the mesh
    only) with fewer particles so the oracle finishes quickly: bitwise E, G and
    CG iteration count, far fewer iterations than plain CG."""
    w = cavity_2d(n=256, kn=1.0, particles=400_000)
    Dx, Dy = _diff(w)
    kw = dict(newton=True, diff_x=Dx, diff_y=Dy, tally_faces=oracle_mod.FACES_EVERY,
              rng_mode=oracle_mod.CRN)
    o = oracle_mod.Oracle(w, cg_precond=oracle_mod.PRECOND_MG, **kw)
    s = gpu.Solver(w, cg_precond=gpu.PRECOND_MG, **kw)
    p = gpu.Solver(w, **kw)
    assert o.step(1) == 0 and s.step(1) == 0 and p.step(1) == 0
    _, _, E, G = s.state()
    assert np.array_equal(o.E(), _np(E)) and np.array_equal(o.G(), _np(G))
    its = s.stats()["cg_iters_last"]
    assert its == o.info().cg_iters_last
    assert 20 * its < p.stats()["cg_iters_last"]
    # both solvers meet the same stopping rule: the two Newton states agree to
    # the CG tolerance relative to the correction
    Ep = _np(p.state()[2])
    assert np.abs(_np(E) - Ep).max() <= 1e-6 * np.abs(Ep).max()


def test_mg_solve_and_group(gpu, oracle_mod):
    """A CRN solve to 1e-6 and grouped stepping on own streams: the same bits as
    the oracle's solve and as the same solver stepped alone."""
    w = cavity_2d(n=48, ny=40, kn=0.01, particles=100_000)
    Dx, Dy = _diff(w)
    kw = dict(newton=True, diff_x=Dx, diff_y=Dy, rng_mode=oracle_mod.CRN, max_iters=30,
              res_tol=1e-6, tally_faces=oracle_mod.FACES_FINAL, cg_precond=oracle_mod.PRECOND_MG)
    o = oracle_mod.Oracle(w, **kw)
    s = gpu.Solver(w, **kw)
    rco, To, qxo, qyo = o.solve()
    rcs, Ts, qxs, qys, st = s.solve()
    assert rco == rcs and o.info().iter == st["iters"]
    assert np.array_equal(To, _np(Ts)) and np.array_equal(qxo, _np(qxs))
    a = gpu.Solver(w, own_stream=True, **kw)
    b = gpu.Solver(w, **kw)
    assert gpu.step_group([a], 3) == 0 and b.step(3) == 0
    assert torch.equal(a.state()[2], b.state()[2])
    assert a.stats()["cg_iters_total"] == b.stats()["cg_iters_total"]


def test_mg_rejections(gpu):
    from paper_2506_09465_amd import _lib as L
    w = slab_1d(n=20, kn=0.01, particles=5000)
    Dx, _ = _diff(w)
    with pytest.raises(L.IugkpError):
        gpu.Solver(w, newton=True, diff_x=Dx, cg_precond=2)


def test_mg_batch_equals_single_solves(gpu, oracle_mod):
    """Batched solves with the multigrid-preconditioned CG (one workgroup per
    instance) beside instances with the plain CG pool and without Newton:
    every instance's status, iteration count, CG iterations, T and q equal its
    own single solve (a group of 8-wave workgroups), and the first instance
    equals the oracle's multigrid solve."""
    ws = [cavity_2d(n=48, ny=40, kn=0.01, particles=100_000, seed=3),
          cavity_2d(n=100, ny=77, kn=0.003, particles=400_000, seed=4),
          slab_1d(n=3000, kn=0.001, particles=60_000, seed=5),
          cavity_2d(n=256, kn=0.05, particles=600_000, seed=6),
          cavity_2d(n=33, kn=0.2, particles=40_000, seed=7),
          cavity_2d(n=40, kn=1.0, particles=60_000, seed=8)]
    kws = []
    for i, w in enumerate(ws):
        Dx, Dy = _diff(w)
        kw = dict(newton=True, diff_x=Dx, diff_y=Dy, rng_mode=oracle_mod.CRN, max_iters=30,
                  res_tol=1e-6, tally_faces=oracle_mod.FACES_FINAL)
        if i == 4:
            kw["cg_precond"] = oracle_mod.PRECOND_NONE        # the pool beside the multigrid
        elif i == 5:
            kw["newton"] = False
        else:
            kw["cg_precond"] = oracle_mod.PRECOND_MG
        kws.append(kw)
    singles = []
    for w, k in zip(ws, kws):
        s = gpu.Solver(w, **k)
        try:
            rc, T, qx, qy, st = s.solve()
        except gpu.IugkpError as e:
            rc, T, qx, qy, st = e.code, None, None, None, s.stats()
        singles.append((rc, T, qx, qy, st))
    bs = gpu.BatchSolver(ws, per_instance=kws)
    rc, outs = bs.solve()
    for i, ((rc1, T1, qx1, qy1, st1), (Tb, qxb, qyb, stb)) in enumerate(zip(singles, outs)):
        assert stb["status"] == rc1, f"instance {i}"
        assert stb["iters"] == st1["iters"], f"instance {i}"
        assert stb["cg_iters_total"] == st1["cg_iters_total"], f"instance {i}"
        if rc1 >= 0:
            assert torch.equal(Tb, T1) and torch.equal(qxb, qx1) and torch.equal(qyb, qy1), i
    o = oracle_mod.Oracle(ws[0], **kws[0])
    rco, To, qxo, qyo = o.solve()
    assert rco == singles[0][0] and o.info().cg_iters_total == outs[0][3]["cg_iters_total"]
    assert np.array_equal(To, _np(outs[0][0])) and np.array_equal(qxo, _np(outs[0][1]))
