"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element on the same seeded inputs.  Integer tallies and the fixed-point state
must agree bit for bit; floating-point state too (same IEEE operations in the
same order, contraction off on both sides)."""
import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_two_tau, cavity_2d, two_material_2d, uniform_field_1d

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
    Dx = np.array([cp.d_eff(l, w.dx) for l in lam])
    Dy = np.array([cp.d_eff(l, w.dy) for l in lam]) if w.dim == 2 else None
    return Dx, Dy


_LAUNCH_KEYS = ("cg_waves", "block_size", "march")   # GPU launch shape only, no effect on results


def _pair(oracle_mod, gpu, w, **kw):
    o = oracle_mod.Oracle(w, **{k: v for k, v in kw.items() if k not in _LAUNCH_KEYS})
    s = gpu.Solver(w, **kw)
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


# ----------------------------------------------------------------- building blocks
def test_philox_bitwise(oracle_mod, gpu):
    rng = np.random.default_rng(0)
    n = 1_000_000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ref = oracle_mod.philox_batch(ctr, (0x12345678, 0x9abcdef0))
    ct = torch.from_numpy(ctr.view(np.int32)).cuda()
    got = gpu.dev_philox(ct, 0x12345678, 0x9abcdef0).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("op", [0, 1, 2, 3, 4, 5])
def test_elementary_ops_bitwise(oracle_mod, gpu, op):
    rng = np.random.default_rng(10 + op)
    n = 1_000_000
    y = None
    if op == 0:      # log on eta = 1 - U, the values the free-path sampler sees
        x = 1.0 - rng.integers(0, 2**53, n) * 2.0 ** -53
        x[:4] = [1.0, 2.0 ** -53, 0.5, 1.0 - 2.0 ** -53]
    elif op == 1:
        x = rng.integers(0, 2**53, n) * 2.0 ** -53
        x[:4] = [0.0, 0.25, 0.5, 0.75]
    elif op == 2:
        x = np.concatenate([rng.uniform(0, 1, n // 2), np.exp(rng.uniform(-700, 700, n // 2))])
    elif op == 3:
        x = rng.normal(size=n) * np.exp(rng.uniform(-50, 50, n))
        y = rng.normal(size=n) * np.exp(rng.uniform(-50, 50, n))
    elif op == 4:
        x = rng.integers(-(2**62), 2**62, n).view(np.float64)
    else:
        x = rng.normal(size=n) * 1e-3
        y = np.full(n, 60.0)
    ref = oracle_mod.math_batch(op, x, y)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yt = None if y is None else torch.from_numpy(y).cuda()
    got = gpu.dev_math(op, xt, yt).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


# ----------------------------------------------------------------- per-iteration tallies
CASES_1D = {
    "slab_kn1": lambda: slab_1d(kn=1.0, particles=100_000),
    "slab_kn0.01": lambda: slab_1d(kn=0.01, particles=100_000),
    "slab_two_tau": lambda: slab_1d_two_tau(particles=100_000),
    "uniform_field": lambda: uniform_field_1d(particles=50_000),
}


@pytest.mark.parametrize("name", sorted(CASES_1D))
@pytest.mark.parametrize("mode", ["fresh", "crn"])
def test_tallies_bitwise_1d(oracle_mod, gpu, name, mode):
    w = CASES_1D[name]()
    rm = oracle_mod.FRESH if mode == "fresh" else oracle_mod.CRN
    o, s = _pair(oracle_mod, gpu, w, rng_mode=rm, epoch=3, tally_faces=oracle_mod.FACES_EVERY)
    assert o.info().F == s.stats()["fixed_point_F"]
    for i in range(4):
        assert o.step(1) == 0 and s.step(1) == 0
        _same_iteration(o, s, f"{name} it{i}")


CASES_2D = {
    "ragged_kn0.02": lambda: cavity_2d(n=37, ny=23, kn=0.02, particles=300_000, newton=False),
    "ragged_kn0.3": lambda: cavity_2d(n=37, ny=23, kn=0.3, particles=300_000, newton=False),
    "ragged_kn5": lambda: cavity_2d(n=37, ny=23, kn=5.0, particles=300_000, newton=False),
    "two_material": lambda: two_material_2d(n=40, kn_right=0.02, ratio=100.0, particles=200_000),
    "tiny_1x1": lambda: cavity_2d(n=1, kn=0.5, particles=1000, newton=False),
    "strip_1x9": lambda: cavity_2d(n=1, ny=9, kn=0.5, particles=5000, newton=False),
}


@pytest.mark.parametrize("name", sorted(CASES_2D))
def test_tallies_bitwise_2d(oracle_mod, gpu, name):
    w = CASES_2D[name]()
    o, s = _pair(oracle_mod, gpu, w, tally_faces=oracle_mod.FACES_EVERY, seed=12345678901)
    for i in range(3):
        assert o.step(1) == 0 and s.step(1) == 0
        _same_iteration(o, s, f"{name} it{i}")


@pytest.mark.parametrize("bs", [64, 128, 512, 1024])
def test_launch_shape_independence(gpu, bs):
    """Integer tallies are order-independent: any workgroup size, same bits."""
    w = cavity_2d(n=33, ny=21, kn=0.7, particles=200_000, newton=False)
    a = gpu.Solver(w, block_size=256)
    b = gpu.Solver(w, block_size=bs)
    a.step(2)
    b.step(2)
    ta, tb = a.tallies(), b.tallies()
    for k in ta:
        assert torch.equal(ta[k], tb[k])


@pytest.mark.parametrize("kind", ["1d", "2d"])
def test_newton_bitwise(oracle_mod, gpu, kind):
    if kind == "1d":
        w = slab_1d(kn=0.01, particles=100_000)
    else:
        w = cavity_2d(n=24, ny=19, kn=0.02, particles=200_000)
    Dx, Dy = _diff(w)
    o, s = _pair(oracle_mod, gpu, w, newton=True, diff_x=Dx, diff_y=Dy,
                 tally_faces=oracle_mod.FACES_EVERY)
    for i in range(3):
        assert o.step(1) == 0 and s.step(1) == 0
        _same_iteration(o, s, f"newton {kind} it{i}")
        assert o.info().cg_iters_last == s.stats()["cg_iters_last"]


def test_solve_bitwise_c0(oracle_mod, gpu):
    """The 1D slab (100 cells, Kn = 1, 1e5 particles, seed 0) solved to 1e-6 in
    common-random-numbers mode: same iteration count, same T and q bits."""
    w = slab_1d(kn=1.0, particles=100_000)
    kw = dict(rng_mode=oracle_mod.CRN, tally_faces=oracle_mod.FACES_FINAL)
    o, s = _pair(oracle_mod, gpu, w, **kw)
    rc_o, T_o, qx_o, _ = o.solve()
    rc_s, T_s, qx_s, _, st = s.solve()
    assert rc_o == rc_s == 0
    assert o.info().iter == st["iters"]
    assert np.array_equal(T_o, _np(T_s)) and np.array_equal(qx_o, _np(qx_s))
    assert np.array_equal(o.residuals(st["iters"]), s.residuals())
    # the one-call form gives the same answer
    T1, (qx1, _), st1, rc1 = gpu.solve(w, **kw)
    assert rc1 == 0 and torch.equal(T1, T_s) and torch.equal(qx1, qx_s)


def test_solve_bitwise_newton_avg(oracle_mod, gpu):
    w = cavity_2d(n=20, ny=16, kn=0.05, particles=100_000)
    Dx, Dy = _diff(w)
    kw = dict(newton=True, diff_x=Dx, diff_y=Dy, tally_faces=oracle_mod.FACES_EVERY,
              avg_iters=3, max_iters=5)
    o, s = _pair(oracle_mod, gpu, w, **kw)
    rc_o, T_o, qx_o, qy_o = o.solve()
    rc_s, T_s, qx_s, qy_s, st = s.solve()
    assert rc_o == rc_s
    assert np.array_equal(T_o, _np(T_s))
    assert np.array_equal(qx_o, _np(qx_s)) and np.array_equal(qy_o, _np(qy_s))


def test_checkpoint_resume_bitwise_gpu(gpu):
    w = two_material_2d(n=24, kn_right=0.05, ratio=20.0, particles=100_000)
    a = gpu.Solver(w)
    a.step(6)
    ref = a.tallies()
    b = gpu.Solver(w)
    b.step(3)
    it, d0, E, G = b.state()
    c = gpu.Solver(w)
    assert c.set_state(it, d0, E, G) == 0
    c.step(3)
    for k, v in c.tallies().items():
        assert torch.equal(v, ref[k])
    assert torch.equal(c.state()[2], a.state()[2])


def test_library_d_eff_matches_scipy(gpu):
    for lam, d in [(1.0, 0.01), (0.01, 0.01), (0.001, 0.01), (10.0, 1 / 256), (0.37, 0.1)]:
        assert gpu.d_eff(lam, d) == pytest.approx(cp.d_eff(lam, d), rel=1e-12)


def test_gpu_error_paths(gpu):
    w = slab_1d(n=10)
    w.tau[2] = -1.0
    with pytest.raises(gpu.IugkpError) as e:
        gpu.Solver(w)
    assert e.value.code == -1
    w = slab_1d(n=10)
    with pytest.raises(gpu.IugkpError):
        gpu.Solver(w, block_size=96)
    s = gpu.Solver(slab_1d(n=10, particles=5000), max_iters=2, res_tol=1e-12)
    rc, T, *_ = s.solve()
    assert rc == 1 and torch.isfinite(T).all()
    w = slab_1d(n=30, kn=0.01, particles=5000)
    s = gpu.Solver(w, newton=True, cg_max_iters=1)
    assert s.step(1) == -7


NEWTON_LAYOUTS = {
    # name: (workload factory, cg_waves) -- the CG group layouts: one workgroup,
    # ragged tree blocks, groups whose workgroups own less than a mesh row (the
    # halo spans several owners), 1D halos, state in registers (cg_waves > 0)
    # or in global memory (cg_waves < 0)
    "strip_1x9": (lambda: cavity_2d(n=1, ny=9, kn=0.05, particles=5000), 0),
    "slab_100": (lambda: slab_1d(n=100, kn=0.003, particles=20_000), 0),
    "slab_1000_w1": (lambda: slab_1d(n=1000, kn=0.003, particles=50_000), 1),
    "slab_1000_g1": (lambda: slab_1d(n=1000, kn=0.003, particles=50_000), -1),
    "ragged_37x23": (lambda: cavity_2d(n=37, ny=23, kn=0.01, particles=50_000), 0),
    "ragged_37x23_g3": (lambda: cavity_2d(n=37, ny=23, kn=0.01, particles=50_000), -3),
    "wide_300x50_w1": (lambda: cavity_2d(n=300, ny=50, kn=0.01, particles=100_000), 1),
    "wide_300x50_g1": (lambda: cavity_2d(n=300, ny=50, kn=0.01, particles=100_000), -1),
    "groups_300": (lambda: cavity_2d(n=300, kn=0.01, particles=200_000), 0),
    "groups_300_w12": (lambda: cavity_2d(n=300, kn=0.01, particles=200_000), 12),
    "groups_300_g12": (lambda: cavity_2d(n=300, kn=0.01, particles=200_000), -12),
    "groups_512": (lambda: cavity_2d(n=512, kn=0.005, particles=300_000), 0),
    "groups_600": (lambda: cavity_2d(n=600, kn=0.005, particles=300_000), 0),
}


@pytest.mark.parametrize("name", list(NEWTON_LAYOUTS))
def test_newton_cg_layouts_bitwise(oracle_mod, gpu, name):
    """One Newton iteration: CG iteration count, E and G bit-identical for every
    workgroup layout of the CG kernel."""
    make, waves = NEWTON_LAYOUTS[name]
    w = make()
    Dx, Dy = _diff(w)
    o, s = _pair(oracle_mod, gpu, w, newton=True, diff_x=Dx, diff_y=Dy,
                 tally_faces=oracle_mod.FACES_EVERY, cg_waves=waves)
    assert o.step(2) == 0 and s.step(2) == 0
    _same_iteration(o, s, name)
    assert o.info().cg_iters_total == s.stats()["cg_iters_total"]


def _batch_cases():
    ws = []
    kw = []
    w = cavity_2d(n=40, ny=33, kn=0.05, particles=150_000)
    ws.append(w); kw.append(dict(rng_mode=1, tally_faces=2, newton=True, max_iters=40, res_tol=1e-6))
    w = cavity_2d(n=17, kn=2.0, particles=40_000, newton=False, seed=5)
    ws.append(w); kw.append(dict(rng_mode=0, tally_faces=1, newton=False, max_iters=4, res_tol=0.0, avg_iters=3))
    w = slab_1d(kn=1.0, particles=100_000)
    ws.append(w); kw.append(dict(rng_mode=1, tally_faces=2, newton=False, max_iters=60, res_tol=1e-6))
    w = two_material_2d(n=24, kn_right=0.05, ratio=20.0, particles=80_000, seed=9)
    ws.append(w); kw.append(dict(rng_mode=0, tally_faces=0, newton=True, max_iters=3, res_tol=0.0))
    w = cavity_2d(n=64, kn=0.003, particles=2_000_000, seed=2)   # resolved: converges in 18
    ws.append(w); kw.append(dict(rng_mode=1, tally_faces=2, newton=True, max_iters=40, res_tol=1e-6))
    w = cavity_2d(n=9, ny=31, kn=0.5, particles=30_000, newton=False, seed=77)
    ws.append(w); kw.append(dict(rng_mode=1, tally_faces=1, newton=False, max_iters=0, res_tol=1e-6, avg_iters=2))
    return ws, kw


def test_batch_equals_single_solves(gpu):
    """The batched driver (one launch per phase for all instances, replayed from
    a captured graph, one-workgroup CG) gives every instance the bits of its
    own single solve: same iteration count, T and q."""
    ws, kws = _batch_cases()
    singles = []
    for w, k in zip(ws, kws):
        s = gpu.Solver(w, **k)
        rc, T, qx, qy, st = s.solve()
        singles.append((rc, T, qx, qy, st))
    bs = gpu.BatchSolver(ws, per_instance=kws)
    rc, outs = bs.solve()
    assert rc >= 0
    for i, ((rc_s, T, qx, qy, sst), (Tb, qxb, qyb, stb)) in enumerate(zip(singles, outs)):
        assert stb["iters"] == sst["iters"], f"instance {i} iterations"
        assert torch.equal(Tb, T), f"instance {i} T"
        assert torch.equal(qxb, qx), f"instance {i} qx"
        assert torch.equal(qyb, qy), f"instance {i} qy"
        assert stb["cg_iters_total"] == sst["cg_iters_total"]


def test_batch_solver_wrapper(gpu):
    """Uneven synthetic batch (sizes, Kn, walls drawn as for the benchmark, fewer
    particles): per-instance status, iterations and outputs equal the single
    solves, including instances whose Newton iteration diverges."""
    from synth import batch_workloads
    ws = batch_workloads(count=6, seed=11)
    for w in ws:
        w.particles_per_iter = min(w.particles_per_iter, 100_000)
    kw = dict(rng_mode=gpu.RNG_CRN, tally_faces=gpu.FACES_FINAL, max_iters=30, res_tol=1e-5)
    bs = gpu.BatchSolver(ws, **kw)
    rc, outs = bs.solve()
    statuses = []
    for i, (w, (T, qx, qy, st)) in enumerate(zip(ws, outs)):
        s = gpu.Solver(w, **kw)
        try:
            rc1, T1, qx1, qy1, st1 = s.solve()
        except gpu.IugkpError as e:
            assert st["status"] == e.code, f"instance {i}"
            assert st["iters"] == s.stats()["iters"]
            statuses.append(e.code)
            continue
        statuses.append(rc1)
        assert st["status"] == rc1
        assert torch.equal(T, T1) and torch.equal(qx, qx1) and torch.equal(qy, qy1)
        assert st["iters"] == st1["iters"]
    assert rc == (min(statuses) if min(statuses) < 0 else max(statuses))


def test_divergence_rule_matches_oracle(gpu, oracle_mod):
    """Under-resolved sampled maps (few particles leave a cell per iteration):
    the single solve, the batch and the oracle stop at the same iteration with
    DIVERGED and the same residual history; a resolved instance in the same
    batch converges as its single solve does."""
    import cp_model as cp
    ws = [slab_1d(n=100, kn=0.0003, particles=10 * 102, newton=True),
          cavity_2d(n=41, kn=0.00995, particles=10 * (41 * 41 + 164), newton=True, seed=13),
          slab_1d(n=100, kn=0.01, particles=100 * 102, newton=True)]
    kws = []
    for w in ws:
        lam = float(w.vg * w.tau[0])
        D = np.full(w.n_cells, cp.d_eff(lam, w.dx))
        kws.append(dict(rng_mode=1, newton=True, diff_x=D, diff_y=D if w.dim == 2 else None,
                        max_iters=60, res_tol=1e-6, tally_faces=2))
    expect = []
    for w, k in zip(ws, kws):
        o = oracle_mod.Oracle(w, **k)
        rc_o, To, _, _ = o.solve()
        it = o.info().iter
        expect.append((rc_o, it, o.residuals(it)))
        s = gpu.Solver(w, **k)
        try:
            rc_s = s.solve()[0]
        except gpu.IugkpError as e:
            rc_s = e.code
        assert rc_s == rc_o and s.stats()["iters"] == it
        assert np.array_equal(s.residuals(), o.residuals(it))
    assert [e[0] for e in expect] == [oracle_mod.E_DIVERGED, oracle_mod.E_DIVERGED, 0]
    bs = gpu.BatchSolver(ws, per_instance=kws)
    rc, outs = bs.solve()
    assert rc == oracle_mod.E_DIVERGED
    for (rc_o, it, _), (_, _, _, st) in zip(expect, outs):
        assert st["status"] == rc_o and st["iters"] == it
