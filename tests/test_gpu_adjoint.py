"""GPU: the volumetric source in the forward step and the adjoint of the
steady state, through the C ABI, against the CPU oracle (bit for bit) and
against central finite differences / a dense transfer matrix built on the
GPU itself."""
import numpy as np
import pytest

import cp_model as cp
from synth import cavity_2d, slab_1d, gaussian_source, adjoint_case
from test_gpu_parity import _diff, _np, _pair, _same_iteration

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _with_source(w, amp=0.03, width=0.2):
    w.source = gaussian_source(w.nx, w.ny, w.dx, w.dy, amp, width)
    return w


@pytest.mark.parametrize("newton", [False, True])
def test_source_iterations_bitwise(oracle_mod, gpu, newton):
    w = _with_source(cavity_2d(n=37, ny=23, kn=0.05, particles=120_000, newton=False))
    kw = dict(rng_mode=oracle_mod.FRESH, tally_faces=oracle_mod.FACES_EVERY)
    if newton:
        Dx, Dy = _diff(w)
        kw.update(newton=True, diff_x=Dx, diff_y=Dy)
    o, s = _pair(oracle_mod, gpu, w, **kw)
    assert o.step(3) == 0 and s.step(3) == 0
    _same_iteration(o, s, f"source newton={newton}")


def test_source_solve_bitwise_1d(oracle_mod, gpu):
    w = slab_1d(n=60, kn=0.2, particles=60_000)
    w.source = 0.05 * np.ones(60)
    o, s = _pair(oracle_mod, gpu, w, rng_mode=oracle_mod.CRN, max_iters=60, res_tol=1e-9,
                 tally_faces=oracle_mod.FACES_FINAL)
    rc_o, To, qxo, _ = o.solve()
    rc, T, qx, _, st = s.solve()
    assert rc_o == rc          # the iteration cap is reached on both sides
    assert st["iters"] == o.info().iter
    assert np.array_equal(To, _np(T)) and np.array_equal(qxo, _np(qx))


def test_batch_with_source_equals_single(gpu):
    ws, kws = [], []
    for i, (n, kn) in enumerate(((24, 0.2), (40, 0.02), (17, 1.5))):
        w = _with_source(cavity_2d(n=n, kn=kn, particles=80_000, seed=i))
        ws.append(w)
        kws.append(dict(rng_mode=gpu.RNG_CRN, tally_faces=gpu.FACES_FINAL, newton=(i != 2),
                        max_iters=50, res_tol=1e-7))
    singles = [gpu.Solver(w, **k).solve() for w, k in zip(ws, kws)]
    rc, outs = gpu.BatchSolver(ws, per_instance=kws).solve()
    assert rc >= 0
    for (rc_s, T, qx, qy, st), (Tb, qxb, qyb, stb) in zip(singles, outs):
        assert st["iters"] == stb["iters"]
        assert torch.equal(T, Tb) and torch.equal(qx, qxb) and torch.equal(qy, qyb)


@pytest.mark.parametrize("newton", [False, True, "mg"])
def test_adjoint_bitwise_vs_oracle(oracle_mod, gpu, newton):
    """Forward solve and adjoint against the oracle, without the Newton step,
    with it (plain CG) and with the multigrid-preconditioned CG."""
    w = _with_source(cavity_2d(n=14, ny=11, kn=0.3, particles=50_000, newton=False))
    kw = dict(rng_mode=oracle_mod.CRN, max_iters=400, res_tol=1e-10,
              tally_faces=oracle_mod.FACES_OFF)
    if newton:
        Dx, Dy = _diff(w)
        kw.update(newton=True, diff_x=Dx, diff_y=Dy)
    if newton == "mg":
        kw.update(cg_precond=oracle_mod.PRECOND_MG)
    o, s = _pair(oracle_mod, gpu, w, **kw)
    rc_o, To, _, _ = o.solve()
    rc, T, _, _, _ = s.solve()
    assert rc_o == rc == 0 and np.array_equal(To, _np(T))
    rng = np.random.default_rng(1)
    dLdT = np.zeros(w.n_cells)
    probes = rng.choice(w.n_cells, 9, replace=False)
    dLdT[probes] = rng.normal(size=9)
    rc_o, gw_o, gs_o, it_o = o.adjoint(dLdT, max_iters=500, tol=1e-11)
    rc, gw, gs, it = s.adjoint(torch.tensor(dLdT), max_iters=500, tol=1e-11)
    assert rc_o == rc == 0 and it_o == it
    assert np.array_equal(gw_o, _np(gw)), np.max(np.abs(gw_o - _np(gw)))
    assert np.array_equal(gs_o, _np(gs)), np.max(np.abs(gs_o - _np(gs)))


def test_adjoint_dense_transfer_16x16(gpu):
    """Gradient of the probe misfit against a dense transfer matrix assembled on
    the GPU from unit-impulse iterations (one emitter emitting at a time)."""
    n = 16
    w = _with_source(cavity_2d(n=n, kn=0.1, particles=64_000, newton=False), 0.02, 0.05)
    nc, nb = w.n_cells, w.n_bfaces
    ne = nc + nb
    imp = gpu.Solver(w, rng_mode=gpu.RNG_CRN, tally_faces=gpu.FACES_OFF)
    N = imp.stats()["n_per_emitter"]
    q = 1 << 20
    Tm = np.zeros((nc, ne))
    for e in range(ne):
        G = np.zeros(ne, np.int64)
        G[e] = q * N
        assert imp.set_state(0, 0.0, np.zeros(nc), G) == 0
        assert imp.step(1, faces=False) == 0
        Tm[:, e] = _np(imp.tallies()["D"]) / float(q * N)
    s = gpu.Solver(w, rng_mode=gpu.RNG_CRN, tally_faces=gpu.FACES_OFF, max_iters=3000,
                   res_tol=1e-13)
    rc, T, _, _, st = s.solve()
    assert rc == 0
    F = st["fixed_point_F"]
    V = w.dx * w.dy
    tmin = float(w.tau[0])
    lam = w.vg * tmin
    A_f = np.where(np.arange(nb) < 2 * w.ny, w.dy, w.dx)
    Gw = np.ldexp(w.cv * (w.wall_T - w.t_ref) * lam * A_f / 4.0, F)
    Gs = np.ldexp(w.source * V * tmin, F)
    Tcc, Tcw = Tm[:, :nc], Tm[:, nc:]
    Dst = np.linalg.solve(np.eye(nc) - Tcc, Tcc @ Gs + Tcw @ Gw)
    Tst = w.t_ref + np.ldexp(Dst, -F) / V / w.cv
    assert np.max(np.abs(_np(T) - Tst)) < 1e-12
    rng = np.random.default_rng(2)
    probes = rng.choice(nc, 12, replace=False)
    target = rng.uniform(0.99, 1.01, 12)
    dLdT = np.zeros(nc)
    dLdT[probes] = 2.0 * (Tst[probes] - target)
    psi = np.linalg.solve((np.eye(nc) - Tcc).T, np.ldexp(dLdT / w.cv / V, -F))
    g_src = (Tcc.T @ psi) * np.ldexp(V * tmin, F)
    g_wall = (Tcw.T @ psi) * np.ldexp(w.cv * lam * A_f / 4.0, F)
    rc, gw, gs, _ = s.adjoint(torch.tensor(dLdT), max_iters=3000, tol=1e-13)
    assert rc == 0
    assert np.max(np.abs(_np(gs) - g_src)) < 1e-9 * np.max(np.abs(g_src))
    assert np.max(np.abs(_np(gw) - g_wall)) < 1e-9 * np.max(np.abs(g_wall))


def test_adjoint_vs_finite_differences_256(gpu):
    """The adjoint workload: 256 x 256 cavity at Kn = 0.1 with a Gaussian source,
    misfit at 64 random probes; autograd gradient vs central differences with
    common random numbers (h = 1e-4) for the four walls and four source cells."""
    case = adjoint_case(n=256, kn=0.1, n_probes=64, particles=10_000_000)
    w = case.workload
    dev = torch.device("cuda")
    probes = torch.tensor(case.probes, device=dev)
    target = torch.tensor(case.target, device=dev)
    opts = dict(max_iters=200, res_tol=1e-9, newton=True)

    def loss_of(walls, src):
        T = gpu.steady_temperature(walls, src, w, **opts)
        return ((T[probes] - target) ** 2).sum()

    walls = torch.tensor(case.walls4, device=dev, requires_grad=True)
    src = torch.tensor(w.source, device=dev, requires_grad=True)
    L0 = loss_of(walls, src)
    L0.backward()
    gwalls, gsrc = walls.grad.clone(), src.grad.clone()
    h = 1e-4
    with torch.no_grad():
        for i in range(4):
            wp, wm = walls.detach().clone(), walls.detach().clone()
            wp[i] += h
            wm[i] -= h
            fd = (loss_of(wp, src.detach()) - loss_of(wm, src.detach())).item() / (2 * h)
            assert abs(gwalls[i].item() - fd) <= 1e-3 * abs(fd), (i, gwalls[i].item(), fd)
        cells = [int(case.probes[0]), int(case.probes[1]), 128 * 256 + 128, 37]
        for c in cells:
            sp, sm = src.detach().clone(), src.detach().clone()
            sp[c] += h
            sm[c] -= h
            fd = (loss_of(walls.detach(), sp) - loss_of(walls.detach(), sm)).item() / (2 * h)
            assert abs(gsrc[c].item() - fd) <= 1e-3 * abs(fd) + 1e-18, (c, gsrc[c].item(), fd)


def test_adjoint_rejects_unsupported(gpu):
    w = cavity_2d(n=8, kn=0.5, particles=5_000, newton=False)
    s = gpu.Solver(w, rng_mode=gpu.RNG_FRESH)
    with pytest.raises(gpu.IugkpError) as e:
        s.adjoint(torch.ones(64))
    assert e.value.code == -1
    w.tau[5] *= 3.0
    s = gpu.Solver(w, rng_mode=gpu.RNG_CRN)
    with pytest.raises(gpu.IugkpError) as e:
        s.adjoint(torch.ones(64))
    assert e.value.code == -1
