"""Grouped stepping of independent solvers on their own streams
(iugkp_step_group): every result equals the same solver stepped alone, and
the group checks its arguments."""
import numpy as np
import pytest

from synth import cavity_2d, slab_1d, two_material_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _problems():
    return [(cavity_2d(n=64, kn=0.05, particles=300_000, seed=1), dict()),
            (cavity_2d(n=48, kn=3.0, particles=200_000, seed=2), dict(newton=False)),
            (slab_1d(n=80, kn=0.1, particles=50_000, seed=3), dict()),
            (two_material_2d(n=40, kn_right=0.02, ratio=30.0, particles=200_000, seed=4),
             dict(estimator=1))]


def test_group_equals_single_bitwise(gpu):
    import cp_model as cp

    def diff(w):
        lam = w.vg * np.asarray(w.tau)
        Dx = np.array([cp.d_eff(l, w.dx) for l in lam])
        Dy = np.array([cp.d_eff(l, w.dy) for l in lam]) if w.dim == 2 else None
        return Dx, Dy

    grouped, single = [], []
    for w, kw in _problems():
        kw = dict(kw)
        if kw.get("newton", w.newton):
            kw["diff_x"], kw["diff_y"] = diff(w)
        grouped.append(gpu.Solver(w, own_stream=True, tally_faces=gpu.FACES_EVERY, **kw))
        single.append(gpu.Solver(w, tally_faces=gpu.FACES_EVERY, **kw))
    assert gpu.step_group(grouped, 1) == 0
    assert gpu.step_group(grouped, 2) == 0
    for s in single:
        assert s.step(3) == 0
    for a, b in zip(grouped, single):
        ta, tb = a.tallies(), b.tallies()
        assert all(torch.equal(ta[k], tb[k]) for k in ta)
        sa, sb = a.state(), b.state()
        assert sa[0] == sb[0] and sa[1] == sb[1]
        assert torch.equal(sa[2], sb[2]) and torch.equal(sa[3], sb[3])
        assert a.stats()["cg_iters_total"] == b.stats()["cg_iters_total"]


def test_group_arguments(gpu):
    from paper_2506_09465_amd import _lib as L
    w = slab_1d(n=20, particles=5000)
    s = gpu.Solver(w, own_stream=True)
    assert gpu.step_group([s, s], 1) == L.E_INVALID_ARG
    assert gpu.step_group([s], 2) == 0
    assert s.stats()["iters"] == 2


def test_group_larger_than_the_device(gpu):
    """More multigrid CGs than fit on the device at once (ten 256^2 cavities,
    32 workgroups of one compute unit each): grouped stepping admits an
    iteration only while the CGs in flight fit, so every problem steps without
    a barrier time-out and equals the same problem stepped alone."""
    import cp_model as cp
    ws = [cavity_2d(n=256, kn=kn, particles=300_000, seed=i)
          for i, kn in enumerate((0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0))]
    kws = []
    for w in ws:
        D = np.full(w.n_cells, cp.d_eff(float(w.vg * w.tau[0]), w.dx))
        kws.append(dict(newton=True, diff_x=D, diff_y=D, tally_faces=gpu.FACES_EVERY,
                        cg_precond=gpu.PRECOND_MG))
    grouped = [gpu.Solver(w, own_stream=True, **k) for w, k in zip(ws, kws)]
    assert gpu.step_group(grouped, 3) == 0
    for w, k, a in zip(ws, kws, grouped):
        b = gpu.Solver(w, **k)
        assert b.step(3) == 0
        sa, sb = a.state(), b.state()
        assert torch.equal(sa[2], sb[2]) and torch.equal(sa[3], sb[3])
        assert a.stats()["cg_iters_total"] == b.stats()["cg_iters_total"]
        b.close()
    for a in grouped:
        a.close()
