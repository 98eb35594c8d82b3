"""The benchmark configurations at full size, in the launch configuration
bench.py times, checked through properties that hold exactly at any size
(integer tallies, so every check is an equality):

  * energy: every emitted weight ends in a cell or a wall face,
    sum D + sum B = sum G;
  * face balance: the net inflow through each cell's faces is D - G;
  * emission: the next emission is rint(2^F (E V) tau_min / tau) after the
    Newton step (uniform tau: ratio 1), or D without it;
  * the 2D gray cavity's four Kn problems stepped as a group equal the same
    problems stepped alone;
  * the emitter-tile and row-stripe particle steps give equal tallies.
"""
import numpy as np
import pytest

from synth import cavity_2d, two_material_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KNS = (0.01, 0.1, 1.0, 10.0)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _face_balance(w, t, G):
    nx, ny, nc = w.nx, w.ny, w.nx * w.ny
    Px = t["Phix"].view(ny, nx + 1)
    inflow = (Px[:, :-1] - Px[:, 1:]).reshape(-1)
    if w.dim == 2:
        Py = t["Phiy"].view(ny + 1, nx)
        inflow = inflow + (Py[:-1, :] - Py[1:, :]).reshape(-1)
    assert torch.equal(inflow, t["D"] - G[:nc])


def test_cavity_256_grouped_bench_configuration(gpu):
    """The four 256^2 cavities at 1e7 particles, Newton on, face tallies every
    iteration, own streams, iugkp_step_group: exact energy and face balance per
    problem and iteration, the Newton emission rule, and bitwise equality with
    the same problems stepped one at a time."""
    ws = [cavity_2d(n=256, kn=kn, particles=10_000_000, newton=True, seed=0) for kn in KNS]
    grouped = [gpu.Solver(w, tally_faces=gpu.FACES_EVERY, own_stream=True,
                          cg_precond=gpu.PRECOND_MG) for w in ws]
    for it in range(2):
        G0 = [s.state()[3] for s in grouped]
        assert gpu.step_group(grouped, 1) == 0
        for w, s, g in zip(ws, grouped, G0):
            t = s.tallies()
            assert int(t["D"].sum()) + int(t["B"].sum()) == int(g.sum())
            _face_balance(w, t, g)
            st = s.stats()
            F = st["fixed_point_F"]
            _, _, E, G1 = s.state()
            want = torch.round(torch.ldexp(E * (w.dx * w.dy), torch.tensor(F, device=E.device)))
            assert torch.equal(G1[: w.nx * w.ny], want.to(torch.int64))
    single = [gpu.Solver(w, tally_faces=gpu.FACES_EVERY, cg_precond=gpu.PRECOND_MG) for w in ws]
    for s in single:
        assert s.step(2) == 0
    for a, b in zip(grouped, single):
        sa, sb = a.state(), b.state()
        assert torch.equal(sa[2], sb[2]) and torch.equal(sa[3], sb[3])


@pytest.mark.parametrize("kn", (0.03, 0.1, 1.0))
def test_cavity_256_tiles_equal_stripes(gpu, kn):
    """The two particle-step kernels on the 256^2 cavity at 1e7 particles,
    from the same state: emitter tiles walking every flight face by face, and
    row stripes marching pre-sampled records with closed-form segment ends
    (the automatic choice from Kn 0.03 here).  Two Newton iterations give
    bitwise equal cell, wall and face tallies, energy and emission."""
    w = cavity_2d(n=256, kn=kn, particles=10_000_000, newton=True, seed=0)
    a = gpu.Solver(w, tally_faces=gpu.FACES_EVERY, cg_precond=gpu.PRECOND_MG, march=1)
    bs = [gpu.Solver(w, tally_faces=gpu.FACES_EVERY, cg_precond=gpu.PRECOND_MG, march=m)
          for m in (2, 3)]     # row stripes; row stripes with the crossings in pieces
    for it in range(2):
        assert a.step(1) == 0
        ta, sa = a.tallies(), a.state()
        for b in bs:
            assert b.step(1) == 0
            tb = b.tallies()
            for k in ("D", "B", "Phix", "Phiy"):
                assert torch.equal(ta[k], tb[k]), (kn, it, k)
            sb = b.state()
            assert torch.equal(sa[2], sb[2]) and torch.equal(sa[3], sb[3]), (kn, it)
            assert a.stats()["flights"] == b.stats()["flights"]
    for h in [a] + bs:
        h.close()


def test_two_material_512_gray_full_size(gpu):
    """512^2 two-material square, left-half tau 100x the right (99% null
    collisions there), Kn 0.01 on the right, 5e7 particles per iteration, no
    Newton: exact energy and face balance, and re-emission of D."""
    w = two_material_2d(n=512, kn_right=0.01, ratio=100.0, particles=50_000_000)
    s = gpu.Solver(w, tally_faces=gpu.FACES_EVERY, newton=False)
    for _ in range(2):
        G0 = s.state()[3]
        assert s.step(1) == 0
        t = s.tallies()
        assert int(t["D"].sum()) + int(t["B"].sum()) == int(G0.sum())
        _face_balance(w, t, G0)
        G1 = s.state()[3]
        assert torch.equal(G1[: w.nx * w.ny], t["D"])
    st = s.stats()
    assert 0 < st["flights"] <= 49_932_288
    assert st["segments"] > st["flights"]          # the left half's null segments
