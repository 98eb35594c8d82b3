"""The particle-step form search of a single solve (emitter tiles of 256 or
512 threads, row stripes, or row stripes with the crossings in pieces, timed
one iteration each, then the fastest):
every form gives the tallies of the forced tile march bit for bit, the choice
is kept for later handles of the same class, and a handle with a set block
size or march does not search."""
import numpy as np
import pytest

from synth import cavity_2d, two_material_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _same_tallies(a, b):
    ta, tb = a.tallies(), b.tallies()
    assert ta.keys() == tb.keys()
    for k in ta:
        assert np.array_equal(ta[k].cpu().numpy(), tb[k].cpu().numpy()), k


# (row stripes in pieces are a form only without null collisions)
@pytest.mark.parametrize("make,n_forms", [
    (lambda: cavity_2d(n=61, ny=47, kn=0.05, particles=200_000, newton=False, seed=21), 4),
    (lambda: two_material_2d(n=53, kn_right=0.2, ratio=10.0, particles=200_000, seed=22), 3),
], ids=["cavity_61x47", "two_material_53"])
def test_form_search_equals_tiles_and_is_kept(gpu, make, n_forms):
    w = make()
    kw = dict(tally_faces=gpu.FACES_EVERY, rng_mode=gpu.RNG_CRN, newton=False)
    s = gpu.Solver(w, **kw)
    ref = gpu.Solver(w, march=1, **kw)               # the tile march, forced
    form, ms = s.march_tuning()
    assert form is None and all(v is None for v in ms.values())
    for it in range(n_forms + 2):
        assert s.step(1) == 0 and ref.step(1) == 0
        _same_tallies(s, ref)
        if it < n_forms:
            assert s.march_tuning()[0] is None       # still measuring
    form, ms = s.march_tuning()
    measured = {k: v for k, v in ms.items() if v is not None}
    assert len(measured) == n_forms and all(v > 0.0 for v in measured.values())
    assert form in measured and ms[form] == min(measured.values())
    # a later handle of the same class starts with the choice
    s2 = gpu.Solver(w, **kw)
    assert s2.march_tuning()[0] == form
    assert s2.step(2) == 0
    s3 = gpu.Solver(w, **kw)
    assert s3.step(2) == 0
    _same_tallies(s2, s3)
    # a set block size (or march) keeps the planner's form: no search
    s4 = gpu.Solver(w, block_size=256, **kw)
    f4, ms4 = s4.march_tuning()
    assert f4 is not None and all(v is None for v in ms4.values())
    for h in (s, ref, s2, s3, s4):
        h.close()


def test_batch_tile_edges_are_measured_then_kept(gpu):
    """A batch measures the tile edge of each instance class (8 or 16 cells,
    replays two and three), a second batch of the same classes starts with
    the edges, and both batches give the single solves' temperatures."""
    ws = [cavity_2d(n=71, ny=43, kn=0.02, particles=150_000, seed=31),
          two_material_2d(n=57, kn_right=0.05, ratio=20.0, particles=150_000, seed=32),
          cavity_2d(n=37, ny=29, kn=0.3, particles=60_000, seed=33)]
    kw = dict(rng_mode=gpu.RNG_CRN, tally_faces=gpu.FACES_FINAL, max_iters=8, res_tol=0.0,
              newton=False)
    singles = []
    for w in ws:
        s = gpu.Solver(w, block_size=256, **kw)
        rc, T, qx, qy, _ = s.solve()
        singles.append((rc, T.cpu().numpy(), qx.cpu().numpy(), qy.cpu().numpy()))
        s.close()
    edges = []
    for _ in range(2):
        bs = gpu.BatchSolver(ws, **kw)
        rc, outs = bs.solve()
        e = bs.tile_edges()
        assert set(e.tolist()) <= {8, 16}
        edges.append(e.tolist())
        for (rc1, T1, qx1, qy1), (T2, qx2, qy2, st) in zip(singles, outs):
            assert st["status"] == rc1
            assert np.array_equal(T1, T2.cpu().numpy())
            assert np.array_equal(qx1, qx2.cpu().numpy())
            assert np.array_equal(qy1[:len(qy2)], qy2.cpu().numpy()[:len(qy1)])
        bs.close()
    assert edges[0] == edges[1]
