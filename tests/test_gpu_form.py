"""The particle-step form search of a single solve (emitter tiles of 256 or
512 threads, or row stripes, timed one iteration each, then the fastest):
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


@pytest.mark.parametrize("make", [
    lambda: cavity_2d(n=61, ny=47, kn=0.05, particles=200_000, newton=False, seed=21),
    lambda: two_material_2d(n=53, kn_right=0.2, ratio=10.0, particles=200_000, seed=22),
], ids=["cavity_61x47", "two_material_53"])
def test_form_search_equals_tiles_and_is_kept(gpu, make):
    w = make()
    kw = dict(tally_faces=gpu.FACES_EVERY, rng_mode=gpu.RNG_CRN, newton=False)
    s = gpu.Solver(w, **kw)
    ref = gpu.Solver(w, march=1, **kw)               # the tile march, forced
    form, ms = s.march_tuning()
    assert form is None and all(v is None for v in ms.values())
    for it in range(5):
        assert s.step(1) == 0 and ref.step(1) == 0
        _same_tallies(s, ref)
        if it < 3:
            assert s.march_tuning()[0] is None       # still measuring
    form, ms = s.march_tuning()
    assert form in ("tiles256", "tiles512", "stripes")
    assert all(v is not None and v > 0.0 for v in ms.values())
    assert ms[form] == min(ms.values())
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
