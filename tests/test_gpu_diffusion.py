"""The Newton step's increment equation solved through the stateless entry
point iugkp_diffusion_solve, against the oracle's CG (Sec. 3.3 operator, the
plain CG of reading R6) on the same inputs: every component of x and the
iteration count bit for bit, on 1D and 2D meshes that span several tree
blocks with a ragged tail, with varying tau and diffusion coefficients, and
the stopping rule's error."""
import numpy as np
import pytest

from synth import cavity_2d, slab_1d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


def _case(name):
    rng = np.random.default_rng(["one_cell", "slab_777", "rect_45x37", "cavity_256"].index(name))
    if name == "slab_777":
        w = slab_1d(n=777, kn=0.01)
    elif name == "rect_45x37":
        w = cavity_2d(n=45, ny=37, kn=0.05)
    elif name == "cavity_256":
        w = cavity_2d(n=256, kn=0.1)
    else:
        w = cavity_2d(n=1, ny=1, kn=0.3)
    w.tau = w.tau * rng.uniform(0.5, 2.0, size=w.tau.size)
    Dx = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-4
    Dy = rng.uniform(0.5, 2.0, size=w.tau.size) * 1e-4
    b = rng.normal(size=w.tau.size)
    return w, Dx, Dy, b


@pytest.mark.parametrize("name", ["one_cell", "slab_777", "rect_45x37", "cavity_256"])
def test_diffusion_solve_bitwise(gpu, oracle_mod, name):
    w, Dx, Dy, b = _case(name)
    rc_o, x_o, its_o = oracle_mod.cg(w, Dx, Dy if w.dim == 2 else None, b, tol=1e-10)
    rc, x, its = gpu.diffusion_solve(w, Dx, Dy, b, tol=1e-10)
    assert rc == rc_o == 0
    assert its == its_o
    assert np.array_equal(x.cpu().numpy(), x_o)


def test_diffusion_solve_stopping_rule(gpu, oracle_mod):
    w, Dx, Dy, b = _case("rect_45x37")
    _, _, its = oracle_mod.cg(w, Dx, Dy, b, tol=1e-10)
    rc_o, x_o, its_o = oracle_mod.cg(w, Dx, Dy, b, tol=1e-10, max_iters=its - 1)
    rc, x, its_g = gpu.diffusion_solve(w, Dx, Dy, b, tol=1e-10, max_iters=its - 1)
    assert rc == rc_o == oracle_mod.E_CG_NOT_CONVERGED
    assert its_g == its_o == its - 1
    assert np.array_equal(x.cpu().numpy(), x_o)
