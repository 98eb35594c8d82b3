"""The no-allocation entry point iugkp_diffusion_solve_noalloc through the C
ABI against iugkp_diffusion_solve (which allocates its scratch per call): the
same x bit for bit and the same CG iteration count on two calls in a row, the
second on a smaller mesh (the shared scratch keeps the first call's contents),
and a mesh whose scratch does not fit is refused before any device work."""
import ctypes as C

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


def _inputs(w, seed):
    rng = np.random.default_rng(seed)
    w.tau = w.tau * rng.uniform(0.5, 2.0, size=w.tau.size)
    n = w.tau.size
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    return (f(w.tau), f(rng.uniform(0.5, 2.0, size=n) * 1e-4),
            f(rng.uniform(0.5, 2.0, size=n) * 1e-4), f(rng.normal(size=n)))


def _call(L, name, w, tau, Dx, Dy, b, tol=1e-10, max_iters=200_000):
    x = torch.full_like(b, float("nan"))
    its = C.c_int(-1)
    fn = getattr(L.lib(), name)
    rc = fn(int(w.dim), int(w.nx), int(w.ny), float(w.dx), float(w.dy), float(w.vg),
            tau.data_ptr(), Dx.data_ptr(), Dy.data_ptr() if w.dim == 2 else None, b.data_ptr(),
            x.data_ptr(), float(tol), int(max_iters), C.addressof(its),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, x, its.value


def test_no_alloc_equals_allocating_entry_point(gpu):
    from paper_2506_09465_amd import _lib as L
    cases = [(cavity_2d(n=200, ny=150, kn=0.02), 1),      # 30000 cells
             (slab_1d(n=777, kn=0.01), 2)]               # then a smaller one
    for w, seed in cases:
        tau, Dx, Dy, b = _inputs(w, seed)
        rc_a, x_a, its_a = _call(L, "iugkp_diffusion_solve", w, tau, Dx, Dy, b)
        rc_n, x_n, its_n = _call(L, "iugkp_diffusion_solve_noalloc", w, tau, Dx, Dy, b)
        assert rc_a == rc_n == L.OK
        assert its_a == its_n > 0
        assert torch.equal(x_a, x_n)
    # the stopping rule's error, also from the no-allocation entry point
    w, seed = cases[0]
    tau, Dx, Dy, b = _inputs(cavity_2d(n=200, ny=150, kn=0.02), 1)
    rc_a, x_a, its_a = _call(L, "iugkp_diffusion_solve", w, tau, Dx, Dy, b, max_iters=7)
    rc_n, x_n, its_n = _call(L, "iugkp_diffusion_solve_noalloc", w, tau, Dx, Dy, b, max_iters=7)
    assert rc_a == rc_n == L.E_CG_NOT_CONVERGED and its_a == its_n == 7
    assert torch.equal(x_a, x_n)


def test_no_alloc_refuses_oversized_mesh(gpu):
    from paper_2506_09465_amd import _lib as L
    w = cavity_2d(n=300, kn=0.02)                        # 90000 cells: scratch too small
    tau, Dx, Dy, b = _inputs(w, 3)
    rc, x, its = _call(L, "iugkp_diffusion_solve_noalloc", w, tau, Dx, Dy, b)
    assert rc == L.E_INVALID_ARG
    assert "no-allocation scratch" in L.lib().iugkp_last_error().decode()
    assert torch.isnan(x).all()                          # nothing was written
    # the allocating entry point takes it, and the no-allocation one still works after
    rc, _, _ = _call(L, "iugkp_diffusion_solve", w, tau, Dx, Dy, b)
    assert rc == L.OK
    w2 = slab_1d(n=300, kn=0.02)
    t2 = _inputs(w2, 4)
    rc_a, x_a, _ = _call(L, "iugkp_diffusion_solve", w2, *t2)
    rc_n, x_n, _ = _call(L, "iugkp_diffusion_solve_noalloc", w2, *t2)
    assert rc_a == rc_n == L.OK and torch.equal(x_a, x_n)
