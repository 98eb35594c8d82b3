"""GPU: the closed-form segment walk (iterations without face tallies) against
the oracle's face-by-face walk, on adversarial rays and on whole iterations."""
import numpy as np
import pytest

from synth import cavity_2d, slab_1d, two_material_2d
from test_gpu_parity import _diff, _np, _pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


class _Mesh:
    def __init__(self, dim, nx, ny, dx, dy):
        self.dim, self.nx, self.ny, self.dx, self.dy = dim, nx, ny, dx, dy
        self.tau = np.ones(nx * ny)
        self.wall_T = np.ones(2 * ny + (2 * nx if dim == 2 else 0))
        self.t_ref, self.cv, self.vg, self.T_init = 1.0, 1.0, 1.0, None


def _rays(mesh, rng, n):
    """Random rays plus the degenerate cases the walk has to get right."""
    nx, ny, dx, dy = mesh.nx, mesh.ny, mesh.dx, mesh.dy
    out = []
    for _ in range(n):
        ix, iy = int(rng.integers(nx)), int(rng.integers(ny))
        x0 = (ix + rng.random()) * dx
        y0 = (iy + rng.random()) * dy if mesh.dim == 2 else 0.5 * dy
        th = rng.uniform(0, 2 * np.pi)
        sx, sy = np.cos(th), (np.sin(th) if mesh.dim == 2 else 0.0)
        if mesh.dim == 1:
            sx = rng.choice([-1.0, 1.0]) * rng.random()
        ell = rng.exponential(rng.choice([0.3, 3.0, 30.0, 300.0])) * dx
        out.append((x0, y0, ix, iy, sx, sy, ell))
    if mesh.dim == 2:
        # vertex ties (dx == dy): start at a cell centre, 45 degrees
        for ix in range(0, nx, max(1, nx // 7)):
            for iy in range(0, ny, max(1, ny // 5)):
                for sx, sy in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
                    for ell in (0.5 * dx, 1.5 * dx, 3 * dx, 1e3 * dx):
                        out.append(((ix + 0.5) * dx, (iy + 0.5) * dy, ix, iy,
                                    sx / np.sqrt(2), sy / np.sqrt(2), ell))
        # axis-aligned rays, rays on a face line, lengths ending exactly on faces
        for ix in range(nx):
            iy = ix % ny
            out.append(((ix + 0.25) * dx, iy * dy, ix, iy, 1.0, 0.0, 7.75 * dx))
            out.append(((ix + 0.25) * dx, (iy + 0.5) * dy, ix, iy, 0.0, -1.0, 5.5 * dy))
            out.append(((ix + 0.25) * dx, (iy + 0.5) * dy, ix, iy, 1.0, 0.0, 0.75 * dx))
            out.append(((ix + 0.5) * dx, (iy + 0.5) * dy, ix, iy, 0.6, 0.8, 40.0 * dx))
        # wall starts (as wall emission) into the domain, and towards the corners
        for iy in range(ny):
            out.append((0.0, (iy + 0.5) * dy, 0, iy, 0.8, 0.6, 1e4 * dx))
            out.append((nx * dx, (iy + 0.5) * dy, nx - 1, iy, -0.8, -0.6, 1e4 * dx))
        cx, cy = nx * dx, ny * dy
        for ix in range(nx):
            x0 = (ix + 0.5) * dx
            d = np.array([cx - x0, cy - 0.5 * dy])
            d /= np.linalg.norm(d)
            out.append((x0, 0.5 * dy, ix, 0, d[0], d[1], 1e4 * dx))
    return np.array(out, dtype=np.float64)


@pytest.mark.parametrize("shape", [(2, 16, 16, 1 / 16, 1 / 16), (2, 37, 23, 0.01, 0.01),
                                   (2, 9, 31, 0.3, 0.07), (2, 1, 9, 0.5, 0.5),
                                   (1, 100, 1, 0.01, 1.0)])
def test_segment_jump_equals_walk(oracle_mod, gpu, shape):
    mesh = _Mesh(*shape)
    rays = _rays(mesh, np.random.default_rng(sum(shape[:3])), 3000)
    got = _np(gpu.dev_segments(mesh.dim, mesh.nx, mesh.ny, mesh.dx, mesh.dy,
                               torch.tensor(rays, device="cuda")))
    for i, r in enumerate(rays):
        ev, kind, cell = oracle_mod.trace_ray(mesh, r[0], r[1], int(r[2]), int(r[3]), r[4], r[5],
                                              r[6], max_events=200000)
        assert (got[i, 0], got[i, 1], got[i, 2]) == (kind, cell, len(ev)), (i, r, got[i], kind,
                                                                            cell, len(ev))


@pytest.mark.parametrize("case", ["cavity_kn10", "cavity_kn1_ragged", "two_material_null",
                                  "slab_kn5", "strip_1x9"])
def test_iterations_without_faces_bitwise(oracle_mod, gpu, case):
    w = {"cavity_kn10": lambda: cavity_2d(n=40, kn=10.0, particles=200_000, newton=False),
         "cavity_kn1_ragged": lambda: cavity_2d(n=37, ny=23, kn=1.0, particles=150_000,
                                                newton=False),
         "two_material_null": lambda: two_material_2d(n=32, kn_right=0.5, ratio=20.0,
                                                      particles=150_000),
         "slab_kn5": lambda: slab_1d(n=100, kn=5.0, particles=100_000),
         "strip_1x9": lambda: cavity_2d(n=1, ny=9, kn=3.0, particles=20_000, newton=False)}[case]()
    o, s = _pair(oracle_mod, gpu, w, tally_faces=oracle_mod.FACES_OFF)
    assert o.step(3, faces=False) == 0 and s.step(3, faces=False) == 0
    to = o.tallies()
    ts = {k: _np(v) for k, v in s.tallies().items()}
    for k in ("D", "W", "B"):
        assert np.array_equal(to[k], ts[k]), f"{case} {k}"
    oi, st = o.info(), s.stats()
    assert (oi.flights, oi.segments, oi.crossings) == (st["flights"], st["segments"], st["crossings"])
    it, d0, E, G = s.state()
    assert np.array_equal(o.E(), _np(E)) and np.array_equal(o.G(), _np(G))


STRIPE_CASES = {
    # name: (workload, options) -- face-tallied iterations on the row-stripe particle step
    "cavity_kn10": (lambda: cavity_2d(n=40, kn=10.0, particles=300_000, newton=False), {}),
    "cavity_kn0.3_ragged": (lambda: cavity_2d(n=37, ny=23, kn=0.3, particles=200_000,
                                              newton=False), {}),
    "two_material_null": (lambda: two_material_2d(n=48, kn_right=0.3, ratio=10.0,
                                                  particles=300_000), {}),
    "strip_1x9": (lambda: cavity_2d(n=1, ny=9, kn=3.0, particles=20_000, newton=False), {}),
    "wide_300x7": (lambda: cavity_2d(n=300, ny=7, kn=2.0, particles=200_000, newton=False), {}),
    "tall_9x300": (lambda: cavity_2d(n=9, ny=300, kn=2.0, particles=200_000, newton=False), {}),
    "newton_kn1": (lambda: cavity_2d(n=64, kn=1.0, particles=400_000, newton=False), "newton"),
    # rows 2400 cells long: a few rows per stripe, several stripes, flights
    # crossing them and ending on the y walls (without and with null collisions)
    "wide_2400x30_stripes": (lambda: cavity_2d(n=2400, ny=30, kn=0.05, particles=300_000,
                                               newton=False), {}),
    "wide_2400x30_null": (lambda: _wide_null(), {}),
}


def _wide_null():
    w = cavity_2d(n=2400, ny=30, kn=0.05, particles=300_000, newton=False)
    ix = np.tile(np.arange(2400), 30)
    w.tau = np.where(ix < 800, 10.0 * np.asarray(w.tau), np.asarray(w.tau))
    return w


# march 2: each lane runs its particles' crossings; march 3: the crossings cut
# into pieces, one per lane (flights without null collisions; with them as 2)
@pytest.mark.parametrize("name", list(STRIPE_CASES))
@pytest.mark.parametrize("march", [2, 3])
def test_stripe_march_bitwise(oracle_mod, gpu, name, march):
    """Row stripes (forced) against the oracle, faces tallied every iteration:
    all tallies, counters and the state bit for bit."""
    make, extra = STRIPE_CASES[name]
    w = make()
    kw = dict(tally_faces=oracle_mod.FACES_EVERY)
    if extra == "newton":
        Dx, Dy = _diff(w)
        kw.update(newton=True, diff_x=Dx, diff_y=Dy)
    o, s = _pair(oracle_mod, gpu, w, march=march, **kw)
    assert o.step(2) == 0 and s.step(2) == 0
    to = o.tallies()
    ts = {k: _np(v) for k, v in s.tallies().items()}
    for k in ("D", "W", "Phix", "Phiy", "B"):
        assert np.array_equal(to[k], ts[k]), f"{name} {k}"
    oi, st = o.info(), s.stats()
    assert (oi.flights, oi.segments, oi.crossings) == (st["flights"], st["segments"], st["crossings"])
    it, d0, E, G = s.state()
    assert np.array_equal(o.E(), _np(E)) and np.array_equal(o.G(), _np(G))


def test_stripe_and_tile_marches_agree_256(gpu):
    """On the 256 x 256 cavity at Kn = 10 both particle steps give identical
    tallies (forced tiles vs forced stripes)."""
    w = cavity_2d(n=256, kn=10.0, particles=10_000_000, newton=False)
    out = []
    for march in (1, 2, 3):
        s = gpu.Solver(w, march=march, tally_faces=gpu.FACES_EVERY)
        assert s.step(2) == 0
        out.append({k: _np(v) for k, v in s.tallies().items()} | {"st": s.stats()})
    for o in out[1:]:
        for k in ("D", "Phix", "Phiy", "B"):
            assert np.array_equal(out[0][k], o[k]), k
        assert out[0]["st"]["crossings"] == o["st"]["crossings"]
