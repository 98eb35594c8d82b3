"""The benchmark's full-size workloads against the oracle, bit for bit.

The expected values are SHA-256 digests of the oracle's arrays, written by
tests/golden/make_fullsize.py (which calls only the oracle):

  * the 256 x 256 gray cavity at Kn 0.01, 0.1, 1 and 10 with 1e7 particles per
    iteration, the Newton step with the multigrid-preconditioned CG and face
    tallies every iteration, in the launch configuration the benchmark times
    (automatic choice of emitter tiles or row stripes, own stream): the
    third iteration's D, W, Phi_x, Phi_y, B, then E and the next emission G,
    and the iteration's flight, segment and crossing counts and CG iterations;
  * the 512 x 512 gray two-material square (left half tau 100x the right) with
    5e7 particles, null collisions, from a seeded temperature field: the first
    iteration's tallies, E and G.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import cp_model as cp
from synth import cavity_2d, seeded_temperature, two_material_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_oracle.json")
KNS = (0.01, 0.1, 1.0, 10.0)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09465_amd as P
    P.library()
    return P


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _digest(t) -> str:
    a = np.ascontiguousarray(t.detach().cpu().numpy())
    return hashlib.sha256(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes()).hexdigest()


def _diffusion(w):
    lam = w.vg * np.asarray(w.tau)
    u, inv = np.unique(lam, return_inverse=True)
    Dx = np.array([cp.d_eff(l, w.dx) for l in u])[inv]
    Dy = np.array([cp.d_eff(l, w.dy) for l in u])[inv]
    return Dx, Dy


def _check(s, ref, name):
    t = s.tallies()
    _, _, E, G = s.state()
    st = s.stats()
    got = {k: _digest(v) for k, v in t.items()}
    got["E"] = _digest(E)
    got["G"] = _digest(G)
    for k in ("flights", "segments", "crossings"):
        assert st[k] == ref[k], f"{name}: {k} {st[k]} != {ref[k]}"
    assert st["iters"] == ref["iter"]
    bad = [k for k in ("D", "W", "Phix", "Phiy", "B", "E", "G") if got[k] != ref[k]]
    assert not bad, f"{name}: {bad} differ from the oracle"


@pytest.mark.parametrize("kn", KNS)
def test_cavity256_bench_configuration_vs_oracle(gpu, golden, kn):
    ref = golden[f"cavity256_kn{kn}"]
    w = cavity_2d(n=256, kn=kn, particles=10_000_000, newton=True, seed=0)
    Dx, Dy = _diffusion(w)
    s = gpu.Solver(w, newton=True, diff_x=Dx, diff_y=Dy, tally_faces=gpu.FACES_EVERY,
                   own_stream=True, cg_precond=gpu.PRECOND_MG)
    for _ in range(ref["iter"]):
        assert s.step(1) == 0
    assert s.stats()["cg_iters_last"] == ref["cg_iters_last"]
    _check(s, ref, f"cavity Kn {kn}")
    s.close()


def test_two_material512_vs_oracle(gpu, golden):
    ref = golden["two_material512"]
    w = two_material_2d(n=512, kn_right=0.01, ratio=100.0, particles=50_000_000, seed=0)
    s = gpu.Solver(w, newton=False, tally_faces=gpu.FACES_EVERY,
                   T_init=seeded_temperature(512 * 512))
    assert s.step(1) == 0
    _check(s, ref, "two-material 512")
    s.close()
