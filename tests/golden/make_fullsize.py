"""Write fullsize_oracle.json: the oracle's results on the benchmark's full-size
workloads, as SHA-256 digests of the little-endian bytes of every array plus
the counters of the pinned iteration.

  * 256 x 256 gray cavity (hot top wall 1.01, others 0.99), Kn 0.01, 0.1, 1,
    10, 1e7 particles per iteration, seed 0, fresh random numbers, Newton step
    with the multigrid-preconditioned CG (tol 1e-10), face tallies every
    iteration, started from T = T_ref: tallies D, W, Phi_x, Phi_y, B of the
    third iteration, then E and the next emission G.
  * 512 x 512 gray two-material square (left half tau 100x the right half,
    Kn 0.01 on the right), 5e7 particles per iteration, seed 0, no Newton step,
    face tallies, started from the seeded field `synth.seeded_temperature`:
    the first iteration's tallies, E and G.

The diffusion coefficient of the Newton operator is problem data given to
both sides (the flat-cell second moment, tests/cp_model.py).  Only the oracle
computes the values stored here.  Run from the repository root:

    python tests/golden/make_fullsize.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

from oracle import oracle as O          # noqa: E402
import cp_model as cp                   # noqa: E402
from synth import cavity_2d, seeded_temperature, two_material_2d   # noqa: E402

OUT = os.path.join(HERE, "fullsize_oracle.json")
KNS = (0.01, 0.1, 1.0, 10.0)
CAVITY_ITERS = 3


def digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes()).hexdigest()


def diffusion(w):
    lam = w.vg * np.asarray(w.tau)
    u, inv = np.unique(lam, return_inverse=True)
    Dx = np.array([cp.d_eff(l, w.dx) for l in u])[inv]
    Dy = np.array([cp.d_eff(l, w.dy) for l in u])[inv]
    return Dx, Dy


def record(o) -> dict:
    t = o.tallies()
    info = o.info()
    r = {k: digest(v) for k, v in t.items()}
    r["E"] = digest(o.E())
    r["G"] = digest(o.G())
    r.update(iter=info.iter, flights=info.flights, segments=info.segments,
             crossings=info.crossings, cg_iters_last=info.cg_iters_last, F=info.F,
             n_per_emitter=info.n_per_emitter)
    return r


def main():
    O.build()
    out = {}
    for kn in KNS:
        w = cavity_2d(n=256, kn=kn, particles=10_000_000, newton=True, seed=0)
        Dx, Dy = diffusion(w)
        t = time.time()
        o = O.Oracle(w, newton=True, diff_x=Dx, diff_y=Dy, tally_faces=O.FACES_EVERY,
                     cg_precond=O.PRECOND_MG)
        for _ in range(CAVITY_ITERS):
            rc = o.step(1)
            assert rc == 0, rc
        out[f"cavity256_kn{kn}"] = record(o)
        print(f"cavity Kn {kn}: {time.time() - t:.1f} s", flush=True)
    w = two_material_2d(n=512, kn_right=0.01, ratio=100.0, particles=50_000_000, seed=0)
    t = time.time()
    o = O.Oracle(w, newton=False, tally_faces=O.FACES_EVERY, T_init=seeded_temperature(512 * 512))
    rc = o.step(1)
    assert rc == 0, rc
    out["two_material512"] = record(o)
    print(f"two-material 512: {time.time() - t:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
