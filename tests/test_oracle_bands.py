"""Oracle: frequency bands (beyond the paper's gray model; readings in the
oracle header).  Pins: the expected steady state from the exact E_3 kernels
of every band (collision-probability model, dense solve), the equilibrium
case, exact per-band energy conservation, and the gray limit."""
import math

import numpy as np
import pytest

import cp_model as cp
from synth import slab_1d, slab_1d_bands, nongray_two_material_2d


def _fresh_average(o, burn, n, nb=6):
    o.step(burn, faces=False)
    Es = []
    for _ in range(n):
        assert o.step(1, faces=False) == 0
        Es.append(o.E())
    Es = np.array(Es)
    bm = Es.reshape(nb, n // nb, -1).mean(axis=1)
    return Es.mean(axis=0), bm.std(axis=0, ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("left", [1.0, 4.0])
def test_bands_fixed_point_matches_cp(oracle_mod, left):
    """Three bands of different C, v, Kn (and a two-tau film with null
    collisions): FRESH iterations averaged vs the CP steady state."""
    w = slab_1d_bands(n=16, kn_left_factor=left, particles=240_000)
    E_star, _ = cp.bands_fixed_point_1d(w)
    o = oracle_mod.Bands(w, tally_faces=oracle_mod.FACES_OFF)
    Em, se = _fresh_average(o, 40, 60)
    z = (Em - E_star) / np.maximum(se, 1e-7)
    assert np.abs(z).max() < 6.0, np.abs(z).max()
    # the spectrum matters: a gray film with the mean properties differs
    assert np.max(np.abs(E_star - E_star.mean())) > 1e-3


def test_bands_source_matches_cp(oracle_mod):
    w = slab_1d_bands(n=16, particles=240_000, t_hot=1.0, t_cold=1.0)
    S = 0.05 * np.ones(16)
    w.source = S
    E_star, _ = cp.bands_fixed_point_1d(w, source=S)
    o = oracle_mod.Bands(w, tally_faces=oracle_mod.FACES_OFF)
    Em, se = _fresh_average(o, 60, 60)
    z = (Em - E_star) / np.maximum(se, 1e-7)
    assert np.abs(z).max() < 6.0
    assert E_star.min() > 1e-3


def test_bands_equilibrium_is_uniform(oracle_mod):
    """Walls all at T_w and no source: the steady state is T_w everywhere, for
    any spectrum (CP model exactly, oracle within the noise)."""
    w = slab_1d_bands(n=12, particles=120_000, t_hot=1.01, t_cold=1.01)
    E_star, _ = cp.bands_fixed_point_1d(w)
    assert np.allclose(E_star, 0.01 * sum(w.band_C), rtol=1e-12)
    o = oracle_mod.Bands(w, tally_faces=oracle_mod.FACES_OFF)
    Em, se = _fresh_average(o, 30, 30)
    assert np.abs((Em - E_star) / np.maximum(se, 1e-7)).max() < 6.0


def test_bands_conserve_energy_per_band(oracle_mod):
    w = nongray_two_material_2d(n=8, K=5, particles=40_000)
    o = oracle_mod.Bands(w, tally_faces=oracle_mod.FACES_EVERY)
    G0 = [o.band(k)["G"] for k in range(5)]
    assert o.step(1) == 0
    for k in range(5):
        t = o.band(k)
        assert int(G0[k].sum()) == int(t["D"].sum()) + int(t["B"].sum())
        # candidates include the real collisions
        assert np.all(np.abs(t["W"]) >= np.abs(t["D"]))


def test_bands_identical_bands_equal_gray_statistically(oracle_mod):
    """K identical bands behave as the gray film with the same properties."""
    w = slab_1d_bands(n=16, C=(0.25, 0.25, 0.25, 0.25), vg=(1.0,) * 4, kn=(0.5,) * 4,
                      particles=200_000)
    E_b, _ = cp.bands_fixed_point_1d(w)
    g = slab_1d(n=16, kn=0.5, particles=200_000)
    E_g, _ = cp.Slab(g).fixed_point()
    assert np.allclose(E_b, E_g, rtol=1e-10, atol=1e-13)
    o = oracle_mod.Bands(w, tally_faces=oracle_mod.FACES_OFF)
    Em, se = _fresh_average(o, 30, 60)
    assert np.abs((Em - E_g) / np.maximum(se, 1e-7)).max() < 6.0


def test_bands_rejects(oracle_mod):
    w = slab_1d_bands(n=8)
    w.band_C = np.array([0.5, -0.3, 0.2])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Bands(w)
