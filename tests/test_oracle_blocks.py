"""Pins of the oracle's building blocks: Philox, uniforms, log, cos(2 pi u),
weight split, fixed-order sum, fixed-point exponent."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import slab_1d, cavity_2d

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    for ctr, key, want in _kat():
        got = oracle_mod.philox(np.array([ctr], dtype=np.uint32), key)[0]
        assert [int(x) for x in got] == want


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_header(oracle_mod, tmp_path):
    """Cross-check against the open-source rocRAND Philox engine (host build)."""
    exe = tmp_path / "rocrand_check"
    subprocess.run(["hipcc", "-O1", "--cuda-host-only", "-o", str(exe),
                    os.path.join(HERE, "rocrand_philox_check.cpp")], check=True,
                   capture_output=True)
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    inp = "\n".join(" ".join(f"{x:x}" for x in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x, 16) for x in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    for i in range(ctr.shape[0]):
        got = oracle_mod.philox(ctr[i:i + 1], (int(key[i, 0]), int(key[i, 1])))[0]
        assert np.array_equal(got.astype(np.uint64), ref[i])


def test_u53_range_and_resolution(oracle_mod):
    assert oracle_mod.u53(0, 0) == 0.0
    assert oracle_mod.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle_mod.u53(0, 1 << 6) == 2.0 ** -53
    assert oracle_mod.u53(1 << 5, 0) == 2.0 ** -27


def test_philox_uniformity_chi2(oracle_mod):
    n = 20000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 1] = np.arange(n)
    out = oracle_mod.philox(ctr, (12345, 678))
    u = np.array([oracle_mod.u53(int(a), int(b)) for a, b in out[:, :2]])
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    exp = n / 50
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert chi2 < 100.0      # 49 dof: P(chi2 > 100) ~ 2e-5
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)


def _ulp(x):
    return np.spacing(np.abs(np.float64(x)))


def test_log_accuracy(oracle_mod):
    rng = np.random.default_rng(3)
    xs = np.concatenate([1.0 - rng.integers(0, 2**53, 4000) * 2.0 ** -53,
                         np.exp(rng.uniform(-36.0, 0.0, 4000)),
                         np.exp(rng.uniform(-5.0, 5.0, 2000)),
                         [1.0, 0.5, 2.0 ** -53, 1.0 - 2.0 ** -53, 0.7071067811865476, 1.4142135623730951]])
    worst = 0.0
    for x in xs:
        got = oracle_mod.log(float(x))
        ref = np.log(np.longdouble(x))
        err = abs(np.longdouble(got) - ref) / np.longdouble(_ulp(float(ref)) if ref != 0 else 2.0 ** -1074)
        worst = max(worst, float(err))
    assert worst <= 2.0
    assert oracle_mod.log(1.0) == 0.0
    for k in range(1, 54):
        assert abs(oracle_mod.log(2.0 ** -k) + k * math.log(2.0)) <= 2 * _ulp(k * math.log(2.0))


def test_cos2pi_accuracy_and_symmetry(oracle_mod):
    rng = np.random.default_rng(4)
    us = rng.integers(0, 2**53, 6000) * 2.0 ** -53
    twopi = 2 * np.arccos(np.longdouble(-1.0))
    worst = 0.0
    for u in us:
        got = oracle_mod.cos2pi(float(u))
        ref = np.cos(twopi * np.longdouble(u))
        worst = max(worst, float(abs(np.longdouble(got) - ref)))
        # exact symmetries of the construction
        assert oracle_mod.cos2pi(1.0 - u) == got or u == 0.0
        if u < 0.5:
            assert oracle_mod.cos2pi(u + 0.5) == -got
    assert worst <= 2.3e-16
    assert oracle_mod.cos2pi(0.0) == 1.0
    assert oracle_mod.cos2pi(0.5) == -1.0
    assert oracle_mod.cos2pi(0.25) == 0.0 and oracle_mod.cos2pi(0.75) == 0.0
    assert abs(oracle_mod.cos2pi(1.0 / 6.0) - 0.5) <= 2.3e-16


def test_expm_accuracy(oracle_mod):
    """exp(-T) built from + - * / and exact scaling: within 2 ulp of the long
    double value over [0, 700], exact at 0, monotone, and zero beyond 700."""
    rng = np.random.default_rng(5)
    Ts = np.concatenate([rng.uniform(0.0, 1.0, 3000), rng.uniform(0.0, 50.0, 3000),
                         rng.uniform(50.0, 700.0, 1000), np.arange(0, 60) * math.log(2.0),
                         [1e-300, 1e-17, 0.34657359027997264, 0.3465735902799727]])
    worst = 0.0
    for T in Ts:
        got = oracle_mod.expm(float(T))
        ref = np.exp(-np.longdouble(T))
        err = abs(np.longdouble(got) - ref) / np.longdouble(_ulp(float(ref)))
        worst = max(worst, float(err))
    assert worst <= 2.0
    assert oracle_mod.expm(0.0) == 1.0
    assert oracle_mod.expm(700.5) == 0.0 and oracle_mod.expm(1e6) == 0.0
    g = sorted(rng.uniform(0.0, 40.0, 2000))
    v = [oracle_mod.expm(float(t)) for t in g]
    assert all(a >= b for a, b in zip(v, v[1:]))
    # products: exp(-a) exp(-b) = exp(-(a + b)) to rounding (the rounded sum's
    # error enters as a relative error of up to ulp(a + b))
    for a_, b_ in rng.uniform(0.0, 20.0, (200, 2)):
        lhs = oracle_mod.expm(a_) * oracle_mod.expm(b_)
        assert abs(lhs - oracle_mod.expm(a_ + b_)) <= 4 * _ulp(lhs) + lhs * _ulp(a_ + b_)


@pytest.mark.parametrize("G", [0, 1, 7, 149, 150, 151, -1, -7, -151, 10**17 + 3, -(10**17) - 5,
                               2**62 - 1, -(2**62) + 1])
def test_split_weight_exact(oracle_mod, G):
    n = 150
    q = [oracle_mod.split_weight(G, n, k) for k in range(n)]
    assert sum(q) == G
    lo = G // n    # python floor division
    assert all(x in (lo, lo + 1) for x in q)
    assert q == sorted(q, reverse=True)


def test_tree_sum_order(oracle_mod):
    # pairing s = 2 then s = 1 on a zero-padded block: (v0 + v2) + (v1 + v3)
    assert oracle_mod.tree_sum(np.array([1e16, 1.0, -1e16, 1.0])) == 2.0
    # a left-to-right sum would lose the first 1.0
    assert ((1e16 + 1.0) - 1e16) + 1.0 == 1.0
    rng = np.random.default_rng(5)
    for n in (1, 2, 255, 256, 257, 1000, 65536, 65537):
        v = rng.normal(size=n)
        s = oracle_mod.tree_sum(v)
        assert abs(s - math.fsum(v)) <= 1e-15 * n * np.abs(v).sum() / max(1, n) * 64
        iv = rng.integers(-1000, 1000, size=n).astype(np.float64)
        assert oracle_mod.tree_sum(iv) == float(iv.sum())
    assert oracle_mod.tree_sum(np.zeros(0)) == 0.0


def test_fixed_exponent(oracle_mod):
    # 1D slab, walls +-0.01, lam = 1: B = 4 * 0.01 * (1 + 1*2/4) = 0.06 -> ceil(log2) = -4
    w = slab_1d(kn=1.0)
    assert oracle_mod.fixed_exponent(w) == 66
    # power-of-two boundary: B = 0.25 exactly -> ceil(log2 B) = -2
    w = slab_1d(n=4, kn=1.0, t_hot=1.0 + 1.0 / 24.0, t_cold=1.0)
    w.tau[:] = 2.0     # lam = 2: B = 4 (1/24)(1 + 2*2/4) = 1/3 -> ceil(log2) = -1
    assert oracle_mod.fixed_exponent(w) == 63
    w = cavity_2d(n=16, kn=1.0)
    # B = 4 * 0.01 * (1 + 1 * 4 / 4) = 0.08 -> ceil(log2 0.08) = -3
    assert oracle_mod.fixed_exponent(w) == 65
