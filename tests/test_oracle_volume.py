"""Pins of the volume-kernel definitions of the Section 5.4 cost comparison (oracle side):

* brute force: pure-Python loops over (element, row, column) on tiny inputs reproduce the
  vectorised definitions, with the fluxes written out again from the shallow-water
  equations (physical flux) and from the entropy-conservative flux's closed form;
* consistency: for a constant state on an element, F(u, u) = f(u), so the entropy-stable
  term is exactly twice the traditional one;
* conservation: with a skew-symmetric matrix the entropy-stable rows of an element sum to
  zero (F is symmetric), while the traditional ones need not;
* the C versions (the CPU side of the cost ratio) agree with the numpy definitions.
"""
import numpy as np
import pytest

from oracle import volume_kernels as V


def _inputs(n, K, seed):
    rng = np.random.default_rng(seed)
    Qx, Qy = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    h = rng.uniform(1.0, 2.0, (K, n))
    u = np.stack([h, h * rng.uniform(-0.5, 0.5, (K, n)), h * rng.uniform(-0.5, 0.5, (K, n))])
    return Qx, Qy, u


def _brute(kind, Qx, Qy, u, g):
    n, K = Qx.shape[0], u.shape[1]
    r = np.zeros_like(u)
    for k in range(K):
        for m in range(n):
            for j in range(n):
                hm, hum, hvm = u[:, k, m]
                hj, huj, hvj = u[:, k, j]
                if kind == "dg":
                    uu, vv = huj / hj, hvj / hj
                    fx = [huj, huj * uu + g * hj * hj / 2, huj * vv]
                    fy = [hvj, hvj * uu, hvj * vv + g * hj * hj / 2]
                    w = 1.0
                else:
                    ha, hua, hva = (hm + hj) / 2, (hum + huj) / 2, (hvm + hvj) / 2
                    ua, va = (hum / hm + huj / hj) / 2, (hvm / hm + hvj / hj) / 2
                    p = g * ha * ha - g * (hm * hm + hj * hj) / 4
                    fx = [hua, hua * ua + p, hua * va]
                    fy = [hva, hva * ua, hva * va + p]
                    w = 2.0
                for c in range(3):
                    r[c, k, m] += w * (Qx[m, j] * fx[c] + Qy[m, j] * fy[c])
    return r


@pytest.mark.parametrize("kind", ["dg", "esdg"])
def test_brute_force_tiny(kind):
    Qx, Qy, u = _inputs(4, 3, seed=1)
    ref = _brute(kind, Qx, Qy, u, 9.81)
    got = (V.dg_volume if kind == "dg" else V.esdg_volume)(Qx, Qy, u, 9.81)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_consistency_constant_state():
    Qx, Qy, u = _inputs(12, 5, seed=2)
    u = np.repeat(u[:, :, :1], 12, axis=2)                 # constant on each element
    assert np.allclose(V.esdg_volume(Qx, Qy, u, 1.0), 2.0 * V.dg_volume(Qx, Qy, u, 1.0), rtol=1e-13, atol=1e-12)


def test_skew_matrix_conserves():
    Qx, Qy, u = _inputs(20, 4, seed=3)
    Sx, Sy = Qx - Qx.T, Qy - Qy.T
    r = V.esdg_volume(Sx, Sy, u, 1.0)
    assert np.abs(r.sum(axis=2)).max() < 1e-12 * np.abs(r).max()
    rd = V.dg_volume(Sx, Sy, u, 1.0)
    assert np.abs(rd.sum(axis=2)).max() > 1e-3 * np.abs(rd).max()


@pytest.mark.parametrize("n", [7, 50])
def test_c_versions_match(n):
    import os
    if not os.path.exists(V.C_LIBRARY):
        V.build_c()
    Qx, Qy, u = _inputs(n, 6, seed=4)
    for kind, fn in (("dg", V.dg_volume), ("esdg", V.esdg_volume)):
        ref = fn(Qx, Qy, u, 1.0)
        got = V.c_volume(kind, Qx, Qy, u, 1.0)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), kind
