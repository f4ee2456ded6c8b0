"""Pins of the DG-SBP oracle (Section 3) and of the SBP quadrature rules it runs on.

* rules (Section 3.1): positive weights, exactness for degree 2N-1 (against a high-degree
  collapsed Gauss-Jacobi rule from scipy), the N+1 Gauss-Legendre points of every face
  among the nodes, and no other boundary nodes;
* operators (the theorem of Section 3.2): Q_SBP + Q_SBP^T = I_f^T B I_f, and W^{-1} Q_SBP
  differentiates every polynomial of degree N exactly at the nodes; on curved elements the
  physical operators keep the SBP property and annihilate constants;
* scheme: lake at rest, entropy conservation with the EC flux (dissipation with LF) on a
  curved periodic mesh with varying bathymetry, conservation of mass, free stream, and a
  planted mistake in the surface term caught by them.
"""
import math

import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import esdg_oracle as O
from paper_2005_02516_amd import sbp_rules
from paper_2005_02516_amd import workloads as wl


def reference_integral(f):
    """int over the triangle (-1,-1), (1,-1), (-1,1) of f(r, s) by a 12x12 collapsed
    Gauss-Jacobi rule built from scipy's nodes (exact to degree 23)."""
    xa, wa = roots_jacobi(12, 0.0, 0.0)
    xb, wb = roots_jacobi(12, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = np.outer(wa, wb) / 2.0
    return float(np.sum(W * f((1 + A) * (1 - B) / 2 - 1, B)))


def sbp_disc(w, N, b=None):
    r, s, q = sbp_rules.load(N)
    return O.Discretization(N, w.xg, w.yg, w.b_nodes if b is None else b, w.g, w.Lx, w.Ly,
                            quad={"rule": (r, s, q), "vol_degree": 2 * N - 1})


def random_state(w, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    x, y = w.xf, w.yf
    f = lambda a: a * np.sin(np.pi * (rng.integers(1, 3) * x + rng.uniform(0, 2))) * np.cos(
        np.pi * (rng.integers(1, 3) * y + rng.uniform(0, 2)))
    h = 2.3 - w.b_nodes + f(amp)
    return np.stack([h, h * (0.2 + f(0.3)), h * (-0.1 + f(0.3))])


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_sbp_rule_conditions(N):
    r, s, w = sbp_rules.load(N)
    assert w.size == {1: 6, 2: 10, 3: 18, 4: 22}[N]
    assert np.all(w > 0)
    for d in range(2 * N):                       # degree 2N-1
        for a in range(d + 1):
            ex = reference_integral(lambda rr, ss: rr ** a * ss ** (d - a))
            assert abs(np.sum(w * r ** a * s ** (d - a)) - ex) < 1e-13, (a, d - a)
    # the N+1 Gauss-Legendre points of every face are nodes, and the only boundary nodes
    t, _ = np.polynomial.legendre.leggauss(N + 1)
    faces = [(t, -np.ones_like(t)), (-t, t), (-np.ones_like(t), -t)]
    for fr, fs in faces:
        dmin = np.min(np.hypot(fr[:, None] - r[None], fs[:, None] - s[None]), axis=1)
        assert np.all(dmin < 1e-13)
    on_bnd = (np.abs(s + 1) < 1e-12) | (np.abs(r + 1) < 1e-12) | (np.abs(r + s) < 1e-12)
    assert on_bnd.sum() == 3 * (N + 1)
    assert abs(np.sum(w) - 2.0) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_sbp_operator_properties(N):
    w = wl.config2(n=3, N=N)
    d = sbp_disc(w, N)
    o = O.SBPOracle(d, "ec")
    ref = d.ref
    P = o.sel
    If = np.eye(ref.Nq)[o.If]
    for j, (Qh, nrm) in enumerate(zip(ref.Qh, (ref.nrJ, ref.nsJ))):
        Q = P.T @ Qh @ P
        np.testing.assert_allclose(Q + Q.T, If.T @ np.diag(ref.wf * nrm) @ If, atol=1e-13)
        # W^{-1} Q differentiates degree-N polynomials exactly at the nodes
        D = Q / ref.wq[:, None]
        for dd in range(N + 1):
            for a in range(dd + 1):
                b = dd - a
                u = ref.rq ** a * ref.sq ** b
                du = (a * ref.rq ** max(a - 1, 0) * ref.sq ** b) if j == 0 else (b * ref.rq ** a * ref.sq ** max(b - 1, 0))
                np.testing.assert_allclose(D @ u, du, atol=1e-11)
    # physical operators on the curved mesh
    ks = np.arange(d.K)
    Qx, Qy = o.Q_sbp(ks)
    Bx = np.einsum("fq,kf,fp->kqp", If, ref.wf[None] * d.nJx, If)
    By = np.einsum("fq,kf,fp->kqp", If, ref.wf[None] * d.nJy, If)
    np.testing.assert_allclose(Qx + np.swapaxes(Qx, 1, 2), Bx, atol=1e-12)
    np.testing.assert_allclose(Qy + np.swapaxes(Qy, 1, 2), By, atol=1e-12)
    assert np.abs(Qx.sum(axis=2)).max() < 1e-12 and np.abs(Qy.sum(axis=2)).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("flux", ["ec", "lf"])
def test_sbp_lake_at_rest(N, flux):
    w = wl.config2(n=4, N=N, bump=0.0)
    d = sbp_disc(w, N)
    o = O.SBPOracle(d, flux)
    u = o.nodal(d.interpolate(w.u_nodes))
    assert np.abs(o.rhs(u)).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_sbp_entropy_and_mass(N):
    """EC: the entropy rate vanishes (relative to its terms); LF: it is negative; the depth's
    integral is conserved with either flux."""
    w = wl.config2(n=4, N=N)
    d = sbp_disc(w, N)
    u0 = random_state(w, seed=N)
    # nodal noise makes the state discontinuous across faces (an interpolant through the
    # shared lattice nodes is continuous, and the LF penalty would vanish)
    noise = 1e-2 * np.random.default_rng(N).uniform(-1, 1, (3, d.K, d.ref.Nq))
    for flux in ("ec", "lf"):
        o = O.SBPOracle(d, flux)
        u = o.nodal(d.interpolate(u0)) + noise
        dg = o.diagnostics(u)
        if flux == "ec":
            assert abs(dg["entropy_rate"]) < 1e-13 * dg["entropy_rate_scale"]
        else:
            assert dg["entropy_rate"] < -1e-8 * dg["entropy_rate_scale"]
        r = o.rhs(u)
        wJ = d.ref.wq[None] * d.Jq
        assert abs(np.sum(wJ * r[0])) < 1e-13 * np.sum(np.abs(wJ * r[0]))


@pytest.mark.parametrize("N", [2, 3])
def test_sbp_free_stream(N):
    w = wl.config2(n=3, N=N)
    xg, yg = w.xg, w.yg
    d = O.Discretization(N, xg, yg, 0 * w.b_nodes + 0.3, 1.0, 2.0, 2.0,
                         quad={"rule": sbp_rules.load(N), "vol_degree": 2 * N - 1})
    o = O.SBPOracle(d, "lf")
    u = np.stack([np.full((d.K, d.ref.Nq), 1.7), np.full((d.K, d.ref.Nq), 0.4), np.full((d.K, d.ref.Nq), -0.2)])
    assert np.abs(o.rhs(u)).max() < 1e-12


def test_sbp_surface_collapse_mutation_caught(monkeypatch):
    """Dropping the face term's collapse onto the volume nodes (adding it to the wrong nodes)
    breaks entropy conservation."""
    w = wl.config2(n=4, N=2)
    d = sbp_disc(w, 2)
    o = O.SBPOracle(d, "ec")
    u = o.nodal(d.interpolate(random_state(w, seed=3))) + 1e-2 * np.random.default_rng(0).uniform(-1, 1, (3, d.K, d.ref.Nq))
    good = o.diagnostics(u)
    assert abs(good["entropy_rate"]) < 1e-13 * good["entropy_rate_scale"]
    o.If = np.roll(o.If, 1)
    bad = o.diagnostics(u)
    assert abs(bad["entropy_rate"]) > 1e-6 * bad["entropy_rate_scale"]


def _sbp_vortex_error(N, n, T=0.1):
    par = dict(g=1.0, hinf=1.0, A=0.1, R=0.3, xc=1.0, yc=1.0, uinf=0.5, vinf=0.25)
    xg, yg, xf, yf = wl.structured_mesh(n, N, warp=0.05)
    d = O.Discretization(N, xg, yg, None, 1.0, 2.0, 2.0, quad={"rule": sbp_rules.load(N), "vol_degree": 2 * N - 1})

    def exact(t):
        def f(x, y):
            h, u, v = wl.vortex_fields(x, y, t, **par)
            return np.stack([h, h * u, h * v])
        return f

    h, u, v = wl.vortex_fields(xf, yf, 0.0, **par)
    dt0 = wl.timestep(np.stack([h, h * u, h * v]), 1.0, N, 2.0 / n, 0.25)
    ns = int(math.ceil(T / dt0))
    o = O.SBPOracle(d, "lf")
    u1, _ = O.run(o, exact(0.0)(d.xh[:, :d.ref.Nq], d.yh[:, :d.ref.Nq]), T / ns, ns)
    # Section 4.2: the nodal solution is projected onto degree-N polynomials first
    return O.l2_error(d, d.project(u1), exact(T))


@pytest.mark.slow
@pytest.mark.parametrize("N", [2, 3])
def test_sbp_vortex_convergence(N):
    """Section 4.2: the DG-SBP scheme converges at about h^N or better on the curved
    vortex (measured 2.3-2.9 at N=2 and 3.6-3.7 at N=3 from 8x8x2 to 16x16x2, with errors
    1.1-1.4x those of the modal scheme at N=3)."""
    rate = np.log2(_sbp_vortex_error(N, 8) / _sbp_vortex_error(N, 16))
    assert np.all(rate > N), rate
