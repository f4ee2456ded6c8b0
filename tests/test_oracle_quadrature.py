"""Pins of the oracle's quadrature options (Section 2.1 fixes only minimum degrees: volume
rules exact to degree 2N, face rules to 2N+1).

* the Stroud rule with N+2 points per direction is exact to degree 2N+3 and the face rule
  with N+2 points to 2N+3 (against scipy's Gauss-Jacobi nodes), and not one degree more;
* with such rules, or with a caller's rule (the Stroud nodes reflected across r = s), the
  scheme keeps the lake at rest, entropy conservation (EC), mass conservation;
* a zero-weight node added to the volume rule leaves the right-hand side unchanged (the
  reading under which a rule may be padded to a fixed node count).
"""
import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import esdg_oracle as O
from paper_2005_02516_amd import workloads as wl


def reference_integral(f):
    xa, wa = roots_jacobi(14, 0.0, 0.0)
    xb, wb = roots_jacobi(14, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    return float(np.sum(np.outer(wa, wb) / 2.0 * f((1 + A) * (1 - B) / 2 - 1, B)))


def exact_to(r, s, w, deg):
    for d in range(deg + 1):
        for a in range(d + 1):
            if abs(np.sum(w * r ** a * s ** (d - a)) - reference_integral(lambda x, y: x ** a * y ** (d - a))) > 1e-13:
                return False
    return True


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_higher_rules_exactness(N):
    (r, s, w), (rf, sf, wf, nr, ns) = O.quadrature_rules(N, {"vol_degree": 2 * N + 2, "face_points": N + 2})
    assert w.size == (N + 2) ** 2 and rf.size == 3 * (N + 2)
    assert exact_to(r, s, w, 2 * N + 3) and not exact_to(r, s, w, 2 * N + 4)
    t = rf[:N + 2]                                   # face 1: s = -1, parameter r
    for d in range(2 * N + 4):
        ex = (1 - (-1) ** (d + 1)) / (d + 1)
        assert abs(np.sum(wf[:N + 2] * t ** d) - ex) < 1e-13
    assert O.rule_degree(r, s, w) == 2 * N + 3


def _state(w, seed):
    rng = np.random.default_rng(seed)
    x, y = w.xf, w.yf
    f = lambda a: a * np.sin(np.pi * (x + rng.uniform(0, 2))) * np.cos(np.pi * (y + rng.uniform(0, 2)))
    h = 2.3 - w.b_nodes + f(0.05)
    return np.stack([h, h * (0.2 + f(0.3)), h * (-0.1 + f(0.3))])


QUADS = {
    "stroud_N+2": lambda N: {"vol_degree": 2 * N + 2, "face_points": N + 2},
    "reflected_rule": lambda N: {"rule": (lambda r, s, w: (s, r, w))(*O.stroud_rule(N))},
    "stroud_N+1_faces_N+2": lambda N: {"face_points": N + 2},
}


@pytest.mark.parametrize("N", [2, 3])
@pytest.mark.parametrize("qname", list(QUADS))
def test_scheme_properties_with_other_rules(N, qname):
    w = wl.config2(n=4, N=N)
    quad = QUADS[qname](N)
    d = O.Discretization(N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad=quad)
    lake = wl.config2(n=4, N=N, bump=0.0)
    for flux in ("ec", "lf"):
        assert np.abs(O.Oracle(d, flux).rhs(d.interpolate(lake.u_nodes))).max() < 1e-12
    uh = d.interpolate(_state(w, 7))
    dg = O.diagnostics(O.Oracle(d, "ec"), uh)
    assert abs(dg["entropy_rate"]) < 1e-13 * dg["entropy_rate_scale"]
    r = O.Oracle(d, "lf").rhs(uh)
    wJ = d.ref.wq[None] * d.Jq
    assert abs(np.sum(wJ * (r[0] @ d.ref.Vq.T))) < 1e-13 * np.abs(r[0]).sum()


@pytest.mark.parametrize("N", [1, 3])
def test_zero_weight_node_changes_nothing(N):
    w = wl.config2(n=3, N=N)
    r, s, q = O.stroud_rule(N)
    padded = (np.r_[r, -1 / 3, 0.2], np.r_[s, -1 / 3, -0.5], np.r_[q, 0.0, 0.0])
    d0 = O.Discretization(N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    d1 = O.Discretization(N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad={"rule": padded})
    uh = d0.interpolate(_state(w, 3))
    r0 = O.Oracle(d0, "lf").rhs(uh)
    r1 = O.Oracle(d1, "lf").rhs(uh)
    assert np.abs(r0 - r1).max() < 1e-13 * np.abs(r0).max()
