"""GPU parity of the quadrature options at the C-ABI boundary (Section 2.1 fixes only
minimum degrees): the Stroud rule with N+2 points per direction and N+2 face points, the
default volume rule with N+2 face points (padded with zero-weight nodes), a caller's rule
(the Stroud nodes reflected across r = s), and the 3-point edge-midpoint rule at N=1
(padded from 3 to 4 nodes), each against the oracle built with the same rule; a batch that
mixes default and (N+2)-point instances."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import esdg_oracle as O
from paper_2005_02516_amd import workloads as wl
from parity_util import EPS32, EPS64, check_rhs, rhs_abs_bound

pytestmark = pytest.mark.gpu

QUADS = {
    "stroud_N+2": lambda N: {"vol_degree": 2 * N + 2, "face_points": N + 2},
    "faces_N+2": lambda N: {"face_points": N + 2},
    "reflected_rule": lambda N: {"rule": (lambda r, s, w: (s, r, w))(*O.stroud_rule(N))},
}


def _solver(ws, precision, quad, **kw):
    from paper_2005_02516_amd.binding import EsdgSwe
    return EsdgSwe(ws, precision=precision, flux="lf", g=ws[0].g, quadrature=quad, **kw)


def _state(w, seed=1):
    rng = np.random.default_rng(seed)
    u = w.u_nodes.copy()
    u[1] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    u[2] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    return u


@pytest.mark.parametrize("qname", list(QUADS))
@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rhs_other_rules(torch_mod, qname, N, precision):
    print(f"quadrature {qname} N={N} {precision}", flush=True)
    w = wl.config2(n=3, N=N)
    quad = QUADS[qname](N)
    d = O.Discretization(N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad=quad)
    o = O.Oracle(d, "lf")
    s = _solver([w], precision, quad)
    s.set_state(0, _state(w))
    uh = s.get_state(0)
    st = s.state_device(0)
    rhs = torch_mod.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_gpu = rhs.cpu().double().numpy()
    s.close()
    ks = np.arange(w.K)
    ok, worst = check_rhs(r_gpu, o.rhs(uh), rhs_abs_bound(o, uh, ks), EPS64 if precision == "fp64" else EPS32)
    print(f"  worst err / (eps * rounding bound) {worst:.2f}", flush=True)
    assert ok, worst


def test_midpoint_rule_padded(torch_mod):
    """N=1 with the 3-point edge-midpoint rule (degree 2): one zero-weight padding node."""
    w = wl.config2(n=4, N=1)
    rule = (np.array([0.0, 0.0, -1.0]), np.array([-1.0, 0.0, 0.0]), np.full(3, 2.0 / 3.0))
    quad = {"rule": rule}
    d = O.Discretization(1, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad=quad)
    o = O.Oracle(d, "lf")
    s = _solver([w], "fp64", quad)
    s.set_state(0, _state(w))
    uh = s.get_state(0)
    st = s.state_device(0)
    rhs = torch_mod.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    ok, worst = check_rhs(rhs.cpu().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), EPS64)
    s.step(w.dt, 10)
    u_gpu = s.get_state(0)
    s.close()
    assert ok, worst
    u_ref, _ = O.run(o, uh, w.dt, 10)
    assert np.linalg.norm(u_gpu - u_ref) < 1e-12 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("fused", [False, True])
def test_steps_stroud_N2_points(torch_mod, fused):
    """10 FP64 steps with (N+2)^2 / N+2 rules against the oracle; FP32 launch modes bitwise."""
    N = 3
    w = wl.config2(n=4, N=N)
    quad = QUADS["stroud_N+2"](N)
    d = O.Discretization(N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad=quad)
    o = O.Oracle(d, "lf")
    s = _solver([w], "fp64", quad, fused=fused)
    s.set_state(0, w.u_nodes)
    uh0 = s.get_state(0)
    s.step(w.dt, 10)
    u_gpu = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 10)
    err = np.linalg.norm(u_gpu - u_ref, axis=(1, 2)) / np.linalg.norm(u_ref[0])
    assert np.all(err < 1e-12), err


def test_mixed_batch_default_and_N2_points(torch_mod):
    """One launch over a default N=2 instance and an (N+2)-point N=3 instance (the build
    with both kinds): 3 FP64 steps of each against its own oracle."""
    ws = [wl.config2(n=3, N=2), wl.config2(n=4, N=3)]
    quads = [None, QUADS["stroud_N+2"](3)]
    s = _solver(ws, "fp64", quads)
    for i, w in enumerate(ws):
        s.set_state(i, w.u_nodes)
    uh0 = [s.get_state(i) for i in range(2)]
    dts = np.array([w.dt for w in ws])
    s.step(dts, 3)
    for i, w in enumerate(ws):
        d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, quad=quads[i])
        u_ref, _ = O.run(O.Oracle(d, "lf"), uh0[i], dts[i], 3)
        err = np.linalg.norm(s.get_state(i) - u_ref) / np.linalg.norm(u_ref)
        assert err < 1e-12, (i, err)
    s.close()
