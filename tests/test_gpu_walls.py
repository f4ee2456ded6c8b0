"""GPU parity of the reflective wall boundary condition (Section 2.9), through the C ABI:
the closed curved-wall basin (not periodic in x or y) and a free-slip channel (periodic in
y only), against the oracle.

Bars: one RHS within 64 eps of the rounding bound (FP64 and FP32, N=2..4), 10 FP64 steps
within 1e-12, 100 FP32 steps within 1e-5 (rel L2, normalised by ||h||), the multi-stage
launch bitwise equal to per-stage launches, lake at rest, the channel's uniform flow
steady, EC entropy conservation and exact mass conservation in FP64, and the
8192-element basin (the benchmark size) row by row.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import esdg_oracle as O
from paper_2005_02516_amd import workloads as wl
from parity_util import EPS32, EPS64, check_rhs, rhs_abs_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def solver(w, precision, flux, **kw):
    from paper_2005_02516_amd.binding import EsdgSwe
    return EsdgSwe([w], precision=precision, flux=flux, g=w.g, **kw)


def oracle_for(w, flux):
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    return d, O.Oracle(d, flux)


def moving_basin(n, N):
    w = wl.basin(n=n, N=N)
    x, y = w.xg, w.yg
    h = w.u_nodes[0] + 0.05 * np.exp(-20.0 * ((x - 0.8) ** 2 + (y - 1.1) ** 2))
    w.u_nodes = np.ascontiguousarray(np.stack([h, 0.1 * h * np.sin(np.pi * y) * np.cos(0.3 * x),
                                               -0.05 * h * np.cos(np.pi * x)]))
    return w


def rhs_of(torch, s):
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    return rhs.cpu().double().numpy()


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rhs_walls(torch, N, precision):
    w = moving_basin(3, N)
    s = solver(w, precision, "lf")
    s.set_state(0, w.u_nodes)
    uh = s.get_state(0)
    r = rhs_of(torch, s)
    s.close()
    d, o = oracle_for(w, "lf")
    ok, worst = check_rhs(r, o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), EPS64 if precision == "fp64" else EPS32)
    print(f"walls {precision} N={N}: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst


def test_steps_walls_fp64(torch):
    w = moving_basin(4, 3)
    s = solver(w, "fp64", "lf")
    s.set_state(0, w.u_nodes)
    uh0 = s.get_state(0)
    s.step(w.dt, 10)
    u = s.get_state(0)
    s.close()
    d, o = oracle_for(w, "lf")
    u_ref, _ = O.run(o, uh0, w.dt, 10)
    hn = np.linalg.norm(u_ref[0])
    err = np.array([np.linalg.norm(u[c] - u_ref[c]) / hn for c in range(3)])
    assert np.all(err < 1e-12), err


def test_walls_fp32_100_steps_small(torch):
    w = wl.basin(n=12, N=3)
    s = solver(w, "fp32", "lf")
    s.set_state(0, w.u_nodes)
    s.step(w.dt, 100)
    u = s.get_state(0)
    s.close()
    d, o = oracle_for(w, "lf")
    uh0 = d.interpolate(w.u_nodes)
    u_ref, _ = O.run(o, uh0, w.dt, 100)
    hn = np.linalg.norm(u_ref[0])
    err = np.array([np.linalg.norm(u[c] - u_ref[c]) / hn for c in range(3)])
    print("walls fp32 100-step rel-L2 (by ||h||):", err, flush=True)
    assert np.all(err < 1e-5), err


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_walls_fused_steps_bitwise(torch, precision):
    w = wl.basin(n=8, N=3)
    out = []
    for fused in (False, True):
        s = solver(w, precision, "lf", fused=fused)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 7)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])


def test_walls_steady_states(torch):
    """Lake at rest in the curved basin, and uniform flow along the walls of a channel."""
    w = wl.basin(n=6, N=3)
    w.u_nodes = np.ascontiguousarray(np.stack([1.2 - w.b_nodes, 0 * w.b_nodes, 0 * w.b_nodes]))
    xg, yg, xf, yf = wl.structured_mesh(4, 3, warp=0.05)
    h = 1.5 + 0 * xg
    ch = wl.Workload(name="channel", N=3, n=4, K=xg.shape[0], xg=xg, yg=yg, xf=xf, yf=yf, Lx=0.0, Ly=2.0, g=1.0,
                     b_nodes=np.zeros_like(xg), u_nodes=np.ascontiguousarray(np.stack([h, 0 * h, 0.4 * h])),
                     flux="lf", cfl=0.25, steps=1)
    for case in (w, ch):
        for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
            s = solver(case, prec, "lf")
            s.set_state(0, case.u_nodes)
            r = rhs_of(torch, s)
            s.close()
            assert np.abs(r).max() < tol * 2.2, (case.name, prec, np.abs(r).max())


def test_walls_entropy_and_mass_gpu(torch):
    w = moving_basin(4, 3)
    for flux in ("ec", "lf"):
        s = solver(w, "fp64", flux)
        s.set_state(0, w.u_nodes)
        dg0 = s.diagnostics()[0]
        uh = s.get_state(0)
        s.step(w.dt, 5)
        dg1 = s.diagnostics()[0]
        s.close()
        d, o = oracle_for(w, flux)
        ref = O.diagnostics(o, uh)
        assert abs(dg0[4] - ref["entropy_rate"]) < 1e-12 * ref["entropy_rate_scale"]
        if flux == "ec":
            assert abs(dg0[4]) < 1e-12 * dg0[5]
        else:
            assert dg0[4] < 0
        assert abs(dg1[0] - dg0[0]) < 1e-12 * abs(dg0[0])      # no mass through the walls


def test_basin_bench_size_rows(torch):
    """The 64x64x2 = 8192-element basin at N=3 (the benchmark's wall case), FP32, every
    element's RHS within 64 eps of the rounding bound."""
    w = moving_basin(64, 3)
    s = solver(w, "fp32", "lf")
    s.set_state(0, w.u_nodes)
    uh = s.get_state(0)
    r = rhs_of(torch, s)
    s.close()
    d, o = oracle_for(w, "lf")
    ks = np.arange(w.K)
    ok, worst = check_rhs(r, o.rhs(uh), rhs_abs_bound(o, uh, ks), EPS32)
    print(f"basin 8192 fp32: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_walls_with_weight_adjusted_inverse(torch, precision):
    """Walls and the weight-adjusted mass inverse together: one RHS against the oracle with
    both, and the multi-stage launch bitwise equal to per-stage launches."""
    from paper_2005_02516_amd.binding import EsdgSwe
    w = moving_basin(3, 3)
    s = EsdgSwe([w], precision=precision, flux="lf", g=w.g, mass="wadg")
    s.set_state(0, w.u_nodes)
    uh = s.get_state(0)
    r = rhs_of(torch, s)
    s.close()
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, mass="wadg")
    o = O.Oracle(d, "lf", Href=O.mean_free_surface(d, uh))
    ok, worst = check_rhs(r, o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), EPS64 if precision == "fp64" else EPS32)
    assert ok, worst
    out = []
    for fused in (False, True):
        s = EsdgSwe([w], precision=precision, flux="lf", g=w.g, mass="wadg", fused=fused)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 5)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])


def test_walls_in_mixed_ensemble(torch):
    """A walled basin next to periodic instances of other degrees in one handle: each
    instance's 3 FP64 steps match its own oracle."""
    from paper_2005_02516_amd.binding import EsdgSwe
    ws = [moving_basin(3, 2), wl.config2(n=3, N=3), moving_basin(2, 4)]
    s = EsdgSwe(ws, precision="fp64", flux="lf", g=1.0)
    uh0 = []
    for i, w in enumerate(ws):
        s.set_state(i, w.u_nodes)
        uh0.append(s.get_state(i))
    dt = min(w.dt for w in ws)
    s.step(np.full(len(ws), dt), 3)
    got = [s.get_state(i) for i in range(len(ws))]
    s.close()
    for w, u0, u in zip(ws, uh0, got):
        d, o = oracle_for(w, "lf")
        ur, _ = O.run(o, u0, dt, 3)
        hn = np.linalg.norm(ur[0])
        err = max(np.linalg.norm(u[c] - ur[c]) / hn for c in range(3))
        assert err < 1e-12, (w.name, w.N, err)


@pytest.mark.parametrize("mode", ["bf16x3", "fp32_mfma", "fp64_mfma"])
def test_walls_matrix_cores(torch, mode):
    """Walls with the projection and lift contractions on the matrix cores (split-bf16, or in
    the bulk precision): one RHS within 64 eps of the rounding bound (eps_eff = 2^-16 for
    split-bf16), and 3 steps of the multi-stage launch bitwise equal to per-stage launches."""
    prec, kw, eps = {"bf16x3": ("bf16x3", {}, 2.0 ** -16), "fp32_mfma": ("fp32", {"matrix_cores": True}, EPS32),
                     "fp64_mfma": ("fp64", {"matrix_cores": True}, EPS64)}[mode]
    w = moving_basin(3, 3)
    s = solver(w, prec, "lf", **kw)
    s.set_state(0, w.u_nodes)
    uh = s.get_state(0)
    r = rhs_of(torch, s)
    s.close()
    d, o = oracle_for(w, "lf")
    ok, worst = check_rhs(r, o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), eps)
    print(f"walls {mode}: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst
    out = []
    for fused in (False, True):
        s = solver(w, prec, "lf", fused=fused, **kw)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 3)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])
