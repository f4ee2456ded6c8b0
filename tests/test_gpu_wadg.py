"""GPU parity of the weight-adjusted mass inverse (ESDG_MASS_WEIGHT_ADJUSTED): the library
through its C ABI against the oracle's weight-adjusted scheme (the implementation remark
after eq. (dgform) in Section 2.8: M^{-1} M_{1/J} M^{-1} in the entropy projection and the
lift), both taking the projected entropy variables of S - g Href h with Href the mean
free-surface level of the state (the oracle computes it from the state itself).

Bars: one RHS within 64 eps of the rounding bound (FP64 and FP32), 10 FP64 steps within
1e-12, 100 FP32 steps within 1e-5 (rel L2, normalised by ||h||), the multi-stage launch
bitwise equal to per-stage launches, entropy conservation with the EC flux, lake at rest,
and sampled rows at the N=5, K=524288 size.
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
    ws = w if isinstance(w, list) else [w]
    return EsdgSwe(ws, precision=precision, flux=flux, g=ws[0].g, mass="wadg", **kw)


def wadg_oracle(w, flux, uh):
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, mass="wadg")
    return d, O.Oracle(d, flux, Href=O.mean_free_surface(d, uh))


CASES = [
    ("affine_N2", lambda: wl.config1(n=4, N=2)),
    ("curved_N3", lambda: wl.config2(n=5, N=3)),
    ("curved_N4", lambda: wl.config2(n=3, N=4)),
    ("curved_N5", lambda: wl.config2(n=3, N=5)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rhs_wadg(torch, name, make, precision):
    w = make()
    u = w.u_nodes.copy()
    rng = np.random.default_rng(5)
    u[1] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    u[2] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    s = solver(w, precision, "lf")
    s.set_state(0, u)
    uh = s.get_state(0)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    s.close()
    d, o = wadg_oracle(w, "lf", uh)
    ok, worst = check_rhs(rhs.cpu().double().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)),
                          EPS64 if precision == "fp64" else EPS32)
    print(f"wadg {precision} {name}: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst


def test_wadg_equals_stored_on_affine_gpu(torch):
    """J constant per element: the weight-adjusted and the stored inverse give the same RHS."""
    from paper_2005_02516_amd.binding import EsdgSwe
    w = wl.config1(n=4, N=2)
    out = {}
    for mass in ("stored", "wadg"):
        s = EsdgSwe([w], precision="fp64", flux="lf", g=w.g, mass=mass)
        s.set_state(0, w.u_nodes)
        st = s.state_device(0)
        rhs = torch.empty_like(st)
        s.rhs(0, st, rhs)
        s.sync()
        out[mass] = rhs.cpu().numpy()
        s.close()
    assert np.abs(out["wadg"] - out["stored"]).max() < 1e-12 * np.abs(out["stored"]).max()


def test_steps_wadg_fp64(torch):
    w = wl.config2(n=4, N=3)
    s = solver(w, "fp64", "lf")
    s.set_state(0, w.u_nodes)
    uh0 = s.get_state(0)
    s.step(w.dt, 10)
    u = s.get_state(0)
    s.close()
    d, o = wadg_oracle(w, "lf", uh0)
    u_ref, _ = O.run(o, uh0, w.dt, 10)
    hn = np.linalg.norm(u_ref[0])
    err = np.array([np.linalg.norm(u[c] - u_ref[c]) / hn for c in range(3)])
    assert np.all(err < 1e-12), err


def test_wadg_fp32_100_steps_small(torch):
    w = wl.config2(n=16, N=3)
    s = solver(w, "fp32", "lf")
    s.set_state(0, w.u_nodes)
    s.step(w.dt, 100)
    u = s.get_state(0)
    s.close()
    d0 = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, mass="wadg")
    uh0 = d0.interpolate(w.u_nodes)
    d, o = wadg_oracle(w, "lf", uh0)
    u_ref, _ = O.run(o, uh0, w.dt, 100)
    hn = np.linalg.norm(u_ref[0])
    err = np.array([np.linalg.norm(u[c] - u_ref[c]) / hn for c in range(3)])
    print("wadg fp32 100-step rel-L2 (by ||h||):", err, flush=True)
    assert np.all(err < 1e-5), err


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_wadg_fused_steps_bitwise(torch, precision):
    w = wl.config2(n=8, N=3)
    out = []
    for fused in (False, True):
        s = solver(w, precision, "lf", fused=fused)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 7)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])


MC_MODES = {"bf16x3": ("bf16x3", {}, 2.0 ** -16), "fp32_mfma": ("fp32", {"matrix_cores": True}, EPS32),
            "fp64_mfma": ("fp64", {"matrix_cores": True}, EPS64)}


@pytest.mark.parametrize("N,n", [(3, 4), (5, 2)])
@pytest.mark.parametrize("mode", list(MC_MODES))
def test_rhs_wadg_matrix_cores(torch, N, n, mode):
    """The weight-adjusted inverse with the other contractions on the matrix cores (split-bf16,
    or in the bulk precision); its own two passes run on the vector ALUs in every mode.  One
    RHS within 64 eps of the rounding bound (eps_eff = 2^-16 for split-bf16), and 3 steps of
    the multi-stage launch bitwise equal to per-stage launches."""
    prec, kw, eps = MC_MODES[mode]
    w = wl.config2(n=n, N=N)
    u = w.u_nodes.copy()
    rng = np.random.default_rng(7)
    u[1] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    u[2] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    s = solver(w, prec, "lf", **kw)
    s.set_state(0, u)
    uh = s.get_state(0)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    s.close()
    d, o = wadg_oracle(w, "lf", uh)
    ok, worst = check_rhs(rhs.cpu().double().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), eps)
    print(f"wadg {mode} N={N}: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst
    out = []
    for fused in (False, True):
        s = solver(w, prec, "lf", fused=fused, **kw)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 3)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])


def test_wadg_entropy_conservation_gpu(torch):
    """EC flux on a curved periodic mesh: the entropy rate vanishes to round-off (it needs
    the same inverse in the projection and the lift); LF makes it negative."""
    w = wl.config2(n=4, N=3)
    u = w.u_nodes.copy()
    u[1] = 0.2 * u[0] * np.sin(np.pi * w.yf)
    u[2] = -0.1 * u[0] * np.cos(np.pi * w.xf)
    for flux in ("ec", "lf"):
        s = solver(w, "fp64", flux)
        s.set_state(0, u)
        dg = s.diagnostics()[0]
        uh = s.get_state(0)
        s.close()
        d, o = wadg_oracle(w, flux, uh)
        ref = O.diagnostics(o, uh)
        assert abs(dg[4] - ref["entropy_rate"]) < 1e-12 * ref["entropy_rate_scale"]
        if flux == "ec":
            assert abs(dg[4]) < 1e-12 * dg[5]
        else:
            assert dg[4] < 0


def test_wadg_lake_at_rest_gpu(torch):
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
        w = wl.config2(n=6, N=3, bump=0.0)
        s = solver(w, prec, "lf")
        s.set_state(0, w.u_nodes)
        st = s.state_device(0)
        rhs = torch.empty_like(st)
        s.rhs(0, st, rhs)
        s.sync()
        s.close()
        assert float(rhs.abs().max()) < tol * 2.2, (prec, float(rhs.abs().max()))


def test_config5_full_sampled_wadg(torch):
    """N=5, K=524288 (where the stored inverses are the largest per-element data): sampled
    rows against the oracle's weight-adjusted scheme, FP32, 64 eps of the rounding bound."""
    w = wl.config5()
    s = solver(w, "fp32", w.flux)
    s.set_state(0, w.u_nodes)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_gpu = rhs.cpu().double().numpy()
    uh = s.get_state(0)
    s.close()
    d, o = wadg_oracle(w, w.flux, uh)
    (cx, cy) = w.meta["center"]
    dx = (w.xg.mean(axis=1) - cx + 1.0) % 2.0 - 1.0
    dy = (w.yg.mean(axis=1) - cy + 1.0) % 2.0 - 1.0
    ks = np.union1d(np.random.default_rng(2).choice(w.K, 256, replace=False),
                    np.nonzero(dx * dx + dy * dy < 0.15 ** 2)[0])
    r_ref = o.rhs(uh, ks)
    ok, worst = check_rhs(r_gpu[:, ks], r_ref, rhs_abs_bound(o, uh, ks), EPS32)
    print(f"config5 wadg fp32: {ks.size} sampled elements, worst err / (eps * bound) {worst:.3f}", flush=True)
    assert ok, worst


def test_wadg_mixed_ensemble(torch):
    """Instances of degrees 2, 3 and 4 (periodic and walled) in one handle with the
    weight-adjusted inverse: each instance's 3 FP64 steps match its own oracle (each with its
    own Href), and the FP32 multi-stage launch is bitwise equal to per-stage launches."""
    from paper_2005_02516_amd.binding import EsdgSwe
    ws = [wl.config2(n=3, N=2), wl.basin(n=3, N=3), wl.config2(n=2, N=4)]
    s = EsdgSwe(ws, precision="fp64", flux="lf", g=1.0, mass="wadg")
    uh0 = []
    for i, w in enumerate(ws):
        s.set_state(i, w.u_nodes)
        uh0.append(s.get_state(i))
    dt = min(w.dt for w in ws)
    s.step(np.full(len(ws), dt), 3)
    got = [s.get_state(i) for i in range(len(ws))]
    s.close()
    for w, u0, u in zip(ws, uh0, got):
        d, o = wadg_oracle(w, "lf", u0)
        ur, _ = O.run(o, u0, dt, 3)
        hn = np.linalg.norm(ur[0])
        err = max(np.linalg.norm(u[c] - ur[c]) / hn for c in range(3))
        assert err < 1e-12, (w.name, w.N, err)
    out = []
    for fused in (False, True):
        s = EsdgSwe(ws, precision="fp32", flux="lf", g=1.0, mass="wadg", fused=fused)
        for i, w in enumerate(ws):
            s.set_state(i, w.u_nodes)
        s.step(np.full(len(ws), dt), 3)
        out.append([s.get_state(i) for i in range(len(ws))])
        s.close()
    assert all(np.array_equal(a, b) for a, b in zip(out[0], out[1]))
