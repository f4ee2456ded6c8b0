"""GPU parity of the DG-SBP scheme (Section 3.2) through the C ABI against the DG-SBP oracle:
one RHS within 64 eps of the rounding bound (FP64 and FP32, N=1..4, LF and EC, periodic
curved mesh and the walled basin), steps (FP64 to 1e-12, FP32 to 1e-5 after 100 steps),
lake at rest, FP64 diagnostics (entropy conservation with the EC flux), and the
no-allocation RHS bitwise equal to the RHS."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import esdg_oracle as O
from paper_2005_02516_amd import sbp_rules
from paper_2005_02516_amd import workloads as wl
from parity_util import EPS32, EPS64, check_rhs, sbp_rhs_abs_bound

pytestmark = pytest.mark.gpu


def _quad(N):
    return {"rule": sbp_rules.load(N)}


def _pair(w, precision, flux="lf", **kw):
    from paper_2005_02516_amd.binding import EsdgSwe
    s = EsdgSwe([w], precision=precision, flux=flux, g=w.g, quadrature=_quad(w.N), scheme="sbp", **kw)
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly,
                         quad={"rule": sbp_rules.load(w.N), "vol_degree": 2 * w.N - 1})
    return s, O.SBPOracle(d, flux)


def _moving(w, seed=1):
    rng = np.random.default_rng(seed)
    u = w.u_nodes.copy()
    u[1] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    u[2] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    return u


def _rhs(torch, s, inst=0, noalloc=False):
    st = s.state_device(inst)
    out = torch.empty_like(st)
    (s.rhs_noalloc if noalloc else s.rhs)(inst, st, out)
    s.sync()
    return out.cpu().double().numpy()


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("flux", ["ec", "lf"])
def test_sbp_rhs(torch_mod, N, precision, flux):
    print(f"DG-SBP rhs N={N} {precision} {flux}", flush=True)
    w = wl.config2(n=4, N=N)
    s, o = _pair(w, precision, flux)
    s.set_state(0, _moving(w))
    u = s.get_state(0)
    r_gpu = _rhs(torch_mod, s)
    s.close()
    ok, worst = check_rhs(r_gpu, o.rhs(u), sbp_rhs_abs_bound(o, u), EPS64 if precision == "fp64" else EPS32)
    print(f"  worst err / (eps * rounding bound) {worst:.2f}", flush=True)
    assert ok, worst


def test_sbp_walls_rhs(torch_mod):
    """The walled basin (Section 2.9 exterior state at the face nodes)."""
    for N, precision in ((2, "fp64"), (3, "fp32")):
        w = wl.basin(n=6, N=N)
        s, o = _pair(w, precision)
        s.set_state(0, _moving(w, 4))
        u = s.get_state(0)
        r_gpu = _rhs(torch_mod, s)
        s.close()
        ok, worst = check_rhs(r_gpu, o.rhs(u), sbp_rhs_abs_bound(o, u), EPS64 if precision == "fp64" else EPS32)
        assert ok, (N, precision, worst)


def test_sbp_steps(torch_mod):
    w = wl.config2(n=6, N=3)
    s, o = _pair(w, "fp64")
    s.set_state(0, w.u_nodes)
    u0 = s.get_state(0)
    s.step(w.dt, 10)
    u_gpu = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, u0, w.dt, 10)
    err = np.linalg.norm(u_gpu - u_ref, axis=(1, 2)) / np.linalg.norm(u_ref[0])
    print("DG-SBP 10 FP64 steps, rel L2 by ||h||:", err, flush=True)
    assert np.all(err < 1e-12), err
    s, o = _pair(w, "fp32")
    s.set_state(0, w.u_nodes)
    s.step(w.dt, 100)
    u32 = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, u0, w.dt, 100)
    err = np.array([np.linalg.norm(u32[c] - u_ref[c]) / np.linalg.norm(u_ref[c]) for c in range(3)])
    print("DG-SBP 100 FP32 steps, rel L2 per field:", err, flush=True)
    assert np.all(err < 1e-5), err


def test_sbp_lake_at_rest_and_diagnostics(torch_mod):
    for N in (1, 4):
        w = wl.config2(n=4, N=N, bump=0.0)
        for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
            s, _ = _pair(w, precision)
            s.set_state(0, w.u_nodes)
            assert np.abs(_rhs(torch_mod, s)).max() < tol, (N, precision)
            s.close()
    w = wl.config2(n=4, N=3)
    s, o = _pair(w, "fp64", "ec")
    s.set_state(0, _moving(w))
    u = s.get_state(0)
    dg = s.diagnostics()[0]
    s.close()
    ref = o.diagnostics(u)
    assert np.allclose(dg[:3], ref["mass"], rtol=1e-13, atol=1e-13)
    assert abs(dg[3] - ref["entropy"]) < 1e-13 * abs(ref["entropy"])
    assert abs(dg[4]) < 1e-12 * dg[5] and abs(ref["entropy_rate"]) < 1e-12 * ref["entropy_rate_scale"]


def test_sbp_noalloc_matches_rhs(torch_mod):
    w = wl.config2(n=5, N=2)
    s, _ = _pair(w, "fp32")
    s.set_state(0, _moving(w))
    a = _rhs(torch_mod, s)
    b = _rhs(torch_mod, s, noalloc=True)
    s.close()
    np.testing.assert_array_equal(a, b)
