"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Both sides start from the same seeded node samples; each interpolates them with its
own code.  Tolerances: FP64 1e-12 relative (per field, against the field's largest
oracle value, or the state scale where the field is ~0), FP32 1e-5 relative L2 per
field after 100 steps (momentum normalised by ||h|| where it starts at zero).
"""
import math

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


def solver(ws, precision, flux, **kw):
    from paper_2005_02516_amd.binding import EsdgSwe
    return EsdgSwe(ws if isinstance(ws, list) else [ws], precision=precision, flux=flux, g=(ws[0] if isinstance(ws, list) else ws).g, **kw)


def oracle_for(w, flux):
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    return d, O.Oracle(d, flux)


def rel_field_err(a, b, scale=None):
    """max |a-b| per field over max |b| per field (or the given scale)."""
    out = []
    for c in range(3):
        s = scale if scale is not None else max(np.abs(b[c]).max(), 1e-300)
        out.append(np.abs(a[c] - b[c]).max() / s)
    return np.array(out)


def rel_l2(a, b, norm_by=None):
    out = []
    for c in range(3):
        nb = np.linalg.norm(b[c]) if norm_by is None else norm_by
        out.append(np.linalg.norm(a[c] - b[c]) / max(nb, 1e-300))
    return np.array(out)


CASES = [
    # (name, workload builder)
    ("affine_N1", lambda: wl.config1(n=3, N=1)),
    ("affine_N2", lambda: wl.config1(n=4, N=2)),
    ("curved_N3", lambda: wl.config2(n=5, N=3)),
    ("curved_N4", lambda: wl.config2(n=3, N=4)),
    ("curved_N5", lambda: wl.config2(n=3, N=5)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("flux", ["ec", "lf"])
def test_rhs_fp64(torch, name, make, flux):
    w = make()
    rng = np.random.default_rng(1)
    u = w.u_nodes.copy()
    u[1] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)      # nonzero velocities everywhere
    u[2] += 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape)
    d, o = oracle_for(w, flux)
    s = solver(w, "fp64", flux)
    s.set_state(0, u)
    uh_gpu = s.get_state(0)
    uh = d.interpolate(u)
    assert np.abs(uh_gpu - uh).max() < 1e-13 * np.abs(uh).max()
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_gpu = rhs.cpu().numpy()
    r_ref = o.rhs(uh_gpu)
    # every entry within 64 eps of the forward rounding bound of its own sum (the RHS of a
    # near-balanced state is a small difference of large pressure terms)
    ok, worst = check_rhs(r_gpu, r_ref, rhs_abs_bound(o, uh_gpu, np.arange(w.K)), EPS64)
    print(f"{name} {flux} fp64: per-field max err / max|rhs| {rel_field_err(r_gpu, r_ref)}, "
          f"worst err / (eps * bound) {worst:.2f}", flush=True)
    assert ok, worst
    s.close()


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_rhs_fp32(torch, name, make):
    w = make()
    d, o = oracle_for(w, "lf")
    s = solver(w, "fp32", "lf")
    s.set_state(0, w.u_nodes)
    uh32 = s.get_state(0)                   # the float state, widened exactly
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_ref = o.rhs(uh32)
    r_gpu = rhs.cpu().double().numpy()
    ok, worst = check_rhs(r_gpu, r_ref, rhs_abs_bound(o, uh32, np.arange(w.K)), EPS32)
    print(f"{name} fp32: per-field max err / max|rhs| {rel_field_err(r_gpu, r_ref)}, "
          f"worst err / (eps * bound) {worst:.2f}", flush=True)
    assert ok, worst
    s.close()


@pytest.mark.parametrize("flux", ["ec", "lf"])
def test_lake_at_rest_gpu(torch, flux):
    """Well-balanced on the GPU: rhs of h = H - b, u = v = 0 is round-off (FP64) / float round-off."""
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
        w = wl.config2(n=6, N=3, bump=0.0)
        s = solver(w, prec, flux)
        s.set_state(0, w.u_nodes)
        st = s.state_device(0)
        rhs = torch.empty_like(st)
        s.rhs(0, st, rhs)
        s.sync()
        assert float(rhs.abs().max()) < tol * 2.2, (prec, float(rhs.abs().max()))
        s.close()


def test_steps_fp64_graph_and_direct(torch):
    """10 LSRK steps in FP64 match the oracle to 1e-12; graph replay equals direct launches bitwise."""
    w = wl.config2(n=4, N=3)
    d, o = oracle_for(w, "lf")
    res = {}
    for use_graph in (True, False):
        s = solver(w, "fp64", "lf", use_graph=use_graph, fused=False)
        s.set_state(0, w.u_nodes)
        uh0 = s.get_state(0)
        s.step(w.dt, 6)
        s.step(w.dt, 4)
        res[use_graph] = s.get_state(0)
        s.close()
    assert np.array_equal(res[True], res[False])
    u_ref, _ = O.run(o, uh0, w.dt, 10)
    err = rel_l2(res[True], u_ref, norm_by=np.linalg.norm(u_ref[0]))
    assert np.all(err < 1e-12), err


def test_config1_fp64_100_steps(torch):
    """Config 1 (affine N=2, 8x8x2, EC flux, flat b): 100 steps, FP64 parity and entropy drift."""
    w = wl.config1()
    d, o = oracle_for(w, "ec")
    s = solver(w, "fp64", "ec")
    s.set_state(0, w.u_nodes)
    uh0 = s.get_state(0)
    dg0 = s.diagnostics()[0]
    s.step(w.dt, 100)
    u_gpu = s.get_state(0)
    dg1 = s.diagnostics()[0]
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 100)
    err = rel_l2(u_gpu, u_ref)
    assert np.all(err < 1e-12), err
    # mass conserved to round-off; entropy changes only by the time-integration error
    assert abs(dg1[0] - dg0[0]) < 1e-12 * abs(dg0[0])
    assert abs(dg1[3] - dg0[3]) < 1e-7 * abs(dg0[3])


def test_fp32_100_steps_small(torch):
    """Config-2 recipe on a 16x16x2 mesh: FP32 after 100 steps within 1e-5 (rel L2 per field)."""
    w = wl.config2(n=16, N=3)
    d, o = oracle_for(w, "lf")
    s = solver(w, "fp32", "lf")
    s.set_state(0, w.u_nodes)
    uh0 = d.interpolate(w.u_nodes)
    s.step(w.dt, 100)
    u_gpu = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 100)
    hn = np.linalg.norm(u_ref[0])
    err = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / np.linalg.norm(u_ref[c]) for c in range(3)])
    err_h = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / hn for c in range(3)])
    print("fp32 100-step rel-L2 per field (own norms):", err, "normalised by ||h||:", err_h, flush=True)
    assert np.all(err < 1e-5), err


def test_diagnostics_parity(torch):
    w = wl.config2(n=4, N=2)
    rng = np.random.default_rng(3)
    u = w.u_nodes.copy()
    u[1] = 0.2 * u[0] * np.sin(np.pi * w.yf)
    u[2] = -0.1 * u[0] * np.cos(np.pi * w.xf)
    for flux in ("ec", "lf"):
        d, o = oracle_for(w, flux)
        s = solver(w, "fp64", flux)
        s.set_state(0, u)
        dg = s.diagnostics()[0]
        ref = O.diagnostics(o, s.get_state(0))
        s.close()
        assert np.allclose(dg[:3], ref["mass"], rtol=1e-13, atol=1e-13)
        assert abs(dg[3] - ref["entropy"]) < 1e-13 * abs(ref["entropy"])
        assert abs(dg[4] - ref["entropy_rate"]) < 1e-12 * ref["entropy_rate_scale"]
        if flux == "ec":
            assert abs(dg[4]) < 1e-12 * dg[5]
        else:
            assert dg[4] < 0
    del rng


def test_ragged_tiles_and_small_meshes(torch):
    """K not a multiple of the tile size, tile size 1, and the 2-element periodic mesh."""
    for n, N, epb in ((1, 2, 0), (3, 3, 0), (3, 3, 5), (2, 4, 1), (5, 1, 7)):
        w = wl.config2(n=n, N=N)
        d, o = oracle_for(w, "lf")
        s = solver(w, "fp64", "lf", elems_per_block=epb)
        s.set_state(0, w.u_nodes)
        st = s.state_device(0)
        rhs = torch.empty_like(st)
        s.rhs(0, st, rhs)
        s.sync()
        uh = s.get_state(0)
        ok, worst = check_rhs(rhs.cpu().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), EPS64)
        s.close()
        assert ok, (n, N, epb, worst)


def test_large_tiles(torch):
    """Tile sizes up to the ABI's 64 elements (the tuned sizes for large N=1 meshes), with
    ragged last tiles: one FP64 RHS against the oracle, and 3 FP32 steps of the multi-stage
    launch bitwise equal to per-stage launches."""
    for n, N, epb in ((8, 1, 32), (7, 1, 48), (9, 1, 64), (6, 2, 32)):
        w = wl.config2(n=n, N=N)
        d, o = oracle_for(w, "lf")
        s = solver(w, "fp64", "lf", elems_per_block=epb)
        s.set_state(0, w.u_nodes)
        st = s.state_device(0)
        rhs = torch.empty_like(st)
        s.rhs(0, st, rhs)
        s.sync()
        uh = s.get_state(0)
        ok, worst = check_rhs(rhs.cpu().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)), EPS64)
        s.close()
        assert ok, (n, N, epb, worst)
        ref = _run_steps([w], "fp32", 3, fused=False, elems_per_block=epb)
        got = _run_steps([w], "fp32", 3, fused=True, elems_per_block=epb)
        assert all(np.array_equal(a, b) for a, b in zip(ref, got)), (n, N, epb)


def test_batched_mixed_instances(torch):
    """Several instances with different N and K in one solver: each matches its own oracle."""
    ws = wl.config4_instances(count=4, n_override=[3, 4, 2, 5], N_override=[2, 3, 4, 3])
    s = solver(ws, "fp64", "lf")
    for i, w in enumerate(ws):
        s.set_state(i, w.u_nodes)
    uh0 = [s.get_state(i) for i in range(len(ws))]
    dts = np.array([w.dt for w in ws])
    s.step(dts, 3)
    for i, w in enumerate(ws):
        d, o = oracle_for(w, "lf")
        u_ref, _ = O.run(o, uh0[i], dts[i], 3)
        err = rel_l2(s.get_state(i), u_ref, norm_by=np.linalg.norm(u_ref[0]))
        assert np.all(err < 1e-12), (i, err)
    s.close()


def test_error_paths(torch):
    from paper_2005_02516_amd.binding import EsdgError, ESDG_ENONPHYS, ESDG_ESTATE, ESDG_EINVAL
    w = wl.config2(n=3, N=2)
    s = solver(w, "fp64", "lf")
    with pytest.raises(EsdgError) as e:
        s.step(w.dt, 1)
    assert e.value.status == ESDG_ESTATE
    bad = w.u_nodes.copy()
    bad[0, 0, 0] = -1.0
    with pytest.raises(EsdgError) as e:
        s.set_state(0, bad)
    assert e.value.status == ESDG_ENONPHYS
    s.set_state(0, w.u_nodes)
    with pytest.raises(EsdgError) as e:
        s.step(-1.0, 1)
    assert e.value.status == ESDG_EINVAL
    s.close()


@pytest.mark.parametrize("N,n", [(3, 4), (5, 2)])
def test_rhs_bf16x3(torch, N, n):
    """Split-bf16 (hi*hi + hi*lo + lo*hi, float accumulate) contractions on the matrix cores:
    one RHS within 64 eps_eff of the rounding bound, eps_eff = 2^-16 (the split's per-product
    relative error)."""
    from parity_util import check_rhs, rhs_abs_bound
    w = wl.config2(n=n, N=N)
    d, o = oracle_for(w, "lf")
    s = solver(w, "bf16x3", "lf")
    s.set_state(0, w.u_nodes)
    uh32 = s.get_state(0)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    s.close()
    ks = np.arange(w.K)
    r_ref = o.rhs(uh32)
    ok, worst = check_rhs(rhs.cpu().double().numpy(), r_ref, rhs_abs_bound(o, uh32, ks), 2.0 ** -16)
    print(f"bf16x3 N={N}: worst err / (2^-16 * bound) = {worst:.3f}", flush=True)
    assert ok, worst


def test_bf16x3_100_steps_small(torch):
    """Config-2 recipe on a 16x16x2 mesh, BF16x3 contractions: state error after 100 steps,
    reported per field (rel L2; momentum also normalised by ||h||)."""
    w = wl.config2(n=16, N=3)
    d, o = oracle_for(w, "lf")
    s = solver(w, "bf16x3", "lf")
    s.set_state(0, w.u_nodes)
    uh0 = d.interpolate(w.u_nodes)
    s.step(w.dt, 100)
    u_gpu = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 100)
    hn = np.linalg.norm(u_ref[0])
    err_h = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / hn for c in range(3)])
    err = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / np.linalg.norm(u_ref[c]) for c in range(3)])
    print("bf16x3 100-step rel-L2 per field:", err, "normalised by ||h||:", err_h, flush=True)
    assert np.all(err_h < 1e-5), err_h


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rhs_matrix_cores(torch, name, make, precision):
    """Projection and lift contractions on the matrix cores in the bulk precision
    (v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32): one RHS within 64 eps of the
    rounding bound, the same bar as a reordered sum in that precision."""
    from parity_util import EPS32, EPS64, check_rhs, rhs_abs_bound
    w = make()
    d, o = oracle_for(w, "lf")
    s = solver(w, precision, "lf", matrix_cores=True)
    s.set_state(0, w.u_nodes)
    uh = s.get_state(0)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    s.close()
    ok, worst = check_rhs(rhs.cpu().double().numpy(), o.rhs(uh), rhs_abs_bound(o, uh, np.arange(w.K)),
                          EPS64 if precision == "fp64" else EPS32)
    print(f"matrix cores {precision} {name}: worst err / (eps * bound) = {worst:.3f}", flush=True)
    assert ok, worst


def test_steps_fp64_matrix_cores(torch):
    """10 LSRK steps in FP64 with matrix-core contractions match the oracle to 1e-12."""
    w = wl.config2(n=4, N=3)
    d, o = oracle_for(w, "lf")
    s = solver(w, "fp64", "lf", matrix_cores=True)
    s.set_state(0, w.u_nodes)
    uh0 = s.get_state(0)
    s.step(w.dt, 10)
    u = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 10)
    err = rel_l2(u, u_ref, norm_by=np.linalg.norm(u_ref[0]))
    assert np.all(err < 1e-12), err


def _run_steps(ws, precision, nsteps, **kw):
    s = solver(ws, precision, "lf", **kw)
    for i, w in enumerate(ws):
        s.set_state(i, w.u_nodes)
    s.step(np.array([w.dt for w in ws]), nsteps)
    out = [s.get_state(i) for i in range(len(ws))]
    s.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_steps_bitwise(torch, precision):
    """All RK stages of a step call in one cooperative launch (tiles wait on their face
    neighbours' progress instead of a kernel boundary): bitwise the per-stage result."""
    w = wl.config2(n=8, N=3)
    ref = _run_steps([w], precision, 7, fused=False)
    got = _run_steps([w], precision, 7, fused=True)
    assert np.array_equal(ref[0], got[0])


def test_fused_steps_many_tiles_per_block(torch):
    """More tiles than resident workgroups (2 elements per tile on K = 32768): each workgroup
    walks several tiles per stage, some of them neighbours of each other."""
    w = wl.config2(n=128, N=3)
    ref = _run_steps([w], "fp32", 3, fused=False, elems_per_block=2)
    got = _run_steps([w], "fp32", 3, fused=True, elems_per_block=2)
    assert np.array_equal(ref[0], got[0])


def test_fused_steps_mixed_ensemble(torch):
    """Mixed degrees (cost-balanced tile ranges) in one fused launch: bitwise per instance."""
    ws = wl.config4_instances(count=4, n_override=[3, 4, 2, 5], N_override=[2, 3, 4, 3])
    ref = _run_steps(ws, "fp32", 4, fused=False)
    got = _run_steps(ws, "fp32", 4, fused=True)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_fused_residency_counts_static_lds(torch):
    """FP64, N=2, 12 elements per tile on 8192 elements (683 tiles): 54240 bytes of dynamic
    LDS plus the multi-stage build's own 256 bytes fit twice per CU in 1 KiB granules of
    160 KiB, not three times, so the automatic plan must not make it a resident
    multi-stage launch; a forced multi-stage launch (two tiles per workgroup on the grid
    that is really resident) matches per-stage launches bitwise."""
    w = wl.config2(n=64, N=2)
    s = solver(w, "fp64", "lf", elems_per_block=12)
    info = s.launch_info()
    s.close()
    assert info["tiles"] == 683 and info["step_mode"] == 0, info
    assert info["resident_workgroups"] < info["tiles"], info
    ref = _run_steps([w], "fp64", 3, fused=False, elems_per_block=12)
    auto = _run_steps([w], "fp64", 3, elems_per_block=12)
    forced = _run_steps([w], "fp64", 3, fused=True, elems_per_block=12)
    assert np.array_equal(ref[0], auto[0]) and np.array_equal(ref[0], forced[0])
