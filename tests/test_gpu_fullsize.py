"""GPU parity at the full workload sizes, in the launch configuration bench.py uses.

The oracle evaluates the RHS only on a seeded sample of elements (its entropy
projection covers all elements, which the sampled rows need through their neighbours),
so these run at K = 8192 (N=3), 131072 (N=4) and 524288 (N=5), and on a stratified
subset of the ensemble (two instances per degree, smallest and largest K drawn).
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


def _solver(ws, precision):
    from paper_2005_02516_amd.binding import EsdgSwe
    return EsdgSwe(ws, precision=precision, flux=ws[0].flux, g=ws[0].g)


def _sampled_rhs_check(torch, w, precision, nsample, seed=0, near=None):
    """Sampled elements' RHS against the oracle, within 64 eps of the rounding bound."""
    s = _solver([w], precision)
    s.set_state(0, w.u_nodes)
    st = s.state_device(0)
    rhs = torch.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_gpu = rhs.cpu().double().numpy()
    uh = s.get_state(0)
    s.close()
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    o = O.Oracle(d, w.flux)
    ks = np.random.default_rng(seed).choice(w.K, size=min(nsample, w.K), replace=False)
    if near is not None:
        # add every element whose centroid lies within `radius` of `center` (periodic)
        (cx, cy), radius = near
        dx = (w.xg.mean(axis=1) - cx + 1.0) % 2.0 - 1.0
        dy = (w.yg.mean(axis=1) - cy + 1.0) % 2.0 - 1.0
        ks = np.union1d(ks, np.nonzero(dx * dx + dy * dy < radius * radius)[0])
    ks = np.sort(ks)
    r_ref = o.rhs(uh, ks)
    bound = rhs_abs_bound(o, uh, ks)
    ok, worst = check_rhs(r_gpu[:, ks], r_ref, bound, EPS64 if precision == "fp64" else EPS32)
    rel = np.abs(r_gpu[:, ks] - r_ref).max() / np.abs(r_ref).max()
    print(f"{w.name} K={w.K} N={w.N} {precision}: {ks.size} sampled elements, max err / max|rhs| {rel:.2e}, "
          f"worst err / (eps * rounding bound) {worst:.2f}", flush=True)
    assert ok, worst


def test_config2_full(torch_mod):
    w = wl.config2()
    _sampled_rhs_check(torch_mod, w, "fp64", 8192)
    _sampled_rhs_check(torch_mod, w, "fp32", 8192)


def test_config2_full_steps_fp32(torch_mod):
    """5 LSRK steps at full size: FP32 state against the FP64 oracle (rel L2 per field)."""
    w = wl.config2()
    s = _solver([w], "fp32")
    s.set_state(0, w.u_nodes)
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    o = O.Oracle(d, w.flux)
    uh0 = d.interpolate(w.u_nodes)
    s.step(w.dt, 5)
    u_gpu = s.get_state(0)
    s.close()
    u_ref, _ = O.run(o, uh0, w.dt, 5)
    err = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / np.linalg.norm(u_ref[c]) for c in range(3)])
    print("config2 5 steps fp32 rel L2:", err, flush=True)
    assert np.all(err < 1e-5), err


def test_config3_full_sampled(torch_mod):
    _sampled_rhs_check(torch_mod, wl.config3(), "fp32", 512)


def test_config5_full_sampled(torch_mod):
    w = wl.config5()
    _sampled_rhs_check(torch_mod, w, "fp32", 256, near=(w.meta["center"], 0.15))


def test_ensemble_subset(torch_mod):
    """Two instances per degree (smallest and largest K drawn) in one solver, one launch
    per stage; sampled RHS and one LSRK step against each instance's oracle."""
    # draw the ensemble's (N, K) without building meshes, then build the stratified subset
    draws = []
    for i in range(256):
        rng = np.random.Generator(np.random.PCG64(1000 + i))
        K = int(rng.integers(2048, 32769))
        n = max(2, int(round(np.sqrt(K / 2.0))))
        N = int(rng.integers(2, 5))
        draws.append((i, N, n))
    pick = []
    for N in (2, 3, 4):
        sub = sorted([d for d in draws if d[1] == N], key=lambda d: d[2])
        pick += [sub[0][0], sub[-1][0]]
    ws = []
    for i in pick:
        ws += wl.config4_instances(count=1, seed0=1000 + i)
    s = _solver(ws, "fp32")
    for j, w in enumerate(ws):
        s.set_state(j, w.u_nodes)
    uh0 = [s.get_state(j) for j in range(len(ws))]
    dts = np.array([w.dt for w in ws])
    s.step(dts, 1)
    for j, w in enumerate(ws):
        d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
        o = O.Oracle(d, w.flux)
        # one step with the oracle on every element is affordable for the small instances only
        if w.K <= 8192:
            u_ref, _ = O.run(o, uh0[j], dts[j], 1)
            u_gpu = s.get_state(j)
            err = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / max(np.linalg.norm(u_ref[c]), 1e-12)
                            for c in range(3)])
            hn = np.linalg.norm(u_ref[0])
            err_h = np.array([np.linalg.norm(u_gpu[c] - u_ref[c]) / hn for c in range(3)])
            print(f"ensemble instance {pick[j]} N={w.N} K={w.K}: 1-step rel L2 {err} (by ||h||: {err_h})",
                  flush=True)
            assert np.all(err < 1e-5), (pick[j], err, err_h)
        ks = np.sort(np.random.default_rng(j).choice(w.K, size=128, replace=False))
        r_ref = o.rhs(s.get_state(j), ks)
        import torch
        st = s.state_device(j)
        rhs = torch.empty_like(st)
        s.rhs(j, st, rhs)
        s.sync()
        r_gpu = rhs.cpu().double().numpy()[:, ks]
        ok, worst = check_rhs(r_gpu, r_ref, rhs_abs_bound(o, s.get_state(j), ks), EPS32)
        assert ok, (pick[j], worst)
    s.close()


def test_graph_replay_matches_direct_fp32(torch_mod):
    """Graph replays of the stage launches give bit-identical states to direct launches,
    replayed several times with host work and synchronisation in between."""
    from paper_2005_02516_amd.binding import EsdgSwe
    w = wl.config2(n=32)
    out = []
    for g in (True, False):
        s = EsdgSwe([w], precision="fp32", flux="lf", g=w.g, use_graph=g, fused=False)
        s.set_state(0, w.u_nodes)
        for _ in range(3):
            s.step(w.dt, 4)
            s.sync()
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])


def test_config5_full_sampled_bf16x3(torch_mod):
    """Config 5's own mode: split-bf16 projection and lift contractions, float flux
    differencing, double entropy round trip (eps_eff = 2^-16 in the rounding bound)."""
    w = wl.config5()
    s = _solver([w], "bf16x3")
    s.set_state(0, w.u_nodes)
    st = s.state_device(0)
    rhs = torch_mod.empty_like(st)
    s.rhs(0, st, rhs)
    s.sync()
    r_gpu = rhs.cpu().double().numpy()
    uh = s.get_state(0)
    s.close()
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
    o = O.Oracle(d, w.flux)
    (cx, cy) = w.meta["center"]
    dx = (w.xg.mean(axis=1) - cx + 1.0) % 2.0 - 1.0
    dy = (w.yg.mean(axis=1) - cy + 1.0) % 2.0 - 1.0
    ks = np.union1d(np.random.default_rng(1).choice(w.K, 256, replace=False),
                    np.nonzero(dx * dx + dy * dy < 0.15 ** 2)[0])
    r_ref = o.rhs(uh, ks)
    ok, worst = check_rhs(r_gpu[:, ks], r_ref, rhs_abs_bound(o, uh, ks), 2.0 ** -16)
    print(f"config5 bf16x3: worst err / (2^-16 bound) {worst:.3f}, max err / max|rhs| "
          f"{np.abs(r_gpu[:, ks] - r_ref).max() / np.abs(r_ref).max():.2e}", flush=True)
    assert ok, worst


def test_config2_fused_steps_bitwise(torch_mod):
    """Config 2 at full size, 20 steps in one fused launch against per-stage graph replays."""
    from paper_2005_02516_amd.binding import EsdgSwe
    w = wl.config2()
    out = []
    for fused in (False, True):
        s = EsdgSwe([w], precision="fp32", flux=w.flux, g=w.g, fused=fused)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, 20)
        out.append(s.get_state(0))
        s.close()
    assert np.array_equal(out[0], out[1])
