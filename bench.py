#!/usr/bin/env python3
"""Throughput benchmark: DOF-updates/s per RK stage of the ESDG shallow-water solver.

Workload (N=3, the degree the metric is quoted at): periodic [0,2]^2, 64x64 squares split
into 8192 curved triangles (nodes warped by 0.05 sin(pi x) sin(pi y)), bathymetry
b = 0.1 sin(pi x) cos(pi y) + 0.1, lake at rest H = 2.2 plus a seeded Gaussian bump of
amplitude 0.01, Lax-Friedrichs interface flux, g = 1.  A step is one LSRK4(5) step (five
RK stages); the library's automatic plan runs all stages of a step call in one launch of
resident workgroups when every tile gets one (this mesh in FP32), else one launch per
stage replayed from HIP graphs.  Inputs are resident in HBM before the timed region.
value = K * Np / (time per RK stage), FP32 bulk path with FP64 entropy round trip; the
FP64 path is timed on the same workload for the speedup.

Prints one JSON line.  Only one GPU is supported: --gpus > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import glob
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6        # MI355X vector FP64 (published)


def pairs(N):
    Nq, Nfq = (N + 1) ** 2, 3 * (N + 1)
    return Nq * (Nq - 1) // 2 + Nq * Nfq


def dims(N):
    Np = (N + 1) * (N + 2) // 2
    Nq, Nfq = (N + 1) ** 2, 3 * (N + 1)
    return Np, Nq, Nfq, Nq + Nfq


def alg_flops_per_elem(N, wadg=False):
    """35 FLOP per unordered nonzero node pair (flux differencing) + projection and lift
    contractions 6(2 Nq Np + Np^2 + Nh Np) + 6(Np Nh + Np^2); with the weight-adjusted mass
    inverse each Np^2 (the stored inverse) becomes 2 Nq Np (two contractions with V_q)."""
    Np, Nq, Nfq, Nh = dims(N)
    m = 2 * Nq * Np if wadg else Np * Np
    return 35 * pairs(N) + 6 * (2 * Nq * Np + m + Nh * Np) + 6 * (Np * Nh + m)


def alg_bytes_per_elem(N, word, wadg=False):
    """Minimum HBM bytes per element per stage: state 12 Np words (read u_h; read and write
    du; write u_h), face exchange 6 Nfq, geometry 2 Np (node coordinates), bathymetry Np,
    and the curved inverse mass matrix Np^2 (with the weight-adjusted inverse: w/J, Nq)."""
    Np, Nq, Nfq, Nh = dims(N)
    return word * (12 * Np + 6 * Nfq + 2 * Np + Np + (Nq if wadg else Np * Np))


TRAFFIC_FILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt")))
FUSED_ARG = {"auto": "auto", "per-stage": False, "fused": True}
STEP_MODES = {0: "one launch per RK stage (HIP graph replays)",
              1: "one launch of resident workgroups per step call, tiles re-read every stage",
              2: "one launch of resident workgroups per step call, tiles resident in LDS across stages"}


def kernel_source_hash():
    """sha256 of the stage kernel's device code: kernels.hip up to its host launchers, and
    device_types.hpp, with // comments, trailing blanks and empty lines removed, so that a
    comment or a host-side change does not void a counter summary taken on the same kernel
    (which kernel build a launch plan uses is part of the plan a summary records)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_types.hpp"):
        with open(os.path.join(ROOT, "paper_2005_02516_amd", "csrc", f)) as fh:
            for line in fh:
                if f == "kernels.hip" and "-- host launchers" in line:
                    break
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(w, prec, epb, step_mode, stages_per_launch):
    """HBM bytes per RK stage (FETCH_SIZE and WRITE_SIZE, copy-calibrated) from a committed
    counter summary taken for this kernel source, workload, tile size and launch mode, or
    None when there is none.  A one-launch-per-stage summary gives the bytes of one stage.
    A multi-stage summary gives a fixed part (the first stage's full fetch, the last one's
    write-back) and a per-stage part, fitted from launches of two stage counts, so the
    bytes per stage of a launch of S stages are fixed / S + per_stage."""
    for path in TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        kv = {}
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k] = v
        if kv.get("kernel_source_sha256") != kernel_source_hash() or int(kv.get("step_mode", -1)) != step_mode:
            continue
        if (int(kv.get("N", -1)), int(kv.get("K", -1)), kv.get("precision"), int(kv.get("epb", -1))) != \
                (w.N, w.K, prec, epb):
            continue
        if "per_stage_fetch_bytes" in kv:
            S = float(stages_per_launch)
            fetch = float(kv["fixed_fetch_bytes"]) / S + float(kv["per_stage_fetch_bytes"])
            write = float(kv["fixed_write_bytes"]) / S + float(kv["per_stage_write_bytes"])
        elif int(kv.get("stages_per_launch", -1)) == stages_per_launch:
            fetch, write = float(kv["fetch_bytes"]), float(kv["write_bytes"])
        else:
            continue
        return {"fetch": int(round(fetch)), "write": int(round(write)), "source": os.path.relpath(path, ROOT)}
    return None


def kernel_trace_summary(w, args):
    """The committed rocprofv3 kernel-trace summary of this workload, if there is one."""
    name = None
    if args.matrix_cores:
        name = None
    elif args.precision == "bf16x3":
        name = "stage_kernel_bf16x3_N5_K524288.md" if (w.N, w.K) == (5, 524288) else None
    elif args.walls:
        name = "stage_kernel_walls_basin_N3_K8192.md" if (w.N, w.K) == (3, 8192) else None
    elif args.mass == "wadg":
        name = {(3, 8192): "stage_kernel_wadg_N3_K8192.md", (5, 524288): "stage_kernel_wadg_N5_K524288.md"}.get((w.N, w.K))
    else:
        name = {(3, 8192): "stage_kernel_curved_N3_K8192.md", (5, 524288): "stage_kernel_curved_N5_K524288.md"}.get((w.N, w.K))
    return f"profiles/{name}" if name and os.path.exists(os.path.join(ROOT, "profiles", name)) else None


def time_steps(s, dt, steps, torch):
    """Event-timed region on the solver's stream: returns milliseconds for `steps` steps."""
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.step(dt, steps)
    ev1.record(s.stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


_POOL_ORACLE = None


def _pool_init(w, mass, Href):
    """Worker of the CPU baseline: its own oracle for the workload, BLAS on one thread."""
    global _POOL_ORACLE
    from threadpoolctl import threadpool_limits
    from oracle import esdg_oracle as O
    threadpool_limits(1)
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, mass="wadg" if mass == "wadg" else "exact")
    _POOL_ORACLE = O.Oracle(d, w.flux, Href=Href)


def _pool_rhs(args):
    uh, ks = args
    return _POOL_ORACLE.rhs(uh, ks)


def host_cpu():
    """(usable cores, CPU model) of this host."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def cpu_baseline(w, stages_pool=200, mass="stored", stages_single=25, max_workers=16):
    """The FP64 oracle as it stands, timed on this host's cores: the RK stages of the same
    workload with each stage's right-hand side split into element chunks over a process
    pool (one worker per core, at most the host share of one GPU, 16; each worker calls the
    oracle's rhs on its chunk, which projects the whole state and evaluates its chunk's rows;
    the main process adds the chunks and does the LSRK axpy).  Also a one-core run (BLAS on
    one thread) for reference."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import esdg_oracle as O
    d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly, mass="wadg" if mass == "wadg" else "exact")
    uh0 = d.interpolate(w.u_nodes)
    Href = O.mean_free_surface(d, uh0)
    o = O.Oracle(d, w.flux, Href=Href)
    Np = dims(w.N)[0]
    ncores, model = host_cpu()
    P = max(1, min(max_workers, ncores))
    chunks = np.array_split(np.arange(w.K), P)

    def rk(stages, rhs):
        uh, du = uh0.copy(), np.zeros_like(uh0)
        t0 = time.perf_counter()
        for s in range(stages):
            du = O.LSRK_A[s % 5] * du + w.dt * rhs(uh)
            uh = uh + O.LSRK_B[s % 5] * du
        return time.perf_counter() - t0

    with mp.get_context("fork").Pool(P, initializer=_pool_init, initargs=(w, mass, Href)) as pool:
        def rhs_pool(uh):
            parts = pool.map(_pool_rhs, [(uh, ks) for ks in chunks])
            return np.concatenate(parts, axis=1)
        rk(1, rhs_pool)                         # workers built and warm
        t = rk(stages_pool, rhs_pool)
    with threadpool_limits(1):
        t1 = rk(stages_single, o.rhs)
    return {"value": w.K * Np * stages_pool / t, "unit": "DOF-updates/s per RK stage", "cores": P, "kind": "oracle",
            "sample": f"{stages_pool} RK stages ({stages_pool // 5} LSRK steps) of the same {w.K}-element N={w.N} "
                      f"workload, dense FP64 numpy oracle, each stage's RHS over {P} worker processes by element "
                      f"chunks, {t:.1f} s",
            "host": {"nproc": ncores, "cpu_model": model},
            "single_core": {"value": w.K * Np * stages_single / t1, "cores": 1,
                            "sample": f"{stages_single} RK stages, one process, BLAS on one thread, {t1:.1f} s"}}


# FLOPs per matrix entry and element in the Section 5.4 volume terms: traditional, 2 matrices x
# 3 fields multiply-adds (12); entropy-stable, the same plus the two-point flux (six averages
# 12, pressure 4, flux products 6): 34
VOLUME_FLOPS = {"traditional": 12, "entropy_stable": 34}


def volume_ratio(args, torch):
    """Section 5.4: time of the entropy-stable volume term over the traditional one for random
    n x n matrices, on the GPU (HIP events, median of 5 launches, FP64 and FP32) and on one
    host core (the oracle's plain C versions, FP64), for n = 10..250."""
    from paper_2005_02516_amd.binding import esdg_volume_kernel
    sizes = [int(x) for x in args.volume_sizes.split(",")]
    rows = []
    for n in sizes:
        K = max(64, min(1 << 22, (1 << 28) // (n * n)))
        rng = np.random.default_rng(n)
        Qx, Qy = rng.standard_normal((n, n)), rng.standard_normal((n, n))
        h = rng.uniform(1.0, 2.0, (K, n))
        u = np.stack([h, h * rng.uniform(-0.5, 0.5, (K, n)), h * rng.uniform(-0.5, 0.5, (K, n))])
        row = {"n": n, "K_gpu": K}
        for prec, tdt in (("fp64", torch.float64), ("fp32", torch.float32)):
            QxT = torch.tensor(np.ascontiguousarray(Qx.T), dtype=tdt, device="cuda:0")
            QyT = torch.tensor(np.ascontiguousarray(Qy.T), dtype=tdt, device="cuda:0")
            ud = torch.tensor(u, dtype=tdt, device="cuda:0")
            r = torch.empty_like(ud)
            t = {}
            for kind in ("traditional", "entropy_stable"):
                esdg_volume_kernel(kind, QxT, QyT, ud, r, 9.81)
                times = []
                for _ in range(5):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    esdg_volume_kernel(kind, QxT, QyT, ud, r, 9.81)
                    e1.record()
                    e1.synchronize()
                    times.append(e0.elapsed_time(e1) * 1e3)
                t[kind] = float(np.median(times))
            row[prec] = {"t_traditional_us": round(t["traditional"], 2), "t_entropy_stable_us": round(t["entropy_stable"], 2),
                         "R_GPU": round(t["entropy_stable"] / t["traditional"], 3),
                         "TFLOPs_traditional": round(VOLUME_FLOPS["traditional"] * K * n * n / t["traditional"] / 1e6, 3),
                         "TFLOPs_entropy_stable": round(VOLUME_FLOPS["entropy_stable"] * K * n * n / t["entropy_stable"] / 1e6, 3)}
            del QxT, QyT, ud, r
        if not args.no_cpu_baseline:
            from oracle import volume_kernels as V
            if not os.path.exists(V.C_LIBRARY):
                V.build_c()
            Kc = max(1, min(K, (1 << 21) // (n * n)))
            tc = {}
            for kind, key in (("dg", "traditional"), ("esdg", "entropy_stable")):
                t0 = time.perf_counter()
                V.c_volume(kind, Qx, Qy, u[:, :Kc], 9.81)
                tc[key] = (time.perf_counter() - t0) / Kc
            row["cpu_fp64_one_core"] = {"K": Kc, "t_traditional_us_per_element": round(tc["traditional"] * 1e6, 3),
                                        "t_entropy_stable_us_per_element": round(tc["entropy_stable"] * 1e6, 3),
                                        "R_CPU": round(tc["entropy_stable"] / tc["traditional"], 3)}
        print(f"# n={n}: R_GPU fp64 {row['fp64']['R_GPU']}, fp32 {row['fp32']['R_GPU']}"
              + (f", R_CPU {row['cpu_fp64_one_core']['R_CPU']}" if "cpu_fp64_one_core" in row else ""),
              file=sys.stderr, flush=True)
        rows.append(row)
    print(json.dumps({"metric": "entropy-stable / traditional DG volume-kernel time ratio (Section 5.4)",
                      "value": rows[[r["n"] for r in rows].index(50)]["fp64"]["R_GPU"] if 50 in sizes else None,
                      "unit": "ratio (R_GPU, FP64, n=50)", "higher_is_better": False, "n_gpus": 1,
                      "data": "synthetic: random matrices and states, seeded", "per_size": rows,
                      "flops_per_entry": VOLUME_FLOPS}), flush=True)


def ensemble(args, torch):
    """Batched ensemble: independent instances (K ~ U{2048..32768}, N ~ U{2,3,4}, seeded
    bathymetry and Gaussian perturbations) advanced together, one launch per RK stage."""
    from paper_2005_02516_amd import workloads as wl
    from paper_2005_02516_amd.binding import EsdgSwe
    t0 = time.perf_counter()
    ws = wl.config4_instances(count=args.ensemble)
    print(f"# ensemble: {len(ws)} instances, {sum(w.K for w in ws)} elements, built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dts = np.array([w.dt for w in ws])
    dof = sum(w.K * dims(w.N)[0] for w in ws)
    dof3 = sum(w.K * dims(w.N)[0] for w in ws if w.N == 3)
    res = {}
    for prec in ([args.precision] + ([] if args.no_fp64 else ["fp64"])):
        t0 = time.perf_counter()
        s = EsdgSwe(ws, precision=prec, flux="lf", g=1.0, use_graph=not args.no_graph,
                    matrix_cores=args.matrix_cores, fused=FUSED_ARG[args.launch], mass=args.mass)
        for i, w in enumerate(ws):
            s.set_state(i, w.u_nodes)
        print(f"# {prec}: planned and set in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        s.step(dts, args.warmup)
        s.sync()
        ms = time_steps(s, dts, args.steps, torch)
        s.sync()
        res[prec] = ms
        print(f"# {prec}: {ms / args.steps * 1e3:.1f} us/step, {ms / (5 * args.steps) * 1e3:.1f} us/stage",
              file=sys.stderr, flush=True)
        s.close()
    t_stage = res[args.precision] * 1e-3 / (5 * args.steps)
    out = {"metric": "DOF-updates/s per RK stage, batched ensemble (all instances, one launch per stage)",
           "value": dof / t_stage, "unit": "DOF-updates/s per RK stage", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res[args.precision] / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64",
           "data": "synthetic",
           "config": {"workload": f"ensemble of {len(ws)} periodic curved instances, K~U{{2048..32768}}, "
                                  f"N~U{{2,3,4}}, LF flux, LSRK4(5)",
                      "instances": len(ws), "elements": int(sum(w.K for w in ws)), "DOF": int(dof),
                      "DOF_N3": int(dof3)}}
    if "fp64" in res and args.precision != "fp64":
        out["fp64_value"] = dof / (res["fp64"] * 1e-3 / (5 * args.steps))
        out["speedup_vs_fp64"] = out["value"] / out["fp64_value"]
    # roofline of the one stage kernel launch that serves every instance, on algorithmic
    # FLOPs and bytes summed over the instances (no counter summary is taken for this mix)
    wadg = args.mass == "wadg"
    word = 8 if args.precision == "fp64" else 4
    flops = sum(alg_flops_per_elem(w.N, wadg) * w.K for w in ws)
    byts = sum(alg_bytes_per_elem(w.N, word, wadg) * w.K for w in ws)
    tf, gbs = flops / t_stage / 1e12, byts / t_stage / 1e9
    peak_alu = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
    if tf / peak_alu >= gbs / PEAK_HBM_GBS:
        roof = {"bound": "alu", "achieved": round(tf, 3), "peak": peak_alu, "unit": "TFLOP/s",
                "frac": round(tf / peak_alu, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None}
    roof["per_stage"] = {"alg_flops": flops, "alg_bytes": byts, "duration_us": round(t_stage * 1e6, 3),
                         "other_bound": ({"hbm_GBs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
                                         if roof["bound"] == "alu" else
                                         {"alu_TFLOPs": round(tf, 3), "frac": round(tf / peak_alu, 4)})}
    trace = os.path.join(ROOT, "profiles", "stage_kernel_ensemble_256.md")
    if args.ensemble == 256 and not args.matrix_cores and not wadg and os.path.exists(trace):
        roof["per_stage"]["duration_source"] = ("HIP events on the solver stream over the timed steps, per RK "
                                                "stage (rocprofv3 kernel trace of this workload: "
                                                "profiles/stage_kernel_ensemble_256.md)")
    out["roofline"] = roof
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--n", type=int, default=64, help="squares per side (64 -> 8192 triangles)")
    ap.add_argument("--N", type=int, default=3)
    ap.add_argument("--epb", type=int, default=0, help="elements per workgroup (0 = tuned default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--launch", choices=["auto", "per-stage", "fused"], default="auto",
                    help="per-stage: one launch per RK stage (graph replays); fused: all stages of a step "
                         "call in one launch of resident workgroups with neighbour-tile waits; auto (default): fused "
                         "when every workgroup holds one tile, which then stays in LDS")
    ap.add_argument("--volume-ratio", action="store_true",
                    help="the Section 5.4 volume-kernel cost ratio (entropy-stable / traditional) instead")
    ap.add_argument("--volume-sizes", default="10,25,50,100,150,200,250")
    ap.add_argument("--walls", action="store_true",
                    help="the closed curved-wall basin (reflective walls) instead of the periodic workload")
    ap.add_argument("--mass", choices=["stored", "wadg"], default="stored",
                    help="inverse curved mass matrices: stored per element (default), or the "
                         "weight-adjusted inverse (w/J per volume node)")
    ap.add_argument("--matrix-cores", action="store_true",
                    help="projection/lift contractions on the matrix cores in the bulk precision")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="time the batched ensemble of this many instances instead (256 = the full ensemble)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this solver runs on a single MI355X "
              "(multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4,
                          "launches": 5}), flush=True)
        return
    from paper_2005_02516_amd import workloads as wl
    from paper_2005_02516_amd.binding import EsdgSwe

    if args.ensemble:
        return ensemble(args, torch)
    if args.volume_ratio:
        return volume_ratio(args, torch)
    w = wl.basin(n=args.n, N=args.N) if args.walls else wl.config2(n=args.n, N=args.N)
    Np, Nq, Nfq, Nh = dims(w.N)
    dof = w.K * Np
    print(f"# workload: K={w.K} N={w.N} Np={Np} DOF={dof} dt={w.dt:.4e}", file=sys.stderr, flush=True)

    results = {}
    states = {}
    epb_used = {}
    plans = {}
    precs = [args.precision] + ([] if args.no_fp64 or args.precision == "fp64" else ["fp64"])
    for prec in precs:
        s = EsdgSwe([w], precision=prec, flux=w.flux, g=w.g, elems_per_block=args.epb, use_graph=not args.no_graph,
                    matrix_cores=args.matrix_cores, fused=FUSED_ARG[args.launch], mass=args.mass)
        plans[prec] = s.launch_info()
        e = s.elems_per_block
        epb_used[prec] = int(e.get(w.N, 0)) if isinstance(e, dict) else int(e or 0)
        s.set_state(0, w.u_nodes)
        s.step(w.dt, args.warmup)
        s.sync()
        ms = time_steps(s, w.dt, args.steps, torch)
        s.sync()
        states[prec] = s.get_state(0)
        results[prec] = ms
        print(f"# {prec}: {ms:.3f} ms for {args.steps} steps -> {ms / args.steps * 1e3:.2f} us/step, "
              f"{ms / (5 * args.steps) * 1e3:.2f} us/stage", file=sys.stderr, flush=True)
        s.close()

    prec = args.precision
    ms = results[prec]
    t_stage = ms * 1e-3 / (5 * args.steps)
    value = dof / t_stage
    word = 8 if prec == "fp64" else 4
    wadg = args.mass == "wadg"
    flops = alg_flops_per_elem(w.N, wadg) * w.K
    byts = alg_bytes_per_elem(w.N, word, wadg) * w.K
    achieved_tf = flops / t_stage / 1e12
    achieved_gbs = byts / t_stage / 1e9
    peak_alu = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
    frac_alu = achieved_tf / peak_alu
    frac_hbm = achieved_gbs / PEAK_HBM_GBS
    step_mode = plans[prec]["step_mode"]
    stages_per_launch = 1 if step_mode == 0 else 5 * args.steps
    tr = None if (wadg or args.walls) else measured_traffic(w, prec, epb_used.get(prec, 0), step_mode, stages_per_launch)
    # which roof binds: with measured traffic, the HBM side is what the kernel really moves
    # (tiles resident in LDS move far less than the algorithmic bytes); else the larger of
    # the two algorithmic fractions
    frac_hbm_real = (tr["fetch"] + tr["write"]) / t_stage / 1e9 / PEAK_HBM_GBS if tr else frac_hbm
    if frac_alu >= frac_hbm_real:
        roof = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": peak_alu, "unit": "TFLOP/s",
                "frac": round(frac_alu, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(frac_hbm, 4), "traffic": None}
    if tr is not None:
        roof["traffic"] = tr["fetch"] + tr["write"]
        roof["traffic_detail"] = {"fetch_bytes": tr["fetch"], "write_bytes": tr["write"],
                                  "GBs_at_this_duration": round((tr["fetch"] + tr["write"]) / t_stage / 1e9, 1),
                                  "counters": "FETCH_SIZE x2.0 + WRITE_SIZE x1.0 (copy-calibrated)",
                                  "source": tr["source"]}
    roof["kernel"] = "stage_kernel (fused RK stage: flux differencing + interface + lift + update + projection)"
    trace_summary = kernel_trace_summary(w, args)
    # a multi-stage launch covers 5 * steps stages: its algorithmic work and its duration are
    # both that many stages', so the per-stage figures give the same rates
    roof["per_stage"] = {"alg_flops": flops, "alg_bytes": byts, "duration_us": round(t_stage * 1e6, 3),
                         "stages_per_launch": stages_per_launch,
                         "duration_source": "HIP events on the solver stream over the timed steps, per RK stage"
                                            + (f" (rocprofv3 kernel trace of this workload: {trace_summary})"
                                               if trace_summary else ""),
                         "other_bound": ({"hbm_GBs": round(achieved_gbs, 1), "frac": round(frac_hbm, 4)}
                                         if roof["bound"] == "alu" else
                                         {"alu_TFLOPs": round(achieved_tf, 3), "frac": round(frac_alu, 4)})}
    out = {
        "metric": "DOF-updates/s per RK stage at N=3; FP32/batched vs FP64 speedup at stated error",
        "value": value,
        "unit": "DOF-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "f32 (bf16x3 contractions)"}[prec],
        "data": "synthetic",
        "config": {"workload": (f"closed curved-wall basin (reflective walls), smoothed dam-break start, "
                                if args.walls else "curved periodic lake at rest + Gaussian bump, ") +
                               f"{args.n}x{args.n}x2={w.K} triangles, "
                               f"N={w.N} (Np={Np}, Nq={Nq}, Nfq={Nfq}), LF flux, LSRK4(5)",
                   "K": w.K, "N": w.N, "DOF": dof, "precision": prec,
                   "hip_graph": (not args.no_graph) and plans[prec]["step_mode"] == 0,
                   "elements_per_workgroup": epb_used.get(prec, 0),
                   "matrix_cores": bool(args.matrix_cores or prec == "bf16x3"),
                   "mass_inverse": {"stored": "stored per element", "wadg": "weight-adjusted"}[args.mass],
                   "launch": STEP_MODES[plans[prec]["step_mode"]],
                   "workgroups": plans[prec]["resident_workgroups"], "tiles": plans[prec]["tiles"]},
        "roofline": roof,
    }
    if "fp64" in results and prec != "fp64":
        v64 = dof / (results["fp64"] * 1e-3 / (5 * args.steps))
        a, b = states[prec], states["fp64"]
        hn = float(np.linalg.norm(b[0]))
        out["fp64_value"] = v64
        out["speedup_vs_fp64"] = value / v64
        out["rel_l2_vs_fp64_after_steps"] = {
            "steps": args.steps + args.warmup,
            "h": float(np.linalg.norm(a[0] - b[0]) / hn),
            "hu_over_norm_h": float(np.linalg.norm(a[1] - b[1]) / hn),
            "hv_over_norm_h": float(np.linalg.norm(a[2] - b[2]) / hn),
            "hu": float(np.linalg.norm(a[1] - b[1]) / max(np.linalg.norm(b[1]), 1e-300)),
            "hv": float(np.linalg.norm(a[2] - b[2]) / max(np.linalg.norm(b[2]), 1e-300)),
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, mass=args.mass)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
