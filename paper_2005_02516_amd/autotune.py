"""Autotuner for the elements-per-workgroup tile size of the RK-stage kernel.

The stage kernel's LDS footprint, and so its occupancy, grows with the number of elements
per workgroup E, while small E leaves threads idle in every phase; the best E depends on
the degree N, the precision and how many elements there are in total.  ``tune`` times a
few LSRK steps for every candidate E (HIP events on the solver's stream) and records the
fastest in a JSON cache keyed by precision, N and a size class of the element count;
``lookup`` reads it when a solver is created without an explicit tile size.

Run ``python -m paper_2005_02516_amd.autotune --write`` on the GPU to refresh the cache.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from typing import Dict, Iterable, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache_gfx950.json")
CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64)


def size_class(K: int) -> str:
    """S: < 32768 elements, M: < 262144, L: larger."""
    return "S" if K < 32768 else ("M" if K < 262144 else "L")


def _key(precision: str, N: int, K: int) -> str:
    return f"{precision}:N{N}:{size_class(K)}"


def _load() -> dict:
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        return json.load(f)


def ref_words(N: int) -> int:
    """LDS reals of the reference block of degree N (rounded up to 4, as the library does)."""
    Np, Nq, Nfq = (N + 1) * (N + 2) // 2, (N + 1) ** 2, 3 * (N + 1)
    Nh = Nq + Nfq
    return (Nh * Np + 2 * Nh * Nq + 2 * Nq * Nfq + 3 * Nfq + 3) // 4 * 4


def tile_words(N: int, E: int) -> int:
    """LDS reals of one tile of E elements of degree N (stored mass inverse)."""
    Np, Nq, Nfq = (N + 1) * (N + 2) // 2, (N + 1) ** 2, 3 * (N + 1)
    Nh = Nq + Nfq
    return E * (Nh * 12 + 8 * Nh + 4 * Nfq + 6 * Np + Np * Np + 2 * Nq + Nh + Nfq)


# LDS per workgroup at which four workgroups share a CU (160 KiB), the residency the stage
# kernel's register budget allows, and the static LDS the kernel adds to the dynamic request
LDS_FOUR_PER_CU = 40 * 1024
STATIC_LDS = 256


def fit_mixed(precision: str, epb: Dict[int, int]) -> Dict[int, int]:
    """One launch serves every degree with the LDS of the largest reference block plus the
    largest tile, so a tile size tuned for a degree alone can lower the residency of all of
    them.  Shrink each degree's E (through the candidate sizes) until the shared LDS fits
    the larger of four workgroups per CU and what the degrees needed on their own."""
    if len(epb) < 2:
        return dict(epb)
    word = 8 if precision == "fp64" else 4
    ref_max = max(ref_words(N) for N in epb)
    alone = max((ref_words(N) + tile_words(N, E)) * word + STATIC_LDS for N, E in epb.items())
    budget = max(LDS_FOUR_PER_CU, alone)
    out = {}
    for N, E in epb.items():
        while E > 1 and (ref_max + tile_words(N, E)) * word + STATIC_LDS > budget:
            E = max(c for c in CANDIDATES if c < E)
        out[N] = E
    return out


def lookup(precision: str, sizes: Iterable[Tuple[int, int]]) -> Optional[Dict[int, int]]:
    """Tuned E per degree for instances of (N, K); the total K of each degree picks the class
    (with several degrees, fitted to their shared LDS: fit_mixed)."""
    cache = _load().get("entries", {})
    totals: Dict[int, int] = {}
    for N, K in sizes:
        totals[N] = totals.get(N, 0) + K
    out = {}
    order = {"S": ("S", "M", "L"), "M": ("M", "L", "S"), "L": ("L", "M", "S")}
    for N, K in totals.items():
        # nearest tuned size class; the bf16x3 mode has the float LDS footprint
        for prec in ((precision, "fp32") if precision == "bf16x3" else (precision,)):
            e = next((cache[f"{prec}:N{N}:{cls}"] for cls in order[size_class(K)]
                      if f"{prec}:N{N}:{cls}" in cache), None)
            if e:
                out[N] = int(e["epb"])
                break
    return fit_mixed("fp32" if precision == "bf16x3" else precision, out) if out else None


def time_config(w, precision: str, epb: int, steps: int = 4, warmup: int = 1) -> float:
    """Milliseconds per RK stage for one workload at tile size epb."""
    import torch
    from .binding import EsdgSwe
    s = EsdgSwe([w], precision=precision, flux=w.flux, g=w.g, elems_per_block=epb, tuned=False)
    try:
        s.set_state(0, w.u_nodes)
        s.step(w.dt, warmup)
        s.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(w.dt, steps)
        e1.record(s.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / (5 * steps)
    finally:
        s.close()


def lds_ok(N: int, E: int, precision: str) -> bool:
    Nh = (N + 1) ** 2 + 3 * (N + 1)
    word = 8 if precision == "fp64" else 4
    return (ref_words(N) + tile_words(N, E)) * word <= 160 * 1024 and E * Nh <= 2048


def tune(cases: List[Tuple[int, int]], precisions=("fp32", "fp64"), write: bool = True, log=sys.stderr,
         out: Optional[str] = None):
    from . import workloads as wl
    data = _load()
    entries = data.setdefault("entries", {})
    for N, n in cases:
        w = wl.config2(n=n, N=N)
        for prec in precisions:
            timings = {}
            for E in CANDIDATES:
                if not lds_ok(N, E, prec):
                    continue
                timings[E] = time_config(w, prec, E, steps=4 if w.K < 100000 else 2)
                print(f"# tune {prec} N={N} K={w.K} E={E}: {timings[E] * 1e3:.1f} us/stage", file=log, flush=True)
            best = min(timings, key=timings.get)
            entries[_key(prec, N, w.K)] = {"epb": best, "K": w.K, "us_per_stage": {str(k): round(v * 1e3, 2)
                                                                                      for k, v in timings.items()}}
    data["device"] = "gfx950 (MI355X)"
    data["note"] = "written by `python -m paper_2005_02516_amd.autotune --write` on the GPU"
    if write:
        with open(out or CACHE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return data


DEFAULT_CASES = [(1, 64), (2, 64), (3, 64), (4, 64), (5, 64), (1, 256), (2, 256), (3, 256), (4, 256), (5, 256)]


def parse_cases(text: Optional[str]) -> List[Tuple[int, int]]:
    """"N:n,N:n,..." (degree, squares per side of the config-2 mesh) -> cases; empty: all."""
    if not text:
        return list(DEFAULT_CASES)
    cases = []
    for item in text.split(","):
        N, n = (int(v) for v in item.split(":"))
        if not (1 <= N <= 5 and n >= 1):
            raise ValueError(f"bad case {item!r}: need 1 <= N <= 5 and n >= 1")
        cases.append((N, n))
    return cases


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--precisions", default="fp32,fp64", help="comma-separated: fp32, fp64")
    ap.add_argument("--out", default=None, help="write the cache here instead of the package's file")
    ap.add_argument("--cases", default=None,
                    help="comma-separated N:n (degree, squares per side of the config-2 mesh); default: all")
    args = ap.parse_args()
    tune(parse_cases(args.cases), precisions=tuple(args.precisions.split(",")), write=args.write, out=args.out)
