"""Autotuner for the tiles of the RK-stage kernel: elements per workgroup E and the
residual phase's tile shape (R rows per thread, P column parts).

The stage kernel's LDS footprint, and so its occupancy, grows with the number of elements
per workgroup E, while small E leaves threads idle in every phase; the residual phase
deals (element, R rows, column part) tasks to the 256 threads, so R and P set how evenly
its rounds fill and how often a column's node record is reused; P also sizes the partial
sums in LDS.  The best choice depends on the degree N, the precision and how many
elements there are in total.  ``tune`` times a few LSRK steps for every candidate E with
the default shape, then every shape the kernel is compiled for at the best few E (HIP
events on the solver's stream), and records the fastest (E, R, P) in a JSON cache keyed by
precision, N and a size class of the element count; ``lookup_shapes`` reads it when a
solver is created without an explicit tile size.

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
CANDIDATES = (1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 48, 64)


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


def tile_words(N: int, E: int, P: int = 2) -> int:
    """LDS reals of one tile of E elements of degree N (stored mass inverse) with P column
    parts: the raw block holds the fetched values [8][Nh] and then the P partial sums
    [P][3][Nh] and the lift's output [3][Np]."""
    Np, Nq, Nfq = (N + 1) * (N + 2) // 2, (N + 1) ** 2, 3 * (N + 1)
    Nh = Nq + Nfq
    raw = max(8 * Nh, 3 * P * Nh + 3 * Np)
    rec = Nh * 12 + (4 if Nh % 2 == 0 else 0)      # node records, padded as the library pads them
    return E * (rec + raw + 4 * Nfq + 6 * Np + Np * Np + 2 * Nq + Nh + Nfq)


def shape_code(R: int, P: int) -> int:
    """Packed tile shape, as the library takes it: (R << 4) | P."""
    return (R << 4) | P


def default_shape(N: int, precision: str) -> Tuple[int, int]:
    """The library's default (R, P)."""
    return (2 if precision != "fp64" and N in (1, 3) else 1), (1 if N == 5 else 2)


def shapes(N: int, precision: str) -> List[Tuple[int, int]]:
    """(R, P) the stage kernel is compiled for: R = 1, or 2 in float where 2 divides
    Nq = (N+1)^2 and Nfq = 3(N+1); P = 1..4."""
    rows = [1] + ([2] if precision != "fp64" and (N + 1) % 2 == 0 else [])
    return [(R, P) for R in rows for P in (1, 2, 3, 4)]


# LDS per workgroup at which four workgroups share a CU (160 KiB), the residency the stage
# kernel's register budget allows, and the static LDS the kernel adds to the dynamic request
LDS_FOUR_PER_CU = 40 * 1024
STATIC_LDS = 256


def fit_mixed(precision: str, epb: Dict[int, int], shp: Optional[Dict[int, int]] = None) -> Dict[int, int]:
    """One launch serves every degree with the LDS of the largest reference block plus the
    largest tile, so a tile size tuned for a degree alone can lower the residency of all of
    them.  Shrink each degree's E (through the candidate sizes) until the shared LDS fits
    the larger of four workgroups per CU and what the degrees needed on their own."""
    if len(epb) < 2:
        return dict(epb)
    word = 8 if precision == "fp64" else 4
    parts = {N: ((shp or {}).get(N, 0) & 15) or default_shape(N, precision)[1] for N in epb}
    ref_max = max(ref_words(N) for N in epb)
    alone = max((ref_words(N) + tile_words(N, E, parts[N])) * word + STATIC_LDS for N, E in epb.items())
    budget = max(LDS_FOUR_PER_CU, alone)
    out = {}
    for N, E in epb.items():
        while E > 1 and (ref_max + tile_words(N, E, parts[N])) * word + STATIC_LDS > budget:
            E = max(c for c in CANDIDATES if c < E)
        out[N] = E
    return out


def lookup(precision: str, sizes: Iterable[Tuple[int, int]]) -> Optional[Dict[int, int]]:
    """Tuned E per degree for instances of (N, K); the total K of each degree picks the class
    (with several degrees, fitted to their shared LDS: fit_mixed)."""
    return lookup_shapes(precision, sizes)[0]


def lookup_shapes(precision: str, sizes: Iterable[Tuple[int, int]], valu: bool = True):
    """(E per degree, packed tile shape per degree) for instances of (N, K), or (None,
    None) without cache entries; a degree whose entry has no shape gets the library's
    default.  The shapes were timed on single-degree workloads with vector-ALU
    contractions, so a launch of several degrees, the split-bf16 mode or matrix-core
    contractions (valu False) take the default shape and the best E timed with it; several degrees then have E fitted to the shared
    LDS (fit_mixed)."""
    cache = _load().get("entries", {})
    totals: Dict[int, int] = {}
    for N, K in sizes:
        totals[N] = totals.get(N, 0) + K
    own_shape = len(totals) == 1 and precision != "bf16x3" and valu
    out, shp = {}, {}
    order = {"S": ("S", "M", "L"), "M": ("M", "L", "S"), "L": ("L", "M", "S")}
    for N, K in totals.items():
        # nearest tuned size class; the bf16x3 mode has the float LDS footprint
        for prec in ((precision, "fp32") if precision == "bf16x3" else (precision,)):
            e = next((cache[f"{prec}:N{N}:{cls}"] for cls in order[size_class(K)]
                      if f"{prec}:N{N}:{cls}" in cache), None)
            if e:
                if "rows" in e and own_shape:
                    out[N] = int(e["epb"])
                    shp[N] = shape_code(int(e["rows"]), int(e["parts"]))
                elif "rows" in e:           # the fastest E with the default shape
                    t = e["us_per_stage"]
                    out[N] = int(min(t, key=lambda E: t[E]))
                else:
                    out[N] = int(e["epb"])
                break
    if not out:
        return None, None
    return fit_mixed("fp32" if precision == "bf16x3" else precision, out, shp), (shp or None)


def time_config(w, precision: str, epb: int, steps: int = 4, warmup: int = 1, shape: Optional[int] = None) -> float:
    """Milliseconds per RK stage for one workload at tile size epb (and packed tile shape)."""
    import torch
    from .binding import EsdgSwe
    s = EsdgSwe([w], precision=precision, flux=w.flux, g=w.g, elems_per_block=epb, tuned=False, tile_shape=shape)
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


def lds_ok(N: int, E: int, precision: str, P: Optional[int] = None) -> bool:
    """The tile of E elements fits the LDS with P column chunks (default: the library's
    default shape)."""
    P = default_shape(N, precision)[1] if P is None else P
    Nh = (N + 1) ** 2 + 3 * (N + 1)
    word = 8 if precision == "fp64" else 4
    return (ref_words(N) + tile_words(N, E, P)) * word <= 160 * 1024 and E * Nh <= 2048


def tune(cases: List[Tuple[int, int]], precisions=("fp32", "fp64"), write: bool = True, log=sys.stderr,
         out: Optional[str] = None, around_cached: bool = False, top: int = 3):
    """around_cached: time only the candidate E within a factor of two of the cached entry's
    (when there is one), to refresh large classes in less time; top: how many of the best E
    get every tile shape timed."""
    from . import workloads as wl
    data = _load()
    entries = data.setdefault("entries", {})
    for N, n in cases:
        w = wl.config2(n=n, N=N)
        steps = 4 if w.K < 100000 else 2
        for prec in precisions:
            # E with the default shape, then every compiled shape at the three best E
            timings = {}
            R0, P0 = default_shape(N, prec)
            cached = entries.get(_key(prec, N, w.K), {}).get("epb") if around_cached else None
            for E in CANDIDATES:
                if not lds_ok(N, E, prec, P0) or (cached and not cached / 2 <= E <= cached * 2):
                    continue
                timings[E] = time_config(w, prec, E, steps=steps, shape=shape_code(R0, P0))
                print(f"# tune {prec} N={N} K={w.K} E={E}: {timings[E] * 1e3:.1f} us/stage", file=log, flush=True)
            shaped = {(E, R0, P0): timings[E] for E in timings}
            for E in sorted(timings, key=timings.get)[:top]:
                for R, P in shapes(N, prec):
                    if (E, R, P) in shaped or not lds_ok(N, E, prec, P):
                        continue
                    shaped[(E, R, P)] = time_config(w, prec, E, steps=steps, shape=shape_code(R, P))
                    print(f"# tune {prec} N={N} K={w.K} E={E} R={R} P={P}: {shaped[(E, R, P)] * 1e3:.1f} us/stage",
                          file=log, flush=True)
            E, R, P = min(shaped, key=shaped.get)
            entries[_key(prec, N, w.K)] = {
                "epb": E, "rows": R, "parts": P, "K": w.K,
                "us_per_stage": {str(k): round(v * 1e3, 2) for k, v in timings.items()},
                "shape_us_per_stage": {f"{e}:{r}:{p}": round(v * 1e3, 2) for (e, r, p), v in shaped.items()}}
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
    ap.add_argument("--around-cached", action="store_true",
                    help="time only E within a factor of two of the cached entry's")
    ap.add_argument("--top", type=int, default=3, help="E values whose tile shapes are all timed")
    args = ap.parse_args()
    tune(parse_cases(args.cases), precisions=tuple(args.precisions.split(",")), write=args.write, out=args.out,
         around_cached=args.around_cached, top=args.top)
