"""Seeded synthetic inputs for the shallow-water ESDG solver.

This module places points and evaluates analytic fields at them.  It holds none of
the discretisation's arithmetic (no basis, quadrature, projection, flux or time
integration), so both the CPU oracle and the HIP library can start from exactly the
same inputs:

* a structured periodic triangulation of a rectangle, optionally warped, given as
  the equispaced isoparametric geometry nodes of every element;
* the bathymetry ``b`` and the initial conservative state ``(h, hu, hv)`` sampled at
  those nodes (``b`` sampled at shared nodes is therefore C0 across elements, as the
  lake-at-rest experiment of Section 4.1 requires);
* a time step following the CFL rule of Section 4 (``dt = CFL * h / C_N``, scaled by
  the largest wave speed, because that rule leaves the wave speed implicit).

Reference-element node convention (used by the library header as well): the
reference triangle has counter-clockwise vertices v1=(-1,-1), v2=(1,-1), v3=(-1,1);
the order-N equispaced nodes are listed as ``for j in 0..N: for i in 0..N-j:
(r, s) = (-1 + 2 i / N, -1 + 2 j / N)``, so node 0 is v1, node N is v2 and the last
node is v3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload",
    "equispaced_index",
    "structured_mesh",
    "timestep",
    "config1",
    "config2",
    "config3",
    "config4_instances",
    "config5",
    "basin",
    "basin_mesh",
    "vortex_fields",
    "make_config",
]


def npts(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def equispaced_index(N: int):
    """Integer lattice offsets (i, j) of the equispaced nodes in the documented order."""
    ij = [(i, j) for j in range(N + 1) for i in range(N + 1 - j)]
    return np.array(ij, dtype=np.int64)


@dataclass
class Workload:
    """One shallow-water instance: mesh, bathymetry, initial state and run recipe."""

    name: str
    N: int
    n: int                      # squares per side
    K: int
    xg: np.ndarray              # [K, Np] geometry node x (warped)
    yg: np.ndarray              # [K, Np] geometry node y (warped)
    xf: np.ndarray              # [K, Np] x where fields are sampled (periodic image)
    yf: np.ndarray              # [K, Np]
    Lx: float
    Ly: float
    g: float
    b_nodes: np.ndarray         # [K, Np]
    u_nodes: np.ndarray         # [3, K, Np]: h, hu, hv
    flux: str                   # "ec" (no dissipation) or "lf" (Lax-Friedrichs)
    cfl: float
    steps: int
    dt: float = 0.0
    precision: str = "fp64"
    seed: int = 0
    meta: dict = field(default_factory=dict)


def structured_mesh(n: int, N: int, L: float = 2.0, warp: float = 0.0, x0: float = 0.0, y0: float = 0.0):
    """n x n squares on [x0, x0+L]^2, each split along its lower-left/upper-right diagonal.

    Square (i, j) gives the two counter-clockwise triangles
    (p00, p10, p11) and (p00, p11, p01).  Element nodes are points of the global
    (nN+1)^2 lattice, so nodes shared by two elements get bit-identical coordinates.
    The warp (when nonzero) moves every node by ``warp * sin(pi x) sin(pi y)`` in x and
    in y, evaluated at the unwarped position; it vanishes on the boundary of [0,2]^2, so
    the periodic matching survives it.

    Returns (xg, yg, xf, yf) as [K, Np] arrays: the warped geometry nodes, and the warped
    coordinates of the periodic image (lattice index mod nN) used to sample fields.
    """
    ij = equispaced_index(N)
    M = n * N
    hl = L / M
    # squares in the order (jq, iq) row-major; each gives its lower then its upper triangle
    jq, iq = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    bi = (iq.reshape(-1) * N)[:, None]
    bj = (jq.reshape(-1) * N)[:, None]
    i_, j_ = ij[None, :, 0], ij[None, :, 1]
    # lower triangle: v1=p00, v2=p10, v3=p11  -> lattice (bi + i + j, bj + j)
    # upper triangle: v1=p00, v2=p11, v3=p01  -> lattice (bi + i, bj + i + j)
    I = np.stack([bi + i_ + j_, bi + i_], axis=1).reshape(-1, ij.shape[0])
    J = np.stack([bj + j_, bj + i_ + j_], axis=1).reshape(-1, ij.shape[0])

    def place(Ii, Jj):
        x = x0 + Ii * hl
        y = y0 + Jj * hl
        if warp != 0.0:
            d = warp * np.sin(np.pi * (x - x0)) * np.sin(np.pi * (y - y0))
            x, y = x + d, y + d
        return x, y

    xg, yg = place(I.astype(np.float64), J.astype(np.float64))
    xf, yf = place((I % M).astype(np.float64), (J % M).astype(np.float64))
    return xg, yg, xf, yf


def basin_mesh(n: int, N: int, wall: float = 0.15, warp: float = 0.05):
    """Closed basin: the image of [0,2]^2 under
    x' = x + wall sin(pi y / 2)(1 - x / 2) + d,  y' = y + wall sin(pi x / 2)(1 - y / 2) + d,
    d = warp sin(pi x) sin(pi y), all evaluated at the unwarped lattice position.  The left
    (x = 0) and bottom (y = 0) walls bulge into the domain along sin(pi s / 2); the right and
    top walls stay straight; d vanishes on the boundary.  Same triangulation and node order
    as structured_mesh; no periodic images (xf, yf are the node positions themselves).
    Returns (xg, yg)."""
    ij = equispaced_index(N)
    M = n * N
    hl = 2.0 / M
    jq, iq = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    bi = (iq.reshape(-1) * N)[:, None]
    bj = (jq.reshape(-1) * N)[:, None]
    i_, j_ = ij[None, :, 0], ij[None, :, 1]
    I = np.stack([bi + i_ + j_, bi + i_], axis=1).reshape(-1, ij.shape[0]).astype(np.float64)
    J = np.stack([bj + j_, bj + i_ + j_], axis=1).reshape(-1, ij.shape[0]).astype(np.float64)
    x, y = I * hl, J * hl
    d = warp * np.sin(np.pi * x) * np.sin(np.pi * y)
    xg = x + wall * np.sin(0.5 * np.pi * y) * (1.0 - 0.5 * x) + d
    yg = y + wall * np.sin(0.5 * np.pi * x) * (1.0 - 0.5 * y) + d
    return xg, yg


def timestep(u_nodes: np.ndarray, g: float, N: int, hmesh: float, cfl: float) -> float:
    """dt = CFL * hmesh / (C_N * a_max), C_N = (N+1)(N+2)/2 (Section 4), a_max = max |u| + sqrt(g h)."""
    h = u_nodes[0]
    u = u_nodes[1] / h
    v = u_nodes[2] / h
    amax = float(np.max(np.sqrt(u * u + v * v) + np.sqrt(g * h)))
    CN = (N + 1) * (N + 2) / 2.0
    return cfl * hmesh / (CN * amax)


def _finish(w: Workload) -> Workload:
    w.dt = timestep(w.u_nodes, w.g, w.N, (w.Lx / w.n), w.cfl)
    return w


def _mk(name, n, N, warp, g, b, h, hu, hv, flux, cfl, steps, precision, seed, xg, yg, xf, yf, meta=None):
    K = xg.shape[0]
    u = np.stack([h, hu, hv]).astype(np.float64)
    return _finish(Workload(name=name, N=N, n=n, K=K, xg=xg, yg=yg, xf=xf, yf=yf, Lx=2.0, Ly=2.0, g=g,
                            b_nodes=np.ascontiguousarray(b, dtype=np.float64), u_nodes=np.ascontiguousarray(u),
                            flux=flux, cfl=cfl, steps=steps, precision=precision, seed=seed, meta=meta or {}))


def config1(n: int = 8, N: int = 2) -> Workload:
    """Plain FP64: affine periodic [0,2]^2, flat b, h = 2 + 0.1 sin(pi x) sin(pi y), u=0.5, v=0.25, EC flux."""
    xg, yg, xf, yf = structured_mesh(n, N)
    h = 2.0 + 0.1 * np.sin(np.pi * xf) * np.sin(np.pi * yf)
    b = np.zeros_like(h)
    return _mk("config1", n, N, 0.0, 1.0, b, h, 0.5 * h, 0.25 * h, "ec", 0.25, 100, "fp64", 0, xg, yg, xf, yf)


def _periodic_d2(x, y, cx, cy, L=2.0):
    dx = (x - cx + 0.5 * L) % L - 0.5 * L
    dy = (y - cy + 0.5 * L) % L - 0.5 * L
    return dx * dx + dy * dy


def config2(n: int = 64, N: int = 3, seed: int = 0, bump: float = 0.01, steps: int = 500) -> Workload:
    """Curved N=3 lake at rest H=2.2 over b = 0.1 sin(pi x) cos(pi y) + 0.1 with a seeded Gaussian bump (sigma 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy = rng.uniform(0.5, 1.5, size=2)
    xg, yg, xf, yf = structured_mesh(n, N, warp=0.05)
    b = 0.1 * np.sin(np.pi * xf) * np.cos(np.pi * yf) + 0.1
    h = 2.2 - b + bump * np.exp(-50.0 * _periodic_d2(xf, yf, cx, cy))
    z = np.zeros_like(h)
    return _mk("config2", n, N, 0.05, 1.0, b, h, z, z.copy(), "lf", 0.25, steps, "fp32", seed, xg, yg, xf, yf,
               meta={"center": (float(cx), float(cy)), "H": 2.2})


def basin(n: int = 64, N: int = 3, wall: float = 0.15, dam: float = 0.2, width: float = 0.1,
          steps: int = 200) -> Workload:
    """Reflective-wall case (Section 2.9) on a boundary-fitted curved mesh: the closed basin of
    basin_mesh (periods 0: not periodic, every boundary face a wall) over
    b = 0.1 + 0.05 cos(pi x / 2) cos(pi y / 2), still water whose free surface steps down
    smoothly across x = 1 (a dam-break-like start): h + b = 1.2 + dam (1 - tanh((x - 1) /
    width)) / 2, u = v = 0, LF flux."""
    xg, yg = basin_mesh(n, N, wall=wall)
    b = 0.1 + 0.05 * np.cos(0.5 * np.pi * xg) * np.cos(0.5 * np.pi * yg)
    h = 1.2 + dam * 0.5 * (1.0 - np.tanh((xg - 1.0) / width)) - b
    z = np.zeros_like(h)
    u = np.ascontiguousarray(np.stack([h, z, z.copy()]))
    w = Workload(name="basin", N=N, n=n, K=xg.shape[0], xg=xg, yg=yg, xf=xg, yf=yg, Lx=0.0, Ly=0.0, g=1.0,
                 b_nodes=np.ascontiguousarray(b), u_nodes=u, flux="lf", cfl=0.25, steps=steps, precision="fp32",
                 seed=0, meta={"walls": True})
    w.dt = timestep(u, w.g, N, 2.0 / n, w.cfl)
    return w


def near_dry(n: int = 8, N: int = 3, hmin: float = 1e-3, speed: float = 0.05, steps: int = 5) -> Workload:
    """Shallow water over a bump: the config-2 mesh, b = 0.2 + 0.1 sin(pi x) sin(pi y) (0.1 to
    0.3), free surface level 0.3 + hmin (depth hmin over the bump's top, about 0.2 elsewhere),
    moving water u = speed cos(pi y), v = speed sin(pi x), LF flux."""
    xg, yg, xf, yf = structured_mesh(n, N, warp=0.05)
    b = 0.2 + 0.1 * np.sin(np.pi * xf) * np.sin(np.pi * yf)
    h = 0.3 + hmin - b
    u = speed * np.cos(np.pi * yf)
    v = speed * np.sin(np.pi * xf)
    return _mk("near_dry", n, N, 0.05, 1.0, b, h, h * u, h * v, "lf", 0.25, steps, "fp32", 0, xg, yg, xf, yf,
               meta={"hmin": hmin})


def _fourier(rng, x, y, nmodes, amax, kmax=4):
    out = np.zeros_like(x)
    for _ in range(nmodes):
        a = rng.uniform(0.0, amax)
        while True:
            k, l = rng.integers(-kmax, kmax + 1, size=2)
            if k != 0 or l != 0:
                break
        ph = rng.uniform(0.0, 2.0 * np.pi)
        out = out + a * np.sin(np.pi * (k * x + l * y) + ph)
    return out


def config3(n: int = 256, N: int = 4, seed: int = 0, steps: int = 200) -> Workload:
    """Large single instance: 16-mode random Fourier b (amplitudes <= 0.05), h = 2.5 - b + eta, smooth u, v."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xg, yg, xf, yf = structured_mesh(n, N, warp=0.05)
    b = _fourier(rng, xf, yf, 16, 0.05)
    eta = _fourier(rng, xf, yf, 4, 0.05)
    h = 2.5 - b + eta
    u = _fourier(rng, xf, yf, 4, 0.075)
    v = _fourier(rng, xf, yf, 4, 0.075)
    return _mk("config3", n, N, 0.05, 1.0, b, h, h * u, h * v, "lf", 0.25, steps, "fp32", seed, xg, yg, xf, yf)


def config4_instances(count: int = 256, seed0: int = 1000, kmin: int = 2048, kmax: int = 32768,
                      steps: int = 100, n_override: Optional[List[int]] = None,
                      N_override: Optional[List[int]] = None) -> List[Workload]:
    """Ensemble: instance i draws K ~ U{kmin..kmax} (rounded to 2 n^2) and N ~ U{2,3,4} from PCG64(seed0 + i)."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        K = int(rng.integers(kmin, kmax + 1))
        n = max(2, int(round(math.sqrt(K / 2.0))))
        N = int(rng.integers(2, 5))
        if n_override is not None:
            n = n_override[i]
        if N_override is not None:
            N = N_override[i]
        xg, yg, xf, yf = structured_mesh(n, N, warp=0.05)
        b = _fourier(rng, xf, yf, 16, 0.05)
        h = 2.2 - b
        for _ in range(3):
            cx, cy = rng.uniform(0.0, 2.0, size=2)
            h = h + 0.01 * np.exp(-50.0 * _periodic_d2(xf, yf, cx, cy))
        z = np.zeros_like(h)
        out.append(_mk(f"config4[{i}]", n, N, 0.05, 1.0, b, h, z, z.copy(), "lf", 0.25, steps, "fp32", seed0 + i,
                       xg, yg, xf, yf))
    return out


def vortex_fields(x, y, t, g, hinf, A, R, xc, yc, uinf, vinf, L=2.0):
    """Translating vortex (steady in the frame moving with (uinf, vinf)), periodic minimum image.

    h = hinf - A^2/(4g) e^{2(1 - r^2/R^2)}, u = uinf - A (y_t/R) e^{1 - r^2/R^2},
    v = vinf + A (x_t/R) e^{1 - r^2/R^2}, with (x_t, y_t) the offset from the moving centre.
    This satisfies g dh/dr = u_theta^2 / r exactly.
    """
    xt = (x - xc - uinf * t + 0.5 * L) % L - 0.5 * L
    yt = (y - yc - vinf * t + 0.5 * L) % L - 0.5 * L
    r2 = (xt * xt + yt * yt) / (R * R)
    e = np.exp(1.0 - r2)
    h = hinf - (A * A / (4.0 * g)) * e * e
    u = uinf - A * (yt / R) * e
    v = vinf + A * (xt / R) * e
    return h, u, v


def config5(n: int = 512, N: int = 5, seed: int = 0, steps: int = 100) -> Workload:
    """High order: translating vortex (g=1, h_inf=1, A=0.2, R=0.1), seeded centre and direction, b=0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy = rng.uniform(0.5, 1.5, size=2)
    th = rng.uniform(0.0, 2.0 * np.pi)
    uinf, vinf = 0.5 * math.cos(th), 0.5 * math.sin(th)
    xg, yg, xf, yf = structured_mesh(n, N, warp=0.05)
    h, u, v = vortex_fields(xf, yf, 0.0, 1.0, 1.0, 0.2, 0.1, cx, cy, uinf, vinf)
    b = np.zeros_like(h)
    return _mk("config5", n, N, 0.05, 1.0, b, h, h * u, h * v, "lf", 0.25, steps, "fp32", seed, xg, yg, xf, yf,
               meta={"center": (float(cx), float(cy)), "uinf": (uinf, vinf), "A": 0.2, "R": 0.1})


def make_config(name: str, **kw) -> Workload:
    return {"config1": config1, "config2": config2, "config3": config3, "config5": config5}[name](**kw)
