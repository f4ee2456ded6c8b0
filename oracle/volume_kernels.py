"""Volume-kernel cost comparison of Section 5.4: oracle definitions.

TEST INFRASTRUCTURE ONLY.  The plain definitions the HIP micro-benchmark kernels are checked
against (and, through the C versions in volume_kernels.c, the CPU side of the cost ratio).
Only ``tests/`` and ``bench.py``'s CPU-baseline leg of the volume-kernel ratio (skipped by
--no-cpu-baseline) use this module; the library never does.

Section 5.4 compares the volume term of a traditional DG scheme, a matrix-vector product
of a differentiation-type matrix with the flux evaluated at each node, against the
entropy-stable volume term, the Hadamard product of that matrix with the matrix of two-point
entropy-conservative fluxes between every pair of nodes, summed along rows (flux
differencing).  As in the paper the matrices are random square matrices of size n, not SBP
operators.  For the shallow-water fluxes of Section 2.8, per element k and node m:

    traditional  r[c,k,m] = sum_n Qx[m,n] f^x_c(u_kn) + Qy[m,n] f^y_c(u_kn)
    entropy-stable  r[c,k,m] = sum_n 2 (Qx[m,n] f^x_{S,c}(u_km, u_kn) + Qy[m,n] f^y_{S,c}(u_km, u_kn))

u has shape [3, K, n] (h, hu, hv); the result has the same shape.  FP64.
"""
from __future__ import annotations

import os

import numpy as np

from .esdg_oracle import ec_flux, physical_flux


def dg_volume(Qx: np.ndarray, Qy: np.ndarray, u: np.ndarray, g: float) -> np.ndarray:
    """Traditional DG volume term: one flux evaluation per node, then a matrix-vector product."""
    fx, fy = physical_flux(u[0], u[1], u[2], g)
    return np.stack([fx[c] @ Qx.T + fy[c] @ Qy.T for c in range(3)])


def esdg_volume(Qx: np.ndarray, Qy: np.ndarray, u: np.ndarray, g: float) -> np.ndarray:
    """Entropy-stable volume term: 2 (Q o F) 1 with F[m, n] the two-point EC flux."""
    uL = tuple(u[c][:, :, None] for c in range(3))
    uR = tuple(u[c][:, None, :] for c in range(3))
    Fx, Fy = ec_flux(uL, uR, g)
    return np.stack([2.0 * np.sum(Qx[None] * Fx[c] + Qy[None] * Fy[c], axis=2) for c in range(3)])


# -- the C versions (volume_kernels.c), compiled by __graft_entry__.build() ----------------

HERE = os.path.dirname(os.path.abspath(__file__))
C_LIBRARY = os.path.join(HERE, "_lib", "libvolume_oracle.so")


def build_c(cc: str = "gcc") -> str:
    """Compile volume_kernels.c into oracle/_lib/ (plain -O2, no vectorisation flags)."""
    import subprocess
    os.makedirs(os.path.dirname(C_LIBRARY), exist_ok=True)
    tmp = C_LIBRARY + ".tmp"
    subprocess.run([cc, "-O2", "-fPIC", "-shared", os.path.join(HERE, "volume_kernels.c"), "-o", tmp], check=True)
    os.replace(tmp, C_LIBRARY)
    return C_LIBRARY


def c_volume(kind: str, Qx: np.ndarray, Qy: np.ndarray, u: np.ndarray, g: float) -> np.ndarray:
    """Run the C version of the traditional ("dg") or entropy-stable ("esdg") volume term."""
    import ctypes as C
    lib = C.CDLL(C_LIBRARY)
    fn = lib.dg_volume_c if kind == "dg" else lib.esdg_volume_c
    dp = C.POINTER(C.c_double)
    fn.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, dp]
    n, K = Qx.shape[0], u.shape[1]
    Qx = np.ascontiguousarray(Qx, dtype=np.float64)
    Qy = np.ascontiguousarray(Qy, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    r = np.empty_like(u)
    fn(n, K, Qx.ctypes.data_as(dp), Qy.ctypes.data_as(dp), u.ctypes.data_as(dp), float(g), r.ctypes.data_as(dp))
    return r
