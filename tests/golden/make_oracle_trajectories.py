"""Writes oracle_trajectories.npz: FP64 oracle states after the configured number of LSRK
steps, on a seeded sample of elements, for the GPU trajectory tests.  It calls only the
oracle (and the seeded input generators); nothing here comes from the HIP library.

Cases (the input recipes of the workloads module):
  config2      : 64x64x2 curved mesh, N=3, lake at rest + Gaussian bump, LF, 100 steps
  config3_n32  : config 3's recipe on 32x32x2, N=4, 200 steps
  config5_n32  : config 5's recipe (translating vortex) on 32x32x2, N=5, 100 steps
Each entry stores the sampled element indices, the state there, and a fingerprint of the
inputs (nodes, bathymetry, initial state, dt) so that a stale file is detected.

Run: python tests/golden/make_oracle_trajectories.py   (a few minutes on one core)
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import esdg_oracle as O  # noqa: E402
from paper_2005_02516_amd import workloads as wl  # noqa: E402

PATH = os.path.join(HERE, "oracle_trajectories.npz")
NSAMPLE = 512

CASES = {
    "config2": (lambda: wl.config2(), 100),
    "config3_n32": (lambda: wl.config3(n=32), 200),
    "config5_n32": (lambda: wl.config5(n=32), 100),
}


def fingerprint(w) -> str:
    h = hashlib.sha256()
    for a in (w.xg, w.yg, w.b_nodes, w.u_nodes, np.array([w.dt])):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def sample(w):
    return np.sort(np.random.default_rng(12345).choice(w.K, size=min(NSAMPLE, w.K), replace=False))


def main():
    out = {}
    for name, (make, steps) in CASES.items():
        w = make()
        d = O.Discretization(w.N, w.xg, w.yg, w.b_nodes, w.g, w.Lx, w.Ly)
        o = O.Oracle(d, w.flux)
        u, _ = O.run(o, d.interpolate(w.u_nodes), w.dt, steps)
        ks = sample(w)
        out[f"{name}/elements"] = ks
        out[f"{name}/state"] = u[:, ks]
        out[f"{name}/norms"] = np.linalg.norm(u, axis=(1, 2))
        out[f"{name}/steps"] = np.array(steps)
        out[f"{name}/fingerprint"] = np.array(fingerprint(w))
        print(name, w.K, "elements,", steps, "steps", flush=True)
    np.savez_compressed(PATH, **out)


if __name__ == "__main__":
    main()
