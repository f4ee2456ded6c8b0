"""Rounding-error bound for comparing one RHS evaluation against the oracle.

The RHS is a sum of many terms that nearly cancel on smooth, near-balanced states (lake
at rest, a weak vortex on a uniform flow), so "error / max |rhs|" says little.  The
standard forward bound for a computed sum is |fl(sum) - sum| <= n eps sum |terms|; here
the terms are those of the dense semi-discrete form (Section 2.8), pushed through the
lift with absolute values:

    bound = |M_h^-1| |V_h^T| ( sum_n 2 (|Qx_mn| |Fx_mn| + |Qy_mn| |Fy_mn|) + |source| + |interface| )

(with the weight-adjusted mass inverse, |M_h^-1| is replaced by its factored form
|V_q^T| diag(w/J) |V_q|).

A result within c * eps * bound (c of order the accumulation length) is as accurate as
the arithmetic allows.  Built from oracle quantities only.
"""
import numpy as np

from oracle import esdg_oracle as O


def rhs_abs_bound(o: "O.Oracle", uh: np.ndarray, ks: np.ndarray) -> np.ndarray:
    d, ref, g = o.d, o.d.ref, o.d.g
    ut, _ = o.entropy_projection(uh)
    Nq = ref.Nq
    Qx, Qy = o.physical_Qh(ks)
    uL = tuple(ut[c, ks][:, :, None] for c in range(3))
    uR = tuple(ut[c, ks][:, None, :] for c in range(3))
    Fx, Fy = O.ec_flux(uL, uR, g)
    r = np.zeros((3, ks.size, ref.Nh))
    for c in range(3):
        r[c] = 2.0 * np.sum(np.abs(Qx) * np.abs(Fx[c]) + np.abs(Qy) * np.abs(Fy[c]), axis=2)
    bt = np.abs(d.b_hyb[ks])
    r[1] += g * np.abs(ut[0, ks]) * np.einsum("kmn,kn->km", np.abs(Qx), bt)
    r[2] += g * np.abs(ut[0, ks]) * np.einsum("kmn,kn->km", np.abs(Qy), bt)
    uf = ut[:, ks, Nq:]
    up = O.exterior_state(d, ut, ks)
    fS_x, fS_y = O.ec_flux(tuple(up), tuple(uf), g)
    f_x, f_y = O.physical_flux(uf[0], uf[1], uf[2], g)
    nJx, nJy, sJ = np.abs(d.nJx[ks]), np.abs(d.nJy[ks]), d.sJ[ks]
    speed = lambda u: np.abs(u[1] / u[0]) + np.abs(u[2] / u[0]) + np.sqrt(g * np.abs(u[0]))
    lam = np.maximum(speed(uf), speed(up))
    for c in range(3):
        r[c, :, Nq:] += ref.wf[None] * (nJx * (np.abs(fS_x[c]) + np.abs(f_x[c])) +
                                        nJy * (np.abs(fS_y[c]) + np.abs(f_y[c])) +
                                        0.5 * lam * sJ * (np.abs(up[c]) + np.abs(uf[c])))
    y = r @ np.abs(ref.Vh)                                     # [3, k, Np]
    if d.mass == "wadg":                                       # |V_q|^T diag(w/J) |V_q| (M = I)
        return ((y @ np.abs(ref.Vq).T) * d.w_over_J[ks]) @ np.abs(ref.Vq)
    Minv = np.abs(np.linalg.inv(d.Mh[ks]))                     # [k, Np, Np]
    return np.einsum("kij,ckj->cki", Minv, y)


def check_rhs(r_gpu: np.ndarray, r_ref: np.ndarray, bound: np.ndarray, eps: float, c: float = 64.0):
    """Returns (ok, worst ratio |r_gpu - r_ref| / (eps * bound))."""
    ratio = np.abs(r_gpu - r_ref) / (eps * bound + 1e-300)
    return bool(np.all(ratio <= c)), float(ratio.max())


EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


def sbp_rhs_abs_bound(o: "O.SBPOracle", u: np.ndarray) -> np.ndarray:
    """The same bound for the DG-SBP scheme (Section 3.2): the absolute terms of
    sum_i (2 Q_SBP^i o F^i) 1 + source + I_f^T (interface terms), divided by w J (the
    diagonal mass matrix).  u: nodal state [3, K, Nq]."""
    d, ref, g = o.d, o.d.ref, o.d.g
    ks = np.arange(d.K)
    Qx, Qy = o.Q_sbp(ks)
    uL = tuple(u[c][:, :, None] for c in range(3))
    uR = tuple(u[c][:, None, :] for c in range(3))
    Fx, Fy = O.ec_flux(uL, uR, g)
    r = np.zeros_like(u)
    for c in range(3):
        r[c] = 2.0 * np.sum(np.abs(Qx) * np.abs(Fx[c]) + np.abs(Qy) * np.abs(Fy[c]), axis=2)
    bq = np.abs(d.b_q)
    r[1] += g * np.abs(u[0]) * np.einsum("kmn,kn->km", np.abs(Qx), bq)
    r[2] += g * np.abs(u[0]) * np.einsum("kmn,kn->km", np.abs(Qy), bq)
    uh = u[:, :, np.r_[np.arange(ref.Nq), o.If]]
    uf = uh[:, :, ref.Nq:]
    up = O.exterior_state(d, uh, ks)
    fS_x, fS_y = O.ec_flux(tuple(up), tuple(uf), g)
    f_x, f_y = O.physical_flux(uf[0], uf[1], uf[2], g)
    nJx, nJy, sJ = np.abs(d.nJx), np.abs(d.nJy), d.sJ
    speed = lambda v: np.abs(v[1] / v[0]) + np.abs(v[2] / v[0]) + np.sqrt(g * np.abs(v[0]))
    lam = np.maximum(speed(uf), speed(up))
    sel = np.eye(ref.Nq)[o.If]
    for c in range(3):
        t = ref.wf[None] * (nJx * (np.abs(fS_x[c]) + np.abs(f_x[c])) + nJy * (np.abs(fS_y[c]) + np.abs(f_y[c])) +
                            0.5 * lam * sJ * (np.abs(up[c]) + np.abs(uf[c])))
        r[c] += t @ sel
    return r / (ref.wq[None, :] * d.Jq)[None]
