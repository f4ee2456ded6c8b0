"""FP64 CPU oracle for the modal entropy-stable DG (ESDG) shallow-water right-hand side.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the HIP
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the library never does, and it
shares no code with the library (its own basis, quadrature, operators, geometry,
connectivity, fluxes and time stepper).

Source: Wu, Kubatko & Chan, "High-order entropy stable discontinuous Galerkin
methods for the shallow water equations: curved triangular meshes and GPU
acceleration" (arXiv 2005.02516).  Every function names the section / equation it
follows.  It evaluates the *literal dense* semi-discrete form, eq. (dgform) of
Section 2.8, with the Lax-Friedrichs penalty of Section 2.8 and the five-stage
low-storage RK4 of Section 4, in float64, vectorised over elements with numpy.

Readings where the paper is silent, garbled or ambiguous:

* modal basis (Section 2.1 leaves it open): orthonormal Dubiner (PKDO) basis,
  modes ordered ``for i in 0..N: for j in 0..N-i``;
* quadrature (Section 2.1 gives only minimum degrees): Stroud collapsed rule with
  (N+1)^2 points (exact to degree 2N+1) and N+1 Gauss-Legendre points per face;
* reference vertices taken counter-clockwise (-1,-1), (1,-1), (-1,1); face 1 is
  s=-1, face 2 is r+s=0, face 3 is r=-1, each parametrised counter-clockwise;
* geometric factors G_ij (Section 2.7) are the Jacobian-scaled cofactors
  rxJ = y_s, sxJ = -y_r, ryJ = -x_s, syJ = x_r, so that
  B^{i,k} = W_f diag(nJ_i) with nJ = G * nhat;
* entropy projection on curved elements uses the J-weighted L2 projection
  (M_h^k)^{-1} V_q^T W diag(J) (Section 2.6 with the curved mass matrix of Section 2.7);
* the flux matrix is F^i[m, n] = f_S^i(u~_m, u~_n) over all hybridized nodes;
* the bathymetry source is -g V_h^T [0; diag(h~) Q_h^{x,k} b; diag(h~) Q_h^{y,k} b]
  with b evaluated at the hybridized nodes (the y-momentum source uses b_y);
* Lax-Friedrichs penalty (Section 2.8): -1/2 lambda sJ W_f (u~+ - u~) on the
  entropy-projected conservative variables, lambda = max over both sides of
  |u.n| + sqrt(g h);
* LSRK coefficients: the published Carpenter-Kennedy (1994) 2N-storage values;
* optional weight-adjusted mass inverse (the implementation remark after eq. (dgform),
  Section 2.8): M^{-1} M_{1/J} M^{-1} in both the entropy projection and the lift, with
  the projected entropy variables those of S - g Href h (Href a fixed reference level);
* optional quadrature (Section 2.1 fixes only minimum degrees): the Stroud rule with more
  points per direction, more Gauss-Legendre points per face, or a caller's volume rule;
* the DG-SBP scheme of Section 3.2 (SBPOracle): the bathymetry source and the LF penalty
  are those of the modal scheme, with the nodal values in place of the entropy-projected
  ones, and the curved SBP mass matrix is W diag(J).
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Tuple

import numpy as np

# ----------------------------------------------------------------------------------
# 1D orthogonal polynomials and Gauss rules
# ----------------------------------------------------------------------------------


def jacobi_normalized(x: np.ndarray, alpha: float, beta: float, n: int) -> np.ndarray:
    """Orthonormal Jacobi polynomial P~_n^{(alpha,beta)}(x) on [-1, 1].

    Normalised so that int_{-1}^{1} (1-x)^alpha (1+x)^beta P~_m P~_n dx = delta_mn.
    Built with the three-term recurrence of the normalised Jacobi family.
    """
    x = np.asarray(x, dtype=np.float64)
    a, b = float(alpha), float(beta)
    g0 = 2.0 ** (a + b + 1) / (a + b + 1) * math.gamma(a + 1) * math.gamma(b + 1) / math.gamma(a + b + 1)
    p_prev = np.full_like(x, 1.0 / math.sqrt(g0))
    if n == 0:
        return p_prev
    g1 = (a + 1) * (b + 1) / (a + b + 3) * g0
    p = ((a + b + 2) * x / 2 + (a - b) / 2) / math.sqrt(g1)
    if n == 1:
        return p
    a_old = 2.0 / (2 + a + b) * math.sqrt((a + 1) * (b + 1) / (a + b + 3))
    for i in range(1, n):
        h1 = 2 * i + a + b
        a_new = 2.0 / (h1 + 2) * math.sqrt((i + 1) * (i + 1 + a + b) * (i + 1 + a) * (i + 1 + b) / ((h1 + 1) * (h1 + 3)))
        b_new = -(a * a - b * b) / (h1 * (h1 + 2))
        p_next = ((x - b_new) * p - a_old * p_prev) / a_new
        p_prev, p = p, p_next
        a_old = a_new
    return p


def jacobi_normalized_deriv(x: np.ndarray, alpha: float, beta: float, n: int) -> np.ndarray:
    """d/dx P~_n^{(alpha,beta)} = sqrt(n (n + alpha + beta + 1)) P~_{n-1}^{(alpha+1,beta+1)}."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return math.sqrt(n * (n + alpha + beta + 1)) * jacobi_normalized(x, alpha + 1, beta + 1, n - 1)


def gauss_jacobi(n: int, alpha: float, beta: float) -> Tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Jacobi rule for weight (1-x)^alpha (1+x)^beta by Golub-Welsch.

    The nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
    monic recurrence; the weights are mu0 times the squared first eigenvector entries.
    """
    a, b = float(alpha), float(beta)
    i = np.arange(n, dtype=np.float64)
    diag = np.empty(n)
    for k in range(n):
        s = 2 * k + a + b
        diag[k] = (b - a) / (a + b + 2) if k == 0 else (b * b - a * a) / (s * (s + 2))
    off = np.empty(max(n - 1, 0))
    for k in range(1, n):
        s = 2 * k + a + b
        off[k - 1] = 2.0 / s * math.sqrt(k * (k + a) * (k + b) * (k + a + b) / ((s - 1) * (s + 1)))
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    lam, vec = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1) * math.gamma(a + 1) * math.gamma(b + 1) / math.gamma(a + b + 2)
    w = mu0 * vec[0, :] ** 2
    del i
    return lam, w


# ----------------------------------------------------------------------------------
# Reference triangle (Section 2.1)
# ----------------------------------------------------------------------------------


def n_modes(N: int) -> int:
    """N_p = dim P^N on a triangle."""
    return (N + 1) * (N + 2) // 2


def rs_to_ab(r: np.ndarray, s: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Collapsed coordinates a = 2(1+r)/(1-s) - 1, b = s (a = -1 at the top vertex)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    a = np.where(np.abs(1.0 - s) > 1e-14, 2.0 * (1.0 + r) / np.where(np.abs(1.0 - s) > 1e-14, 1.0 - s, 1.0) - 1.0, -1.0)
    return a, s.copy()


def mode_list(N: int):
    """Mode ordering: for i in 0..N, for j in 0..N-i."""
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def dubiner(N: int, r: np.ndarray, s: np.ndarray, grad: bool = False):
    """Orthonormal Dubiner basis phi_ij = sqrt(2) P~_i(a) P~_j^{(2i+1,0)}(b) (1-b)^i.

    Returns V[p, m] = phi_m(r_p, s_p) and, with ``grad``, the r and s derivatives by the
    chain rule (a_r = 2/(1-s), a_s = (1+a)/(1-s), b_s = 1).  Derivatives are only
    requested at points with s < 1.
    """
    a, b = rs_to_ab(r, s)
    modes = mode_list(N)
    V = np.zeros((a.size, len(modes)))
    Vr = np.zeros_like(V)
    Vs = np.zeros_like(V)
    for m, (i, j) in enumerate(modes):
        fa = jacobi_normalized(a, 0, 0, i)
        gb = jacobi_normalized(b, 2 * i + 1, 0, j)
        V[:, m] = math.sqrt(2.0) * fa * gb * (1.0 - b) ** i
        if grad:
            dfa = jacobi_normalized_deriv(a, 0, 0, i)
            dgb = jacobi_normalized_deriv(b, 2 * i + 1, 0, j)
            # d/dr: sqrt2 f'(a) a_r g (1-b)^i = sqrt2 f'(a) g 2 (1-b)^(i-1)
            pw1 = (1.0 - b) ** (i - 1) if i > 0 else np.zeros_like(b)
            Vr[:, m] = math.sqrt(2.0) * dfa * gb * 2.0 * pw1
            # d/ds: sqrt2 [ f'(a) (1+a) g (1-b)^(i-1) + f(a) (g'(b) (1-b)^i - i g (1-b)^(i-1)) ]
            Vs[:, m] = math.sqrt(2.0) * (dfa * (1.0 + a) * gb * pw1
                                         + fa * (dgb * (1.0 - b) ** i - i * gb * pw1))
    if grad:
        return V, Vr, Vs
    return V


def stroud_rule(N: int, q: Optional[int] = None):
    """Volume rule: q-point Gauss-Legendre in a times q-point Gauss-Jacobi(1,0) in b (q = N+1
    by default).

    Collapsed map r = (1+a)(1-b)/2 - 1, s = b, weight w = w_a w_b / 2 (sum w = 2, the
    reference area).  Exact for total degree 2q-1 (2N+1 by default, which covers the 2N
    volume rule of Section 2.1).
    """
    q = N + 1 if q is None else int(q)
    xa, wa = gauss_jacobi(q, 0.0, 0.0)
    xb, wb = gauss_jacobi(q, 1.0, 0.0)
    A, Bm = np.meshgrid(xa, xb, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    r = ((1.0 + A) * (1.0 - Bm) / 2.0 - 1.0).ravel()
    s = Bm.ravel()
    w = (0.5 * WA * WB).ravel()
    return r, s, w


def face_rule(N: int, npts: Optional[int] = None):
    """npts (default N+1) Gauss-Legendre points on each face, faces listed 1, 2, 3, each
    counter-clockwise.

    Face 1: s=-1 from v1 to v2, scaled normal (0,-1).
    Face 2: r+s=0 from v2 to v3, scaled normal (1, 1) (unit normal times the face Jacobian sqrt 2).
    Face 3: r=-1 from v3 to v1, scaled normal (-1, 0).
    The weights are the Gauss-Legendre weights in the face parameter t in [-1, 1].
    """
    t, wt = gauss_jacobi(N + 1 if npts is None else int(npts), 0.0, 0.0)
    rf = np.concatenate([t, -t, -np.ones_like(t)])
    sf = np.concatenate([-np.ones_like(t), t, -t])
    wf = np.concatenate([wt, wt, wt])
    one = np.ones_like(t)
    nr = np.concatenate([0 * one, one, -one])
    ns = np.concatenate([-one, one, 0 * one])
    return rf, sf, wf, nr, ns


def quadrature_rules(N: int, quad: Optional[dict] = None):
    """The volume and face rules of degree N selected by ``quad`` (Section 2.1 fixes only
    minimum degrees): None gives the Stroud rule with N+1 points per direction and N+1
    Gauss-Legendre points per face; a mapping may give "vol_degree" (the Stroud rule with
    ceil((vol_degree+1)/2) points per direction, at least N+1), "face_points" (default N+1)
    and "rule" = (r, s, w), a caller's volume rule used as given."""
    quad = quad or {}
    npf = int(quad.get("face_points") or N + 1)
    if quad.get("rule") is not None:
        r, s, w = (np.asarray(a, dtype=np.float64) for a in quad["rule"])
    else:
        deg = int(quad.get("vol_degree") or 2 * N)
        r, s, w = stroud_rule(N, max(N + 1, (deg + 2) // 2))
    return (r, s, w), face_rule(N, npf)


def monomial_integral(a: int, b: int) -> float:
    """Exact integral of r^a s^b over the reference triangle:
    int_{-1}^{1} s^b ((-s)^(a+1) - (-1)^(a+1)) / (a+1) ds (rational arithmetic)."""
    from fractions import Fraction
    def pint(p):
        return Fraction(0) if p % 2 else Fraction(2, p + 1)
    sg = -1 if (a + 1) % 2 else 1
    return float(Fraction(sg, a + 1) * (pint(a + b + 1) - pint(b)))


def rule_degree(r, s, w, max_degree: int = 30, tol: float = 1e-13) -> int:
    """Largest d such that the rule integrates every r^a s^b with a + b <= d exactly."""
    d = -1
    for deg in range(max_degree + 1):
        for a in range(deg + 1):
            b = deg - a
            if abs(np.sum(w * r ** a * s ** b) - monomial_integral(a, b)) > tol * max(1.0, np.sum(np.abs(w))):
                return d
        d = deg
    return d


class ReferenceElement:
    """Reference-element operators of Sections 2.1-2.3 for degree N (quadrature as selected
    by ``quad``, see quadrature_rules)."""

    def __init__(self, N: int, quad: Optional[dict] = None):
        self.N = N
        self.Np = n_modes(N)
        (rq, sq, wq), (rf, sf, wf, nr, ns) = quadrature_rules(N, quad)
        self.rq, self.sq, self.wq = rq, sq, wq
        self.rf, self.sf, self.wf, self.nrJ, self.nsJ = rf, sf, wf, nr, ns
        self.Nq, self.Nfq = rq.size, rf.size
        self.Nh = self.Nq + self.Nfq
        self.Nfp = self.Nfq // 3
        Vq, Vrq, Vsq = dubiner(N, rq, sq, grad=True)
        Vf, Vrf, Vsf = dubiner(N, rf, sf, grad=True)
        self.Vq, self.Vf = Vq, Vf
        self.Vrq, self.Vsq, self.Vrf, self.Vsf = Vrq, Vsq, Vrf, Vsf
        W = np.diag(wq)
        Wf = np.diag(wf)
        self.W, self.Wf = W, Wf
        # Section 2.1: mass matrix and quadrature L2 projection
        self.M = Vq.T @ W @ Vq
        self.Pq = np.linalg.solve(self.M, Vq.T @ W)
        # modal differentiation: coefficients of the derivative (exact: d phi in P^{N-1})
        self.Dr = self.Pq @ Vrq
        self.Ds = self.Pq @ Vsq
        # Section 2.2
        self.Qhat = [self.M @ self.Dr, self.M @ self.Ds]
        self.B = [Wf @ np.diag(nr), Wf @ np.diag(ns)]
        self.Q = [self.Pq.T @ Qh @ self.Pq for Qh in self.Qhat]
        self.E = Vf @ self.Pq
        self.Vh = np.vstack([Vq, Vf])
        # Section 2.3: hybridized SBP operators
        self.Qh = []
        for Qi, Bi in zip(self.Q, self.B):
            top = np.hstack([Qi - Qi.T, self.E.T @ Bi])
            bot = np.hstack([-Bi @ self.E, Bi])
            self.Qh.append(0.5 * np.vstack([top, bot]))


# ----------------------------------------------------------------------------------
# Mesh geometry and connectivity (Section 2.7)
# ----------------------------------------------------------------------------------


def equispaced_rs(N: int):
    """Equispaced nodes in the input convention: for j in 0..N, for i in 0..N-j."""
    pts = [(-1.0 + 2.0 * i / N, -1.0 + 2.0 * j / N) for j in range(N + 1) for i in range(N + 1 - j)]
    a = np.array(pts)
    return a[:, 0], a[:, 1]


class Discretization:
    """Per-mesh data for one instance: geometry, connectivity and curved mass matrices.

    ``mass`` selects how (M_h^k)^{-1} is applied wherever the scheme needs it (the
    J-weighted entropy projection of Section 2.6 and the lift of Section 2.8):
    "exact" solves with the curved mass matrix M_h^k = V_q^T W diag(J) V_q (Section 2.7);
    "wadg" uses the weight-adjusted inverse that the paper names as the way to avoid
    storing the per-element inverses (the implementation remark after eq. (dgform) in
    Section 2.8, citing Chan & Wilcox): (M_h^k)^{-1} ~ M^{-1} M_{1/J} M^{-1}, with the reference
    mass matrix M and M_{1/J} = V_q^T W diag(1/J) V_q.  It is exact where J is constant
    on the element, and used in both places so that the projected entropy variables and
    the time derivative see the same (approximate) mass matrix.
    """

    def __init__(self, N: int, xg: np.ndarray, yg: np.ndarray, b_nodes: Optional[np.ndarray], g: float,
                 Lx: float, Ly: float, mass: str = "exact", quad: Optional[dict] = None):
        if mass not in ("exact", "wadg"):
            raise ValueError("mass must be 'exact' or 'wadg'")
        self.mass = mass
        ref = ReferenceElement(N, quad)
        self.ref, self.N, self.g = ref, N, float(g)
        self.K = xg.shape[0]
        self.Lx, self.Ly = float(Lx), float(Ly)
        req, seq = equispaced_rs(N)
        self.Vgeo = dubiner(N, req, seq)                        # interpolation nodes -> modes
        self.Vgeo_inv = np.linalg.inv(self.Vgeo)
        # isoparametric map: modal coefficients of x and y
        xm = xg @ self.Vgeo_inv.T
        ym = yg @ self.Vgeo_inv.T
        self.xm, self.ym = xm, ym
        Vrh = np.vstack([ref.Vrq, ref.Vrf])
        Vsh = np.vstack([ref.Vsq, ref.Vsf])
        xr, xs = xm @ Vrh.T, xm @ Vsh.T
        yr, ys = ym @ Vrh.T, ym @ Vsh.T
        # Jacobian-scaled metric cofactors at all hybridized nodes
        self.rxJ, self.sxJ = ys, -yr
        self.ryJ, self.syJ = -xs, xr
        self.J = xr * ys - xs * yr
        self.Jq = self.J[:, :ref.Nq]
        # physical node positions at the hybridized nodes
        self.xh = xm @ ref.Vh.T
        self.yh = ym @ ref.Vh.T
        # scaled physical normals at face nodes: nJ_i = sum_j G_ij nhat_j
        f = slice(ref.Nq, ref.Nh)
        self.nJx = self.rxJ[:, f] * ref.nrJ + self.sxJ[:, f] * ref.nsJ
        self.nJy = self.ryJ[:, f] * ref.nrJ + self.syJ[:, f] * ref.nsJ
        self.sJ = np.sqrt(self.nJx ** 2 + self.nJy ** 2)
        # curved mass matrices M_h^k = Vq^T W diag(J^k) Vq and their Cholesky factors
        wJ = ref.wq[None, :] * self.Jq
        self.Mh = np.einsum("qi,kq,qj->kij", ref.Vq, wJ, ref.Vq)
        self.Mh_chol = np.linalg.cholesky(self.Mh)
        # weight-adjusted inverse: quadrature weights over J at the volume nodes
        self.w_over_J = ref.wq[None, :] / self.Jq
        self.mapP = self._connect()
        # bathymetry: C0 nodal samples -> modes -> hybridized nodes
        if b_nodes is None:
            b_nodes = np.zeros_like(xg)
        self.bh = b_nodes @ self.Vgeo_inv.T
        self.b_hyb = self.bh @ ref.Vh.T
        self.b_q = self.b_hyb[:, :ref.Nq]

    # -- connectivity ---------------------------------------------------------------
    def _connect(self) -> np.ndarray:
        """mapP[k, f]: flat index k'*Nfq + f' of the neighbour's face node at the same point.

        Faces are paired by their midpoints (rounded to a fine grid; wrapped by the period in
        each periodic direction, a period <= 0 meaning none); the nodes of two paired faces are
        matched by nearest distance (periodic where periodic).  A face whose midpoint no other
        face shares is a reflective wall (Section 2.9) when some direction is not periodic,
        and an error otherwise; its nodes map to themselves and are marked in self.wall.
        """
        ref = self.ref
        K, Nfp, Nq = self.K, ref.Nfp, ref.Nq
        xf = self.xh[:, Nq:].reshape(K * 3, Nfp)
        yf = self.yh[:, Nq:].reshape(K * 3, Nfp)
        hscale = float(np.max(np.hypot(xf[:, -1] - xf[:, 0], yf[:, -1] - yf[:, 0])))
        tol = 1e-7 * hscale
        cell = 1e-4 * hscale
        px, py = self.Lx > 0, self.Ly > 0
        mx, my = xf.mean(axis=1), yf.mean(axis=1)
        if px:
            mx = mx % self.Lx
        if py:
            my = my % self.Ly
        kx = np.round(mx / cell).astype(np.int64)
        ky = np.round(my / cell).astype(np.int64)
        if px:
            kx %= int(round(self.Lx / cell))
        if py:
            ky %= int(round(self.Ly / cell))
        key = (kx - kx.min()) * (int(ky.max() - ky.min()) + 1) + (ky - ky.min())
        uniq, inverse, counts = np.unique(key, return_inverse=True, return_counts=True)
        if np.any(counts > 2):
            raise ValueError("more than two faces share a midpoint")
        single = counts[inverse] == 1
        if np.any(single) and px and py:
            raise ValueError("every face needs exactly one periodic partner")
        partner = np.arange(K * 3)
        order = np.argsort(key, kind="stable")
        ks = key[order]
        first = np.nonzero(np.r_[True, ks[1:] != ks[:-1]])[0]
        for a in first:
            if a + 1 < ks.size and ks[a + 1] == ks[a]:
                partner[order[a]], partner[order[a + 1]] = order[a + 1], order[a]
        # node matching: nearest node of the partner face (distances periodic where periodic)
        dx = xf[partner][:, None, :] - xf[:, :, None]
        dy = yf[partner][:, None, :] - yf[:, :, None]
        if px:
            dx -= self.Lx * np.round(dx / self.Lx)
        if py:
            dy -= self.Ly * np.round(dy / self.Ly)
        d = np.hypot(dx, dy)                                 # [face, my node, partner node]
        j = np.argmin(d, axis=2)
        j[single] = np.arange(Nfp)[None, :]                  # wall faces: each node itself
        if np.max(np.take_along_axis(d, j[:, :, None], axis=2)) > tol:
            raise ValueError("unmatched face node")
        mapP = partner[:, None] * Nfp + j                      # flat face-node index
        self.wall = np.repeat(single, Nfp).reshape(K, 3 * Nfp)
        return mapP.reshape(K, 3 * Nfp)

    # -- nodal <-> modal --------------------------------------------------------------
    def interpolate(self, u_nodes: np.ndarray) -> np.ndarray:
        """Modal coefficients of the degree-N interpolant of samples at the equispaced nodes."""
        return u_nodes @ self.Vgeo_inv.T

    def project(self, f_q: np.ndarray) -> np.ndarray:
        """J-weighted quadrature L2 projection (M_h^k)^{-1} V_q^T W diag(J^k) f_q, per element
        (the weight-adjusted inverse with mass="wadg")."""
        ref = self.ref
        rhs = (f_q * (ref.wq[None, :] * self.Jq)) @ ref.Vq
        return self.mh_solve(rhs)

    def ref_solve(self, r: np.ndarray) -> np.ndarray:
        """Solve M x = r with the reference mass matrix, along the last axis of r."""
        Np = self.ref.Np
        flat = r.reshape(-1, Np)
        return np.linalg.solve(self.ref.M, flat.T).T.reshape(r.shape)

    def wadg_apply(self, r: np.ndarray, ks: np.ndarray) -> np.ndarray:
        """x = M^{-1} M_{1/J} M^{-1} r for the elements ks (r has shape [..., len(ks), Np]):
        the weight-adjusted approximation of (M_h^k)^{-1} r, applied as written, one
        factor after the other."""
        ref = self.ref
        y = self.ref_solve(r)
        t = (y @ ref.Vq.T) * self.w_over_J[ks]            # W diag(1/J) V_q y at the volume nodes
        return self.ref_solve(t @ ref.Vq)

    def mh_solve_subset(self, r: np.ndarray, ks: np.ndarray) -> np.ndarray:
        """Solve M_h^k x = r for the listed elements ks (r has shape [3, len(ks), Np]);
        with mass="wadg", apply the weight-adjusted inverse instead."""
        if self.mass == "wadg":
            return self.wadg_apply(r, ks)
        L = self.Mh_chol[ks]
        out = np.empty_like(r)
        for c in range(r.shape[0]):
            y = np.linalg.solve(L, r[c][..., None])[..., 0]
            out[c] = np.linalg.solve(np.swapaxes(L, 1, 2), y[..., None])[..., 0]
        return out

    def mh_solve(self, r: np.ndarray) -> np.ndarray:
        """Solve M_h^k x = r for every element (r has shape [..., K, Np]); with
        mass="wadg", apply the weight-adjusted inverse instead."""
        if self.mass == "wadg":
            return self.wadg_apply(r, np.arange(self.K))
        L = self.Mh_chol
        shp = r.shape
        rr = r.reshape(-1, self.K, self.ref.Np)
        out = np.empty_like(rr)
        for c in range(rr.shape[0]):
            y = np.linalg.solve(L, rr[c][..., None])[..., 0]
            out[c] = np.linalg.solve(np.swapaxes(L, 1, 2), y[..., None])[..., 0]
        return out.reshape(shp)


# ----------------------------------------------------------------------------------
# Shallow-water entropy, entropy variables and fluxes (Sections 2.4, 2.8)
# ----------------------------------------------------------------------------------


def entropy(h, hu, hv, b, g):
    """S(u) = 1/2 h (u^2 + v^2) + 1/2 g h^2 + g h b."""
    u, v = hu / h, hv / h
    return 0.5 * h * (u * u + v * v) + 0.5 * g * h * h + g * h * b


def entropy_variables(h, hu, hv, b, g):
    """v = (g (h + b) - (u^2 + v^2)/2, u, v)."""
    u, v = hu / h, hv / h
    return g * (h + b) - 0.5 * (u * u + v * v), u, v


def conservative_from_entropy(v1, v2, v3, b, g):
    """Inverse map of entropy_variables: h = (v1 + (v2^2 + v3^2)/2)/g - b, hu = h v2, hv = h v3."""
    h = (v1 + 0.5 * (v2 * v2 + v3 * v3)) / g - b
    return h, h * v2, h * v3


def exterior_state(d: "Discretization", ut: np.ndarray, ks: np.ndarray) -> np.ndarray:
    """u~+ at the face nodes of elements ks, shape [3, len(ks), Nfq]: the neighbour's value at
    the matching node, or on a reflective wall (Section 2.9) the mirror state h+ = h,
    (hu, hv)+ = (hu, hv) - 2 ((hu, hv) . n) n with n the unit outward normal."""
    Nq = d.ref.Nq
    up = ut[:, :, Nq:].reshape(3, -1)[:, d.mapP[ks].reshape(-1)].reshape(3, ks.size, d.ref.Nfq).copy()
    w = d.wall[ks]
    if np.any(w):
        nx, ny = d.nJx[ks] / d.sJ[ks], d.nJy[ks] / d.sJ[ks]
        h, hu, hv = ut[0, ks, Nq:], ut[1, ks, Nq:], ut[2, ks, Nq:]
        mn = hu * nx + hv * ny
        up[0][w] = h[w]
        up[1][w] = (hu - 2.0 * mn * nx)[w]
        up[2][w] = (hv - 2.0 * mn * ny)[w]
    return up


def physical_flux(h, hu, hv, g):
    """f^x = (hu, hu^2/h + g h^2/2, hu hv/h), f^y = (hv, hu hv/h, hv^2/h + g h^2/2)."""
    u, v = hu / h, hv / h
    fx = (hu, hu * u + 0.5 * g * h * h, hu * v)
    fy = (hv, hv * u, hv * v + 0.5 * g * h * h)
    return fx, fy


def ec_flux(uL, uR, g):
    """Entropy-conservative fluxes f^x_S, f^y_S of Section 2.8 with arithmetic averages {.}.

    uL, uR are tuples (h, hu, hv) of broadcastable arrays.
    """
    hL, huL, hvL = uL
    hR, huR, hvR = uR
    uL_, vL_ = huL / hL, hvL / hL
    uR_, vR_ = huR / hR, hvR / hR
    avg = lambda a, b: 0.5 * (a + b)
    h_avg = avg(hL, hR)
    h2_avg = avg(hL * hL, hR * hR)
    hu_avg, hv_avg = avg(huL, huR), avg(hvL, hvR)
    u_avg, v_avg = avg(uL_, uR_), avg(vL_, vR_)
    p = g * h_avg * h_avg - 0.5 * g * h2_avg
    fx = (hu_avg, hu_avg * u_avg + p, hu_avg * v_avg)
    fy = (hv_avg, hv_avg * u_avg, hv_avg * v_avg + p)
    return fx, fy


# ----------------------------------------------------------------------------------
# Semi-discrete right-hand side (Sections 2.6-2.8), literal dense form
# ----------------------------------------------------------------------------------


class Oracle:
    """Dense FP64 evaluation of eq. (dgform) with bathymetry source and optional LF penalty."""

    def __init__(self, disc: Discretization, flux: str = "lf", chunk: int = 2048, Href: float = 0.0):
        """``Href``: the entropy whose variables are projected (Section 2.6) is taken as
        S - g Href h, with entropy variables v - (g Href, 0, 0).  It differs from S by a
        multiple of the conserved depth, so it is an entropy of the same system, and with
        the exact mass inverse the result does not depend on Href (the J-weighted projection
        reproduces constants).  The weight-adjusted inverse does not reproduce constants on
        curved elements, so there the result depends on Href at the level of the
        weight-adjustment error; a lake at rest at level Href then stays exactly at rest."""
        if flux not in ("ec", "lf"):
            raise ValueError("flux must be 'ec' or 'lf'")
        self.d = disc
        self.flux = flux
        self.chunk = chunk
        self.Href = float(Href)

    # Section 2.6: entropy projection
    def entropy_projection(self, uh: np.ndarray):
        """u_q = V_q u_h, v_q = v(u_q), v_h = P^k v_q, v~ = V_h v_h, u~ = u(v~).

        Returns u~ at the hybridized nodes, shape [3, K, Nh], and v_h [3, K, Np].
        """
        d, ref, g = self.d, self.d.ref, self.d.g
        uq = uh @ ref.Vq.T                                     # [3,K,Nq]
        vq = np.stack(entropy_variables(uq[0], uq[1], uq[2], d.b_q, g))
        vq[0] -= g * self.Href                                 # variables of S - g Href h
        vh = d.project(vq)
        vt = vh @ ref.Vh.T
        vt[0] += g * self.Href
        vh[0, :, 0] += g * self.Href * math.sqrt(2.0)          # depth field only; 1 = sqrt(2) phi_0
        ut = np.stack(conservative_from_entropy(vt[0], vt[1], vt[2], d.b_hyb, g))
        return ut, vh

    def physical_Qh(self, ks):
        """Q_h^{i,k}[m,n] = 1/2 sum_j (G_ij[m] + G_ij[n]) Qhat_h^j[m,n] (Section 2.7)."""
        d, ref = self.d, self.d.ref
        Qr, Qs = ref.Qh
        def op(Gr, Gs):
            return 0.5 * ((Gr[:, :, None] + Gr[:, None, :]) * Qr[None] + (Gs[:, :, None] + Gs[:, None, :]) * Qs[None])
        Qx = op(d.rxJ[ks], d.sxJ[ks])
        Qy = op(d.ryJ[ks], d.syJ[ks])
        return Qx, Qy

    def residual(self, uh: np.ndarray, elements: Optional[np.ndarray] = None) -> np.ndarray:
        """Hybridized-node residual r_h such that M_h du/dt = -V_h^T r_h.

        r_h = sum_i 2 (Q_h^{i,k} o F^i) 1 + [0; B^{i,k} (f_S^i(u~+, u~) - f^i(u~_f))] - S (+ LF penalty).
        With ``elements`` (an index array) only those elements' rows are evaluated; the
        result then has shape [3, len(elements), Nh].
        """
        d, ref, g = self.d, self.d.ref, self.d.g
        ut, _ = self.entropy_projection(uh)
        Nq, Nh = ref.Nq, ref.Nh
        ks_all = np.arange(d.K) if elements is None else np.asarray(elements, dtype=np.int64)
        r = np.zeros((3, ks_all.size, Nh))
        for c0 in range(0, ks_all.size, self.chunk):
            sel = slice(c0, min(ks_all.size, c0 + self.chunk))
            ks = ks_all[sel]
            Qx, Qy = self.physical_Qh(ks)
            uL = tuple(ut[c, ks][:, :, None] for c in range(3))
            uR = tuple(ut[c, ks][:, None, :] for c in range(3))
            Fx, Fy = ec_flux(uL, uR, g)
            for c in range(3):
                r[c, sel] += 2.0 * np.sum(Qx * Fx[c] + Qy * Fy[c], axis=2)
            # bathymetry source S = -g [0; diag(h~) Q^x b; diag(h~) Q^y b] moved to the left
            bt = d.b_hyb[ks]
            r[1, sel] += g * ut[0, ks] * np.einsum("kmn,kn->km", Qx, bt)
            r[2, sel] += g * ut[0, ks] * np.einsum("kmn,kn->km", Qy, bt)
        # interface terms on the face rows
        uf = ut[:, ks_all, Nq:]                                   # [3,k,Nfq]
        up = exterior_state(d, ut, ks_all)
        fS_x, fS_y = ec_flux(tuple(up), tuple(uf), g)
        f_x, f_y = physical_flux(uf[0], uf[1], uf[2], g)
        wf = ref.wf[None, :]
        nJx, nJy, sJ = d.nJx[ks_all], d.nJy[ks_all], d.sJ[ks_all]
        for c in range(3):
            r[c, :, Nq:] += wf * (nJx * (fS_x[c] - f_x[c]) + nJy * (fS_y[c] - f_y[c]))
        if self.flux == "lf":
            nx, ny = nJx / sJ, nJy / sJ
            def speed(u):
                return np.abs((u[1] * nx + u[2] * ny) / u[0]) + np.sqrt(g * u[0])
            lam = np.maximum(speed(uf), speed(up))
            for c in range(3):
                r[c, :, Nq:] -= wf * 0.5 * lam * sJ * (up[c] - uf[c])
        return r

    def rhs(self, uh: np.ndarray, elements: Optional[np.ndarray] = None) -> np.ndarray:
        """du_h/dt = -(M_h^k)^{-1} V_h^T r_h, solved with the Cholesky factors of M_h^k.

        With ``elements``, only those elements (shape [3, len(elements), Np]).
        """
        r = self.residual(uh, elements)
        if elements is None:
            return -self.d.mh_solve(r @ self.d.ref.Vh)
        return -self.d.mh_solve_subset(r @ self.d.ref.Vh, np.asarray(elements, dtype=np.int64))


# ----------------------------------------------------------------------------------
# DG-SBP scheme (Section 3): traditional SBP operators from the hybridized ones
# ----------------------------------------------------------------------------------


class SBPOracle:
    """Dense FP64 evaluation of the entropy-conservative DG-SBP form at the end of Section
    3.2, with the bathymetry source and the LF penalty of the modal scheme:

        M_SBP du/dt + sum_i (2 Q_SBP^i o F^i) 1 + I_f^T B^i (f_S^i - f^i) = S,

    with Q_SBP^i = [I; I_f]^T Q_h^i [I; I_f] (the theorem of Section 3.2) built from the
    physical hybridized operator of Section 2.7 on the rule's nodes, I_f the selection of the
    face nodes among the volume nodes, M_SBP^k = W diag(J) (the SBP mass matrix on curved
    elements), u the nodal values at the volume nodes, F^i[m, n] = f_S^i(u_m, u_n) over the
    volume nodes, and S = -g [0; diag(h) Q_SBP^x b; diag(h) Q_SBP^y b] with b at the volume
    nodes.  The state has shape [3, K, Nq].  ``disc`` must be built with a volume rule
    containing the face nodes (quad = {"rule": ..., "vol_degree": 2N-1}).
    """

    def __init__(self, disc: "Discretization", flux: str = "lf"):
        if flux not in ("ec", "lf"):
            raise ValueError("flux must be 'ec' or 'lf'")
        self.d, self.flux = disc, flux
        self.modal = Oracle(disc, flux)        # for the physical hybridized operators
        ref = disc.ref
        # I_f: face node f is volume node If[f] (same reference point)
        dist = np.hypot(ref.rf[:, None] - ref.rq[None, :], ref.sf[:, None] - ref.sq[None, :])
        self.If = np.argmin(dist, axis=1)
        if np.max(dist[np.arange(ref.Nfq), self.If]) > 1e-12:
            raise ValueError("the volume rule does not contain the face nodes")
        self.sel = np.vstack([np.eye(ref.Nq), np.eye(ref.Nq)[self.If]])   # [I; I_f], Nh x Nq

    def nodal(self, uh: np.ndarray) -> np.ndarray:
        """Values at the volume nodes of the modal coefficients uh (the initial state)."""
        return uh @ self.d.ref.Vq.T

    def Q_sbp(self, ks):
        """Q_SBP^{x,k}, Q_SBP^{y,k} of the elements ks, each [len(ks), Nq, Nq]."""
        Qx_h, Qy_h = self.modal.physical_Qh(ks)
        P = self.sel
        return P.T @ Qx_h @ P, P.T @ Qy_h @ P

    def rhs(self, u: np.ndarray) -> np.ndarray:
        d, ref, g = self.d, self.d.ref, self.d.g
        K = d.K
        ks = np.arange(K)
        Qx, Qy = self.Q_sbp(ks)
        uL = tuple(u[c][:, :, None] for c in range(3))
        uR = tuple(u[c][:, None, :] for c in range(3))
        Fx, Fy = ec_flux(uL, uR, g)
        r = np.zeros_like(u)
        for c in range(3):
            r[c] = 2.0 * np.sum(Qx * Fx[c] + Qy * Fy[c], axis=2)
        bq = d.b_q
        r[1] += g * u[0] * np.einsum("kmn,kn->km", Qx, bq)
        r[2] += g * u[0] * np.einsum("kmn,kn->km", Qy, bq)
        # I_f^T B (f_S(u+, u_f) - f(u_f)) and the LF penalty, at the face nodes
        uh = u[:, :, np.r_[np.arange(ref.Nq), self.If]]          # values at the hybridized nodes
        uf = uh[:, :, ref.Nq:]
        up = exterior_state(d, uh, ks)
        fS_x, fS_y = ec_flux(tuple(up), tuple(uf), g)
        f_x, f_y = physical_flux(uf[0], uf[1], uf[2], g)
        wf = ref.wf[None, :]
        surf = np.zeros_like(uf)
        for c in range(3):
            surf[c] = wf * (d.nJx * (fS_x[c] - f_x[c]) + d.nJy * (fS_y[c] - f_y[c]))
        if self.flux == "lf":
            nx, ny = d.nJx / d.sJ, d.nJy / d.sJ
            def speed(v):
                return np.abs((v[1] * nx + v[2] * ny) / v[0]) + np.sqrt(g * v[0])
            lam = np.maximum(speed(uf), speed(up))
            for c in range(3):
                surf[c] -= wf * 0.5 * lam * d.sJ * (up[c] - uf[c])
        for c in range(3):
            r[c] += surf[c] @ np.eye(ref.Nq)[self.If]                # I_f^T
        return -r / (ref.wq[None, :] * d.Jq)[None]

    def diagnostics(self, u: np.ndarray) -> Dict[str, float]:
        """Mass sum w J h, entropy sum w J S(u), entropy rate sum w J v(u).du/dt."""
        d, ref, g = self.d, self.d.ref, self.d.g
        wJ = ref.wq[None, :] * d.Jq
        dudt = self.rhs(u)
        v = entropy_variables(u[0], u[1], u[2], d.b_q, g)
        terms = wJ[None] * np.stack(v) * dudt
        return {"mass": np.array([np.sum(wJ * u[c]) for c in range(3)]),
                "entropy": float(np.sum(wJ * entropy(u[0], u[1], u[2], d.b_q, g))),
                "entropy_rate": float(np.sum(terms)), "entropy_rate_scale": float(np.sum(np.abs(terms)))}


# ----------------------------------------------------------------------------------
# Time stepping (Section 4: five-stage fourth-order low-storage RK)
# ----------------------------------------------------------------------------------

LSRK_A = np.array([0.0,
                   -567301805773.0 / 1357537059087.0,
                   -2404267990393.0 / 2016746695238.0,
                   -3550918686646.0 / 2091501179385.0,
                   -1275806237668.0 / 842570457699.0])
LSRK_B = np.array([1432997174477.0 / 9575080441904.0,
                   5161836677717.0 / 13612068292357.0,
                   1720146321549.0 / 2090206949498.0,
                   3134564353537.0 / 4481467310338.0,
                   2277821191437.0 / 14882151754819.0])
LSRK_C = np.array([0.0,
                   1432997174477.0 / 9575080441904.0,
                   2526269341429.0 / 6820363962896.0,
                   2006345519317.0 / 3224310063776.0,
                   2802321613138.0 / 2924317926251.0])


def lsrk_step(rhs, u: np.ndarray, du: np.ndarray, dt: float):
    """One 2N-storage step: for each stage du = a_s du + dt rhs(u); u = u + b_s du."""
    for s in range(5):
        du = LSRK_A[s] * du + dt * rhs(u)
        u = u + LSRK_B[s] * du
    return u, du


def run(oracle, uh: np.ndarray, dt: float, nsteps: int):
    du = np.zeros_like(uh)
    u = uh.copy()
    for _ in range(nsteps):
        u, du = lsrk_step(oracle.rhs, u, du, dt)
    return u, du


# ----------------------------------------------------------------------------------
# Diagnostics (Sections 2.4 and 2.7): conserved totals, entropy and its rate
# ----------------------------------------------------------------------------------


def mean_free_surface(disc: Discretization, uh: np.ndarray) -> float:
    """J-weighted mean of h + b over the volume quadrature nodes (the reference level of a
    state: sum w J (h + b) / sum w J)."""
    wJ = disc.ref.wq[None, :] * disc.Jq
    hq = uh[0] @ disc.ref.Vq.T
    return float(np.sum(wJ * (hq + disc.b_q)) / np.sum(wJ))


def diagnostics(oracle: Oracle, uh: np.ndarray) -> Dict[str, np.ndarray]:
    """Mass sum_k 1^T W J V_q u_h, entropy sum w J S(u_q), entropy rate sum w J v(u_q).(V_q du/dt)."""
    d, ref, g = oracle.d, oracle.d.ref, oracle.d.g
    wJ = ref.wq[None, :] * d.Jq
    uq = uh @ ref.Vq.T
    mass = np.array([np.sum(wJ * uq[c]) for c in range(3)])
    S = np.sum(wJ * entropy(uq[0], uq[1], uq[2], d.b_q, g))
    dudt = oracle.rhs(uh) @ ref.Vq.T
    vq = entropy_variables(uq[0], uq[1], uq[2], d.b_q, g)
    terms = wJ[None] * np.stack(vq) * dudt
    return {"mass": mass, "entropy": float(S), "entropy_rate": float(np.sum(terms)),
            "entropy_rate_scale": float(np.sum(np.abs(terms)))}


def l2_error(disc: Discretization, uh: np.ndarray, exact_fn) -> np.ndarray:
    """Per-field L2 error with a volume rule exact to degree >= 2N+2 (Section 4.2).

    ``exact_fn(x, y)`` returns the exact (h, hu, hv) at physical points.
    """
    N = disc.N
    r, s, w = stroud_rule(N + 1)                        # (N+2)^2 points, exact to 2N+3
    V, Vr, Vs = dubiner(N, r, s, grad=True)
    x, y = disc.xm @ V.T, disc.ym @ V.T
    J = (disc.xm @ Vr.T) * (disc.ym @ Vs.T) - (disc.xm @ Vs.T) * (disc.ym @ Vr.T)
    ue = exact_fn(x, y)
    uq = uh @ V.T
    return np.array([math.sqrt(np.sum(w[None, :] * J * (uq[c] - ue[c]) ** 2)) for c in range(3)])
