"""Pins of the oracle's reference-element layer against facts that do not come from it.

Quadrature is checked against exact rational monomial integrals and against scipy's
independent Gauss-Jacobi routine; the basis against orthonormality under those
rules and exact reproduction of monomials and their derivatives; the operators
against the SBP identities of Sections 2.2-2.3.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

from oracle import esdg_oracle as O

NS = [1, 2, 3, 4, 5]


def exact_triangle_integral(a: int, b: int) -> Fraction:
    """int over the reference triangle of (1+r)^a (1+s)^b = 4 * 2^(a+b) a! b! / (a+b+2)!."""
    return Fraction(4 * 2 ** (a + b) * math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))


@pytest.mark.parametrize("N", NS)
def test_gauss_jacobi_matches_scipy(N):
    for (al, be) in [(0.0, 0.0), (1.0, 0.0), (3.0, 0.0), (2.0, 1.0)]:
        x, w = O.gauss_jacobi(N + 1, al, be)
        xs, ws = scipy.special.roots_jacobi(N + 1, al, be)
        assert np.allclose(np.sort(x), np.sort(xs), atol=1e-14, rtol=0)
        assert np.allclose(w[np.argsort(x)], ws[np.argsort(xs)], atol=1e-14, rtol=1e-13)


@pytest.mark.parametrize("N", NS)
def test_volume_rule_exact_to_2N_plus_1(N):
    """PIN-1: Stroud rule integrates every degree <= 2N+1 monomial exactly; sum w = 2."""
    r, s, w = O.stroud_rule(N)
    assert r.size == (N + 1) ** 2
    assert np.all(w > 0)
    assert abs(w.sum() - 2.0) < 1e-14
    for a in range(2 * N + 2):
        for b in range(2 * N + 2 - a):
            q = np.sum(w * (1 + r) ** a * (1 + s) ** b)
            ex = float(exact_triangle_integral(a, b))
            assert abs(q - ex) <= 1e-14 * max(1.0, abs(ex)) * 4, (a, b, q, ex)
    # and it is not exact one degree higher (a sanity check that the test can fail)
    a = 2 * N + 2
    q = np.sum(w * (1 + s) ** a)
    assert abs(q - float(exact_triangle_integral(0, a))) > 1e-10


@pytest.mark.parametrize("N", NS)
def test_face_rule_exact_to_2N_plus_1(N):
    """PIN-1 (faces): N+1 Gauss-Legendre points per face integrate degree 2N+1 exactly."""
    rf, sf, wf, nr, ns = O.face_rule(N)
    Nfp = N + 1
    for f in range(3):
        sl = slice(f * Nfp, (f + 1) * Nfp)
        for p in range(2 * N + 2):
            ex = (1 - (-1) ** (p + 1)) / (p + 1)
            # every face is parametrised by t in [-1,1]; test the parameter directly
            param = (rf[sl], sf[sl], -sf[sl])[f]      # face parameter t of faces 1, 2, 3
            assert abs(np.sum(wf[sl] * param ** p) - ex) < 1e-14
    # scaled normals integrate to zero around the boundary (divergence of a constant)
    assert abs(np.sum(wf * nr)) < 1e-14 and abs(np.sum(wf * ns)) < 1e-14


@pytest.mark.parametrize("al,be", [(0.0, 0.0), (1.0, 0.0), (3.0, 0.0), (5.0, 0.0), (1.0, 1.0)])
def test_jacobi_orthonormal(al, be):
    x, w = scipy.special.roots_jacobi(20, al, be)
    P = np.stack([O.jacobi_normalized(x, al, be, n) for n in range(8)])
    G = (P * w) @ P.T
    assert np.allclose(G, np.eye(8), atol=1e-13)
    # derivative against the scipy Jacobi polynomial derivative
    for n in range(1, 8):
        c = O.jacobi_normalized(np.array([0.3]), al, be, n)[0] / scipy.special.eval_jacobi(n, al, be, 0.3)
        xx = np.linspace(-0.9, 0.9, 7)
        d_ref = c * 0.5 * (n + al + be + 1) * scipy.special.eval_jacobi(n - 1, al + 1, be + 1, xx)
        assert np.allclose(O.jacobi_normalized_deriv(xx, al, be, n), d_ref, atol=1e-12, rtol=1e-12)


@pytest.mark.parametrize("N", NS)
def test_basis_orthonormal_and_spans_PN(N):
    """PIN-2: M = I under a rule of higher degree; monomials and their gradients are reproduced."""
    r, s, w = O.stroud_rule(N + 2)
    V = O.dubiner(N, r, s)
    assert np.allclose((V.T * w) @ V, np.eye(O.n_modes(N)), atol=1e-13)
    rng = np.random.default_rng(0)
    # random interior points (s < 1) for pointwise checks
    pr = rng.uniform(-1, 1, 40)
    ps = rng.uniform(-1, 1, 40)
    keep = pr + ps < -0.05
    pr, ps = pr[keep], ps[keep]
    Vp, Vrp, Vsp = O.dubiner(N, pr, ps, grad=True)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f = r ** a * s ** b
            c = np.linalg.lstsq(V, f, rcond=None)[0]
            assert np.allclose(V @ c, f, atol=1e-13)
            assert np.allclose(Vp @ c, pr ** a * ps ** b, atol=1e-13)
            fr = a * pr ** max(a - 1, 0) * ps ** b if a > 0 else 0 * pr
            fs = b * pr ** a * ps ** max(b - 1, 0) if b > 0 else 0 * pr
            assert np.allclose(Vrp @ c, fr, atol=1e-12)
            assert np.allclose(Vsp @ c, fs, atol=1e-12)


@pytest.mark.parametrize("N", NS)
def test_projection_and_sbp(N):
    """PIN-2/3/4: PqVq=I, M=I, SBP identities, Q_h 1 = 0, zero surface-surface skew block."""
    ref = O.ReferenceElement(N)
    Np, Nq, Nh = ref.Np, ref.Nq, ref.Nh
    assert np.allclose(ref.Pq @ ref.Vq, np.eye(Np), atol=1e-14)
    assert np.allclose(ref.M, np.eye(Np), atol=1e-13)
    for i in range(2):
        lhs = ref.Qhat[i] + ref.Qhat[i].T
        assert np.allclose(lhs, ref.Vf.T @ ref.B[i] @ ref.Vf, atol=1e-13)
        assert np.allclose(ref.Q[i] + ref.Q[i].T, ref.E.T @ ref.B[i] @ ref.E, atol=1e-13)
        Bh = np.zeros((Nh, Nh))
        Bh[Nq:, Nq:] = ref.B[i]
        assert np.allclose(ref.Qh[i] + ref.Qh[i].T, Bh, atol=1e-13)
        assert np.allclose(ref.Qh[i] @ np.ones(Nh), 0.0, atol=1e-13)
        S = ref.Qh[i] - ref.Qh[i].T
        assert np.all(S[Nq:, Nq:] == 0.0)
        assert np.all(np.diag(S) == 0.0)
    # D^r, D^s exact on P^N: derivative of monomials
    rng = np.random.default_rng(1)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            c = ref.Pq @ (ref.rq ** a * ref.sq ** b)
            dr = ref.Vq @ (ref.Dr @ c)
            ds = ref.Vq @ (ref.Ds @ c)
            er = a * ref.rq ** max(a - 1, 0) * ref.sq ** b if a else 0 * ref.rq
            es = b * ref.rq ** a * ref.sq ** max(b - 1, 0) if b else 0 * ref.rq
            assert np.allclose(dr, er, atol=1e-12) and np.allclose(ds, es, atol=1e-12)
    del rng


def test_dimensions_table():
    """Sizes used throughout: Np, Nq=(N+1)^2, Nfq=3(N+1), Nh."""
    for N, (Np, Nq, Nfq, Nh) in {1: (3, 4, 6, 10), 2: (6, 9, 9, 18), 3: (10, 16, 12, 28),
                                 4: (15, 25, 15, 40), 5: (21, 36, 18, 54)}.items():
        ref = O.ReferenceElement(N)
        assert (ref.Np, ref.Nq, ref.Nfq, ref.Nh) == (Np, Nq, Nfq, Nh)
