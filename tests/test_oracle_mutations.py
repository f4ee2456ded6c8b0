"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch them.

Each mutation is applied to a fresh oracle instance; the property checks used are the
lake-at-rest residual, the entropy production of the EC scheme, and mass conservation.
A mutation that none of them detects would mean the pins leave that part unpinned.
"""
import numpy as np
import pytest

from oracle import esdg_oracle as O
from paper_2005_02516_amd import workloads as wl


def _setup(N=2):
    xg, yg, xf, yf = wl.structured_mesh(4, N, warp=0.05)
    b = 0.1 * np.sin(np.pi * xf) * np.cos(np.pi * yf) + 0.1
    d = O.Discretization(N, xg, yg, b, 1.0, 2.0, 2.0)
    rng = np.random.default_rng(4)
    h = 2.3 - b + 0.05 * np.sin(np.pi * (xf + rng.uniform())) * np.cos(np.pi * yf)
    u = np.stack([h, h * (0.2 + 0.1 * np.sin(np.pi * yf)), h * (-0.1 + 0.1 * np.cos(np.pi * xf))])
    lake = np.stack([2.2 - b, 0 * b, 0 * b])
    return d, u, lake


def properties_hold(d, u, lake):
    """True if lake-at-rest, EC entropy conservation and mass conservation all hold."""
    o_ec = O.Oracle(d, "ec")
    ok_lake = np.abs(o_ec.rhs(d.interpolate(lake))).max() < 1e-12
    dg = O.diagnostics(o_ec, d.interpolate(u))
    ok_ent = abs(dg["entropy_rate"]) < 1e-12 * dg["entropy_rate_scale"]
    r = o_ec.rhs(d.interpolate(u))
    wJ = d.ref.wq[None] * d.Jq
    ok_mass = abs(np.sum(wJ * (r[0] @ d.ref.Vq.T))) < 1e-12 * np.abs(r[0]).sum()
    return ok_lake and ok_ent and ok_mass


def test_unmutated_oracle_passes():
    d, u, lake = _setup()
    assert properties_hold(d, u, lake)


def _mut_transpose_Q(d):
    d.ref.Qh[0] = d.ref.Qh[0].T.copy()


def _mut_swap_metric(d):
    d.rxJ, d.ryJ = d.ryJ, d.rxJ


def _mut_unweighted_projection(d):
    def project(f_q, d=d):
        return f_q @ d.ref.Pq.T
    d.project = project


def _mut_discontinuous_b(d):
    """Bathymetry at the hybridized nodes that is no longer C0 across elements."""
    rng = np.random.default_rng(0)
    d.b_hyb = d.b_hyb + 1e-3 * rng.uniform(size=(d.K, 1))


def _mut_normal_sign(d):
    d.nJx = -d.nJx


def _mut_lift_with_Vq_only(d):
    Vh = d.ref.Vh.copy()
    Vh[d.ref.Nq:] = 0.0
    d.ref.Vh = Vh


@pytest.mark.parametrize("mut", [_mut_transpose_Q, _mut_swap_metric, _mut_unweighted_projection,
                                 _mut_discontinuous_b, _mut_normal_sign, _mut_lift_with_Vq_only])
def test_mutation_is_caught(mut):
    d, u, lake = _setup()
    mut(d)
    with np.errstate(all="ignore"):
        assert not properties_hold(d, u, lake)


def test_pressure_mutation_caught_by_tadmor(monkeypatch):
    """A wrong pressure average (g{h}^2 instead of g{h}^2 - 1/2 g{h^2}) breaks Tadmor's condition."""
    real = O.ec_flux

    def bad(uL, uR, g):
        fx, fy = real(uL, uR, g)
        extra = 0.5 * g * 0.5 * (uL[0] ** 2 + uR[0] ** 2)
        return (fx[0], fx[1] + extra, fx[2]), (fy[0], fy[1], fy[2] + extra)

    monkeypatch.setattr(O, "ec_flux", bad)
    d, u, lake = _setup()
    assert not properties_hold(d, u, lake)


def test_source_sign_flip_caught(monkeypatch):
    """Adding the bathymetry source with the wrong sign breaks the lake at rest."""
    real = O.Oracle.residual

    def flipped(self, uh, elements=None):
        r = real(self, uh, elements)
        ut, _ = self.entropy_projection(uh)
        Qx, Qy = self.physical_Qh(slice(0, self.d.K))
        g = self.d.g
        r[1] -= 2 * g * ut[0] * np.einsum("kmn,kn->km", Qx, self.d.b_hyb)
        r[2] -= 2 * g * ut[0] * np.einsum("kmn,kn->km", Qy, self.d.b_hyb)
        return r

    monkeypatch.setattr(O.Oracle, "residual", flipped)
    d, u, lake = _setup()
    assert not properties_hold(d, u, lake)


def _vh_consistent(d, u, Href):
    """V_h v_h equals the entropy variables of u~ (both from entropy_projection)."""
    ut, vh = O.Oracle(d, "lf", Href=Href).entropy_projection(d.interpolate(u))
    v = np.stack(O.entropy_variables(ut[0], ut[1], ut[2], d.b_hyb, d.g))
    return np.abs(vh @ d.ref.Vh.T - v).max() < 1e-12 * np.abs(v).max()


def test_reference_level_shift_on_momentum_caught(monkeypatch):
    """Shifting the projected momentum variables by the reference level as well as the depth
    variable breaks V_h v_h = v(u~)."""
    real = O.Oracle.entropy_projection

    def shifted(self, uh):
        ut, vh = real(self, uh)
        vh = vh.copy()
        vh[1:, :, 0] += self.d.g * self.Href * np.sqrt(2.0)
        return ut, vh

    d, u, _ = _setup()
    assert _vh_consistent(d, u, 2.2)
    monkeypatch.setattr(O.Oracle, "entropy_projection", shifted)
    assert not _vh_consistent(d, u, 2.2)
