"""Pins of the oracle's Roe flux (Harten-Hyman entropy fix) and Sutherland
viscosity, the face flux and viscosity law of the paper's solver
(§Governing Equations and Numerical Method; §Compressible Taylor-Green-Vortex).

Roe: the signed linearisation reproduces the flux jump exactly (Roe's
property), it vanishes for equal states, stationary contacts carry no
dissipation, supersonic states are upwinded, and the entropy fix changes the
dissipation only at transonic acoustic waves.  Sutherland: the reference
value, tabulated air viscosity at 300 K, and the T^(1/2) / T^(3/2) limits.
Residual level: free-stream preservation, conservation and rotation
invariance with the Roe flux and with Sutherland's law.
"""
import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from tests.helpers import quad_weights3

G = 1.4
PI = np.pi


def cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u])


def rand_state(rng):
    return cons(rng.uniform(0.5, 2.0), rng.uniform(-1, 1, 3), rng.uniform(0.5, 2.0))


def unit(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def test_roe_property(orc):
    """A~(UR - UL) = f(UR).n - f(UL).n for any two states (signed speeds)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        UL, UR, nh = rand_state(rng), rand_state(rng), unit(rng)
        got = orc.roe_matrix(UL, UR, nh, mode=1)
        want = orc.flux_adv(UR, nh) - orc.flux_adv(UL, nh)
        assert np.abs(got - want).max() < 1e-13 * (1 + np.abs(want).max()), (got, want)


def test_roe_consistency_and_contact(orc):
    rng = np.random.default_rng(12)
    for _ in range(20):
        U, nh = rand_state(rng), unit(rng)
        for mode in (0, 1, 2):
            assert np.abs(orc.roe_matrix(U, U, nh, mode)).max() == 0.0
    # stationary contact: equal pressure, zero velocity, different density
    for _ in range(20):
        nh = unit(rng)
        UL, UR = cons(rng.uniform(0.5, 2), [0, 0, 0], 1.3), cons(rng.uniform(0.5, 2), [0, 0, 0], 1.3)
        assert np.abs(orc.roe_matrix(UL, UR, nh, 0)).max() < 1e-15


def test_roe_supersonic_upwinding(orc):
    """All wave speeds of one sign: |A~| = +-A~, so the weak-form Roe flux
    {f}.n - 1/2 |A~| dU is the upwind state's flux."""
    rng = np.random.default_rng(13)
    for sgn in (1.0, -1.0):
        for _ in range(20):
            nh = unit(rng)
            UL = cons(rng.uniform(0.8, 1.2), sgn * 4.0 * nh + 0.1 * rng.normal(size=3), rng.uniform(0.8, 1.2))
            UR = cons(rng.uniform(0.8, 1.2), sgn * 4.0 * nh + 0.1 * rng.normal(size=3), rng.uniform(0.8, 1.2))
            D = orc.roe_matrix(UL, UR, nh, 0)
            F = 0.5 * (orc.flux_adv(UL, nh) + orc.flux_adv(UR, nh)) - 0.5 * D
            up = orc.flux_adv(UL if sgn > 0 else UR, nh)
            assert np.abs(F - up).max() < 1e-12 * np.abs(up).max()
            assert np.abs(D - orc.roe_matrix(UL, UR, nh, 2)).max() == 0.0


def test_entropy_fix_acts_only_at_transonic_acoustic_waves(orc):
    rng = np.random.default_rng(14)
    # subsonic, well away from sonic points: fix inactive
    for _ in range(20):
        nh = unit(rng)
        UL = cons(1.0, 0.2 * rng.normal(size=3), 1.0)
        UR = cons(1.1, 0.2 * rng.normal(size=3), 1.05)
        assert np.abs(orc.roe_matrix(UL, UR, nh, 0) - orc.roe_matrix(UL, UR, nh, 2)).max() == 0.0
    # transonic expansion in the first acoustic wave: un - c goes from -0.1 to +0.1;
    # the Roe speed is near zero and the fix adds dissipation along r1
    c = np.sqrt(G)
    nh = np.array([0.0, 0.0, 1.0])
    UL, UR = cons(1.0, [0, 0, c - 0.1], 1.0), cons(1.0, [0, 0, c + 0.1], 1.0)
    d = orc.roe_matrix(UL, UR, nh, 0) - orc.roe_matrix(UL, UR, nh, 2)
    assert np.abs(d).max() > 1e-3
    # the added part is a multiple of the first acoustic eigenvector (1, u~ - c~ n, H~ - un~ c~)
    # at the Roe averages (equal densities: plain means of u and H)
    um = 0.5 * (UL[1:4] + UR[1:4])
    Hm = 0.5 * ((UL[4] + 1.0) + (UR[4] + 1.0))
    cm = np.sqrt((G - 1) * (Hm - 0.5 * um @ um))
    r1 = np.array([1.0, *(um - cm * nh), Hm - (um @ nh) * cm])
    coef = d[0] / r1[0]
    assert np.abs(d - coef * r1).max() < 1e-12 * np.abs(d).max()


def test_sutherland_law(orc):
    # reference value
    assert orc.viscosity(1.0, mu=0.3, Tref=1.0, Ts=0.4) == pytest.approx(0.3, rel=1e-15)
    # air: mu_ref = 1.716e-5 Pa s at 273.15 K, S = 110.4 K; tabulated 1.846e-5 Pa s at 300 K
    mu300 = orc.viscosity(300.0, mu=1.716e-5, Tref=273.15, Ts=110.4 / 273.15)
    assert abs(mu300 / 1.846e-5 - 1.0) < 2e-3
    # limits: mu ~ T^(1/2) for T >> S, ~ T^(3/2) for T << S
    hi = orc.viscosity(4e6, Ts=0.4) / orc.viscosity(1e6, Ts=0.4)
    lo = orc.viscosity(4e-6, Ts=0.4) / orc.viscosity(1e-6, Ts=0.4)
    assert abs(hi - 2.0) < 1e-5 and abs(lo - 8.0) < 1e-4
    # constant law: the viscous flux of the Sutherland law at T = Tref equals the constant-mu flux
    rng = np.random.default_rng(15)
    U = cons(1.0, [0.1, 0.2, 0.3], 1.0)          # T = p/(rho R) = 1
    g = rng.normal(size=12)
    for n in range(3):
        a = orc.flux_visc_law(U, g, n, mu=0.02, law=1, Tref=1.0)
        b = orc.flux_visc(U, g, n, mu=0.02)
        assert np.abs(a - b).max() < 1e-15 * np.abs(b).max() + 1e-300


VARIANTS = [
    dict(riemann=2),
    dict(riemann=2, viscosity=1, Tref=1.0 / (G * 0.01), Ts=0.4),
    dict(viscosity=1, Tref=1.0, Ts=0.4),
]


@pytest.mark.parametrize("N,nodes,form,physics,extra", [
    (5, 1, 1, 0, VARIANTS[0]), (4, 0, 0, 0, VARIANTS[0]), (5, 1, 1, 1, VARIANTS[1]), (4, 1, 0, 1, VARIANTS[2])])
def test_free_stream_preservation(orc, N, nodes, form, physics, extra):
    curved = nodes == 1
    mesh = I.box_mesh((3, 3, 3), (-PI,) * 3, (PI,) * 3, Ngeo=N if curved else 1,
                      curved_amp=0.1 if curved else 0.0, rotate_seed=21)
    o = orc.Oracle(dict(N=N, nodes=nodes, form=form, physics=physics, mu=1.0 / 1600, **extra), mesh)
    rho, u, p = 1.0, np.array([0.1, 0.2, -0.1]), 1.0 / (G * 0.01)
    U = np.zeros(o.state_shape)
    U[:] = cons(rho, u, p)[:, None, None, None, None]
    R = o.rhs(U)
    _, J, Ja = o.geometry()
    b = orc.basis(N, nodes)
    Dhat = (b["w"][:, None] / b["w"][None, :]) * b["D"]
    f = np.abs(orc.flux_adv(U[:, 0, 0, 0, 0], np.ones(3))).max() + np.abs(U[:, 0, 0, 0, 0]).max()
    scale = 3 * f * np.abs(Ja).max() * np.abs(Dhat).sum(0).max() / J.min()
    assert np.abs(R).max() < 1e-13 * scale


@pytest.mark.parametrize("N,nodes,form,physics,rot,extra", [
    (3, 0, 0, 0, None, VARIANTS[0]), (4, 1, 1, 0, 4, VARIANTS[0]), (3, 1, 1, 1, 9, VARIANTS[1]),
    (3, 0, 0, 1, 4, VARIANTS[2])])
def test_conservation(orc, N, nodes, form, physics, rot, extra):
    mesh = I.box_mesh((3, 2, 3), (-PI,) * 3, (PI,) * 3, Ngeo=N if nodes == 1 else 1,
                      curved_amp=0.1 if nodes == 1 else 0.0, rotate_seed=rot)
    o = orc.Oracle(dict(N=N, nodes=nodes, form=form, physics=physics, mu=0.05, **extra), mesh)
    xyz, J, _ = o.geometry()
    U = I.smooth_random_state(xyz, 5, amp=0.2)
    R = o.rhs(U)
    W = quad_weights3(orc.basis(N, nodes)["w"])
    for v in range(5):
        assert abs((W * J * R[v]).sum()) < 1e-13 * (W * J * np.abs(R[v])).sum()


def test_roe_changes_the_residual_and_sutherland_scales_viscosity(orc):
    """The switches reach the residual: Roe differs from Rusanov on a
    non-constant state, and Sutherland at T = Tref equals the constant law."""
    mesh = I.box_mesh((2, 2, 2), (-PI,) * 3, (PI,) * 3)
    base = dict(N=3, nodes=1, form=1, physics=1, mu=0.05)
    xyz = orc.Oracle(base, mesh).coords()
    # per-node random values jump across faces (a continuous nodal field does not on LGL nodes)
    U = I.random_state(xyz.shape[1:], 6)
    R_rus = orc.Oracle(base, mesh).rhs(U)
    R_roe = orc.Oracle(dict(base, riemann=2), mesh).rhs(U)
    assert np.abs(R_roe - R_rus).max() > 1e-3 * np.abs(R_rus).max()
    U = I.smooth_random_state(xyz, 6, amp=0.2)
    # uniform temperature 1 (p = rho R): Sutherland with Tref = 1 gives mu everywhere
    Uc = U.copy()
    rho = Uc[0]
    m = Uc[1:4]
    Uc[4] = rho / (G - 1) + 0.5 * (m * m).sum(0) / rho
    R_c = orc.Oracle(base, mesh).rhs(Uc)
    R_s = orc.Oracle(dict(base, viscosity=1, Tref=1.0, Ts=0.4), mesh).rhs(Uc)
    assert np.abs(R_s - R_c).max() < 1e-12 * np.abs(R_c).max()
