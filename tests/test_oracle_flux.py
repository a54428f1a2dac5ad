"""Pins of the oracle's point fluxes.

* two-point flux: consistency F#(U,U) = f(U), symmetry, Tadmor's entropy
  conservation condition [[v]].F# = [[rho u.n]], and the kinetic-energy-
  preserving structure of the momentum flux;
* logarithmic mean against a 50-digit evaluation of (x-y)/(ln x - ln y);
* viscous flux: symmetry and zero trace of the Stokes stress, pure heat
  conduction for a fluid at rest, linearity in the gradients;
* manufactured-solution source against a finite-difference evaluation of
  U_t + div F(U) from the oracle's own flux functions.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest

G = 1.4


def rand_state(rng, n=None):
    rho = rng.uniform(0.5, 2.0)
    u = rng.uniform(-1, 1, 3)
    p = rng.uniform(0.5, 2.0)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u])


def entropy_vars(U):
    rho = U[0]
    u = U[1:4] / rho
    p = (G - 1) * (U[4] - 0.5 * rho * u @ u)
    s = np.log(p) - G * np.log(rho)
    beta = rho / (2 * p)
    return np.array([(G - s) / (G - 1) - beta * u @ u, *(2 * beta * u), -2 * beta])


def test_twopoint_consistent_and_symmetric(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        Ua, Ub = rand_state(rng), rand_state(rng)
        n = rng.normal(size=3)
        assert np.allclose(orc.flux_twopoint(Ua, Ua, n), orc.flux_adv(Ua, n), rtol=1e-14, atol=1e-14)
        assert np.allclose(orc.flux_twopoint(Ua, Ub, n), orc.flux_twopoint(Ub, Ua, n), rtol=1e-14, atol=1e-14)
        # linear in the direction
        n2 = rng.normal(size=3)
        lhs = orc.flux_twopoint(Ua, Ub, 2.0 * n - 0.5 * n2)
        rhs = 2.0 * orc.flux_twopoint(Ua, Ub, n) - 0.5 * orc.flux_twopoint(Ua, Ub, n2)
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-13)


def test_twopoint_entropy_conservative(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        Ua, Ub = rand_state(rng), rand_state(rng)
        n = rng.normal(size=3)
        F = orc.flux_twopoint(Ua, Ub, n)
        jump_v = entropy_vars(Ub) - entropy_vars(Ua)
        psi = lambda U: U[1:4] @ n
        assert abs(jump_v @ F - (psi(Ub) - psi(Ua))) < 1e-12 * (1 + np.abs(F).max())
    # near-equal states exercise the series branch of the log mean
    for _ in range(50):
        Ua = rand_state(rng)
        Ub = Ua * (1 + 1e-4 * rng.uniform(-1, 1, 5))
        n = rng.normal(size=3)
        F = orc.flux_twopoint(Ua, Ub, n)
        jump_v = entropy_vars(Ub) - entropy_vars(Ua)
        assert abs(jump_v @ F - (Ub[1:4] - Ua[1:4]) @ n) < 1e-12


def test_twopoint_kinetic_energy_structure(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        Ua, Ub = rand_state(rng), rand_state(rng)
        n = rng.normal(size=3)
        F = orc.flux_twopoint(Ua, Ub, n)
        um = 0.5 * (Ua[1:4] / Ua[0] + Ub[1:4] / Ub[0])
        pres = F[1:4] - um * F[0]          # must be a pure pressure term p_hat * n
        ph = pres @ n / (n @ n)
        assert np.allclose(pres, ph * n, rtol=1e-13, atol=1e-13)
        pa = (G - 1) * (Ua[4] - 0.5 * Ua[1:4] @ Ua[1:4] / Ua[0])
        pb = (G - 1) * (Ub[4] - 0.5 * Ub[1:4] @ Ub[1:4] / Ub[0])
        # p_hat = {rho}/(2{beta}) is a rho-weighted harmonic mean of the two pressures
        assert min(pa, pb) - 1e-12 <= ph <= max(pa, pb) + 1e-12


def test_central_switch_is_flux_average(orc):
    rng = np.random.default_rng(4)
    Ua, Ub = rand_state(rng), rand_state(rng)
    n = rng.normal(size=3)
    F = orc.flux_twopoint(Ua, Ub, n, central=True)
    assert np.allclose(F, 0.5 * (orc.flux_adv(Ua, n) + orc.flux_adv(Ub, n)), rtol=1e-15, atol=1e-15)


def _logmean_ref(x, y):
    getcontext().prec = 60
    X, Y = Decimal(float(x)), Decimal(float(y))
    if X == Y:
        return float(X)
    return float((X - Y) / (X.ln() - Y.ln()))


def test_logmean_accuracy(orc):
    """Series branch (|x-y|/(x+y) < 1e-2): a few ulp.  Direct branch: the
    rounding of ln x - ln y bounds the error by ~eps |ln x| / |ln x - ln y|."""
    rng = np.random.default_rng(5)
    worst_series, worst_direct = 0.0, 0.0
    for _ in range(3000):
        x = rng.uniform(0.01, 10.0)
        rel = 10.0 ** rng.uniform(-12, 0)
        y = x * (1 + rel * rng.choice([-1, 1]) * rng.uniform(0.1, 1.0))
        got, ref = orc.logmean(x, y), _logmean_ref(x, y)
        f = abs(x - y) / (x + y)
        if f < 0.0099:
            worst_series = max(worst_series, abs(got - ref) / ref)
        elif f > 0.0101:
            cond = max(abs(np.log(x)), abs(np.log(y)), 1.0) / abs(np.log(x) - np.log(y))
            worst_direct = max(worst_direct, abs(got - ref) / ref / cond)
    assert worst_series < 1e-15
    assert worst_direct < 1e-15
    assert orc.logmean(1.5, 1.5) == 1.5


def test_viscous_flux_properties(orc):
    rng = np.random.default_rng(6)
    mu, Pr = 0.02, 0.72
    lam = mu * G * 1.0 / ((G - 1) * Pr)
    for _ in range(20):
        U = rand_state(rng)
        g = rng.normal(size=12)
        Gs = np.array([orc.flux_visc(U, g, n, mu=mu, Pr=Pr) for n in range(3)])
        tau = Gs[:, 1:4]                       # tau[n][a]
        assert np.allclose(tau, tau.T, rtol=1e-14, atol=1e-15)
        assert abs(np.trace(tau)) < 1e-14
        assert np.all(Gs[:, 0] == 0.0)
        # linear in the gradients
        g2 = rng.normal(size=12)
        Gs2 = np.array([orc.flux_visc(U, g2, n, mu=mu, Pr=Pr) for n in range(3)])
        Gs3 = np.array([orc.flux_visc(U, 3 * g - g2, n, mu=mu, Pr=Pr) for n in range(3)])
        assert np.allclose(Gs3, 3 * Gs - Gs2, rtol=1e-13, atol=1e-13)
    # fluid at rest with a temperature gradient: pure Fourier conduction
    U = np.array([1.0, 0, 0, 0, 2.5])
    g = np.zeros(12)
    g[9:12] = [0.3, -0.2, 0.7]
    for n in range(3):
        Gn = orc.flux_visc(U, g, n, mu=mu, Pr=Pr)
        assert np.allclose(Gn[:4], 0.0) and abs(Gn[4] - lam * g[9 + n]) < 1e-15
    # uniform shear du/dy = s: tau_xy = mu s, energy flux tau.u
    U = np.array([1.0, 0.5, 0.0, 0.0, 2.5])
    g = np.zeros(12)
    g[1] = 0.4
    G1 = orc.flux_visc(U, g, 1, mu=mu, Pr=Pr)
    assert abs(G1[1] - mu * 0.4) < 1e-16 and abs(G1[4] - mu * 0.4 * 0.5) < 1e-16


@pytest.mark.parametrize("mu", [0.0, 1e-2])
def test_mms_source_matches_pde_residual(orc, mu):
    """Q = U_t + div F(U, grad U) for the manufactured solution, by central differences."""
    A, a, Pr, R = 0.1, 1.0, 0.72, 1.0

    def exact(x, y, z, t):
        rho = 2 + A * np.sin(2 * np.pi * (x + y + z - a * t))
        return np.array([rho, rho, rho, rho, rho * rho])

    def prim(U):
        rho = U[0]
        u = U[1:4] / rho
        p = (G - 1) * (U[4] - 0.5 * rho * u @ u)
        return np.array([*u, p / (rho * R)])

    h = 1e-4
    rng = np.random.default_rng(7)
    for _ in range(5):
        x, y, z, t = rng.uniform(-1, 1, 4)
        X = np.array([x, y, z])
        Ut = (exact(*X, t + h) - exact(*X, t - h)) / (2 * h)
        div = np.zeros(5)
        for n in range(3):
            e = np.zeros(3)
            e[n] = h

            def flux(P):
                U = exact(*P, t)
                grad = np.zeros(12)
                for d in range(3):
                    ed = np.zeros(3)
                    ed[d] = h
                    dq = (prim(exact(*(P + ed), t)) - prim(exact(*(P - ed), t))) / (2 * h)
                    grad[d::3] = dq
                nv = np.zeros(3)
                nv[n] = 1.0
                return orc.flux_adv(U, nv) - orc.flux_visc(U, grad, n, mu=mu, Pr=Pr)

            div += (flux(X + e) - flux(X - e)) / (2 * h)
        Q = orc.mms_source(x, y, z, t, mu=mu, Pr=Pr, A=A, a=a)
        assert np.allclose(Q, Ut + div, rtol=1e-5, atol=2e-5)
