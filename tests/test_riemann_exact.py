"""Pins of the exact Riemann solver used as the shock-capturing reference:
Sod's problem against the published star state (Toro, Table 4.2), continuity
of the rarefaction fan at its head and tail, the Rankine-Hugoniot conditions
across the shock, and mirror symmetry."""
import numpy as np

from tests.riemann_exact import sample, star_state

G = 1.4
SOD_L, SOD_R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_sod_star_state():
    p, u = star_state(SOD_L, SOD_R, G)
    assert abs(p - 0.30313) < 5e-6 and abs(u - 0.92745) < 5e-6
    s = np.array([u - 1e-9, u + 1e-9])
    rho = sample(SOD_L, SOD_R, s, G)[0]
    assert abs(rho[0] - 0.42632) < 5e-6 and abs(rho[1] - 0.26557) < 5e-6


def test_fan_is_continuous_and_isentropic():
    p, u = star_state(SOD_L, SOD_R, G)
    cl = np.sqrt(G * SOD_L[2] / SOD_L[0])
    cs = cl * (p / SOD_L[2]) ** ((G - 1) / (2 * G))
    head, tail = -cl, u - cs
    e = 1e-10
    W = sample(SOD_L, SOD_R, np.array([head - e, head + e, tail - e, tail + e]), G)
    assert np.abs(W[:, 0] - W[:, 1]).max() < 1e-8
    assert np.abs(W[:, 2] - W[:, 3]).max() < 1e-8
    fan = sample(SOD_L, SOD_R, np.linspace(head + 1e-3, tail - 1e-3, 9), G)
    # isentropic (p / rho^gamma of the left state), and the left state's Riemann invariant u + 2c/(gamma-1)
    ent = fan[2] / fan[0] ** G
    assert np.abs(ent / (SOD_L[2] / SOD_L[0] ** G) - 1).max() < 1e-12
    c = np.sqrt(G * fan[2] / fan[0])
    assert np.abs(fan[1] + 2 * c / (G - 1) - 2 * cl / (G - 1)).max() < 1e-12


def test_shock_satisfies_rankine_hugoniot():
    p, u = star_state(SOD_L, SOD_R, G)
    rr, ur, pr = SOD_R
    cr = np.sqrt(G * pr / rr)
    S = ur + cr * np.sqrt((G + 1) / (2 * G) * p / pr + (G - 1) / (2 * G))
    rs = sample(SOD_L, SOD_R, np.array([S - 1e-9]), G)[0, 0]
    # mass, momentum and energy fluxes in the shock frame
    Es, Er = p / (G - 1) + 0.5 * rs * u * u, pr / (G - 1) + 0.5 * rr * ur * ur
    assert abs(rs * (u - S) - rr * (ur - S)) < 1e-12
    assert abs(rs * u * (u - S) + p - (rr * ur * (ur - S) + pr)) < 1e-12
    assert abs((Es + p) * u - S * Es - ((Er + pr) * ur - S * Er)) < 1e-12


def test_mirror_symmetry():
    s = np.linspace(-2, 2, 41) + 1e-7
    A = sample(SOD_L, SOD_R, s, G)
    B = sample(SOD_R, SOD_L, -s, G)
    assert np.abs(A[0] - B[0]).max() < 1e-12 and np.abs(A[1] + B[1]).max() < 1e-12
