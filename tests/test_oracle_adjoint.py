"""Pins of the oracle's reverse mode: the taped transposed residual Jacobian,
the gradient of E_k and the reverse sweep of the low-storage RK schemes.

They are checked against what does not share their arithmetic:

* the dual-number tangent (forward mode, itself pinned against finite
  differences): <(dR/dU)^T lam, d> = <lam, (dR/dU) d> for every
  discretisation variant, and the whole matrix entry by entry on one element;
* the closed form of dE_k/dU (drho: -c w J |m|^2/rho^2, dm: 2 c w J m/rho,
  dE: 0, c = 1/(2 rho0 U0^2 |Omega|));
* trajectory tangents and central finite differences of E_k(U(T)) for the
  reverse RK sweep (LSERK4(5) and LSERK4-14).
"""
import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from tests.helpers import quad_weights3

PI = np.pi

VARIANTS = [
    # config, K, curved, rotate_seed, FV mask seed (None: DG only)
    (dict(N=3, nodes=0, form=0, physics=0), (2, 2, 2), 0.0, 7, None),
    (dict(N=3, nodes=1, form=1, physics=1, mu=0.05), (2, 2, 2), 0.1, 2, None),
    (dict(N=3, nodes=0, form=1, physics=1, mu=0.05), (2, 2, 1), 0.0, 3, None),
    (dict(N=2, nodes=1, form=1, physics=1, mu=0.05, riemann=2, viscosity=1, Tref=1.0, Ts=0.4), (2, 1, 2), 0.1, 5,
     None),
    (dict(N=4, nodes=1, form=0, physics=1, mu=0.05), (1, 2, 2), 0.1, 9, None),
    (dict(N=2, nodes=0, form=0, physics=0, fv=1), (2, 2, 2), 0.0, 4, 11),
]


def _oracle(orc, cfg, K, curved, rot, fvseed):
    mesh = I.box_mesh(K, (-PI,) * 3, (PI,) * 3, Ngeo=cfg["N"] if curved else 1, curved_amp=curved, rotate_seed=rot)
    o = orc.Oracle(cfg, mesh)
    if fvseed is not None:
        o.fv_set_mask(np.random.default_rng(fvseed).integers(0, 2, mesh.nElems))
    return o


@pytest.mark.parametrize("cfg,K,curved,rot,fvseed", VARIANTS, ids=[str(v[0]) for v in VARIANTS])
def test_vjp_against_tangent(orc, cfg, K, curved, rot, fvseed):
    o = _oracle(orc, cfg, K, curved, rot, fvseed)
    U = I.smooth_random_state(o.coords(), 5, amp=0.2)
    rng = np.random.default_rng(1)
    for _ in range(2):
        lam, d = rng.uniform(-1, 1, U.shape), rng.uniform(-1, 1, U.shape)
        a = (o.rhs_vjp(U, lam) * d).sum()
        b = (lam * o.rhs_jvp(U, d)[1]).sum()
        assert abs(a - b) <= 1e-13 * (abs(a) + abs(b)), (a, b)


@pytest.mark.parametrize("cfg", [dict(N=2, nodes=1, form=1, physics=1, mu=0.05),
                                 dict(N=2, nodes=0, form=1, physics=0)], ids=str)
def test_vjp_whole_matrix(orc, cfg):
    """One periodic element: every row of (dR/dU)^T from unit seeds equals the
    corresponding column of the tangent, entry by entry."""
    mesh = I.box_mesh((1, 1, 1), (-PI,) * 3, (PI,) * 3, rotate_seed=3)
    o = orc.Oracle(cfg, mesh)
    U = I.smooth_random_state(o.coords(), 8, amp=0.2)
    n = U.size
    Jc = np.empty((n, n))
    Jr = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Jc[:, i] = o.rhs_jvp(U, e.reshape(U.shape))[1].ravel()
        Jr[i, :] = o.rhs_vjp(U, e.reshape(U.shape)).ravel()
    assert np.abs(Jc - Jr).max() <= 1e-13 * np.abs(Jc).max()


def test_kinetic_energy_gradient_closed_form(orc):
    mesh = I.box_mesh((2, 1, 2), (-PI,) * 3, (PI,) * 3, Ngeo=3, curved_amp=0.1, rotate_seed=4)
    o = orc.Oracle(dict(N=3, nodes=0), mesh)
    xyz, J, _ = o.geometry()
    U = I.tgv_state(xyz)
    rho0U0sq = 1.3
    g = o.kinetic_energy_grad(U, rho0U0sq)
    w = orc.basis(3, 0)["w"]
    wJ = quad_weights3(w)[None] * J
    c = 1.0 / (2.0 * rho0U0sq * wJ.sum())
    rho, m = U[0], U[1:4]
    ref = np.zeros_like(U)
    ref[0] = -c * wJ * (m * m).sum(0) / rho ** 2
    ref[1:4] = 2.0 * c * wJ * m / rho
    assert np.abs(g - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("cfg", [dict(N=3, nodes=1, form=1, physics=0),
                                 dict(N=2, nodes=1, form=1, physics=1, mu=0.05)], ids=str)
def test_reverse_sweep_against_trajectory_tangent(orc, cfg, integrator):
    mesh = I.box_mesh((2, 2, 1), (-PI,) * 3, (PI,) * 3, rotate_seed=6)
    o = orc.Oracle(dict(cfg, integrator=integrator), mesh)
    U0 = I.smooth_random_state(o.coords(), 12, amp=0.2)
    dt = o.timestep(U0, 0.9)
    nsteps = 4
    rng = np.random.default_rng(13)
    lamT = rng.uniform(-1, 1, U0.shape)
    lam0 = o.lserk_adjoint(U0, lamT, nsteps, dt)
    for _ in range(3):
        d = rng.uniform(-1, 1, U0.shape)
        _, dT = o.lserk_jvp(U0, d, nsteps, dt)
        a, b = (lam0 * d).sum(), (lamT * dT).sum()
        # rounding scale of the two inner products: the sums of the terms' magnitudes
        scale = np.abs(lam0 * d).sum() + np.abs(lamT * dT).sum()
        assert abs(a - b) <= 1e-13 * scale, (a, b, scale)


def test_reverse_sweep_finite_differences(orc):
    """Gradient of E_k(U(T)) through 6 LSERK4(5) steps against central differences."""
    mesh = I.box_mesh((2, 2, 2), (-PI,) * 3, (PI,) * 3)
    o = orc.Oracle(dict(N=3, nodes=1, form=1, physics=0), mesh)
    U0 = I.smooth_random_state(o.coords(), 14, amp=0.2)
    dt = o.timestep(U0, 0.9)
    nsteps = 6
    grad = o.lserk_adjoint(U0, o.kinetic_energy_grad(o.lserk(U0, nsteps, dt)), nsteps, dt)
    eps = 1e-6
    for d in I.random_directions(U0.size, (100, 101)):
        d = d.reshape(U0.shape)
        fd = (o.kinetic_energy(o.lserk(U0 + eps * d, nsteps, dt)) -
              o.kinetic_energy(o.lserk(U0 - eps * d, nsteps, dt))) / (2 * eps)
        ad = (grad * d).sum()
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (fd, ad)
