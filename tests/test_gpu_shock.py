"""Shock capturing on the GPU: a periodic double Sod shock tube (Euler, N = 3
LG weak form with FV sub-cells, Kx x 1 x 1 elements on [0, 2] x [0, h]^2).

The high state (rho, p) = (1, 1) sits in 0.51 < x < 1.51 and the low state
(0.125, 0.1) around it; the two Riemann problems do not interact before
t = 0.2.  Elements are switched between DG and FV by the Persson indicator
(thresholds -5 / -3.5, with hysteresis) after every LSERK4(5) step.

* against the oracle running the same switching loop (16 elements): the same
  element types after every step and the same final state (1e-10);
* at t = 0.2 (32 and 64 elements): the state stays physical and near the
  initial density range, mass, momentum and energy are conserved, the
  element-mean density is within 0.02 / 0.012 (L1) of the exact solution's
  element averages, and the error falls under refinement.
"""
import sys

import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from tests.riemann_exact import sample

pytestmark = pytest.mark.gpu
G = 1.4
X0, X1 = 0.51, 1.51
HIGH, LOW = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
LO_T, HI_T = -5.0, -3.5
T_END = 0.2
_L1 = {}


def _say(*a):
    print("[gpu-shock]", *a, flush=True)
    sys.stdout.flush()


def _exact_rho(x, t):
    a = sample(LOW, HIGH, (x - X0) / t, G)[0]    # interface at X0: low | high
    b = sample(HIGH, LOW, (x - X1) / t, G)[0]    # interface at X1: high | low
    return np.where(x < 1.01, a, b)


def _initial(xyz):
    inside = (xyz[0] > X0) & (xyz[0] < X1)
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    return I.prim_to_cons(rho, 0 * rho, 0 * rho, 0 * rho, p, G)


def _mesh(Kx):
    h = 2.0 / Kx
    return I.box_mesh((Kx, 1, 1), (0.0, 0.0, 0.0), (2.0, h, h)), h


def _totals(U, mask, h):
    """Integrals of the five conserved variables (affine cubes of side h)."""
    w = np.polynomial.legendre.leggauss(4)[1]
    W3 = w[None, None, :] * w[None, :, None] * w[:, None, None] * (h / 2) ** 3
    dg = (W3 * U).sum(axis=(2, 3, 4))                  # [5][nE]
    fv = U.sum(axis=(2, 3, 4)) * h ** 3 / 64.0
    return np.where(mask[None, :] == 1, fv, dg).sum(axis=1)


def _element_mean_rho(U, mask):
    w = np.polynomial.legendre.leggauss(4)[1]
    W3 = w[None, None, :] * w[None, :, None] * w[:, None, None] / 8.0
    return np.where(mask == 1, U[0].mean(axis=(1, 2, 3)), (W3 * U[0]).sum(axis=(1, 2, 3)))


def _gpu_run(Kx, dt=None, cfl=0.5, record=False):
    import torch
    from paper_2605_28627_amd.solver import DGSolver
    assert torch.cuda.is_available()
    mesh, h = _mesh(Kx)
    s = DGSolver(dict(N=3, nodes=0, form=0, physics=0, fv=1), mesh)
    U = s.init_state(_initial(s.coords()))
    s.fv_switch_by_indicator(U, LO_T, HI_T)
    if dt is None:
        dt = s.timestep(U, cfl)
        n = int(np.ceil(T_END / dt))
        dt = T_END / n
    else:
        n = int(round(T_END / dt))
    dU = torch.zeros_like(U)
    masks = [s.fv_mask().copy()]
    tot0 = _totals(U.cpu().numpy(), masks[0], h)
    for _ in range(n):
        s.rk_step(U, dU, dt, 1)
        s.fv_switch_by_indicator(U, LO_T, HI_T)
        if record:
            masks.append(s.fv_mask().copy())
    ok = s.check_state(U) == 0
    mask = s.fv_mask().copy()
    Uh = U.cpu().numpy()
    s.close()
    return dict(U=Uh, mask=mask, masks=masks, ok=ok, n=n, dt=dt, h=h, tot0=tot0)


def test_switching_run_matches_oracle(orc):
    Kx = 16
    mesh, h = _mesh(Kx)
    o = orc.Oracle(dict(N=3, nodes=0, form=0, physics=0, fv=1), mesh)
    U = _initial(o.coords())
    mask = np.zeros(mesh.nElems, np.int32)

    def decide(U, mask):
        ind = o.indicator(U)
        return np.where(ind > HI_T, 1, np.where(ind < LO_T, 0, mask)).astype(np.int32)

    mask = decide(U, mask)
    U, _ = o.fv_switch(U, None, mask)
    dt = o.timestep(U, 0.5)
    n = int(np.ceil(T_END / dt))
    dt = T_END / n
    masks = [mask]
    for _ in range(n):
        U = o.lserk(U, 1, dt)
        mask = decide(U, mask)
        U, _ = o.fv_switch(U, None, mask)
        masks.append(mask)
    g = _gpu_run(Kx, dt=dt, record=True)
    _say("oracle steps", n, "FV elements per step", [int(m.sum()) for m in masks])
    assert g["n"] == n
    for k, (a, b) in enumerate(zip(g["masks"], masks)):
        assert np.array_equal(a, b), (k, a, b)
    # momentum components against the largest one (m_y, m_z are round-off)
    scale = np.abs(U).max(axis=(1, 2, 3, 4))
    scale[1:4] = scale[1:4].max()
    err = np.abs(g["U"] - U).max(axis=(1, 2, 3, 4)) / scale
    _say("final state relative difference per variable", err)
    assert np.all(err < 1e-10), err


@pytest.mark.parametrize("Kx", [32, 64])
def test_double_sod_against_exact(Kx):
    g = _gpu_run(Kx)
    U, mask, h = g["U"], g["mask"], g["h"]
    assert g["ok"]
    rho = U[0]
    rng = (rho.min(), rho.max())
    tot = _totals(U, mask, h)
    cons = np.abs(tot - g["tot0"]) / np.abs(g["tot0"][[0, 0, 0, 0, 4]])
    xs = (np.arange(Kx)[:, None] + (np.arange(400)[None, :] + 0.5) / 400) * h
    exact = _exact_rho(xs, T_END).mean(axis=1)
    l1 = np.abs(_element_mean_rho(U, mask) - exact).sum() * h
    _say("Kx", Kx, "steps", g["n"], "FV elements", int(mask.sum()), "rho range", rng, "conservation", cons, "L1", l1)
    assert 0.1 < rng[0] and rng[1] < 1.05
    assert np.all(cons < 1e-13), cons
    assert l1 < (0.02 if Kx == 32 else 0.012)
    _L1[Kx] = l1
    if Kx == 64 and 32 in _L1:
        assert l1 < 0.8 * _L1[32], _L1
