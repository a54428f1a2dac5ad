"""GPU parity of the entropy-stable split form on Legendre-Gauss nodes (the
hybridised SBP operator with entropy-projected face states) against the
oracle, through the C-ABI.

* residual on small meshes for N = 1..7: the shuffle-free and the in-wavefront
  line paths, rotated frames, curved elements, Euler and Navier-Stokes, with
  the oracle's metrics uploaded: 1e-12 per variable;
* the central face flux, the central two-point switch, Roe with Sutherland;
* BR1 lifting from the projected traces; LSERK4(5) and LSERK4-14 steps
  (the projected traces of each new stage state come from the RK kernel);
* the FP32-flux path within 1e-4 (L2, per variable);
* on the GPU's own residual: entropy conservation with the central face flux,
  free-stream preservation and conservation with the library's metrics;
* the TGV workload at full size (16^3, N=3): sampled elements;
* a single periodic element and one-element slabs
(the adjoint of this form is checked with the other adjoint tests).
"""
import sys

import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from tests.helpers import quad_weights3, rel_err_per_var
from tests.test_oracle_invariants import _entropy_rate

pytestmark = pytest.mark.gpu
PI = np.pi


def _say(*a):
    print("[gpu-es-gauss]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def S(torch_cuda):
    from paper_2605_28627_amd.solver import DGSolver
    return DGSolver


CASES = [
    # N, physics, curved, rotate_seed   (nodes = Gauss, form = split)
    (1, 0, 0.0, 5),
    (2, 1, 0.1, 5),
    (3, 0, 0.0, 7),
    (3, 1, 0.1, 7),
    (4, 1, 0.0, 9),
    (5, 0, 0.1, 11),
    (6, 1, 0.0, 4),
    (7, 1, 0.0, 3),
    (7, 0, 0.1, 3),
]


def _setup(S, orc, case, K=(3, 2, 2), upload=True, **kw):
    N, physics, curved, rot = case
    mesh = I.box_mesh(K, (-PI,) * 3, (PI,) * 3, Ngeo=N if curved else 1, curved_amp=curved, rotate_seed=rot)
    cfg = dict(N=N, nodes=0, form=1, physics=physics, mu=0.02 if physics else 0.0)
    cfg.update(kw)
    o = orc.Oracle(cfg, mesh)
    s = S(cfg, mesh)
    if upload:
        _, J, Ja = o.geometry()
        s.upload_metrics(Ja, 1.0 / J, o.face_normals())
    return o, s, mesh


@pytest.mark.parametrize("case", CASES, ids=str)
def test_rhs_matches_oracle(S, orc, case):
    _say("rhs", case)
    o, s, _ = _setup(S, orc, case)
    U = I.smooth_random_state(o.coords(), 51, amp=0.1)
    R_orc = o.rhs(U)
    Ug = s.init_state(U)
    R_gpu = s.rhs(Ug).cpu().numpy()
    err = rel_err_per_var(R_gpu, R_orc)
    _say("rhs", case, "rel err", err)
    assert np.all(err < 1e-12), err
    assert np.array_equal(R_gpu, s.rhs(Ug).cpu().numpy())


@pytest.mark.parametrize("case", [CASES[2], CASES[3], CASES[8]], ids=str)
def test_switches_match_oracle(S, orc, case):
    """Central surface flux (riemann 1), the central two-point flux, and Roe with Sutherland."""
    for okw, gkw in ((dict(dissipation=0), dict(riemann=1)), (dict(twopoint=1), dict(twopoint=1)),
                     (dict(riemann=2, viscosity=1, Tref=1.0, Ts=0.4), dict(riemann=2, viscosity=1, Tref=1.0, Ts=0.4))):
        _say("switches", case, gkw)
        o, _, _ = _setup(S, orc, case, upload=False, **okw)
        _, s, _ = _setup(S, orc, case, upload=False, **gkw)
        _, J, Ja = o.geometry()
        s.upload_metrics(Ja, 1.0 / J, o.face_normals())
        U = I.smooth_random_state(o.coords(), 52, amp=0.1)
        err = rel_err_per_var(s.rhs(s.init_state(U)).cpu().numpy(), o.rhs(U))
        _say("switches", case, gkw, err)
        assert np.all(err < 1e-12), (gkw, err)


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[7]], ids=str)
def test_lift_matches_oracle(S, orc, case):
    _say("lift", case)
    o, s, _ = _setup(S, orc, case)
    U = I.smooth_random_state(o.coords(), 53, amp=0.1)
    err = rel_err_per_var(s.lift(s.init_state(U)).cpu().numpy(), o.lift(U))
    _say("lift", case, err.max())
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case,integrator", [(CASES[2], 0), (CASES[3], 0), (CASES[6], 1), (CASES[8], 1)], ids=str)
def test_rk_steps_match_oracle(S, orc, case, integrator):
    _say("rk", case, integrator)
    o, s, _ = _setup(S, orc, case, integrator=integrator)
    U0 = I.smooth_random_state(o.coords(), 54, amp=0.1)
    dt = o.timestep(U0, 0.9)
    Ug = s.init_state(U0)
    assert abs(s.timestep(Ug, 0.9) / dt - 1.0) < 1e-13
    U_orc = o.lserk(U0, 3, dt)
    s.rk_step(Ug, s.empty_state(), dt, 3)
    err = rel_err_per_var(Ug.cpu().numpy() - U0, U_orc - U0)
    _say("rk", case, integrator, err)
    assert np.all(err < 1e-11), err


@pytest.mark.parametrize("case", [CASES[3], CASES[7]], ids=str)
def test_fp32_flux_error(S, orc, case):
    o, s, _ = _setup(S, orc, case, precision=1)
    U = I.smooth_random_state(o.coords(), 55, amp=0.1)
    R_orc = o.rhs(U)
    R32 = s.rhs(s.init_state(U)).cpu().numpy()
    l2 = [np.linalg.norm(R32[v] - R_orc[v]) / np.linalg.norm(R_orc[v]) for v in range(5)]
    _say("fp32", case, l2)
    assert max(l2) < 1e-4, l2


@pytest.mark.parametrize("N", [3, 4])
def test_entropy_conservation_on_gpu(S, orc, N):
    """Central face flux: the GPU residual conserves the total entropy."""
    o, s, _ = _setup(S, orc, (N, 0, 0.0, 13), K=(3, 3, 2), riemann=1)
    _, J, _ = o.geometry()
    U = I.smooth_random_state(o.coords(), 56, amp=0.1)
    R = s.rhs(s.init_state(U)).cpu().numpy()
    rate, mag = _entropy_rate(o, U, R, J, quad_weights3(orc.basis(N, 0)["w"]))
    _say("entropy", N, rate / mag)
    assert abs(rate) < 1e-13 * mag


@pytest.mark.parametrize("case", [(3, 1, 0.0, 21), (6, 0, 0.0, 21)], ids=str)
def test_free_stream_and_conservation(S, orc, case):
    o, s, _ = _setup(S, orc, case, K=(3, 3, 3), upload=False)
    xyz, Ja, sJ, _ = s.metrics()
    U = np.zeros(s.state_shape)
    rho, u, p = 1.0, np.array([0.1, 0.2, -0.1]), 71.43
    U[0], U[1:4] = rho, (rho * u)[:, None, None, None, None]
    U[4] = p / 0.4 + 0.5 * rho * u @ u
    R = s.rhs(s.init_state(U)).cpu().numpy()
    b = orc.basis(case[0], 0)
    Dhat = (b["w"][:, None] / b["w"][None, :]) * b["D"]
    f = np.abs(orc.flux_adv(U[:, 0, 0, 0, 0], np.ones(3))).max() + np.abs(U[:, 0, 0, 0, 0]).max()
    scale = 3 * f * np.abs(Ja).max() * np.abs(Dhat).sum(0).max() * sJ.max()
    _say("fsp", case, np.abs(R).max() / scale)
    assert np.abs(R).max() < 1e-13 * scale
    R2 = s.rhs(s.init_state(I.smooth_random_state(xyz, 57, amp=0.1))).cpu().numpy()
    W = quad_weights3(b["w"]) / sJ
    for v in range(5):
        assert abs((W * R2[v]).sum()) < 1e-13 * (W * np.abs(R2[v])).sum()


def test_tgv_workload_full_size_sampled(S, orc, torch_cuda):
    """NS split form on Gauss nodes, N=3, 16^3 TGV at full size: sampled elements."""
    name = "ns_split_lg_n3_16x16x16_tgv"
    w = I.WORKLOADS[name]
    mesh = I.workload_mesh(name)
    cfg = dict(N=w["N"], nodes=w["nodes"], form=w["form"], physics=w["physics"], mu=w["mu"])
    _say("full size", name)
    o = orc.Oracle(cfg, mesh)
    xyz, J, Ja = o.geometry()
    s = S(cfg, mesh)
    s.upload_metrics(Ja, 1.0 / J, o.face_normals())
    sample = [0, 15, 255, 2047, 4095, 1234, 3000]
    # (a) mild per-node noise (5 % in rho and p): O(1) residual, no cancellation
    U = I.random_state(xyz.shape[1:], 41, rho=(0.95, 1.05), vel=0.1, p=(0.95, 1.05))
    R_gpu = s.rhs(s.init_state(U)).cpu().numpy()[:, sample]
    err = rel_err_per_var(R_gpu, o.rhs_elems(U, sample))
    _say("full size random state", err)
    assert np.all(err < 1e-12), err
    # (b) the Taylor-Green vortex: the residual is a small difference of much
    # larger flux terms, and the projected face states carry the rounding of
    # the inverse entropy map, whose density exp(z - (gamma + ln b)/(gamma-1))
    # (b = rho/p) has an exponent made of terms of size |ln b|/(gamma-1) (about
    # 11 at Ma 0.1): bound 64 eps (1 + |ln b|/(gamma-1)) of the flux-term size
    # plus the 1e-12 relative bound
    U = I.workload_state(name, xyz)
    R_gpu = s.rhs(s.init_state(U)).cpu().numpy()[:, sample]
    R_orc = o.rhs_elems(U, sample)
    b = orc.basis(3, 0)
    fmax = max(np.abs(orc.flux_adv(U[:, e, 0, 0, 0], np.ones(3))).max() for e in sample)
    scale = np.abs(b["DS"]).sum(1).max() * fmax * np.abs(Ja).max() / J.min()
    rho = U[0]
    p = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
    cond = 1.0 + np.abs(np.log(rho / p)).max() / 0.4
    diff = np.abs(R_gpu - R_orc).max(axis=(1, 2, 3, 4))
    _say("full size tgv", "diff", diff, "rel", rel_err_per_var(R_gpu, R_orc), "term scale", scale, "cond", cond)
    assert np.all(diff < 1e-12 * np.abs(R_orc).max(axis=(1, 2, 3, 4)) + 64 * 2.2e-16 * cond * scale)


@pytest.mark.parametrize("case,K", [((3, 1), (1, 1, 1)), ((1, 0), (1, 2, 1)), ((5, 1), (2, 1, 1))], ids=str)
def test_degenerate_meshes_match_oracle(S, orc, case, K):
    """A single periodic element (each face its own element's neighbour) and
    one-element-thick slabs, rotated frames; mild per-node noise (5 %), since
    the entropy projection of unresolved noise is ill-conditioned."""
    N, physics = case
    _say("degenerate", case, K)
    o, s, _ = _setup(S, orc, (N, physics, 0.0, 3), K=K)
    U = I.random_state(s.state_shape[1:], 39, rho=(0.95, 1.05), vel=0.1, p=(0.95, 1.05))
    err = rel_err_per_var(s.rhs(s.init_state(U)).cpu().numpy(), o.rhs(U))
    _say("degenerate", case, K, err)
    assert np.all(err < 1e-12), err
    Ug = s.init_state(U)
    s.rk_step(Ug, s.empty_state(), 1e-3, 0)
    assert np.array_equal(Ug.cpu().numpy(), U)
