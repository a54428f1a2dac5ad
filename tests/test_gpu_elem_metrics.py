"""Per-element metric terms (dg_set_element_metrics) on the GPU.

An affine element's metric terms are constant; the mesh set-up makes them
exactly constant (node mean, when they agree to 1e-12), and the kernels of
such an element then read one copy per element instead of the node arrays.
The values are the same, so Euler residuals, RK steps and the adjoint must be
bitwise equal with the per-element copy on and off.  The lifting of such an
element forms its gradient as Ja^r (Dhat q) instead of Dhat (Ja^r q), equal
in exact arithmetic for constant Ja: Navier-Stokes results agree to rounding
(1e-12 of each output's largest entry).  On curved elements nothing changes
(no element qualifies).
"""
import sys

import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I

pytestmark = pytest.mark.gpu
PI = np.pi


def _say(*a):
    print("[gpu-elem-metrics]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2605_28627_amd.solver import DGSolver
    return DGSolver


CASES = [
    # N, nodes, form, physics, K, curved amplitude, rotation seed
    (3, 0, 0, 0, (3, 4, 5), 0.0, None),    # weak form, Euler, Gauss nodes
    (7, 1, 1, 1, (3, 3, 2), 0.0, None),    # split form, Navier-Stokes, LGL (the benchmark kernels)
    (5, 1, 1, 1, (3, 2, 2), 0.0, 11),      # rotated box: full constant metric matrix
    (3, 0, 1, 1, (3, 3, 3), 0.0, 7),       # entropy-stable split form on Gauss nodes
    (4, 1, 0, 1, (2, 3, 2), 0.0, None),    # weak form, Navier-Stokes, LGL
    (5, 1, 1, 1, (3, 2, 2), 0.1, 11),      # curved: no element qualifies
]


def _run(s, U0, dt):
    import torch
    out = {}
    U = s.init_state(U0)
    out["rhs"] = s.rhs(U).cpu().numpy()
    if s.cfg["physics"] == 1:
        out["lift"] = s.lift(U).cpu().numpy()
    lam = s.to_device(np.cos(np.arange(U0.size) * 0.37).reshape(U0.shape))
    out["adjoint_rhs"] = s.adjoint_rhs(U, lam).cpu().numpy()
    Uw = U.clone()
    dU = torch.zeros_like(Uw)
    s.rk_step(Uw, dU, dt, 2)
    out["rk"] = Uw.cpu().numpy()
    lamU, lamdU = lam.clone(), torch.empty_like(lam)
    s.adjoint_rk_step(U, lamU, lamdU, dt)
    out["adjoint_rk"] = lamU.cpu().numpy()
    return out


@pytest.mark.parametrize("case", CASES)
def test_element_metrics_bitwise_equal(S, case):
    N, nodes, form, physics, K, curved, rot = case
    _say("case", case)
    mesh = I.box_mesh(K, (-PI,) * 3, (PI,) * 3, Ngeo=N if curved else 1, curved_amp=curved, rotate_seed=rot)
    cfg = dict(N=N, nodes=nodes, form=form, physics=physics, mu=1e-2 if physics else 0.0)
    s = S(cfg, mesh, "cuda:0", adjoint=True)
    try:
        n_el = s.element_metric_count()
        if curved:
            assert n_el < mesh.nElems
        else:
            assert n_el == mesh.nElems
        U0 = I.smooth_random_state(s.coords(), 17, amp=0.2)
        dt = 0.2 * s.timestep(s.init_state(U0), 0.9)
        on = _run(s, U0, dt)
        s.set_element_metrics(False)
        assert s.element_metric_count() == 0
        off = _run(s, U0, dt)
        s.set_element_metrics(True)
        assert s.element_metric_count() == n_el
        again = _run(s, U0, dt)
    finally:
        s.close()
    for k in on:
        if physics == 0 or curved:
            assert np.array_equal(on[k], off[k]), (k, np.abs(on[k] - off[k]).max())
        else:
            diff, ref = np.abs(on[k] - off[k]).max(), np.abs(off[k]).max()
            _say(k, "max |diff|", diff, "of", ref)
            assert diff <= 1e-12 * ref, (k, diff, ref)
        assert np.array_equal(on[k], again[k]), k
        assert np.isfinite(on[k]).all(), k


def test_uploaded_metrics_are_examined_again(S):
    """dg_upload_metrics replaces the terms: an element qualifies only if its
    new terms are bitwise constant; per-node noise sends it to the node arrays."""
    N = 3
    mesh = I.box_mesh((2, 2, 3), (-PI,) * 3, (PI,) * 3)
    cfg = dict(N=N, nodes=0, form=0, physics=0, mu=0.0)
    s = S(cfg, mesh, "cuda:0")
    try:
        assert s.element_metric_count() == mesh.nElems
        _, Ja, sJ, nv = s.metrics()
        U = s.init_state(I.smooth_random_state(s.coords(), 5, amp=0.2))
        R0 = s.rhs(U).cpu().numpy()
        Ja2 = Ja.copy()
        Ja2[0, 1, 0, 0, 0] *= 1.0 + 1e-15          # one node of element 1 no longer equal
        s.upload_metrics(Ja2, sJ, nv)
        assert s.element_metric_count() == mesh.nElems - 1
        s.upload_metrics(Ja, sJ, nv)
        assert s.element_metric_count() == mesh.nElems
        R1 = s.rhs(U).cpu().numpy()
    finally:
        s.close()
    assert np.array_equal(R0, R1)
