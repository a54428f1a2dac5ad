"""dg_rk_step_noalloc (static device scratch, no workspace bound) against
dg_rk_step (caller-bound workspace) through the C-ABI: the same steps on the
same seeded inputs give the same states, on two calls in a row, the second
with a smaller mesh; a mesh whose scratch exceeds the static array is
refused."""
import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I

pytestmark = pytest.mark.gpu
PI = np.pi


def _run_pair(cfg, mesh, seed, nsteps):
    import torch
    from paper_2605_28627_amd import dgx
    from paper_2605_28627_amd.solver import DGSolver, config_from_dict
    ref = DGSolver(cfg, mesh, "cuda:0")
    U0 = I.smooth_random_state(ref.coords(), seed, amp=0.2)
    Ua = ref.init_state(U0)
    dUa = torch.empty_like(Ua)
    dt = ref.timestep(Ua, 0.9)
    ref.rk_step(Ua, dUa, dt, nsteps)
    # a context with no workspace bound at all
    ctx = dgx.dg_create(config_from_dict(cfg))
    try:
        with torch.cuda.device(0):
            dgx.dg_upload_mesh(ctx, mesh)
        Ub = torch.from_numpy(U0).to("cuda:0").reshape(Ua.shape).contiguous()
        dUb = torch.full_like(Ub, 7.0)          # not zero: the call zeroes it
        dgx.dg_rk_step_noalloc(ctx, Ub, dUb, 0.0, dt, nsteps)
        torch.cuda.synchronize()
    finally:
        dgx.dg_destroy(ctx)
    a, b = Ua.cpu().numpy(), Ub.cpu().numpy()
    ref.close()
    err = np.abs(a - b).max() / np.abs(a - U0).max()
    return err, np.array_equal(a, b)


def test_noalloc_matches_workspace_path_two_calls():
    big = I.box_mesh((3, 2, 2), (-PI,) * 3, (PI,) * 3, Ngeo=3, curved_amp=0.1, rotate_seed=5)
    err, same = _run_pair(dict(N=3, nodes=1, form=1, physics=1, mu=0.02), big, 71, 3)
    assert err < 1e-12 and same, err
    small = I.box_mesh((2, 1, 2), (-PI,) * 3, (PI,) * 3, rotate_seed=2)
    err, same = _run_pair(dict(N=2, nodes=0, form=0, physics=0), small, 72, 2)
    assert err < 1e-12 and same, err


def test_noalloc_refuses_meshes_beyond_the_static_scratch():
    import torch
    from paper_2605_28627_amd import dgx
    from paper_2605_28627_amd.solver import config_from_dict
    cfg = dict(N=7, nodes=1, form=1, physics=1, mu=1.0 / 1600.0)
    mesh = I.box_mesh((16, 16, 16), (-PI,) * 3, (PI,) * 3)
    ctx = dgx.dg_create(config_from_dict(cfg))
    try:
        with torch.cuda.device(0):
            dgx.dg_upload_mesh(ctx, mesh)
        assert dgx.dg_workspace_bytes(ctx) > 256 << 20
        n = dgx.dg_sizes(ctx)[3]
        U = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dU = torch.zeros_like(U)
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_rk_step_noalloc(ctx, U, dU, 0.0, 1e-4, 1)
        assert ei.value.status == dgx.DG_ERR_ARG
        assert "static" in str(ei.value)
    finally:
        dgx.dg_destroy(ctx)
