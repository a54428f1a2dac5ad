"""CPU tests of the C-ABI library: it loads, exports every symbol declared in
include/dgx.h, validates its arguments, and its host-side mesh set-up
(connectivity, geometry, metric terms, face normals) agrees with the oracle.
No call here launches device work.
"""
import os
import re

import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PI = np.pi


@pytest.fixture(scope="module")
def dgx():
    lib = os.path.join(ROOT, "paper_2605_28627_amd", "libdgx.so")
    if not os.path.exists(lib):
        from paper_2605_28627_amd import build
        build.build()
    from paper_2605_28627_amd import dgx as m
    return m


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "dgx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(dgx):
    declared = _header_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(dgx.lib(), name), name
    assert sorted(dgx.SYMBOLS) == declared


def test_create_validates_config(dgx):
    ok = dgx.make_config(3)
    ctx = dgx.dg_create(ok)
    dgx.dg_destroy(ctx)
    bad = [dict(nodes=2), dict(volume_form=3), dict(physics=-1), dict(precision=2), dict(gamma=1.0),
           dict(mu=-1.0), dict(Pr=0.0), dict(R=0.0), dict(gamma=float("nan"))]
    for kw in bad:
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_create(dgx.make_config(3, **kw))
        assert ei.value.status == dgx.DG_ERR_ARG, kw
    for kw in [dict(N=0), dict(N=8)]:
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_create(dgx.make_config(**({"N": 3} | kw)))
        assert ei.value.status == dgx.DG_ERR_UNSUPPORTED, kw
    # the split form runs on both node sets (entropy-stable hybridised form on Gauss nodes)
    for nodes in (0, 1):
        dgx.dg_destroy(dgx.dg_create(dgx.make_config(3, nodes=nodes, volume_form=1)))
    # FV sub-cells: FP64, Rusanov, any DG form; Euler or Navier-Stokes with
    # constant viscosity
    for kw in [dict(nodes=0), dict(nodes=1), dict(nodes=1, volume_form=1), dict(nodes=0, volume_form=1),
               dict(physics=1, mu=0.01), dict(physics=1, mu=0.01, nodes=1, volume_form=1),
               dict(physics=1, mu=0.01, nodes=0, volume_form=1)]:
        dgx.dg_destroy(dgx.dg_create(dgx.make_config(3, fv=1, **kw)))
    for kw in [dict(precision=1), dict(riemann=2), dict(physics=1, mu=0.01, viscosity=1, Tref=1.0, Ts=0.4)]:
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_create(dgx.make_config(3, fv=1, **kw))
        assert ei.value.status == dgx.DG_ERR_UNSUPPORTED, kw
    with pytest.raises(dgx.DGError) as ei:
        dgx.dg_create(dgx.make_config(3, fv=2))
    assert ei.value.status == dgx.DG_ERR_ARG


def test_lserk_coefficients_match_oracle(dgx, orc):
    A, B, C = dgx.dg_lserk_coefficients()
    Ao, Bo, Co = orc.lserk_coeffs()
    assert np.array_equal(A, Ao) and np.array_equal(B, Bo) and np.array_equal(C, Co)


@pytest.mark.parametrize("integrator", [0, 1])
def test_rk_coefficients_match_oracle(dgx, orc, integrator):
    """The library's tables equal the oracle's (pinned there by the order conditions)."""
    got = dgx.dg_rk_coefficients(integrator)
    want = orc.rk_coeffs(integrator)
    assert len(got[0]) == (5, 14)[integrator]
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    with pytest.raises(dgx.DGError) as ei:
        dgx.dg_rk_coefficients(7)
    assert ei.value.status == dgx.DG_ERR_ARG
    with pytest.raises(dgx.DGError) as ei:
        dgx.dg_create(dgx.make_config(3, integrator=2))
    assert ei.value.status == dgx.DG_ERR_ARG


@pytest.mark.parametrize("N,nodes,curved,rot", [(3, 0, 0.0, None), (5, 1, 0.1, 7), (7, 1, 0.1, 3), (4, 0, 0.0, 9)])
def test_host_metrics_match_oracle(dgx, orc, N, nodes, curved, rot):
    mesh = I.box_mesh((3, 2, 2), (-PI,) * 3, (PI,) * 3, Ngeo=N if curved else 1, curved_amp=curved, rotate_seed=rot)
    ctx = dgx.dg_create(dgx.make_config(N, nodes=nodes))
    try:
        dgx.dg_set_mesh(ctx, mesh)
        xyz, Ja, sJ, nv = dgx.dg_get_metrics(ctx)
    finally:
        dgx.dg_destroy(ctx)
    o = orc.Oracle(dict(N=N, nodes=nodes), mesh)
    xo, Jo, Jao = o.geometry()
    nvo = o.face_normals()
    assert np.abs(xyz - xo).max() < 1e-14 * np.abs(xo).max() + 1e-15
    assert np.abs(1.0 / sJ - Jo).max() < 1e-12 * np.abs(Jo).max()
    # curl-form rounding grows like |D|^2 eps: allow 1e-12 of the largest entry
    assert np.abs(Ja - Jao).max() < 1e-12 * np.abs(Jao).max()
    assert np.abs(nv - nvo).max() < 1e-12 * np.abs(nvo).max()


def test_set_mesh_rejects_bad_meshes(dgx):
    ctx = dgx.dg_create(dgx.make_config(2))
    try:
        mesh = I.box_mesh((2, 2, 2), (0,) * 3, (1,) * 3)
        X = mesh.X.copy()
        X[0, 3] = X[0, 3][:, :, ::-1]                      # fold one element
        folded = I.Mesh(mesh.nElems, mesh.Ngeo, X, mesh.sideElem, mesh.sideLoc, mesh.sideOrient)
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_set_mesh(ctx, folded)
        assert ei.value.status == dgx.DG_ERR_MESH and "Jacobian" in str(ei.value)
        se = mesh.sideElem.copy()
        se[1] = se[3]                                      # one face used twice, another left open
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_set_mesh(ctx, I.Mesh(mesh.nElems, mesh.Ngeo, mesh.X, se, mesh.sideLoc, mesh.sideOrient))
        assert ei.value.status == dgx.DG_ERR_MESH
        so = mesh.sideOrient.copy()
        so[0] = 9
        with pytest.raises(dgx.DGError) as ei:
            dgx.dg_set_mesh(ctx, I.Mesh(mesh.nElems, mesh.Ngeo, mesh.X, mesh.sideElem, mesh.sideLoc, so))
        assert ei.value.status == dgx.DG_ERR_MESH
        import ctypes
        L = dgx.lib()
        z = np.zeros(3 * 8)
        zi = np.zeros(6, dtype=np.int32)
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        assert L.dg_set_mesh(ctx, 0, 1, z.ctypes.data_as(dp), 0, zi.ctypes.data_as(ip), zi.ctypes.data_as(ip),
                             zi.ctypes.data_as(ip)) == dgx.DG_ERR_ARG          # empty mesh
        dgx.dg_set_mesh(ctx, mesh)                         # and a good mesh still works afterwards
        assert dgx.dg_workspace_bytes(ctx) > 0
    finally:
        dgx.dg_destroy(ctx)


def test_hot_path_calls_need_a_device_mesh(dgx):
    """Call-order errors are reported before any device work is attempted."""
    import ctypes
    ctx = dgx.dg_create(dgx.make_config(3))
    try:
        L = dgx.lib()
        p = ctypes.c_void_p(0x1000)
        assert L.dg_rhs(ctx, p, p, 0.0, None) == dgx.DG_ERR_STATE
        assert L.dg_rk_step(ctx, p, p, 0.0, 0.1, 1, None) == dgx.DG_ERR_STATE
        assert L.dg_upload_metrics(ctx, None, None, None) == dgx.DG_ERR_STATE
        assert "no mesh" in dgx.dg_last_error(ctx)
        assert L.dg_bind_workspace(ctx, p, 10) == dgx.DG_ERR_STATE
        dgx.dg_set_mesh(ctx, I.box_mesh((2, 2, 2)))
        assert L.dg_bind_workspace(ctx, ctypes.c_void_p(0x1001), 1 << 30) == dgx.DG_ERR_ARG   # misaligned
        assert L.dg_bind_workspace(ctx, p, 16) == dgx.DG_ERR_ARG                             # too small
        assert L.dg_rhs(None, p, p, 0.0, None) == dgx.DG_ERR_ARG
    finally:
        dgx.dg_destroy(ctx)


@pytest.mark.parametrize("N,nodes,rot", [(3, 0, None), (7, 1, None), (5, 1, 11)])
def test_affine_metrics_snapped_constant(dgx, orc, N, nodes, rot):
    """dg_set_mesh gives every element of an affine mesh (a box, also rotated)
    metric terms that are exactly constant over its nodes (their node mean),
    within the curl form's rounding of the oracle's; curved elements keep
    their node values."""
    mesh = I.box_mesh((3, 2, 2), (-PI,) * 3, (PI,) * 3, rotate_seed=rot)
    ctx = dgx.dg_create(dgx.make_config(N, nodes=nodes))
    try:
        dgx.dg_set_mesh(ctx, mesh)
        _, Ja, sJ, _ = dgx.dg_get_metrics(ctx)
    finally:
        dgx.dg_destroy(ctx)
    nE = Ja.shape[1]
    Jr, s = Ja.reshape(9, nE, -1), sJ.reshape(nE, -1)
    assert (Jr == Jr[:, :, :1]).all() and (s == s[:, :1]).all()
    _, Jo, Jao = orc.Oracle(dict(N=N, nodes=nodes), mesh).geometry()
    assert np.abs(Ja - Jao).max() < 1e-12 * np.abs(Jao).max()
    assert np.abs(1.0 / sJ - Jo).max() < 1e-12 * np.abs(Jo).max()
    curved = I.box_mesh((2, 2, 2), (-PI,) * 3, (PI,) * 3, Ngeo=N, curved_amp=0.1, rotate_seed=rot)
    ctx = dgx.dg_create(dgx.make_config(N, nodes=nodes))
    try:
        dgx.dg_set_mesh(ctx, curved)
        _, Jc, _, _ = dgx.dg_get_metrics(ctx)
    finally:
        dgx.dg_destroy(ctx)
    Jc = Jc.reshape(9, curved.nElems, -1)
    assert not (Jc == Jc[:, :, :1]).all(axis=(0, 2)).any()
