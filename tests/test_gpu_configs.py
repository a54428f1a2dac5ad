"""Every workload configuration at its full size on the GPU against the oracle.

For each configuration the residual of its initial state is evaluated by the
FP64 path and by the FP32-flux path, with the oracle's metrics uploaded so
that both sides use the same geometry, on sampled elements (all elements for
the small meshes):

* FP64: per variable within 1e-12 of the largest oracle entry plus 64 eps of
  the size of the flux terms the residual is made of (on fine meshes a
  smooth state's residual is a small difference of much larger terms);
* FP32 flux: the relative L2 error per variable against the oracle is
  reported (one JSON line per configuration, prefixed "RESULT"), with a loose
  bound that catches a broken mixed path.

A second test runs each configuration with the library's own metrics (host
curl-form metrics, no upload): the oracle computes its geometry for the
sampled elements only.  The two codes round the metric terms independently
(relative differences of about 1e-13), and a Ma 0.1 residual is a small
difference of O(p0) flux terms, so the bound adds the measured metric
difference times the size of those terms.  The 64^3, N=7
configuration (134 M nodes, 5.4 GB per state) is part of both.
"""
import json
import sys

import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I

pytestmark = pytest.mark.gpu

CONFIGS = [
    "euler_weak_lg_n3_4x4x4",
    "euler_weak_lg_n3_64x64x64",
    "ns_split_lgl_n7_16x16x16_tgv",
    "ns_split_lgl_n5_32x32x32_curved_tgv",
    "euler_split_lgl_n5_8x8x8_tgv",
    "ns_split_lgl_n7_64x64x64_tgv",
]


def _say(*a):
    print("[gpu-configs]", *a, flush=True)
    sys.stdout.flush()


def _sample(nE, K, seed=7):
    if nE <= 512:
        return list(range(nE))
    k0, k1, k2 = K
    corners = [0, k0 - 1, k0 * k1 - 1, nE - 1, (k2 // 2) * k0 * k1 + (k1 // 2) * k0 + k0 // 2]
    rng = np.random.default_rng(seed)
    extra = sorted(set(int(x) for x in rng.integers(0, nE, 6)) - set(corners))
    return corners + extra


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2605_28627_amd.solver import DGSolver
    return DGSolver


def _flux_scale(orc, w, U, el, Ja, J):
    """Size of the terms a residual entry is summed from: the largest row sum of
    the volume operator times the largest flux over the sampled elements' first
    nodes, times the largest metric entry over the smallest Jacobian."""
    b = orc.basis(w["N"], w["nodes"])
    # weak-form operator Dhat[a][l] = (w_l / w_a) D[l][a]; split operator D^S
    D = b["DS"] if w["form"] == 1 else (b["w"][None, :] / b["w"][:, None]) * b["D"].T
    fmax = max(np.abs(orc.flux_adv(U[:, e].reshape(5, -1)[:, 0], np.ones(3))).max() for e in el)
    return np.abs(D).sum(1).max() * fmax * np.abs(Ja).max() / J.min()


@pytest.mark.parametrize("name", CONFIGS)
def test_config_fp64_parity_and_fp32_error(S, orc, name):
    import torch
    w = I.WORKLOADS[name]
    cfg = dict(N=w["N"], nodes=w["nodes"], form=w["form"], physics=w["physics"], mu=w["mu"])
    _say(name, "mesh")
    mesh = I.workload_mesh(name)
    _say(name, "oracle geometry,", mesh.nElems, "elements")
    o = orc.Oracle(cfg, mesh)
    xyz, J, Ja = o.geometry()
    nv = o.face_normals()
    U = I.workload_state(name, xyz)
    el = _sample(mesh.nElems, w["K"])
    _say(name, "oracle residual of", len(el), "elements")
    R_orc = o.rhs_sample(U, el)
    del o
    scale = _flux_scale(orc, w, U, el, Ja, J)
    out = {"config": name, "dof": int(mesh.nElems * (w["N"] + 1) ** 3), "sampled_elements": len(el)}
    # FP64; the FP32-flux mode with plain float flux arithmetic; and with the
    # workload's reference state (float rounds deviations from it)
    for prec, refstate in ((0, False), (1, False), (1, True)):
        _say(name, "GPU precision", prec, "reference state" if refstate else "")
        s = S(dict(cfg, precision=prec), mesh)
        s.upload_metrics(Ja, 1.0 / J, nv)
        if refstate:
            s.set_reference_state(*I.workload_reference(name))
        Ug = s.init_state(U)
        R = s.rhs(Ug)
        R_gpu = R[:, torch.as_tensor(el, device=R.device)].cpu().numpy()
        del R, Ug
        s.close()
        diff = np.abs(R_gpu - R_orc).max(axis=(1, 2, 3, 4))
        ref = np.abs(R_orc).max(axis=(1, 2, 3, 4))
        l2 = [float(np.linalg.norm(R_gpu[v] - R_orc[v]) / max(np.linalg.norm(R_orc[v]), 1e-300)) for v in range(5)]
        if prec == 0:
            out["fp64_max_abs_diff_per_var"] = diff.tolist()
            out["fp64_rel_l2_per_var"] = l2
            assert np.all(diff < 1e-12 * ref + 64 * 2.2e-16 * scale), (diff, ref, scale)
        elif not refstate:
            out["fp32_flux_rel_l2_per_var"] = l2
            assert max(l2) < 5e-2, l2
        else:
            out["fp32_flux_reference_state_rel_l2_per_var"] = l2
            assert max(l2) < 1e-3, l2
    _say("RESULT", json.dumps(out))


@pytest.mark.parametrize("name", CONFIGS)
def test_config_library_metrics_sampled(S, orc, name):
    """Full size with the library's own metrics: sampled elements against the oracle."""
    import torch
    w = I.WORKLOADS[name]
    cfg = dict(N=w["N"], nodes=w["nodes"], form=w["form"], physics=w["physics"], mu=w["mu"])
    _say(name, "library metrics: mesh and GPU set-up")
    mesh = I.workload_mesh(name)
    s = S(cfg, mesh)
    xyz = s.coords()
    U = I.workload_state(name, xyz)
    Ug = s.init_state(U)
    R = s.rhs(Ug)
    el = _sample(mesh.nElems, w["K"])
    R_gpu = R[:, torch.as_tensor(el, device=R.device)].cpu().numpy()
    del R, Ug
    _, Ja_lib, sJ_lib, _ = s.metrics()
    Ja_s, J_s = Ja_lib[:, el], 1.0 / sJ_lib[el]
    s.close()
    del Ja_lib, sJ_lib
    _say(name, "oracle residual of", len(el), "elements (oracle geometry of those elements)")
    o = orc.Oracle(cfg, mesh)
    _, J_o, Ja_o = o.geometry_sample(el)
    R_orc = o.rhs_sample(U, el)
    scale = _flux_scale(orc, w, U, el, Ja_s, J_s)
    # the two codes round the metric terms independently; the residual moves by
    # the metric change times the flux terms (volume and surface term, 1/J)
    metric_rel = max(np.abs(Ja_s - Ja_o).max() / np.abs(Ja_o).max(), np.abs(J_s - J_o).max() / np.abs(J_o).max())
    diff = np.abs(R_gpu - R_orc).max(axis=(1, 2, 3, 4))
    ref = np.abs(R_orc).max(axis=(1, 2, 3, 4))
    bound = 1e-12 * ref + (64 * 2.2e-16 + 4 * metric_rel) * scale
    _say("RESULT", json.dumps({"config": name, "library_metrics": True, "sampled_elements": len(el),
                               "metric_rel_diff": float(metric_rel), "flux_scale": float(scale),
                               "fp64_max_abs_diff_per_var": diff.tolist(),
                               "diff_over_metric_scale": (diff / (metric_rel * scale)).tolist(),
                               "bound_per_var": bound.tolist()}))
    assert np.all(diff < bound), (diff, ref, scale, metric_rel)
