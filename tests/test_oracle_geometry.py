"""Pins of the oracle's geometry: node coordinates, Jacobians, metric terms.

* affine boxes: coordinates, J and Ja have closed forms;
* sum of w J is the domain volume (exact on affine meshes, spectrally
  accurate on the curved mesh whose boundary is the undeformed box);
* the conservative curl form equals the cross-product (cofactor) form
  J dxi_r/dx_n wherever the collocated product is exact (N >= 2 Ngeo);
* discrete metric identities sum_r D_r Ja^r = 0 on curved, rotated meshes;
* master face normals are outward and equal to the extrapolated volume
  metrics; a folded element is rejected.
"""
import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from tests.helpers import quad_weights3


def test_affine_box_closed_forms(orc):
    N = 4
    lo, hi, K = (0.5, -1.0, 2.0), (2.5, 0.0, 5.0), (2, 3, 4)
    mesh = I.box_mesh(K, lo, hi, Ngeo=1)
    o = orc.Oracle(dict(N=N, nodes=1), mesh)
    xyz, J, Ja = o.geometry()
    x = orc.basis(N, 1)["x"]
    h = [(hi[d] - lo[d]) / K[d] for d in range(3)]
    half = np.array(h) / 2
    assert np.allclose(J, np.prod(half), rtol=1e-14, atol=0)
    for r in range(3):
        for n in range(3):
            want = np.prod(half) / half[r] if r == n else 0.0
            assert np.abs(Ja[3 * r + n] - want).max() < 1e-14
    e = (1 * K[1] + 2) * K[0] + 1      # kx=1, ky=2, kz=1
    ex = lo[0] + (1 + (x + 1) / 2) * h[0]
    assert np.allclose(xyz[0, e, 0, 0, :], ex, atol=1e-14, rtol=0)
    ey = lo[1] + (2 + (x + 1) / 2) * h[1]
    assert np.allclose(xyz[1, e, 0, :, 0], ey, atol=1e-14, rtol=0)


@pytest.mark.parametrize("nodes", [0, 1])
def test_volume(orc, nodes):
    N = 5
    W = quad_weights3(orc.basis(N, nodes)["w"])
    aff = orc.Oracle(dict(N=N, nodes=nodes), I.box_mesh((3, 2, 2), (0, 0, 0), (1.5, 2.0, 0.5)))
    _, J, _ = aff.geometry()
    assert abs((W * J).sum() - 1.5) < 1e-13
    vols = []
    for N2 in (4, 6, 8):
        W2 = quad_weights3(orc.basis(N2, 1)["w"])
        cur = orc.Oracle(dict(N=N2, nodes=1), I.box_mesh((3, 3, 3), (-np.pi,) * 3, (np.pi,) * 3,
                                                        Ngeo=N2, curved_amp=0.1))
        _, J2, _ = cur.geometry()
        assert J2.min() > 0
        vols.append(abs((W2 * J2).sum() - 8 * np.pi ** 3) / (8 * np.pi ** 3))
    # the elements tile the undeformed box (planar outer faces); the odd symmetry
    # of the displacement cancels the quadrature error of sum w J
    assert max(vols) < 1e-13


def _cofactor_metrics(orc, N, xyz):
    """J dxi_r/dx_n from the cross products of the covariant vectors (textbook form)."""
    D = orc.basis(N, 1)["D"]
    dX = np.zeros((3, 3) + xyz.shape[1:])           # dX[d][r]
    for d in range(3):
        f = xyz[d]
        dX[d, 0] = np.einsum("il,eKJl->eKJi", D, f)
        dX[d, 1] = np.einsum("jl,eKlI->eKjI", D, f)
        dX[d, 2] = np.einsum("kl,elJI->ekJI", D, f)
    a = [dX[:, r] for r in range(3)]                 # covariant vectors a_r = dX/dxi_r
    Ja = np.zeros((9,) + xyz.shape[1:])
    for r in range(3):
        c = np.cross(a[(r + 1) % 3], a[(r + 2) % 3], axis=0)
        for n in range(3):
            Ja[3 * r + n] = c[n]
    return Ja


def test_curl_form_equals_cross_product_when_exact(orc):
    N, Ngeo = 6, 2
    mesh = I.box_mesh((2, 2, 2), (-np.pi,) * 3, (np.pi,) * 3, Ngeo=Ngeo, curved_amp=0.1, rotate_seed=3)
    o = orc.Oracle(dict(N=N, nodes=1), mesh)
    xyz, J, Ja = o.geometry()
    Jc = _cofactor_metrics(orc, N, xyz)
    assert np.abs(Ja - Jc).max() < 1e-12 * np.abs(Jc).max()
    # J = a_1 . (a_2 x a_3) = first row contraction
    assert J.min() > 0


@pytest.mark.parametrize("nodes", [0, 1])
def test_discrete_metric_identities(orc, nodes):
    N = 5
    mesh = I.box_mesh((2, 3, 2), (-np.pi,) * 3, (np.pi,) * 3, Ngeo=N, curved_amp=0.1, rotate_seed=11)
    o = orc.Oracle(dict(N=N, nodes=nodes), mesh)
    _, _, Ja = o.geometry()
    D = orc.basis(N, nodes)["D"]
    for n in range(3):
        div = (np.einsum("il,eKJl->eKJi", D, Ja[0 + n]) + np.einsum("jl,eKlI->eKjI", D, Ja[3 + n]) +
               np.einsum("kl,elJI->ekJI", D, Ja[6 + n]))
        scale = np.abs(D).max() * np.abs(Ja).max()
        assert np.abs(div).max() < 1e-14 * scale


def test_face_normals_outward_and_consistent(orc):
    N = 4
    mesh = I.box_mesh((3, 3, 3), (-np.pi,) * 3, (np.pi,) * 3, Ngeo=N, curved_amp=0.1, rotate_seed=5)
    o = orc.Oracle(dict(N=N, nodes=1), mesh)
    xyz, J, Ja = o.geometry()
    nv = o.face_normals()
    n1 = N + 1
    for s in range(mesh.nSides):
        for m in range(2):
            e, f = mesh.sideElem[2 * s + m], mesh.sideLoc[2 * s + m]
            d = f // 2
            # centre of the element and of the face
            c_el = xyz[:, e].reshape(3, -1).mean(1)
            sl = [slice(None)] * 3
            sl[2 - d] = N if f % 2 else 0                  # arrays are [k][j][i]
            fx = xyz[(slice(None), e) + tuple(sl)]
            c_face = fx.reshape(3, -1).mean(1)
            if m == 0:
                # master: outward means pointing from element centre to face centre
                nm = nv[:, s].reshape(3, -1).mean(1)
                assert nm @ (c_face - c_el) > 0
                # equals +-Ja^d at the boundary nodes, in face-local (p, q) order
                jad = Ja[3 * d:3 * d + 3, e][(slice(None),) + tuple(sl)]
                sg = 1.0 if f % 2 else -1.0
                # [k][j][i] slice with d removed -> (q, p) order already
                assert np.allclose(nv[:, s], sg * jad, rtol=0, atol=1e-13)
    assert n1 == N + 1


def test_folded_element_rejected(orc):
    mesh = I.box_mesh((2, 2, 2), (0, 0, 0), (1, 1, 1), Ngeo=1)
    X = mesh.X.copy()
    X[0, 3] = X[0, 3][:, :, ::-1]                          # mirror one element in x
    mesh.X = X
    o = orc.Oracle(dict(N=2, nodes=1), mesh)
    with pytest.raises(ValueError):
        o.check_jacobians()
