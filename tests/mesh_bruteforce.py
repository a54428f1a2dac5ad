"""Element-by-element construction of the periodic box meshes, for checking
the whole-array builder in paper_2605_28627_amd.inputs.box_mesh on small
boxes.  Same conventions and the same random draws (PCG64(rotate_seed):
nElems rotation indices, then nSides master bits); every element, side and
node is handled in its own loop iteration, with the rotations applied to
reference points one at a time.
"""
import numpy as np

from paper_2605_28627_amd import inputs as I


def box_mesh_loops(K, lo, hi, Ngeo=1, curved_amp=0.0, rotate_seed=None):
    Kx, Ky, Kz = (int(k) for k in K)
    nE = Kx * Ky * Kz
    g1 = Ngeo + 1
    h = [(hi[d] - lo[d]) / K[d] for d in range(3)]
    X = np.empty((3, nE, g1, g1, g1))
    for kz in range(Kz):
        for ky in range(Ky):
            for kx in range(Kx):
                e = (kz * Ky + ky) * Kx + kx
                for c in range(g1):
                    for b in range(g1):
                        for a in range(g1):
                            x = lo[0] + (kx + a / Ngeo) * h[0]
                            y = lo[1] + (ky + b / Ngeo) * h[1]
                            z = lo[2] + (kz + c / Ngeo) * h[2]
                            bump = curved_amp * np.sin(x) * np.sin(y) * np.sin(z) if curved_amp else 0.0
                            X[:, e, c, b, a] = (x + bump, y + bump, z + bump)
    rots = [np.eye(3, dtype=np.int64)] * nE
    masters = None
    if rotate_seed is not None:
        rng = np.random.Generator(np.random.PCG64(rotate_seed))
        rots = [I._ROT[r] for r in rng.integers(0, 24, size=nE)]
        masters = rng.integers(0, 2, size=3 * nE)
        Xr = np.empty_like(X)
        for e in range(nE):
            P = rots[e]
            for cn in range(g1):
                for bn in range(g1):
                    for an in range(g1):
                        # reference point of the new frame, in the undisplaced frame: xi_old = P xi_new
                        xn = np.array([an, bn, cn]) * 2 - Ngeo
                        xo = P @ xn
                        ao, bo, co = ((xo + Ngeo) // 2).astype(int)
                        Xr[:, e, cn, bn, an] = X[:, e, co, bo, ao]
        X = Xr
    sideElem, sideLoc, sideOrient = [], [], []
    for kz in range(Kz):
        for ky in range(Ky):
            for kx in range(Kx):
                e = (kz * Ky + ky) * Kx + kx
                for d in range(3):
                    kk = [kx, ky, kz]
                    kk[d] = (kk[d] + 1) % K[d]
                    en = (kk[2] * Ky + kk[1]) * Kx + kk[0]
                    PE, PN = rots[e], rots[en]
                    up = [0, 0, 0]
                    up[d] = 1
                    dn = [0, 0, 0]
                    dn[d] = -1
                    fe = I._face_of(PE.T @ np.array(up))
                    fn = I._face_of(PN.T @ np.array(dn))
                    m_is_e = True if masters is None else bool(masters[3 * e + d])
                    (mE, mF, mP), (sE, sF, sP) = (((e, fe, PE), (en, fn, PN)) if m_is_e
                                                  else ((en, fn, PN), (e, fe, PE)))
                    sideElem += [mE, sE]
                    sideLoc += [mF, sF]
                    sideOrient.append(I._side_orientation(mP, mF, sP, sF, d))
    return X, np.array(sideElem), np.array(sideLoc), np.array(sideOrient)
