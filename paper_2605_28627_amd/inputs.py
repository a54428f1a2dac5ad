"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the DG method itself.  It produces:

* hexahedral meshes in unstructured form: equispaced geometry nodes per
  element plus side connectivity (master/slave element, local face,
  orientation), optionally with the curved displacement of the curved-mesh
  workload and with every element's local frame turned by a random proper
  cube rotation (to exercise general connectivity);
* analytic initial conditions evaluated at caller-supplied node coordinates:
  the Taylor-Green vortex (paper, TGV section, eq. tgv_ic), the advected
  density wave, the manufactured solution of the convergence section;
* seeded random states and seeded velocity noise (numpy PCG64).

Conventions (shared by every consumer, stated once here):

* state arrays are ``U[v][e][k][j][i]`` with ``v`` in (rho, rho u, rho v,
  rho w, rho e) and ``i`` fastest;
* geometry arrays are ``X[d][e][c][b][a]`` on the equispaced nodes
  ``-1 + 2 a / Ngeo``;
* local face ``f``: ``f // 2`` is the reference direction of its normal,
  ``f % 2 == 1`` the ``+1`` end; face-local indices ``(p, q)`` are the two
  tangential volume indices in increasing direction order;
* orientation ``o`` maps the master's ``(p, q)`` to the slave's ``(p', q')``:
  swap if ``o & 4``, then reverse the first index if ``o & 1`` and the second
  if ``o & 2``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------


@dataclass
class Mesh:
    nElems: int
    Ngeo: int
    X: np.ndarray            # float64 [3][nElems][Ngeo+1]^3, a fastest
    sideElem: np.ndarray     # int32 [2*nSides]: master, slave
    sideLoc: np.ndarray      # int32 [2*nSides]
    sideOrient: np.ndarray   # int32 [nSides]
    volume: float = 0.0      # |Omega| of the undeformed box
    meta: dict = field(default_factory=dict)

    @property
    def nSides(self) -> int:
        return int(self.sideOrient.shape[0])


def _rotations():
    """The 24 proper rotations of the cube as signed 3x3 permutation matrices."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            P = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                P[r, perm[r]] = signs[r]
            if round(np.linalg.det(P)) == 1:
                mats.append(P)
    assert len(mats) == 24
    return mats


_ROT = _rotations()


def _face_of(xi):
    """Local face index of a reference point lying on exactly one face."""
    for r in range(3):
        if abs(xi[r]) == 1:
            return 2 * r + (1 if xi[r] > 0 else 0)
    raise ValueError("point not on a face")


def _tangential(f, xi):
    r = f // 2
    t = [d for d in range(3) if d != r]
    return xi[t[0]], xi[t[1]]


def _embed(f, s, t):
    r = f // 2
    xi = [0, 0, 0]
    xi[r] = 1 if f % 2 else -1
    tt = [d for d in range(3) if d != r]
    xi[tt[0]] = s
    xi[tt[1]] = t
    return xi


def _orient_code(st_map):
    """Orientation code from the images of (1,0) and (0,1) under (s,t) -> (s',t')."""
    (a1, b1), (a2, b2) = st_map((1, 0)), st_map((0, 1))
    if a1 != 0:      # no swap: s' = +-s, t' = +-t
        o = 0
        if a1 < 0:
            o |= 1
        if b2 < 0:
            o |= 2
    else:            # swap: s' = +-t, t' = +-s
        o = 4
        if a2 < 0:
            o |= 1
        if b1 < 0:
            o |= 2
    return o


def _to_new(P, xi_old):
    """Reference coordinates in an element's turned frame: xi_new = P^T xi_old."""
    return [float(v) for v in (P.T @ np.array(xi_old, dtype=np.float64))]


def _new_face(P, d, plus):
    """Local face (in the turned frame P) of the undisplaced face at the +-1 end of direction d."""
    xi = [0, 0, 0]
    xi[d] = 1 if plus else -1
    return _face_of(_to_new(P, xi))


def _side_orientation(PM, fM, PS, fS, d):
    """Orientation code of a side whose master (frame PM, local face fM) and
    slave (frame PS, local face fS) meet across the undisplaced direction d:
    two probe points inside the master face are carried to the slave's face."""
    def st_map(st):
        xi_m_old = PM @ np.array(_embed(fM, 0.5 * st[0], 0.5 * st[1]), dtype=np.float64)
        xi_s_old = xi_m_old.copy()
        xi_s_old[d] = -xi_m_old[d]   # same tangential position, opposite end
        xi_s_new = _to_new(PS, xi_s_old)
        assert _face_of(xi_s_new) == fS
        a, b = _tangential(fS, xi_s_new)
        return (int(round(2 * a)), int(round(2 * b)))
    return _orient_code(st_map)


def _frame_permutation(P, Ngeo):
    """Flat node permutation of a turned element: node (c,b,a) of the new
    frame is node perm[(c g1 + b) g1 + a] of the undisplaced one (xi_old = P xi_new)."""
    g1 = Ngeo + 1
    grid = np.arange(g1)
    an, bn, cn = np.meshgrid(grid, grid, grid, indexing="ij")
    new = [an, bn, cn]
    old = []
    for r in range(3):
        col = int(np.nonzero(P[r])[0][0])
        old.append(new[col] if P[r, col] > 0 else Ngeo - new[col])
    perm = np.empty(g1 ** 3, dtype=np.int64)
    perm[((cn * g1 + bn) * g1 + an).ravel()] = ((old[2] * g1 + old[1]) * g1 + old[0]).ravel()
    return perm


def box_mesh(K=(4, 4, 4), lo=(0.0, 0.0, 0.0), hi=(2.0, 2.0, 2.0), Ngeo=1,
             curved_amp=0.0, rotate_seed=None) -> Mesh:
    """Periodic box of Kx*Ky*Kz hexahedra in lexicographic order.

    Geometry nodes are equispaced (Ngeo+1)^3 per element.  With
    ``curved_amp`` every geometry node is displaced by
    ``amp * sin(x) sin(y) sin(z)`` in each coordinate, evaluated at the
    undisplaced position (the curved-mesh workload uses amp = 0.1 on
    [-pi, pi]^3, which keeps the periodic faces in place).  With
    ``rotate_seed`` each element's local frame is turned by a random proper
    cube rotation (PCG64(rotate_seed), one draw of nElems rotation indices)
    and master/slave roles are drawn at random (one further draw of nSides
    bits).

    Sides are numbered 3 e + d: element e (lexicographic) and its periodic
    neighbour in the + direction d.  Everything is built with whole-array
    operations, so the 64^3 boxes take a fraction of a second.
    """
    Kx, Ky, Kz = (int(k) for k in K)
    nE = Kx * Ky * Kz
    g1 = Ngeo + 1
    h = [(hi[d] - lo[d]) / K[d] for d in range(3)]
    s = np.arange(g1, dtype=np.float64) / Ngeo
    kz, ky, kx = np.meshgrid(np.arange(Kz), np.arange(Ky), np.arange(Kx), indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()        # element e = (kz Ky + ky) Kx + kx
    # element-local undisplaced coordinates, index order [c][b][a]
    X = np.empty((3, nE, g1, g1, g1))
    X[0] = (lo[0] + (kx[:, None] + s[None, :]) * h[0])[:, None, None, :]
    X[1] = (lo[1] + (ky[:, None] + s[None, :]) * h[1])[:, None, :, None]
    X[2] = (lo[2] + (kz[:, None] + s[None, :]) * h[2])[:, :, None, None]
    if curved_amp != 0.0:
        bump = curved_amp * np.sin(X[0]) * np.sin(X[1]) * np.sin(X[2])
        X = X + bump[None]
    # structural sides: element e and its + neighbour in each direction
    e = np.arange(nE)
    nb = [((kz * Ky + ky) * Kx + (kx + 1) % Kx),
          ((kz * Ky + (ky + 1) % Ky) * Kx + kx),
          ((((kz + 1) % Kz) * Ky + ky) * Kx + kx)]
    nS = 3 * nE
    elemA = np.repeat(e, 3)                                  # owner of the + face, side 3e + d
    elemB = np.stack(nb, axis=1).ravel()                     # its neighbour (- face)
    dirs = np.tile(np.arange(3), nE)
    if rotate_seed is None:
        sideElem = np.stack([elemA, elemB], axis=1).ravel()
        sideLoc = np.stack([2 * dirs + 1, 2 * dirs], axis=1).ravel()
        sideOrient = np.zeros(nS, dtype=np.int64)
    else:
        rng = np.random.Generator(np.random.PCG64(rotate_seed))
        rot = rng.integers(0, 24, size=nE)
        master_is_a = rng.integers(0, 2, size=nS).astype(bool)
        flat = X.reshape(3, nE, g1 ** 3)
        for rid in np.unique(rot):
            sel = np.nonzero(rot == rid)[0]
            flat[:, sel] = flat[:, sel][:, :, _frame_permutation(_ROT[rid], Ngeo)]
        X = flat.reshape(3, nE, g1, g1, g1)
        # local faces in the turned frames, per (rotation, direction, end)
        face_tab = np.array([[[_new_face(P, d, pl) for pl in (False, True)] for d in range(3)] for P in _ROT])
        rA, rB = rot[elemA], rot[elemB]
        fA, fB = face_tab[rA, dirs, 1], face_tab[rB, dirs, 0]
        mE = np.where(master_is_a, elemA, elemB)
        sE = np.where(master_is_a, elemB, elemA)
        mF = np.where(master_is_a, fA, fB)
        sF = np.where(master_is_a, fB, fA)
        mR = np.where(master_is_a, rA, rB)
        sR = np.where(master_is_a, rB, rA)
        # orientation per distinct (master frame, master face, slave frame, slave face, direction)
        key = (((mR * 6 + mF) * 24 + sR) * 6 + sF) * 3 + dirs
        ukeys, inv = np.unique(key, return_inverse=True)
        codes = np.empty(ukeys.size, dtype=np.int64)
        for u, kk in enumerate(ukeys):
            kk = int(kk)
            d = kk % 3; kk //= 3
            f_s = kk % 6; kk //= 6
            r_s = kk % 24; kk //= 24
            f_m = kk % 6; r_m = kk // 6
            codes[u] = _side_orientation(_ROT[r_m], f_m, _ROT[r_s], f_s, d)
        sideElem = np.stack([mE, sE], axis=1).ravel()
        sideLoc = np.stack([mF, sF], axis=1).ravel()
        sideOrient = codes[inv.ravel()]
    vol = float(np.prod([hi[d] - lo[d] for d in range(3)]))
    return Mesh(nE, Ngeo, np.ascontiguousarray(X), np.ascontiguousarray(sideElem, np.int32),
                np.ascontiguousarray(sideLoc, np.int32), np.ascontiguousarray(sideOrient, np.int32), vol,
                {"K": (Kx, Ky, Kz), "lo": tuple(lo), "hi": tuple(hi), "curved_amp": curved_amp,
                 "rotate_seed": rotate_seed})


# ---------------------------------------------------------------------------
# Initial states (functions of node coordinates xyz[3][nElems][n][n][n])
# ---------------------------------------------------------------------------


def prim_to_cons(rho, u, v, w, p, gamma):
    """Conserved state from primitive fields (perfect gas, total energy rho e)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E]))


def _by_element_chunks(fn, xyz, chunk=8192):
    """fn(xyz[:, e0:e1]) -> [5][e1-e0][...] evaluated over blocks of elements
    in host threads (numpy releases the GIL inside its array operations), so
    that the 134 M-node states are built in seconds."""
    nE = xyz.shape[1]
    if nE <= chunk:
        return fn(xyz)
    import concurrent.futures as cf
    import os
    out = np.empty((5,) + xyz.shape[1:])
    blocks = [(e0, min(nE, e0 + chunk)) for e0 in range(0, nE, chunk)]

    def work(b):
        out[:, b[0]:b[1]] = fn(xyz[:, b[0]:b[1]])

    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, blocks))
    return out


def tgv_state(xyz, gamma=1.4, Ma=0.1, rho0=1.0, U0=1.0, L=1.0, noise_amp=0.0, noise_seed=3):
    """Taylor-Green vortex (paper eq. tgv_ic) at background Mach number Ma.

    p0 = rho0 U0^2 / (gamma Ma^2); rho = p / (R T0) = rho0 p / p0.  With
    ``noise_amp`` each velocity component gets noise_amp * U(-1,1) per node
    (PCG64(noise_seed), drawn as one array of shape [3][...]) after the
    vortex is set, keeping rho and p.
    """
    p0 = rho0 * U0 * U0 / (gamma * Ma * Ma)

    def prim(xyz):
        x, y, z = xyz[0] / L, xyz[1] / L, xyz[2] / L
        u = U0 * np.sin(x) * np.cos(y) * np.cos(z)
        v = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
        w = np.zeros_like(u)
        p = p0 + rho0 * U0 * U0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (2.0 + np.cos(2 * z))
        return rho0 * p / p0, u, v, w, p

    if noise_amp == 0.0:
        return _by_element_chunks(lambda c: prim_to_cons(*prim(c), gamma), xyz)
    rho, u, v, w, p = prim(xyz)
    rng = np.random.Generator(np.random.PCG64(noise_seed))
    nz = rng.uniform(-1.0, 1.0, size=(3,) + u.shape)
    u = u + noise_amp * nz[0]
    v = v + noise_amp * nz[1]
    w = w + noise_amp * nz[2]
    return prim_to_cons(rho, u, v, w, p, gamma)


def freestream_state(xyz, gamma=1.4, Ma=0.1, rho0=1.0, U0=1.0):
    """Uniform flow along x at Mach Ma (p = rho0 U0^2 / (gamma Ma^2)): the
    paper's performance runs start from a free stream."""
    one = np.ones(xyz.shape[1:])
    p0 = rho0 * U0 ** 2 / (gamma * Ma ** 2)
    return prim_to_cons(rho0 * one, U0 * one, 0 * one, 0 * one, p0 * one, gamma)


def density_wave_state(xyz, t=0.0, gamma=1.4):
    """rho = 2 + 0.1 sin(pi (x+y+z - 3t)), u=v=w=1, p=1: an exact Euler solution."""
    rho = 2.0 + 0.1 * np.sin(np.pi * (xyz[0] + xyz[1] + xyz[2] - 3.0 * t))
    one = np.ones_like(rho)
    return prim_to_cons(rho, one, one, one, one, gamma)


def mms_state(xyz, t=0.0, A=0.1, a=1.0):
    """Manufactured solution of the convergence section: rho u = rho, rho e = rho^2."""
    rho = 2.0 + A * np.sin(2.0 * np.pi * (xyz[0] + xyz[1] + xyz[2] - a * t))
    return np.ascontiguousarray(np.stack([rho, rho, rho, rho, rho * rho]))


def random_state(shape, seed, gamma=1.4, rho=(0.8, 1.2), vel=0.5, p=(0.8, 1.2)):
    """Seeded random physical state: uniform rho, velocity, pressure per node."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.uniform(*rho, size=shape)
    u = rng.uniform(-vel, vel, size=(3,) + tuple(shape))
    pp = rng.uniform(*p, size=shape)
    return prim_to_cons(r, u[0], u[1], u[2], pp, gamma)


def smooth_random_state(xyz, seed, gamma=1.4, amp=0.1, nmodes=3):
    """Seeded smooth state: a few random Fourier modes on a uniform background."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fields = []
    for _ in range(5):
        f = np.zeros(xyz.shape[1:])
        for _m in range(nmodes):
            kv = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            c = rng.uniform(-1, 1)
            f = f + c * np.sin(kv[0] * xyz[0] + kv[1] * xyz[1] + kv[2] * xyz[2] + ph)
        fields.append(f)
    rho = 1.0 + amp * fields[0]
    u, v, w = 0.5 * amp * fields[1], 0.5 * amp * fields[2], 0.5 * amp * fields[3]
    p = 1.0 + amp * fields[4]
    return prim_to_cons(rho, u, v, w, p, gamma)


def random_directions(n_dof_vars, seeds):
    """Seeded directions with entries U(-1,1), one per seed."""
    return [np.random.Generator(np.random.PCG64(s)).uniform(-1.0, 1.0, size=n_dof_vars) for s in seeds]


# ---------------------------------------------------------------------------
# Workload presets (paper-shaped configurations)
# ---------------------------------------------------------------------------

PI = float(np.pi)

WORKLOADS = {
    # advected density wave, Euler, weak form, N=3 on LG nodes, 4^3 on [0,2]^3
    "euler_weak_lg_n3_4x4x4": dict(N=3, nodes=0, form=0, physics=0, mu=0.0, K=(4, 4, 4),
                                   lo=(0.0,) * 3, hi=(2.0,) * 3, curved=0.0, state="density_wave"),
    # same physics at the paper's single-node size (64^3 elements = 16.78 M nodes)
    "euler_weak_lg_n3_64x64x64": dict(N=3, nodes=0, form=0, physics=0, mu=0.0, K=(64, 64, 64),
                                      lo=(0.0,) * 3, hi=(2.0,) * 3, curved=0.0, state="density_wave"),
    # TGV Ma 0.1 Re 1600, NS + BR1, split form, N=7 LGL, 16^3 on [-pi,pi]^3
    "ns_split_lgl_n7_16x16x16_tgv": dict(N=7, nodes=1, form=1, physics=1, mu=1.0 / 1600.0, K=(16, 16, 16),
                                         lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.0, state="tgv"),
    # curved 32^3, N=5, TGV + velocity noise 1e-3 (seed 3)
    "ns_split_lgl_n5_32x32x32_curved_tgv": dict(N=5, nodes=1, form=1, physics=1, mu=1.0 / 1600.0,
                                                K=(32, 32, 32), lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.1,
                                                state="tgv_noise"),
    # Euler split form, N=5 LGL, 8^3, TGV (adjoint workload)
    "euler_split_lgl_n5_8x8x8_tgv": dict(N=5, nodes=1, form=1, physics=0, mu=0.0, K=(8, 8, 8),
                                         lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.0, state="tgv"),
    # entropy-stable split form on Gauss nodes, N=3: the TGV setup (16^3) and the
    # size of the CPU/GPU PID comparison (64^3 elements = 16.78 M DOFs, free stream)
    "ns_split_lg_n3_16x16x16_tgv": dict(N=3, nodes=0, form=1, physics=1, mu=1.0 / 1600.0, K=(16, 16, 16),
                                        lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.0, state="tgv"),
    "ns_split_lg_n3_64x64x64_freestream": dict(N=3, nodes=0, form=1, physics=1, mu=1.0 / 1600.0,
                                               K=(64, 64, 64), lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.0,
                                               state="freestream"),
    # large single-GPU run: NS split N=7 LGL 64^3 (134 M nodes)
    "ns_split_lgl_n7_64x64x64_tgv": dict(N=7, nodes=1, form=1, physics=1, mu=1.0 / 1600.0, K=(64, 64, 64),
                                         lo=(-PI,) * 3, hi=(PI,) * 3, curved=0.0, state="tgv"),
}


def workload_mesh(name, K=None):
    w = WORKLOADS[name]
    K = w["K"] if K is None else K
    Ngeo = w["N"] if w["curved"] else 1
    return box_mesh(K, w["lo"], w["hi"], Ngeo=Ngeo, curved_amp=w["curved"])


def workload_reference(name, gamma=1.4, state=None):
    """(rho0, p0) of a workload's background state: the reference state of
    the FP32-flux arithmetic (Taylor-Green vortex and free stream at Mach 0.1:
    p0 = rho0 U0^2 / (gamma Ma^2); density wave: rho 2, p 1)."""
    w = WORKLOADS[name]
    kind = "freestream" if state == "freestream" else w["state"]
    if kind == "density_wave":
        return 2.0, 1.0
    return 1.0, 1.0 / (gamma * 0.1 * 0.1)


def workload_state(name, xyz, gamma=1.4, state=None):
    """Initial state of a workload; state="freestream" replaces it by a free stream."""
    w = WORKLOADS[name]
    if state == "freestream":
        return freestream_state(xyz, gamma)
    if w["state"] == "density_wave":
        return density_wave_state(xyz, 0.0, gamma)
    if w["state"] == "tgv":
        return tgv_state(xyz, gamma=gamma)
    if w["state"] == "freestream":
        return freestream_state(xyz, gamma)
    if w["state"] == "tgv_noise":
        return tgv_state(xyz, gamma=gamma, noise_amp=1e-3, noise_seed=3)
    raise KeyError(w["state"])
