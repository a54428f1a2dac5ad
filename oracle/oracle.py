"""ctypes wrapper around the serial FP64 oracle (dg_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dg_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (portable x86-64, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
               "-o", tmp, SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def build_native(out_dir: str) -> str:
    """The same source compiled with -O3 -march=native for the host it runs on
    (timing of the CPU baseline only; the parity build above is the one the
    tests use).  Built into out_dir, since the code is specific to this CPU."""
    out = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["g++", "-O3", "-march=native", "-std=c++17", "-fPIC", "-shared", "-o", out, SRC]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def load(path):
    """ctypes handle of an oracle build with every signature declared."""
    L = ctypes.CDLL(path)
    L.orc_last_error.restype = ctypes.c_char_p
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [_ip, _dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _ip]
    for name in ("orc_destroy",):
        getattr(L, name).argtypes = [ctypes.c_void_p]
    L.orc_check_jacobians.argtypes = [ctypes.c_void_p]
    L.orc_geometry.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    L.orc_face_normals.argtypes = [ctypes.c_void_p, _dp]
    L.orc_rhs.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double]
    L.orc_rhs_elems.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip]
    L.orc_lift.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_rhs_jvp.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_double]
    L.orc_lserk.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_lserk_jvp.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_kinetic_energy.restype = ctypes.c_double
    L.orc_kinetic_energy.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
    L.orc_kinetic_energy_jvp.restype = ctypes.c_double
    L.orc_kinetic_energy_jvp.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double]
    L.orc_timestep.restype = ctypes.c_double
    L.orc_timestep.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
    L.orc_rhs_opcount.argtypes = [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_uint64)]
    L.orc_rk_coeffs.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.orc_rk_coeffs.restype = ctypes.c_int
    L.orc_viscosity.argtypes = [_ip, _dp, ctypes.c_double]
    L.orc_viscosity.restype = ctypes.c_double
    L.orc_roe_matrix.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp]
    L.orc_flux_visc_law.argtypes = [_ip, _dp, _dp, _dp, ctypes.c_int, _dp]
    L.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_lserk_coeffs.argtypes = [_dp, _dp, _dp]
    L.orc_flux_twopoint.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    L.orc_flux_adv.argtypes = [_dp, _dp, _dp, _dp]
    L.orc_flux_visc.argtypes = [_dp, _dp, _dp, ctypes.c_int, _dp]
    L.orc_fv_set_mask.argtypes = [ctypes.c_void_p, _ip]
    L.orc_fv_switch.argtypes = [ctypes.c_void_p, _dp, _dp, _ip]
    L.orc_fv_get_mask.argtypes = [ctypes.c_void_p, _ip]
    L.orc_fv_indicator.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_fv_geometry.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    L.orc_fv_operators.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    L.orc_fv_convert.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.orc_entropy_vars.argtypes = [_dp, _dp, _dp]
    L.orc_cons_from_entropy.argtypes = [_dp, _dp, _dp]
    L.orc_logmean.restype = ctypes.c_double
    L.orc_logmean.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_mms_source.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    L.orc_rhs_sample.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip]
    L.orc_opcount_point.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_uint64)]
    L.orc_geometry_sample.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip, _dp, _dp, _dp]
    L.orc_fv_gradients.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_rhs_vjp.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_double]
    L.orc_kinetic_energy_grad.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp]
    L.orc_lserk_adjoint.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    return L


def _d(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def basis(N, nodes):
    n = N + 1
    x, w, Lm, Lp = (np.zeros(n) for _ in range(4))
    D, DS = np.zeros((n, n)), np.zeros((n, n))
    rc = lib().orc_basis(N, nodes, _d(x), _d(w), _d(D), _d(Lm), _d(Lp), _d(DS))
    if rc:
        raise ValueError("bad basis request")
    return dict(x=x, w=w, D=D, Lm=Lm, Lp=Lp, DS=DS)


def rk_coeffs(integrator):
    """A, B, c of the low-storage scheme: 0 = LSERK4(5), 1 = LSERK4-14."""
    A, B, C = np.zeros(14), np.zeros(14), np.zeros(14)
    ns = lib().orc_rk_coeffs(int(integrator), _d(A), _d(B), _d(C))
    if ns == 0:
        raise ValueError("unknown integrator")
    return A[:ns], B[:ns], C[:ns]


def lserk_coeffs():
    A, B, C = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().orc_lserk_coeffs(_d(A), _d(B), _d(C))
    return A, B, C


def _cfg_arrays(cfg):
    # the library's riemann key (0 Rusanov, 1 central, 2 Roe) maps onto the oracle's dissipation switch
    diss = {0: 1, 1: 0, 2: 2}[cfg["riemann"]] if "riemann" in cfg else cfg.get("dissipation", 1)
    icfg = np.array([cfg.get("N", 3), cfg.get("nodes", 0), cfg.get("form", 0), cfg.get("physics", 0),
                     cfg.get("twopoint", 0), diss, cfg.get("mms", 0),
                     cfg.get("integrator", 0), cfg.get("viscosity", 0), cfg.get("hybrid", 0),
                     cfg.get("fv", 0)], dtype=np.int32)
    dcfg = np.array([cfg.get("gamma", 1.4), cfg.get("mu", 0.0), cfg.get("Pr", 0.72), cfg.get("R", 1.0),
                     cfg.get("mms_A", 0.1), cfg.get("mms_a", 1.0), cfg.get("Tref", 1.0),
                     cfg.get("Ts", 110.4 / 273.15)], dtype=np.float64)
    return icfg, dcfg


def flux_twopoint(Ua, Ub, nv, gamma=1.4, central=False):
    icfg, dcfg = _cfg_arrays(dict(twopoint=1 if central else 0, gamma=gamma))
    F = np.zeros(5)
    lib().orc_flux_twopoint(_i(icfg), _d(dcfg), _d(np.ascontiguousarray(Ua, dtype=np.float64)),
                            _d(np.ascontiguousarray(Ub, dtype=np.float64)),
                            _d(np.ascontiguousarray(nv, dtype=np.float64)), _d(F))
    return F


def flux_adv(U, nv, gamma=1.4):
    _, dcfg = _cfg_arrays(dict(gamma=gamma))
    F = np.zeros(5)
    lib().orc_flux_adv(_d(dcfg), _d(np.ascontiguousarray(U, dtype=np.float64)),
                       _d(np.ascontiguousarray(nv, dtype=np.float64)), _d(F))
    return F


def roe_matrix(UL, UR, nh, mode=0, gamma=1.4):
    """mode 0: |A~|(UR-UL) with the Harten-Hyman fix; 1: A~(UR-UL) (signed); 2: |A~|(UR-UL) without the fix."""
    _, dcfg = _cfg_arrays(dict(gamma=gamma))
    D = np.zeros(5)
    lib().orc_roe_matrix(_d(dcfg), _d(np.ascontiguousarray(UL, dtype=np.float64)),
                         _d(np.ascontiguousarray(UR, dtype=np.float64)),
                         _d(np.ascontiguousarray(nh, dtype=np.float64)), int(mode), _d(D))
    return D


def viscosity(temp, mu=1.0, law=1, Tref=1.0, Ts=110.4 / 273.15):
    icfg, dcfg = _cfg_arrays(dict(mu=mu, viscosity=law, Tref=Tref, Ts=Ts))
    return lib().orc_viscosity(_i(icfg), _d(dcfg), float(temp))


def flux_visc_law(U, g, n, gamma=1.4, mu=1e-2, Pr=0.72, R=1.0, law=1, Tref=1.0, Ts=110.4 / 273.15):
    icfg, dcfg = _cfg_arrays(dict(gamma=gamma, mu=mu, Pr=Pr, R=R, viscosity=law, Tref=Tref, Ts=Ts))
    G = np.zeros(5)
    lib().orc_flux_visc_law(_i(icfg), _d(dcfg), _d(np.ascontiguousarray(U, dtype=np.float64)),
                            _d(np.ascontiguousarray(g, dtype=np.float64)), int(n), _d(G))
    return G


def flux_visc(U, g, n, gamma=1.4, mu=1e-2, Pr=0.72, R=1.0):
    _, dcfg = _cfg_arrays(dict(gamma=gamma, mu=mu, Pr=Pr, R=R))
    G = np.zeros(5)
    lib().orc_flux_visc(_d(dcfg), _d(np.ascontiguousarray(U, dtype=np.float64)),
                        _d(np.ascontiguousarray(g, dtype=np.float64)), int(n), _d(G))
    return G


def entropy_vars(U, gamma=1.4):
    """v = dS/dU for S = -rho s/(gamma-1), s = ln p - gamma ln rho."""
    _, dcfg = _cfg_arrays(dict(gamma=gamma))
    v = np.zeros(5)
    lib().orc_entropy_vars(_d(dcfg), _d(np.ascontiguousarray(U, dtype=np.float64)), _d(v))
    return v


def cons_from_entropy(v, gamma=1.4):
    """Inverse of entropy_vars."""
    _, dcfg = _cfg_arrays(dict(gamma=gamma))
    U = np.zeros(5)
    lib().orc_cons_from_entropy(_d(dcfg), _d(np.ascontiguousarray(v, dtype=np.float64)), _d(U))
    return U


def opcount_point(kind, Ua, Ub=None, nv=(1.0, 0.0, 0.0), gamma=1.4):
    """Operation counts of one point function on the counting scalar: kind
    "flux_adv" (Ua, nv), "logmean" (Ua[0], Ub[0]) or "twopoint" (Ua, Ub, nv)."""
    _, dcfg = _cfg_arrays(dict(gamma=gamma))
    k = {"flux_adv": 0, "logmean": 1, "twopoint": 2}[kind]
    a = np.zeros(5)
    a[:len(np.atleast_1d(Ua))] = np.atleast_1d(Ua)
    b = np.zeros(5)
    if Ub is not None:
        b[:len(np.atleast_1d(Ub))] = np.atleast_1d(Ub)
    c = (ctypes.c_uint64 * 5)()
    if lib().orc_opcount_point(k, _d(dcfg), _d(a), _d(b), _d(np.ascontiguousarray(nv, dtype=np.float64)), c):
        raise ValueError(lib().orc_last_error().decode())
    return dict(add=c[0], mul=c[1], div=c[2], sqrt=c[3], log=c[4])


def logmean(x, y):
    return lib().orc_logmean(float(x), float(y))


def mms_source(x, y, z, t, gamma=1.4, mu=1e-3, Pr=0.72, R=1.0, A=0.1, a=1.0):
    _, dcfg = _cfg_arrays(dict(gamma=gamma, mu=mu, Pr=Pr, R=R, mms_A=A, mms_a=a))
    Q = np.zeros(5)
    lib().orc_mms_source(_d(dcfg), float(x), float(y), float(z), float(t), _d(Q))
    return Q


class Oracle:
    """One discretisation (config + mesh) in the oracle."""

    def __init__(self, cfg: dict, mesh, library=None):
        self.L = library if library is not None else lib()
        self.cfg = dict(cfg)
        self.mesh = mesh
        self.N = int(cfg["N"])
        self.n1 = self.N + 1
        self.nElems = mesh.nElems
        self.nSides = mesh.nSides
        icfg, dcfg = _cfg_arrays(cfg)
        X = np.ascontiguousarray(mesh.X, dtype=np.float64)
        self._keep = (X, mesh.sideElem, mesh.sideLoc, mesh.sideOrient)
        h = self.L.orc_create(_i(icfg), _d(dcfg), mesh.nElems, mesh.Ngeo, _d(X), mesh.nSides,
                              _i(mesh.sideElem), _i(mesh.sideLoc), _i(mesh.sideOrient))
        if not h:
            raise ValueError("oracle: " + self.L.orc_last_error().decode())
        self.h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and getattr(self, "L", None) is not None:
            self.L.orc_destroy(h)
            self.h = None

    @property
    def state_shape(self):
        return (5, self.nElems, self.n1, self.n1, self.n1)

    def check_jacobians(self):
        if self.L.orc_check_jacobians(self.h):
            raise ValueError(self.L.orc_last_error().decode())

    def geometry(self):
        n = self.n1
        xyz = np.zeros((3, self.nElems, n, n, n))
        J = np.zeros((self.nElems, n, n, n))
        Ja = np.zeros((9, self.nElems, n, n, n))
        self.L.orc_geometry(self.h, _d(xyz), _d(J), _d(Ja))
        return xyz, J, Ja

    def geometry_sample(self, elems):
        """Node coordinates, Jacobian and metrics of the listed elements only:
        [3][n][...], [n][...], [9][n][...]."""
        el = np.ascontiguousarray(np.asarray(elems, dtype=np.int32))
        n = self.n1
        xyz, J, Ja = np.zeros((3, el.size, n, n, n)), np.zeros((el.size, n, n, n)), np.zeros((9, el.size, n, n, n))
        self._chk(self.L.orc_geometry_sample(self.h, int(el.size), _i(el), _d(xyz), _d(J), _d(Ja)))
        return xyz, J, Ja

    def coords(self):
        return self.geometry()[0]

    def face_normals(self):
        nv = np.zeros((3, self.nSides, self.n1, self.n1))
        self.L.orc_face_normals(self.h, _d(nv))
        return nv

    def rhs(self, U, t=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        Ut = np.zeros_like(U)
        self.L.orc_rhs(self.h, _d(U), _d(Ut), float(t))
        return Ut

    def rhs_elems(self, U, elems, t=0.0):
        """Residual of the listed elements only: array [5][len(elems)][n][n][n]."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        el = np.ascontiguousarray(np.asarray(elems, dtype=np.int32))
        Ut = np.zeros_like(U)
        if self.L.orc_rhs_elems(self.h, _d(U), _d(Ut), float(t), int(el.size), _i(el)):
            raise ValueError(self.L.orc_last_error().decode())
        return Ut[:, el]

    def rhs_sample(self, U, elems, t=0.0):
        """Residual of the listed (distinct) elements, written straight into an
        array [5][len(elems)][n][n][n] (no full-size output)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        el = np.ascontiguousarray(np.asarray(elems, dtype=np.int32))
        n = self.n1
        out = np.empty((5, el.size, n, n, n))
        if self.L.orc_rhs_sample(self.h, _d(U), _d(out), float(t), int(el.size), _i(el)):
            raise ValueError(self.L.orc_last_error().decode())
        return out

    def lift(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        n = self.n1
        g = np.zeros((12, self.nElems, n, n, n))
        self.L.orc_lift(self.h, _d(U), _d(g))
        return g

    def rhs_jvp(self, U, dU, t=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.ascontiguousarray(dU, dtype=np.float64).reshape(U.shape)
        Ut, dUt = np.zeros_like(U), np.zeros_like(U)
        self.L.orc_rhs_jvp(self.h, _d(U), _d(dU), _d(Ut), _d(dUt), float(t))
        return Ut, dUt

    def lserk(self, U, nsteps, dt, t0=0.0):
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        self.L.orc_lserk(self.h, _d(U), int(nsteps), float(dt), float(t0))
        return U

    def lserk_jvp(self, U, dU, nsteps, dt, t0=0.0):
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        dU = np.array(dU, dtype=np.float64, copy=True, order="C").reshape(U.shape)
        self.L.orc_lserk_jvp(self.h, _d(U), _d(dU), int(nsteps), float(dt), float(t0))
        return U, dU

    def rhs_vjp(self, U, lam, t=0.0):
        """(dR/dU)^T lam at U, by reverse-mode differentiation of the residual."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(U.shape)
        out = np.zeros_like(U)
        self.L.orc_rhs_vjp(self.h, _d(U), _d(lam), _d(out), float(t))
        return out

    def kinetic_energy_grad(self, U, rho0U0sq=1.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        g = np.zeros_like(U)
        self.L.orc_kinetic_energy_grad(self.h, _d(U), float(rho0U0sq), _d(g))
        return g

    def lserk_adjoint(self, U0, lamT, nsteps, dt, t0=0.0):
        """(dU(T)/dU0)^T lamT through nsteps steps of the context's RK scheme
        (the reverse sweep of the 2N-storage stages, stage inputs recomputed)."""
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        lam = np.array(lamT, dtype=np.float64, copy=True, order="C").reshape(U0.shape)
        self._chk(self.L.orc_lserk_adjoint(self.h, _d(U0), _d(lam), int(nsteps), float(dt), float(t0)))
        return lam

    def kinetic_energy(self, U, rho0U0sq=1.0):
        return self.L.orc_kinetic_energy(self.h, _d(np.ascontiguousarray(U, dtype=np.float64)), float(rho0U0sq))

    def kinetic_energy_jvp(self, U, dU, rho0U0sq=1.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.ascontiguousarray(dU, dtype=np.float64).reshape(U.shape)
        return self.L.orc_kinetic_energy_jvp(self.h, _d(U), _d(dU), float(rho0U0sq))

    def timestep(self, U, cfl=0.9):
        return self.L.orc_timestep(self.h, _d(np.ascontiguousarray(U, dtype=np.float64)), float(cfl))

    # FV sub-cells (config fv=1, Euler)
    def _chk(self, rc):
        if rc:
            raise ValueError(self.L.orc_last_error().decode())

    def fv_set_mask(self, mask):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int32).reshape(-1))
        assert m.size == self.nElems
        self._chk(self.L.orc_fv_set_mask(self.h, _i(m)))

    def fv_mask(self):
        m = np.zeros(self.nElems, dtype=np.int32)
        self.L.orc_fv_get_mask(self.h, _i(m))
        return m

    def fv_switch(self, U, dU, newmask):
        """Convert U (and dU) to the element types of newmask; returns copies."""
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        dU = None if dU is None else np.array(dU, dtype=np.float64, copy=True, order="C")
        m = np.ascontiguousarray(np.asarray(newmask, dtype=np.int32).reshape(-1))
        self._chk(self.L.orc_fv_switch(self.h, _d(U), _d(dU) if dU is not None else None, _i(m)))
        return U, dU

    def indicator(self, U):
        ind = np.zeros(self.nElems)
        self.L.orc_fv_indicator(self.h, _d(np.ascontiguousarray(U, dtype=np.float64)), _d(ind))
        return ind

    def fv_gradients(self, U):
        """Sub-cell gradients [12][nElems][...] of a Navier-Stokes FV context:
        Green-Gauss for FV elements, sub-cell means of the lifted gradient for DG."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        n = self.n1
        g = np.zeros((12, self.nElems, n, n, n))
        self._chk(self.L.orc_fv_gradients(self.h, _d(U), _d(g)))
        return g

    def fv_geometry(self):
        n = self.n1
        V = np.zeros((self.nElems, n, n, n))
        Si = np.zeros((self.nElems, 3, 3, self.N, n, n))
        Sb = np.zeros((self.nSides, 3, n, n))
        self._chk(self.L.orc_fv_geometry(self.h, _d(V), _d(Si), _d(Sb)))
        return V, Si, Sb

    def fv_operators(self):
        n = self.n1
        B, Bi, Vi = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
        self._chk(self.L.orc_fv_operators(self.h, _d(B), _d(Bi), _d(Vi)))
        return B, Bi, Vi

    def fv_convert(self, e, block, to_fv=True):
        b = np.ascontiguousarray(block, dtype=np.float64)
        out = np.zeros_like(b)
        self._chk(self.L.orc_fv_convert(self.h, int(e), 0 if to_fv else 1, _d(b), _d(out)))
        return out

    def opcount(self, U):
        c = (ctypes.c_uint64 * 5)()
        self.L.orc_rhs_opcount(self.h, _d(np.ascontiguousarray(U, dtype=np.float64)), c)
        return dict(add=c[0], mul=c[1], div=c[2], sqrt=c[3], log=c[4])
