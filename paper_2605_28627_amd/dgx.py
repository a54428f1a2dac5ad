"""Thin ctypes binding of the C-ABI in include/dgx.h (argument marshalling only).

Every function has the name of its C counterpart.  Device arrays are passed
as torch CUDA tensors (float64, contiguous), host arrays as numpy arrays,
streams as torch streams (default: the current stream).  A failing status
raises DGError carrying dg_last_error().  Importing this module raises
ImportError when the HIP library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: it loads its own HIP runtime (libamdhip64 and the HSA runtime),
# and libdgx.so must resolve to that already-loaded copy.  Loaded the other
# way round, the process holds two HIP runtimes and the second sees no device.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdgx.so not found at {LIB_PATH}: build it with __graft_entry__.build() "
                      "(python -m paper_2605_28627_amd.build); there is no CPU fallback")

_L = ctypes.CDLL(LIB_PATH)

DG_OK, DG_ERR_ARG, DG_ERR_MESH, DG_ERR_HIP, DG_ERR_NONPHYSICAL, DG_ERR_NOMEM, DG_ERR_UNSUPPORTED, DG_ERR_STATE = range(8)
DG_RK_LSERK45, DG_RK_LSERK414 = 0, 1
DG_RIEMANN_RUSANOV, DG_RIEMANN_CENTRAL, DG_RIEMANN_ROE = 0, 1, 2
DG_VISC_CONSTANT, DG_VISC_SUTHERLAND = 0, 1
DG_RK_MAX_STAGES = 14
STATUS_NAMES = {0: "DG_OK", 1: "DG_ERR_ARG", 2: "DG_ERR_MESH", 3: "DG_ERR_HIP", 4: "DG_ERR_NONPHYSICAL",
                5: "DG_ERR_NOMEM", 6: "DG_ERR_UNSUPPORTED", 7: "DG_ERR_STATE"}

# public symbols of include/dgx.h
SYMBOLS = ["dg_create", "dg_destroy", "dg_set_reference_state", "dg_last_error", "dg_lserk_coefficients", "dg_rk_coefficients", "dg_set_mesh", "dg_upload_mesh",
           "dg_upload_metrics", "dg_get_metrics", "dg_set_element_metrics", "dg_element_metric_count", "dg_node_coords", "dg_sizes", "dg_workspace_bytes",
           "dg_workspace_bytes_adjoint", "dg_bind_workspace", "dg_init_state", "dg_rhs", "dg_lift", "dg_rk_step", "dg_rk_step_noalloc", "dg_rk_step_stages", "dg_adjoint_rhs", "dg_adjoint_rk_step",
           "dg_adjoint_rk_step_stages",
           "dg_kinetic_energy", "dg_kinetic_energy_grad", "dg_timestep", "dg_check_state", "dg_profile",
           "dg_profile_families", "dg_profile_query", "dg_fv_switch", "dg_fv_indicator", "dg_fv_switch_by_indicator", "dg_fv_mask"]


class dg_config(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("nodes", ctypes.c_int), ("volume_form", ctypes.c_int),
                ("physics", ctypes.c_int), ("riemann", ctypes.c_int), ("twopoint", ctypes.c_int),
                ("precision", ctypes.c_int), ("integrator", ctypes.c_int), ("viscosity", ctypes.c_int),
                ("fv", ctypes.c_int),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("Pr", ctypes.c_double), ("R", ctypes.c_double), ("Tref", ctypes.c_double), ("Ts", ctypes.c_double)]


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
_sz = ctypes.c_size_t
_sig = {
    "dg_create": (ctypes.c_int, [ctypes.POINTER(dg_config), ctypes.POINTER(_vp)]),
    "dg_destroy": (ctypes.c_int, [_vp]),
    "dg_set_reference_state": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
    "dg_last_error": (ctypes.c_char_p, [_vp]),
    "dg_lserk_coefficients": (ctypes.c_int, [_dp, _dp, _dp]),
    "dg_rk_coefficients": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp, _ip]),
    "dg_set_mesh": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _ip]),
    "dg_upload_mesh": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _ip]),
    "dg_upload_metrics": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "dg_get_metrics": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "dg_set_element_metrics": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_element_metric_count": (ctypes.c_int, [_vp, _ip]),
    "dg_node_coords": (ctypes.c_int, [_vp, _dp]),
    "dg_sizes": (ctypes.c_int, [_vp, _ip, _ip, _ip, ctypes.POINTER(_sz)]),
    "dg_workspace_bytes": (_sz, [_vp]),
    "dg_workspace_bytes_adjoint": (_sz, [_vp]),
    "dg_bind_workspace": (ctypes.c_int, [_vp, _vp, _sz]),
    "dg_init_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "dg_rhs": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp]),
    "dg_lift": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "dg_rk_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _vp]),
    "dg_rk_step_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _vp]),
    "dg_adjoint_rhs": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "dg_adjoint_rk_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp]),
    "dg_rk_step_stages": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "dg_adjoint_rk_step_stages": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp]),
    "dg_kinetic_energy": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _vp]),
    "dg_kinetic_energy_grad": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "dg_timestep": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _dp, _vp]),
    "dg_check_state": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_profile_families": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_profile_query": (ctypes.c_int, [_vp, ctypes.c_char_p, _dp, ctypes.POINTER(ctypes.c_long)]),
    "dg_fv_switch": (ctypes.c_int, [_vp, _vp, _vp, _ip, _vp]),
    "dg_fv_indicator": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "dg_fv_switch_by_indicator": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp]),
    "dg_fv_mask": (ctypes.c_int, [_vp, _ip, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _L


def _check(ctx, st):
    if st != DG_OK:
        msg = _L.dg_last_error(ctx)
        raise DGError(st, msg.decode() if msg else "")


def _hd(a):
    """Host float64 array pointer."""
    assert isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _hi(a):
    assert isinstance(a, np.ndarray) and a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def _dev(t, n=None, name="array"):
    """Device pointer of a contiguous float64 CUDA tensor (length checked when n is given)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_config(N, nodes=1, volume_form=0, physics=0, riemann=0, twopoint=0, precision=0, integrator=0, viscosity=0,
                gamma=1.4, mu=0.0, Pr=0.72, R=1.0, Tref=1.0, Ts=110.4 / 273.15, fv=0):
    return dg_config(N, nodes, volume_form, physics, riemann, twopoint, precision, integrator, viscosity, fv, gamma,
                     mu, Pr, R, Tref, Ts)


def dg_create(cfg: dg_config):
    h = ctypes.c_void_p()
    _check(None, _L.dg_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def dg_destroy(ctx):
    _check(None, _L.dg_destroy(ctx))


def dg_set_reference_state(ctx, rho0, p0):
    _check(ctx, _L.dg_set_reference_state(ctx, float(rho0), float(p0)))


def dg_last_error(ctx):
    m = _L.dg_last_error(ctx)
    return m.decode() if m else ""


def dg_lserk_coefficients():
    A, B, C = np.zeros(5), np.zeros(5), np.zeros(5)
    _check(None, _L.dg_lserk_coefficients(_hd(A), _hd(B), _hd(C)))
    return A, B, C


def dg_rk_coefficients(integrator):
    """(A, B, c) of the scheme DG_RK_* (length = its number of stages)."""
    A, B, C = (np.zeros(DG_RK_MAX_STAGES) for _ in range(3))
    ns = ctypes.c_int(0)
    _check(None, _L.dg_rk_coefficients(int(integrator), _hd(A), _hd(B), _hd(C), ctypes.byref(ns)))
    return A[:ns.value], B[:ns.value], C[:ns.value]


def _mesh_args(mesh):
    X = np.ascontiguousarray(mesh.X, dtype=np.float64)
    se = np.ascontiguousarray(mesh.sideElem, dtype=np.int32)
    sl = np.ascontiguousarray(mesh.sideLoc, dtype=np.int32)
    so = np.ascontiguousarray(mesh.sideOrient, dtype=np.int32)
    return X, se, sl, so


def dg_set_mesh(ctx, mesh):
    X, se, sl, so = _mesh_args(mesh)
    _check(ctx, _L.dg_set_mesh(ctx, mesh.nElems, mesh.Ngeo, _hd(X), int(so.size), _hi(se), _hi(sl), _hi(so)))


def dg_upload_mesh(ctx, mesh):
    X, se, sl, so = _mesh_args(mesh)
    _check(ctx, _L.dg_upload_mesh(ctx, mesh.nElems, mesh.Ngeo, _hd(X), int(so.size), _hi(se), _hi(sl), _hi(so)))


def dg_sizes(ctx):
    ne, ns, npe, sl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), _sz()
    _check(ctx, _L.dg_sizes(ctx, ctypes.byref(ne), ctypes.byref(ns), ctypes.byref(npe), ctypes.byref(sl)))
    return ne.value, ns.value, npe.value, sl.value


def dg_upload_metrics(ctx, Ja, sJ, nvec):
    Ja, sJ, nvec = (np.ascontiguousarray(a, dtype=np.float64) for a in (Ja, sJ, nvec))
    _check(ctx, _L.dg_upload_metrics(ctx, _hd(Ja), _hd(sJ), _hd(nvec)))


def dg_get_metrics(ctx):
    ne, ns, npe, _ = dg_sizes(ctx)
    n1 = round(npe ** (1 / 3))
    xyz = np.zeros((3, ne, n1, n1, n1))
    Ja = np.zeros((9, ne, n1, n1, n1))
    sJ = np.zeros((ne, n1, n1, n1))
    nv = np.zeros((3, ns, n1, n1))
    _check(ctx, _L.dg_get_metrics(ctx, _hd(xyz), _hd(Ja), _hd(sJ), _hd(nv)))
    return xyz, Ja, sJ, nv


def dg_set_element_metrics(ctx, enable: bool):
    _check(ctx, _L.dg_set_element_metrics(ctx, 1 if enable else 0))


def dg_element_metric_count(ctx) -> int:
    n = ctypes.c_int(0)
    _check(ctx, _L.dg_element_metric_count(ctx, ctypes.byref(n)))
    return n.value


def dg_node_coords(ctx):
    ne, _, npe, _ = dg_sizes(ctx)
    n1 = round(npe ** (1 / 3))
    xyz = np.zeros((3, ne, n1, n1, n1))
    _check(ctx, _L.dg_node_coords(ctx, _hd(xyz)))
    return xyz


def dg_workspace_bytes(ctx):
    return int(_L.dg_workspace_bytes(ctx))


def dg_workspace_bytes_adjoint(ctx):
    return int(_L.dg_workspace_bytes_adjoint(ctx))


def dg_bind_workspace(ctx, ws_tensor):
    _check(ctx, _L.dg_bind_workspace(ctx, ctypes.c_void_p(ws_tensor.data_ptr()), ws_tensor.numel() * ws_tensor.element_size()))


def dg_init_state(ctx, U_src, U, stream=None):
    """Copies U_src (a float64 numpy array on the host, or a contiguous float64
    CUDA tensor) into the device state U and checks it; DG_ERR_NONPHYSICAL raises."""
    import torch
    n = dg_sizes(ctx)[3]
    if isinstance(U_src, np.ndarray):
        src = np.ascontiguousarray(U_src, dtype=np.float64)
        if src.size != n:
            raise ValueError(f"U_src has {src.size} elements, expected {n}")
        ptr, on_dev = ctypes.cast(src.ctypes.data, _vp), 0
    elif isinstance(U_src, torch.Tensor):
        ptr, on_dev = _dev(U_src, n, "U_src"), 1
    else:
        raise TypeError("U_src must be a numpy array or a CUDA tensor")
    _check(ctx, _L.dg_init_state(ctx, ptr, on_dev, _dev(U, n, "U"), _stream(stream)))


def dg_rhs(ctx, U, Ut, t=0.0, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_rhs(ctx, _dev(U, n, "U"), _dev(Ut, n, "Ut"), float(t), _stream(stream)))


def dg_lift(ctx, U, g, stream=None):
    ne, _, npe, n = dg_sizes(ctx)
    _check(ctx, _L.dg_lift(ctx, _dev(U, n, "U"), _dev(g, 12 * ne * npe, "g"), _stream(stream)))


def dg_rk_step(ctx, U, dU, t, dt, nsteps, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_rk_step(ctx, _dev(U, n, "U"), _dev(dU, n, "dU"), float(t), float(dt), int(nsteps),
                              _stream(stream)))


def dg_rk_step_noalloc(ctx, U, dU, t, dt, nsteps, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_rk_step_noalloc(ctx, _dev(U, n, "U"), _dev(dU, n, "dU"), float(t), float(dt), int(nsteps),
                                      _stream(stream)))


def dg_adjoint_rhs(ctx, U, lam, out, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_adjoint_rhs(ctx, _dev(U, n, "U"), _dev(lam, n, "lam"), _dev(out, n, "out"), _stream(stream)))


def dg_adjoint_rk_step(ctx, Un, lamU, lamdU, t, dt, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_adjoint_rk_step(ctx, _dev(Un, n, "Un"), _dev(lamU, n, "lamU"), _dev(lamdU, n, "lamdU"),
                                      float(t), float(dt), _stream(stream)))


def dg_rk_step_stages(ctx, U, dU, t, dt, Y, nstages, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_rk_step_stages(ctx, _dev(U, n, "U"), _dev(dU, n, "dU"), float(t), float(dt),
                                     _dev(Y, (nstages - 1) * n, "Y"), _stream(stream)))


def dg_adjoint_rk_step_stages(ctx, Un, Y, lamU, lamdU, t, dt, nstages, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_adjoint_rk_step_stages(ctx, _dev(Un, n, "Un"), _dev(Y, (nstages - 1) * n, "Y"),
                                             _dev(lamU, n, "lamU"), _dev(lamdU, n, "lamdU"), float(t), float(dt),
                                             _stream(stream)))


def dg_kinetic_energy(ctx, U, out, rho0U0sq=1.0, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_kinetic_energy(ctx, _dev(U, n, "U"), float(rho0U0sq), _dev(out, 1, "out"), _stream(stream)))


def dg_kinetic_energy_grad(ctx, U, grad, rho0U0sq=1.0, scale=1.0, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_kinetic_energy_grad(ctx, _dev(U, n, "U"), float(rho0U0sq), float(scale),
                                          _dev(grad, n, "grad"), _stream(stream)))


def dg_timestep(ctx, U, cfl=0.9, stream=None):
    n = dg_sizes(ctx)[3]
    dt = ctypes.c_double()
    _check(ctx, _L.dg_timestep(ctx, _dev(U, n, "U"), float(cfl), ctypes.byref(dt), _stream(stream)))
    return dt.value


def dg_check_state(ctx, U, stream=None):
    """Returns the status code (DG_OK or DG_ERR_NONPHYSICAL); other errors raise."""
    n = dg_sizes(ctx)[3]
    st = _L.dg_check_state(ctx, _dev(U, n, "U"), _stream(stream))
    if st not in (DG_OK, DG_ERR_NONPHYSICAL):
        _check(ctx, st)
    return st


def dg_fv_switch(ctx, U, dU, mask, stream=None):
    ne, _, _, n = dg_sizes(ctx)
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.int32).reshape(-1))
    if m.size != ne:
        raise ValueError(f"mask has {m.size} entries, expected {ne}")
    _check(ctx, _L.dg_fv_switch(ctx, _dev(U, n, "U"), None if dU is None else _dev(dU, n, "dU"), _hi(m),
                                _stream(stream)))


def dg_fv_indicator(ctx, U, ind, stream=None):
    ne, _, _, n = dg_sizes(ctx)
    _check(ctx, _L.dg_fv_indicator(ctx, _dev(U, n, "U"), _dev(ind, ne, "ind"), _stream(stream)))


def dg_fv_switch_by_indicator(ctx, U, dU, ind_lo, ind_hi, stream=None):
    n = dg_sizes(ctx)[3]
    _check(ctx, _L.dg_fv_switch_by_indicator(ctx, _dev(U, n, "U"), None if dU is None else _dev(dU, n, "dU"),
                                             float(ind_lo), float(ind_hi), _stream(stream)))


def dg_fv_mask(ctx, stream=None):
    ne = dg_sizes(ctx)[0]
    m = np.zeros(ne, dtype=np.int32)
    _check(ctx, _L.dg_fv_mask(ctx, _hi(m), _stream(stream)))
    return m


def dg_profile(ctx, enable):
    _check(ctx, _L.dg_profile(ctx, int(bool(enable))))


PROFILE_FAMILIES = ("trace", "lift", "volume", "adjoint", "other", "fv")


def dg_profile_families(ctx, families):
    """Events only around the launches of the named kernel families (empty: off)."""
    mask = 0
    for f in families:
        mask |= 1 << PROFILE_FAMILIES.index(f)
    _check(ctx, _L.dg_profile_families(ctx, mask))


def dg_profile_query(ctx, kernel):
    """(total milliseconds, launch count) of a kernel family since profiling was enabled."""
    ms, n = ctypes.c_double(), ctypes.c_long()
    _check(ctx, _L.dg_profile_query(ctx, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
