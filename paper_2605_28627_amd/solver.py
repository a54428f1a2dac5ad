"""DGSolver: one discretisation on the GPU (context, mesh, workspace) over the C-ABI.

PyTorch provides device memory and streams only; every step of the residual,
the time stepping and the adjoint runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dgx

CONFIG_KEYS = ("N", "nodes", "volume_form", "physics", "riemann", "twopoint", "precision", "integrator", "viscosity",
               "gamma", "mu", "Pr", "R", "Tref", "Ts", "fv")


def config_from_dict(d: dict) -> dgx.dg_config:
    """Accepts the library's key names and the short names used by the workloads (form)."""
    kw = {k: d[k] for k in CONFIG_KEYS if k in d}
    if "form" in d and "volume_form" not in d:
        kw["volume_form"] = d["form"]
    if "dissipation" in d and "riemann" not in d:
        kw["riemann"] = 0 if d["dissipation"] else 1
    return dgx.make_config(**kw)


class DGSolver:
    def __init__(self, cfg: dict, mesh, device: str | torch.device = "cuda", adjoint: bool = False):
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.ctx = dgx.dg_create(config_from_dict(cfg))
        try:
            with torch.cuda.device(self.device):
                dgx.dg_upload_mesh(self.ctx, mesh)
            self.nElems, self.nSides, self.npe, self.state_len = dgx.dg_sizes(self.ctx)
            self.n1 = round(self.npe ** (1 / 3))
            self._stages = len(dgx.dg_rk_coefficients(self.cfg.get("integrator", 0))[0])
            nb = dgx.dg_workspace_bytes_adjoint(self.ctx) if adjoint else dgx.dg_workspace_bytes(self.ctx)
            self.adjoint = adjoint
            # over-allocate so the bound pointer is 256-byte aligned
            self._ws_raw = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[off:off + nb]
            dgx.dg_bind_workspace(self.ctx, self.ws)
        except Exception:
            dgx.dg_destroy(self.ctx)
            self.ctx = None
            raise

    def close(self):
        """Destroys the context and drops the workspace (the solver is unusable afterwards)."""
        if getattr(self, "ctx", None) is not None:
            dgx.dg_destroy(self.ctx)
            self.ctx = None
        self.ws = None
        self._ws_raw = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_reference_state(self, rho0: float, p0: float):
        """Reference state of the FP32-flux arithmetic (rounding only)."""
        dgx.dg_set_reference_state(self.ctx, rho0, p0)

    @property
    def state_shape(self):
        return (5, self.nElems, self.n1, self.n1, self.n1)

    # FV sub-cell shock capturing (contexts with fv=1)
    def fv_switch(self, U: torch.Tensor, mask, dU: torch.Tensor | None = None):
        dgx.dg_fv_switch(self.ctx, U, dU, mask)

    def fv_indicator(self, U: torch.Tensor) -> torch.Tensor:
        ind = torch.empty(self.nElems, dtype=torch.float64, device=self.device)
        dgx.dg_fv_indicator(self.ctx, U, ind)
        return ind

    def fv_switch_by_indicator(self, U: torch.Tensor, ind_lo: float, ind_hi: float, dU: torch.Tensor | None = None):
        dgx.dg_fv_switch_by_indicator(self.ctx, U, dU, ind_lo, ind_hi)

    def fv_mask(self) -> np.ndarray:
        return dgx.dg_fv_mask(self.ctx)

    def coords(self) -> np.ndarray:
        return dgx.dg_node_coords(self.ctx)

    def metrics(self):
        return dgx.dg_get_metrics(self.ctx)

    def upload_metrics(self, Ja, sJ, nvec):
        dgx.dg_upload_metrics(self.ctx, Ja, sJ, nvec)

    def set_element_metrics(self, enable: bool):
        """Per-element metric terms for elements whose terms are constant (default on)."""
        dgx.dg_set_element_metrics(self.ctx, enable)

    def element_metric_count(self) -> int:
        return dgx.dg_element_metric_count(self.ctx)

    def to_device(self, U: np.ndarray) -> torch.Tensor:
        """Any host array of the state shape (a state, an adjoint vector, a direction) on the device."""
        return torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64)).to(self.device).reshape(self.state_shape)

    def init_state(self, U, out: torch.Tensor | None = None) -> torch.Tensor:
        """A device state from a host array or a device tensor, copied and checked
        (rho > 0, p > 0, finite) by dg_init_state; a non-physical state raises."""
        out = self.empty_state() if out is None else out
        dgx.dg_init_state(self.ctx, U, out)
        return out

    def empty_state(self) -> torch.Tensor:
        return torch.empty(self.state_shape, dtype=torch.float64, device=self.device)

    def rhs(self, U: torch.Tensor, Ut: torch.Tensor | None = None, t: float = 0.0) -> torch.Tensor:
        Ut = self.empty_state() if Ut is None else Ut
        dgx.dg_rhs(self.ctx, U, Ut, t)
        return Ut

    def lift(self, U: torch.Tensor) -> torch.Tensor:
        g = torch.empty((12, self.nElems, self.n1, self.n1, self.n1), dtype=torch.float64, device=self.device)
        dgx.dg_lift(self.ctx, U, g)
        return g

    def rk_step(self, U: torch.Tensor, dU: torch.Tensor, dt: float, nsteps: int = 1, t: float = 0.0):
        dgx.dg_rk_step(self.ctx, U, dU, t, dt, nsteps)

    @property
    def rk_stages(self) -> int:
        return self._stages

    def stage_buffer(self) -> torch.Tensor:
        """Device buffer for the S-1 stage inputs of one step (rk_step_stages)."""
        return torch.empty((self.rk_stages - 1,) + self.state_shape, dtype=torch.float64, device=self.device)

    def rk_step_stages(self, U: torch.Tensor, dU: torch.Tensor, dt: float, Y: torch.Tensor, t: float = 0.0):
        dgx.dg_rk_step_stages(self.ctx, U, dU, t, dt, Y, self.rk_stages)

    def adjoint_rk_step_stages(self, Un: torch.Tensor, Y: torch.Tensor, lamU: torch.Tensor, lamdU: torch.Tensor,
                               dt: float, t: float = 0.0):
        dgx.dg_adjoint_rk_step_stages(self.ctx, Un, Y, lamU, lamdU, t, dt, self.rk_stages)

    def adjoint_rhs(self, U: torch.Tensor, lam: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.empty_state() if out is None else out
        dgx.dg_adjoint_rhs(self.ctx, U, lam, out)
        return out

    def adjoint_rk_step(self, Un: torch.Tensor, lamU: torch.Tensor, lamdU: torch.Tensor, dt: float, t: float = 0.0):
        dgx.dg_adjoint_rk_step(self.ctx, Un, lamU, lamdU, t, dt)

    def kinetic_energy(self, U: torch.Tensor, rho0U0sq: float = 1.0) -> torch.Tensor:
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        dgx.dg_kinetic_energy(self.ctx, U, out, rho0U0sq)
        return out

    def kinetic_energy_grad(self, U: torch.Tensor, rho0U0sq: float = 1.0, scale: float = 1.0) -> torch.Tensor:
        g = self.empty_state()
        dgx.dg_kinetic_energy_grad(self.ctx, U, g, rho0U0sq, scale)
        return g

    def timestep(self, U: torch.Tensor, cfl: float = 0.9) -> float:
        return dgx.dg_timestep(self.ctx, U, cfl)

    def check_state(self, U: torch.Tensor) -> int:
        return dgx.dg_check_state(self.ctx, U)
