"""Benchmark of the DGSEM residual hot path on one MI355X.

A step is one LSERK4(5) time step (five evaluations of the whole residual:
BR1 lifting, surface fluxes, split-form volume integral, surface lift,
Jacobian scaling, RK update) of the large single-GPU Navier-Stokes
Taylor-Green vortex workload: N=7 on Lobatto nodes, 64^3 periodic
hexahedra on [-pi,pi]^3 (134 M nodes), Ma 0.1, Re 1600, Pr 0.72, FP64.  The
metric is the paper's PID (wall time / (RK stages * DOF), one GPU), lower is
better.  The adjoint/forward cost is taken over a 50-step trajectory whose
checkpoint interval is sized to the free HBM.

Printed as one JSON line.  Besides the contract fields it carries the
FP32-flux PID on the same workload and its error against the FP64 path,
the adjoint/forward cost, the residual kernel's roofline figures (HIP events
around every launch of the timed region; HBM bytes from the algorithmic
count, FP64 FLOPs from the committed rocprofv3 counters) and the serial FP64
oracle timed on a bounded sample of the same workload on the host.

Other workloads (--workload, --K, --state) and repetitions (--reps, median)
serve the per-configuration measurements; --fv checker/all runs a
workload with half or all of its elements on FV sub-cells (shock
capturing; the paper's 50 % FV row uses a checkerboard), --fv zero the same
FV-capable context with no element switched.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "ns_split_lgl_n7_64x64x64_tgv"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
KERNEL_SOURCES = ("dgx_kernels.hpp", "dgx_pointwise.hpp", "dgx_internal.hpp", "dgx_inst.hip", "dgx_tile.hpp",
                  "dgx_fv.hpp")


def _log(*a):
    """Progress on stderr (stdout carries only the JSON line)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=1, help="timed repetitions of --steps steps; the median is reported")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--K", default=None, help="element counts K1,K2,K3 replacing the workload's")
    ap.add_argument("--state", default=None, choices=[None, "freestream"], help="replace the initial state")
    ap.add_argument("--integrator", type=int, default=0, choices=[0, 1],
                    help="0 = LSERK4(5) (5 stages), 1 = LSERK4-14 (14 stages)")
    ap.add_argument("--riemann", default="rusanov", choices=["rusanov", "roe"],
                    help="face flux dissipation: Rusanov, or Roe with the Harten-Hyman entropy fix")
    ap.add_argument("--viscosity", default="constant", choices=["constant", "sutherland"],
                    help="constant mu, or Sutherland's law with Tref = the flow's reference temperature "
                         "and S/Tref = 110.4/273.15 (air)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--fp32-reference", default="workload", choices=["workload", "none"],
                    help="reference state of the FP32-flux arithmetic: the workload's background, or none")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-element-metrics", action="store_true",
                    help="every element reads its metric terms from the node arrays (the paper's per-node "
                         "storage), also where they are constant over the element")
    ap.add_argument("--fv-switch-every-step", action="store_true",
                    help="with --fv: one dg_rk_step call per step, each followed by the indicator and the "
                         "switch (hysteresis window (-inf, inf), so the element types stay as set), as a "
                         "shock-capturing run does")
    ap.add_argument("--fv", default="none", choices=["none", "zero", "checker", "all"],
                    help="FV sub-cell elements (Euler workloads): none (a DG-only context), zero (an FV "
                         "context with every element on DG), a checkerboard half, or all")
    ap.add_argument("--adjoint-steps", type=int, default=50)
    ap.add_argument("--checkpoint-every", type=int, default=None,
                    help="steps between checkpoints (default: sized to the free HBM)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target length of the timed oracle sample (the element count follows from a warm call)")
    ap.add_argument("--cpu-sample-elems", type=int, default=None, help="fixed oracle sample size (elements)")
    ap.add_argument("--cpu-repeats", type=int, default=2)
    ap.add_argument("--cpu-procs", type=int, default=1,
                    help="also run this many independent oracle processes at once (aggregate host throughput)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size: 2^27 doubles (1 GiB read + 1 GiB write) x 5."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                                           "copies": 5}}), flush=True)


def measured_copy_gbs():
    """Read + write rate of a plain 1 GiB device copy (the practical HBM ceiling for context)."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return 16.0 * n / (ms * 1e-3) / 1e9


def kernel_source_hash():
    """sha256[:16] over the sources the residual kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2605_28627_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_path(workload):
    return os.path.join(ROOT, "profiles", f"k_volume_{workload}.md")


def profile_meta(workload):
    """Machine-readable block of the committed rocprofv3 summary of a workload,
    or None when there is none or the kernel sources have changed since it
    was taken."""
    import re
    try:
        txt = open(profile_path(workload)).read()
        meta = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
        if kernel_source_hash() != meta["source_sha256_16"]:
            return None
        return meta
    except (OSError, KeyError, AttributeError, ValueError):
        return None


def profile_counters(workload, kernel):
    """Counters of one kernel from the committed summary: calibrated HBM bytes
    read and written and FP64 FLOPs per launch (None if absent or stale)."""
    meta = profile_meta(workload)
    try:
        return meta["kernels"][kernel] if meta else None
    except KeyError:
        return None


def kernel_counter_table(workload):
    """Per-kernel rates from the committed summary: measured HBM bytes per
    launch over the profiled average duration, and FP64 FLOP/s, each against
    the chip's peak (None if absent or stale)."""
    meta = profile_meta(workload)
    if not meta:
        return None
    out = {}
    for name, k in meta["kernels"].items():
        us = k.get("avg_us") or 0.0
        if us <= 0:
            continue
        gbs = (k["read"] + k["write"]) / (us * 1e-6) / 1e9
        row = {"avg_us": us, "hbm_bytes": k["read"] + k["write"], "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        if k.get("flops"):
            tf = k["flops"] / (us * 1e-6) / 1e12
            row.update(fp64_TFLOPs=tf, fp64_frac=tf / FP64_PEAK_TFLOPS)
        if k.get("alg_bytes"):
            row.update(alg_bytes=k["alg_bytes"], alg_GBs=k["alg_bytes"] / (us * 1e-6) / 1e9)
        out[name] = row
    return {"source": "committed rocprofv3 summary " + os.path.relpath(profile_path(workload), ROOT),
            "kernels": out}


def workload_cfg(name):
    from paper_2605_28627_amd import inputs as I
    w = I.WORKLOADS[name]
    return w, dict(N=w["N"], nodes=w["nodes"], form=w["form"], physics=w["physics"], mu=w["mu"], Pr=0.72,
                   gamma=1.4, R=1.0)


# kernel families timed live (events in the timed region): the residual kernels the roofline is taken on
ROOF_FAMILIES = ("volume", "fv")


def volume_kernel_name(w, precision=0, roe=0):
    return f"void dgx::k_volume<{w['N']}, {w['nodes']}, {w['form']}, {w['physics']}, {precision}, 1, {roe}, 0>"


def metric_values_per_dof(w, elem_frac=0.0, nvals=10):
    """Metric values a kernel reads per node: nvals (Ja 9 and 1/J 1, or 1/J
    alone) at every node of an element that reads the node arrays, and once
    per element (nvals / (N+1)^3 per node) for the fraction elem_frac of
    elements with constant terms, which read the per-element copy."""
    n3 = (w["N"] + 1) ** 3
    return nvals * (1.0 - elem_frac) + nvals * elem_frac / n3


def volume_kernel_bytes_per_dof(w, precision=0, elem_frac=0.0):
    """Compulsory HBM bytes of one launch of the residual/RK kernel, per node.

    Reads: U (5), metrics Ja (9) and 1/J (1) (metric_values_per_dof: once per
    element where they are constant), dU (5, except in the first of
    the five stages, whose A is 0: 4 on average), and per face node of
    each of the element's 6 faces both sides' traces (2 x 5) and the face
    normal + area (4); Navier-Stokes adds the viscous volume term (4) and
    both sides' face-normal viscous fluxes (2 x 4), formed by the lifting
    kernel.  Writes: dU (5), U (5) and the element's own traces of the new
    state (5 per face node).  8 bytes each, except the face viscous fluxes
    in the FP32-flux mode (4 bytes).
    """
    n1 = w["N"] + 1
    fpn = 6 * n1 * n1 / n1 ** 3          # face nodes of one element per volume node
    reads = 5 + metric_values_per_dof(w, elem_frac) + 4 + fpn * (10 + 4)
    writes = 5 + 5 + fpn * 5
    if w["physics"] == 1:
        reads += 4 + fpn * 8 * (0.5 if precision == 1 else 1.0)
    return 8.0 * (reads + writes)


def lift_kernel_bytes_per_dof(w, precision=0, elem_frac=0.0):
    """Compulsory HBM bytes of one launch of the lifting kernel (the forward
    stages' variant), per node.  Reads: U (5), Ja (9), 1/J (1) (as in the
    residual kernel), and per face node the other side's trace (5; on Gauss
    nodes both sides', 2 x 5: on LGL nodes the own trace is the face node's
    state, which the kernel has in LDS) and the face normal + area (4).
    Writes: the viscous volume term (4) and the element's own face-normal
    viscous flux (4 per face node; 4 bytes each in the FP32-flux mode)."""
    n1 = w["N"] + 1
    fpn = 6 * n1 * n1 / n1 ** 3
    traces = 5 if w["nodes"] == 1 else 10
    reads = 5 + metric_values_per_dof(w, elem_frac) + fpn * (traces + 4)
    writes = 4 + fpn * 4 * (0.5 if precision == 1 else 1.0)
    return 8.0 * (reads + writes)


def adjoint_kernel_bytes_per_dof(w, elem_frac=0.0):
    """Compulsory HBM bytes per node of one launch of each kernel of an
    adjoint stage (dg_adjoint_rk_step; the stage's reverse RK update fused
    into its last kernel), 8 bytes per value, per face node values times
    the face nodes per volume node (fpn):
      k_trace (the stage state's traces): U 5; writes 5 fpn;
      k_lift, gradients (Navier-Stokes): U 5, Ja 9, 1/J 1, the traces (as in
        lift_kernel_bytes_per_dof: 5 fpn on LGL nodes, 10 fpn on Gauss nodes),
        face 4 fpn; writes g 12 and the own gradient traces 12 fpn;
      k_adj_trace: lambda 5, 1/J 1; writes the surface adjoint 5 fpn
        (Navier-Stokes: first stage of a step only, the later ones take it
        from the fused update);
      k_adj_volume: lambda 5, 1/J 1, U 5, Ja 9, both traces, both surface
        adjoints and the face 24 fpn (Navier-Stokes: g 12, both gradient
        traces 24 fpn; writes out 5 and the lifting adjoint's face values
        Qbar 4 fpn; Euler: lamU 5 read, lamU and lamdU 10 written);
      k_adj_lift_volume (Navier-Stokes): 1/J 1, the own trace 5 fpn, both
        Qbar 8 fpn, out 5, lamU 5, lamdU 5; writes lamU and lamdU 10 and the
        next stage's surface adjoint 5 fpn.
    Ja and 1/J as in the residual kernel (metric_values_per_dof)."""
    n1 = w["N"] + 1
    fpn = 6 * n1 * n1 / n1 ** 3
    ns = w["physics"] == 1
    m10, m1 = metric_values_per_dof(w, elem_frac), metric_values_per_dof(w, elem_frac, 1)
    b = {"k_trace": 5 + 5 * fpn,
         "k_adj_trace": 5 + m1 + 5 * fpn}
    vol_r = 5 + 5 + m10 + 24 * fpn + (12 + 24 * fpn if ns else 5)
    vol_w = 5 + 4 * fpn if ns else 10
    b["k_adj_volume"] = vol_r + vol_w
    if ns:
        traces = 5 if w["nodes"] == 1 else 10
        b["k_lift_gradients"] = 5 + m10 + (traces + 4) * fpn + 12 + 12 * fpn
        b["k_adj_lift_volume"] = m1 + 15 + 13 * fpn + 10 + 5 * fpn
    return {k: 8.0 * v for k, v in b.items()}


def fv_kernel_bytes_per_dof(w):
    """Compulsory HBM bytes of one RK-stage launch of the FV kernel, per sub-cell.

    Reads: U (5), the sub-cell volume (1), dU (5, 4 on average over the five
    stages), the interior sub-face vectors (9 N / (N+1) per sub-cell), and
    per element face node the sub-face vector (3) and both sides' two-layer
    traces (2 x 10).  Writes: dU (5), U (5) and the element's own two-layer
    traces (10 per face node).  Navier-Stokes adds the sub-cell gradients
    (12) and per element face node both sides' layer-0 gradients (2 x 12).
    8 bytes each.
    """
    n1 = w["N"] + 1
    fpn = 6 * n1 * n1 / n1 ** 3
    reads = 5 + 1 + 4 + 9 * w["N"] / n1 + fpn * (3 + 20)
    writes = 5 + 5 + fpn * 10
    if w["physics"] == 1:
        reads += 12 + fpn * 24
    return 8.0 * (reads + writes)


def fv_mask(kind, K):
    import numpy as np
    ne = K[0] * K[1] * K[2]
    if kind == "all":
        return np.ones(ne, np.int32)
    if kind == "zero":
        return np.zeros(ne, np.int32)
    e = np.arange(ne)
    return ((e % K[0] + (e // K[0]) % K[1] + e // (K[0] * K[1])) % 2).astype(np.int32)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no multi-GPU path "
                                   "(it would shard the mesh by elements, one process per GPU)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2605_28627_amd import dgx
    from paper_2605_28627_amd import inputs as I
    from paper_2605_28627_amd.solver import DGSolver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w, cfg = workload_cfg(args.workload)
    cfg["integrator"] = args.integrator
    cfg["riemann"] = 2 if args.riemann == "roe" else 0
    if args.viscosity == "sutherland":
        # reference temperature of the initial state: T0 = p0 / (rho0 R) at Ma 0.1, rho0 = U0 = 1
        cfg.update(viscosity=1, Tref=1.0 / (1.4 * 0.01), Ts=110.4 / 273.15)
    if args.fv_switch_every_step and args.fv == "none":
        raise SystemExit("--fv-switch-every-step needs --fv")
    if args.fv != "none":
        if args.viscosity == "sutherland" or args.riemann == "roe":
            raise SystemExit("--fv: FV contexts use the Rusanov flux and constant viscosity")
        cfg["fv"] = 1
        args.no_fp32 = True      # FV contexts are FP64
        args.no_adjoint = True   # the adjoint does not cover FV sub-cells
    nst = len(dgx.dg_rk_coefficients(args.integrator)[0])
    K = tuple(int(x) for x in args.K.split(",")) if args.K else tuple(w["K"])
    _log("mesh", args.workload, K)
    mesh = I.workload_mesh(args.workload, K=K)
    _log("solver set-up")
    s = DGSolver(cfg, mesh, dev)
    if args.no_element_metrics:
        s.set_element_metrics(False)
    n_elem_metric = s.element_metric_count()
    dof = s.nElems * s.npe
    xyz = s.coords()
    U_host = I.workload_state(args.workload, xyz, state=args.state)
    U0 = s.init_state(U_host)
    dt = s.timestep(U0, 0.9)
    nfv = 0
    if args.fv != "none":
        mask = fv_mask(args.fv, K)
        s.fv_switch(U0, mask)
        nfv = int(mask.sum())

    def timed(solver, profile, keep=None):
        """args.reps repetitions of (warmup, then args.steps timed steps) from U0;
        returns the wall times and, with profile, the per-family kernel event
        times: the roofline families (volume, fv) from events in the first
        repetition's timed region (events around those launches only, which
        perturbs the timing least), the others from an untimed pass after it."""
        times, prof = [], {}
        for rep in range(args.reps):
            _log("timing", "fp32-flux" if solver.cfg.get("precision") else "fp64", "repetition", rep + 1, "of", args.reps)
            U = U0.clone()
            dU = torch.zeros_like(U)
            if args.warmup:
                solver.rk_step(U, dU, dt, args.warmup)
            torch.cuda.synchronize()
            events = profile and rep == 0
            if events:
                dgx.dg_profile_families(solver.ctx, ROOF_FAMILIES)
            t0 = time.perf_counter()
            if args.fv_switch_every_step:
                for _ in range(args.steps):
                    solver.rk_step(U, dU, dt, 1)
                    solver.fv_switch_by_indicator(U, -math.inf, math.inf, dU=dU)
            else:
                solver.rk_step(U, dU, dt, args.steps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if events:
                for fam in ROOF_FAMILIES:
                    prof[fam] = dgx.dg_profile_query(solver.ctx, fam)
                dgx.dg_profile(solver.ctx, 0)
            if solver.check_state(U) != 0:
                raise RuntimeError("non-physical state after the timed steps")
        if profile:
            _log("kernel breakdown (untimed)")
            Ub = U0.clone()
            dUb = torch.zeros_like(Ub)
            dgx.dg_profile(solver.ctx, 1)
            if args.fv_switch_every_step:
                for _ in range(args.steps):
                    solver.rk_step(Ub, dUb, dt, 1)
                    solver.fv_switch_by_indicator(Ub, -math.inf, math.inf, dU=dUb)
            else:
                solver.rk_step(Ub, dUb, dt, args.steps)
            for fam in ("trace", "lift", "other"):
                prof[fam] = dgx.dg_profile_query(solver.ctx, fam)
            dgx.dg_profile(solver.ctx, 0)
            del Ub, dUb
        if keep is not None:
            keep.append(U)
        return times, prof

    final64 = []
    times64, prof = timed(s, profile=True, keep=final64)
    t64 = statistics.median(times64)
    pid64 = t64 / (nst * args.steps * dof)
    vol_ms, vol_n = prof["volume"]
    vol_avg_s = vol_ms * 1e-3 / max(vol_n, 1)
    lift_ms, lift_n = prof["lift"]
    npe = (w["N"] + 1) ** 3
    # (Navier-Stokes FV contexts: the residual kernel reads the node arrays)
    elem_frac = 0.0 if args.fv != "none" and w["physics"] == 1 else n_elem_metric / s.nElems
    bytes_launch = volume_kernel_bytes_per_dof(w, elem_frac=elem_frac) * (dof - nfv * npe)
    kfam = "k_volume"
    if nfv:
        # the roofline of the dominant family: DG elements (k_volume) or FV elements (k_fv)
        fv_ms, fv_n = prof["fv"]
        fv_avg_s = fv_ms * 1e-3 / max(fv_n, 1)
        if fv_avg_s > vol_avg_s:
            kfam, vol_avg_s, vol_n = "k_fv", fv_avg_s, fv_n
            bytes_launch = fv_kernel_bytes_per_dof(w) * nfv * npe
    achieved_gbs = bytes_launch / vol_avg_s / 1e9
    kname = volume_kernel_name(w, 0, 1 if args.riemann == "roe" else 0)
    default_run = (args.K is None and args.state is None and args.integrator == 0 and args.riemann == "rusanov"
                   and args.viscosity == "constant")
    counters = profile_counters(args.workload, kname) if default_run and args.fv == "none" else None
    form = ("split form" if w["form"] else "weak form") + (", Navier-Stokes" if w["physics"] else ", Euler")

    result = {
        "metric": "PID (s per DOF per RK stage) FP64 vs FP32-mixed; adjoint/forward cost",
        "value": pid64,
        "unit": "s/(DOF*stage)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t64 / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (" + ("free stream" if args.state == "freestream" else
                                 {"tgv": "Taylor-Green vortex", "tgv_noise": "Taylor-Green vortex with seeded "
                                  "velocity noise", "density_wave": "advected density wave",
                                  "freestream": "free stream"}[w["state"]]) +
                " initial condition evaluated at the mesh nodes)",
        "config": {"workload": args.workload, "N": w["N"], "nodes": "LGL" if w["nodes"] else "LG",
                   "elements": list(K), "dof": dof, "physics": "navier-stokes" if w["physics"] else "euler",
                   "volume_form": "split" if w["form"] else "weak", "curved": bool(w["curved"]), "dt": dt,
                   "integrator": ("LSERK4(5)", "LSERK4-14")[args.integrator], "stages_per_step": nst,
                   "riemann": args.riemann, "viscosity": args.viscosity,
                   "state": args.state or w["state"], "fv_elements": nfv,
                   "fv_mask": args.fv, "fv_switch_every_step": bool(args.fv_switch_every_step),
                   "elements_with_element_metrics": n_elem_metric},
        "dof_updates_per_s": 1.0 / pid64,
        "simulated_time_per_wall_s": dt * args.steps / t64,
        "reps": args.reps,
        "ms_per_step_reps": [1e3 * t / args.steps for t in times64],
        "kernels_ms_per_launch": {k: (v[0] / max(v[1], 1)) for k, v in prof.items()},
        "kernel_timing": "HIP events on the launch stream: around the residual kernels (volume, fv) in the "
                         "timed region; around the other kernels in an untimed pass after it",
        "roofline": {
            "bound": "hbm",
            "kernel": (f"k_volume ({form}, RK stage)" if kfam == "k_volume" else
                       "k_fv (FV sub-cell elements, RK stage)"),
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": (counters["read"] + counters["write"]) if counters else None,
            "algorithmic_bytes_per_launch": bytes_launch,
            "avg_launch_ms": vol_avg_s * 1e3,
            "launches": vol_n,
            "measured_copy_GBs": measured_copy_gbs(),
        },
    }
    if counters and counters.get("flops"):
        tf = counters["flops"] / vol_avg_s / 1e12
        result["roofline_fp64_valu"] = {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                        "frac": tf / FP64_PEAK_TFLOPS, "flops_per_launch": counters["flops"],
                                        "source": "SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 x 64 lanes (FMA x 2) "
                                                  "from the committed rocprofv3 summary"}
    if lift_n:
        result["kernels_ms_per_launch"]["lift"] = lift_ms / lift_n
        lb = lift_kernel_bytes_per_dof(w, elem_frac=n_elem_metric / s.nElems) * dof
        lgbs = lb / (lift_ms * 1e-3 / lift_n) / 1e9
        result["roofline_lift"] = {"bound": "hbm", "kernel": "k_lift (BR1 lifting, forward stages)",
                                   "achieved": lgbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": lgbs / HBM_PEAK_GBS,
                                   "algorithmic_bytes_per_launch": lb, "avg_launch_ms": lift_ms / lift_n,
                                   "timing": "HIP events, untimed pass"}
    if default_run and args.fv == "none":
        result["kernel_counters"] = kernel_counter_table(args.workload)
    if not args.no_fp32:
        cfg32 = dict(cfg, precision=1)
        s32 = DGSolver(cfg32, mesh, dev)
        if args.no_element_metrics:
            s32.set_element_metrics(False)
        ref32 = I.workload_reference(args.workload, state=args.state) if args.fp32_reference == "workload" else (0, 0)
        s32.set_reference_state(*ref32)
        result["fp32_reference_state"] = {"rho0": ref32[0], "p0": ref32[1]}
        final32 = []
        times32, prof32 = timed(s32, profile=True, keep=final32)
        t32 = statistics.median(times32)
        result["pid_fp32_flux"] = t32 / (nst * args.steps * dof)
        result["kernels_ms_per_launch_fp32_flux"] = {k: (v[0] / max(v[1], 1)) for k, v in prof32.items()}
        result["fp32_speedup"] = t64 / t32
        # relative L2 error per variable of the FP32-flux path against the FP64 path
        # (which matches the oracle to 1e-12): residual of the initial state, and
        # the state after warmup + timed steps
        R64, R32 = s.rhs(U0), s32.rhs(U0)
        d_state = final32[0] - final64[0]
        d_ref = final64[0] - U0
        result["fp32_l2_error"] = {
            "residual_rel_per_var": [float((R32[v] - R64[v]).norm() / max(float(R64[v].norm()), 1e-300))
                                     for v in range(5)],
            "state_rel_to_change_per_var": [float(d_state[v].norm() / max(float(d_ref[v].norm()), 1e-300))
                                            for v in range(5)],
            "state_rel_per_var": [float(d_state[v].norm() / final64[0][v].norm()) for v in range(5)],
            "steps": args.steps + args.warmup,
        }
        del R64, R32, d_state, d_ref, final32
        s32.close()
        del s32
    del final64
    # (the forward context is done: its workspace goes back to the checkpoints of the adjoint)
    s.close()
    torch.cuda.empty_cache()
    _log("adjoint" if not args.no_adjoint else "adjoint skipped")
    # the adjoint covers every FP64 DG configuration (not FV sub-cells)
    adjoint_ok = args.fv == "none"
    result["adjoint_forward_cost"] = (adjoint_cost(cfg, mesh, dev, U0, dt, args)
                                      if not args.no_adjoint and adjoint_ok else None)
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(args, cfg, mesh, U_host, pid64)
    print(json.dumps(result), flush=True)


def adjoint_cost(cfg, mesh, dev, U0, dt, args):
    """Backward (reverse sweep with recomputation) over forward time of the
    gradient of E_k(T) through args.adjoint_steps steps of the same workload."""
    import torch
    from paper_2605_28627_amd.autograd import checkpoint_plan, kinetic_energy, trajectory
    from paper_2605_28627_amd.solver import DGSolver
    sa = DGSolver(cfg, mesh, dev, adjoint=True)
    if args.no_element_metrics:
        sa.set_element_metrics(False)
    n = args.adjoint_steps
    if args.checkpoint_every:
        every, keep = args.checkpoint_every, args.checkpoint_every - 1
    else:
        every, keep = checkpoint_plan(sa, n)
    times = []
    # a 2-step trajectory loads and warms the adjoint kernels; the 50-step one is timed
    for rep, (ns, ev, kp) in enumerate(((min(2, n), 2, 1), (n, every, keep))):
        _log("adjoint", "warm-up:" if rep == 0 else "timed:", ns, "steps, checkpoints every", ev,
             "stage states kept for", kp, "steps per segment")
        U = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = kinetic_energy(sa, trajectory(sa, U, dt, ns, checkpoint_every=ev, keep_stages=kp))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
        del U, J
    sa.close()
    tf, tb = times[-1]
    return {"value": tb / tf, "steps": n, "checkpoint_every": every, "stage_states_kept_per_segment": keep,
            "forward_s": tf, "backward_s": tb,
            "note": "backward includes the recomputation of the step states from checkpoints, keeping their stage "
                    "states (the last step of each segment recomputes its own)"}


def host_info():
    """Host CPU model, logical CPU count and the CPUs this process may run on."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        info["model"] = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return info


def _oracle_sample(workload, K, state, fv, library, nel, repeats, U=None):
    """Timed oracle residuals of elements 0..nel-1 of a workload, after an
    untimed warm call over the same elements (it builds their lazily computed
    geometry).  Each call writes only the sampled elements' residual."""
    from oracle import oracle as O
    from paper_2605_28627_amd import inputs as I
    _, cfg = workload_cfg(workload)
    mesh = I.workload_mesh(workload, K=K)
    if fv != "none":
        cfg["fv"] = 1
    o = O.Oracle(cfg, mesh, library=O.load(library))
    if fv != "none":
        o.fv_set_mask(fv_mask(fv, K or tuple(I.WORKLOADS[workload]["K"])))
    if U is None:
        U = I.workload_state(workload, o.coords(), state=state)
    el = list(range(nel))
    o.rhs_sample(U, el)
    t0 = time.perf_counter()
    for _ in range(repeats):
        o.rhs_sample(U, el)
    return time.perf_counter() - t0


def cpu_baseline(args, cfg, mesh, U, pid_gpu):
    """The serial FP64 oracle on the host, built -O3 -march=native for this
    CPU: residuals of a contiguous block of elements of the same workload (one
    RK stage's worth of work per node), on one thread, after an untimed warm
    call; with --cpu-procs P > 1 also P such processes at once.  The block is
    sized from a warm call on 64 elements so that the timed loop takes about
    --cpu-seconds."""
    import tempfile
    from oracle import oracle as O
    from paper_2605_28627_amd import inputs as I
    tmp = tempfile.mkdtemp(prefix="dgx_oracle_")
    library = O.build_native(tmp)
    K = tuple(int(x) for x in args.K.split(",")) if args.K else tuple(I.WORKLOADS[args.workload]["K"])
    o = O.Oracle(cfg, mesh, library=O.load(library))
    if args.fv != "none":
        o.fv_set_mask(fv_mask(args.fv, K))
    npe = (cfg["N"] + 1) ** 3
    nel = args.cpu_sample_elems
    if nel is None:
        probe = list(range(min(64, mesh.nElems)))
        o.rhs_sample(U, probe)
        t0 = time.perf_counter()
        o.rhs_sample(U, probe)
        per_el = (time.perf_counter() - t0) / len(probe)
        nel = int(args.cpu_seconds / (args.cpu_repeats * per_el))
    nel = max(1, min(nel, mesh.nElems))
    el = list(range(nel))
    o.rhs_sample(U, el)                      # warm: the sample's geometry
    t0 = time.perf_counter()
    for _ in range(args.cpu_repeats):
        o.rhs_sample(U, el)
    t = time.perf_counter() - t0
    pid = t / (args.cpu_repeats * nel * npe)
    out = {"value": pid, "unit": "s/(DOF*stage)", "cores": 1, "kind": "oracle",
           "sample": f"{args.cpu_repeats} residual evaluations of elements 0..{nel - 1} of the {mesh.nElems}-element "
                     f"workload ({nel * npe} DOF each, serial, one thread, after one untimed warm call; only the "
                     f"sampled elements' residual is written), {t:.1f} s",
           "build": "g++ -O3 -march=native (the oracle source, built on this host)",
           "gpu_over_cpu_per_rank": pid / pid_gpu,
           "host": host_info()}
    if args.cpu_procs > 1:
        import multiprocessing as mp
        P = args.cpu_procs
        Kp = tuple(int(x) for x in args.K.split(",")) if args.K else None
        with mp.get_context("spawn").Pool(P) as pool:
            t0 = time.perf_counter()
            ts = pool.starmap(_oracle_sample, [(args.workload, Kp, args.state, args.fv, library, nel,
                                                args.cpu_repeats)] * P)
            wall = time.perf_counter() - t0
        pid_all = max(ts) / (P * args.cpu_repeats * nel * npe)
        out["all_cores"] = {"procs": P, "pid_aggregate": pid_all, "dof_updates_per_s": 1.0 / pid_all,
                            "per_process_s": ts, "wall_s_incl_setup": wall,
                            "gpu_over_all_cores": pid_all / pid_gpu,
                            "note": "independent oracle processes on the same sample at once; aggregate over the "
                                    "slowest process's timed loop (set-up and warm call excluded)"}
    return out


if __name__ == "__main__":
    main()
