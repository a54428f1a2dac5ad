"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte models the roofline divides by (against the per-node tables of the
kernels' reads and writes), and the FV element masks."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2605_28627_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["n_gpus"] == 2 and "one GPU" in d["error"]


def test_byte_models():
    # 8 B per value; 0.75 face nodes per volume node at N = 7, 1.5 at N = 3
    c2 = I.WORKLOADS["ns_split_lgl_n7_16x16x16_tgv"]
    # U 5, Ja + 1/J 10, dU 4 (five-stage average), viscous volume term 4, traces 2x5 and face viscous
    # fluxes 2x4 and face geometry 4 per face node; writes dU 5, U 5, traces 5 per face node
    assert bench.volume_kernel_bytes_per_dof(c2) == 8 * (5 + 10 + 4 + 4 + 0.75 * (10 + 8 + 4) + 5 + 5 + 0.75 * 5)
    assert bench.volume_kernel_bytes_per_dof(c2) == 426
    c1 = I.WORKLOADS["euler_weak_lg_n3_64x64x64"]
    assert bench.volume_kernel_bytes_per_dof(c1) == 460
    assert bench.fv_kernel_bytes_per_dof(c1) == 610
    es = I.WORKLOADS["ns_split_lg_n3_64x64x64_freestream"]
    assert bench.volume_kernel_bytes_per_dof(es) == 588
    # FP32-flux mode stores the face viscous fluxes as float
    assert bench.volume_kernel_bytes_per_dof(c2, precision=1) == 426 - 4 * 0.75 * 8
    # lifting: reads U 5, Ja + 1/J 10, the other side's trace 5 (LGL: the own trace is the
    # face node's state) and face geometry 4 per face node; writes the viscous volume term 4
    # and the own face viscous flux 4 per face node
    assert bench.lift_kernel_bytes_per_dof(c2) == 8 * (15 + 0.75 * 9 + 4 + 0.75 * 4) == 230
    # Gauss nodes: both sides' traces (2 x 5), 1.5 face nodes per node at N = 3
    assert bench.lift_kernel_bytes_per_dof(es) == 8 * (15 + 1.5 * 14 + 4 + 1.5 * 4)
    # elements with constant metric terms read Ja + 1/J once per element (10 values per 512 nodes)
    assert bench.volume_kernel_bytes_per_dof(c2, elem_frac=1.0) == pytest.approx(426 - 8 * (10 - 10 / 512))
    assert bench.lift_kernel_bytes_per_dof(c2, elem_frac=0.5) == pytest.approx(230 - 8 * 0.5 * (10 - 10 / 512))
    a0, a1 = bench.adjoint_kernel_bytes_per_dof(c2), bench.adjoint_kernel_bytes_per_dof(c2, elem_frac=1.0)
    assert a0["k_adj_volume"] - a1["k_adj_volume"] == pytest.approx(8 * (10 - 10 / 512))
    assert a0["k_adj_trace"] - a1["k_adj_trace"] == pytest.approx(8 * (1 - 1 / 512))


def test_fv_masks():
    K = (4, 3, 2)
    m = bench.fv_mask("checker", K)
    assert m.sum() == 12 and m.dtype == np.int32
    e = np.arange(24)
    i, j, k = e % 4, (e // 4) % 3, e // 12
    assert np.array_equal(m, (i + j + k) % 2)
    assert bench.fv_mask("all", K).sum() == 24
    assert bench.fv_mask("zero", K).sum() == 0


def test_cpu_baseline_leg_runs_on_the_host():
    """The oracle leg of the bench line (native build, warm call, sampled
    residuals) on the smallest workload, with a short time target."""
    import argparse
    w, cfg = bench.workload_cfg("euler_weak_lg_n3_4x4x4")
    mesh = I.workload_mesh("euler_weak_lg_n3_4x4x4")
    from oracle import oracle as O
    U = I.workload_state("euler_weak_lg_n3_4x4x4", O.Oracle(cfg, mesh).coords())
    args = argparse.Namespace(workload="euler_weak_lg_n3_4x4x4", K=None, state=None, fv="none", cpu_seconds=0.2,
                              cpu_sample_elems=None, cpu_repeats=2, cpu_procs=1)
    out = bench.cpu_baseline(args, cfg, mesh, U, 1e-9)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    assert out["host"]["nproc"] >= 1 and "O3" in out["build"]
