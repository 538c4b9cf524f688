"""Benchmark of the MR-LBM hot path on one MI355X.

A step is one full pass of Algorithm 1 (mesh adaptation + transfer, MR
transport, collision) over the whole synthetic state. Prints one JSON line:
leaf updates per second over the timed steps, the roofline of the dominant
kernel (transport + collision, HBM-bound) measured with HIP events on the
library's stream, and the FP64 oracle timed on the host on a bounded sample.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision 8|4]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leaf updates/s + HBM GB/s (% peak) at 1 GPU; FP32/batched/adjoint vs plain FP64"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
KERNEL_SOURCES = ["paper_2103_02903_amd/csrc/mr_kernels.h", "paper_2103_02903_amd/csrc/mr_device.h"]


def workload(name: str):
    """(list of (cfg, m0), description, default precision in bytes)."""
    from paper_2103_02903_amd import workloads as W

    if name == "d2q9_shear_1024":
        items = [W.shear_layer_d2q9()]  # levels 3..10, eps 1e-3, Re 1e4, width 1/80
        desc = "D2Q9 MRT double shear layer, periodic unit square, levels 3..10 (1024^2 finest), gamma=1, " \
               "eps=1e-3, mu_bar=1, Re=1e4, U0=0.1, tanh width 1/80, seeded 0.05 sinusoidal perturbation"
        prec = 8
    elif name == "d2q9_shear_batch96":
        items = W.shear_layer_batch(96)
        desc = "96 independent D2Q9 MRT double shear layers, levels 3..J with J drawn in {7,8,9,10}, " \
               "eps drawn in {1e-2,1e-3,1e-4}, Re uniform in [1e3,3e4], seeded perturbations; one launch " \
               "sequence per step for all instances"
        prec = 4
    elif name == "d1q3_burgers_16384":
        items = [W.burgers_d1q3()]
        desc = "D1Q3 inviscid Burgers, periodic [-1,1], levels 2..14 (16384 finest), gamma=1, eps=1e-4, " \
               "s=1.5, 8 seeded random-amplitude sines"
        prec = 8
    elif name == "d1q2_advection_1024":
        items = [W.advection_d1q2()]
        desc = "D1Q2 advection at Courant 1, periodic [-1,1], levels 2..10, gamma=1, eps=1e-4, s=1.9"
        prec = 8
    else:
        raise SystemExit("unknown workload %s" % name)
    return items, desc, prec


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name: str, precision: int):
    """HBM bytes per transport launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "transport_collide_%s_fp%d_counters.json" % (workload_name, 8 * precision))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, tree, values, seconds: float):
    """The FP64 oracle (single thread) stepping from the GPU's state for about
    `seconds` of host time; leaf updates per second of that sample."""
    import numpy as np

    import oracle

    o = oracle.Oracle(cfg)
    tree = tree.copy()
    values = values.astype(np.float64)
    updates, steps = 0, 0
    t0 = time.perf_counter()
    while True:
        o.step(tree, values)
        updates += int(o.leaf_counts(tree).sum())
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=updates / dt, unit="leaf updates/s", cores=1, kind="oracle",
                sample="%d oracle steps (%.1f s, single thread) from the GPU state at the start of the timed "
                       "region" % (steps, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="d2q9_shear_1024")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 4, 8], help="0: the workload's default")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see the design notes on "
              "sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_02903_amd import mrlbm

    if not os.path.exists(mrlbm.LIB_PATH):
        from paper_2103_02903_amd import build as hip_build

        hip_build.build(force=False)
    items, desc, prec = workload(args.workload)
    precision = args.precision or prec
    sim = mrlbm.Batch([c for c, _ in items], precision=precision)
    for i, (_, m0) in enumerate(items):
        sim.init_equilibrium(i, m0)
    sim.step(args.warmup)
    sim.synchronize()
    # the CPU baseline steps the largest instance from its state at the start of the timed region
    big = max(range(len(items)), key=lambda i: items[i][0]["jmax"])
    state0 = None if args.no_cpu_baseline else sim.get_state(big)

    sim.profile(True)
    stream = sim.stream
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    sim.step(args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    elapsed_ms = t_start.elapsed_time(t_end)
    cnt = sim.counters()
    stats = [sim.stats(i) for i in range(sim.B)]

    q, rs = sim.q, precision
    leaf_updates = int(cnt["leaf_updates"])
    value = leaf_updates / (elapsed_ms * 1e-3)
    bytes_per_leaf = 2 * q * rs  # read q populations, write q (neighbours are cache reuse)
    launches = max(1, int(cnt["timed_launches"]))
    avg_ms = cnt["transport_ms"] / launches
    bytes_per_launch = leaf_updates * bytes_per_leaf / max(1, int(cnt["transport_launches"]))
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    finest = sum(1 << (sim.dim * int(c["jmax"])) for c, _ in items)
    leaves_now = sum(int(st["leaves"].sum()) for st in stats)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "leaf updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "precision": "fp%d" % (8 * precision),
                   "instances": sim.B},
        "roofline": {
            "kernel": "k_transport_collide",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, precision),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_ms,
        },
        "mean_leaves_per_step": leaf_updates / max(1, args.steps),
        "compression_rate_final": 1.0 - leaves_now / finest,
        "compression_rate_mean": 1.0 - leaf_updates / max(1, args.steps) / finest,
        "phase_ms_per_step": {"adapt": cnt["adapt_ms"] / args.steps, "reconstruct": cnt["reconstruct_ms"] / args.steps,
                              "transport_collide": cnt["transport_ms"] / args.steps},
        "transport_kernel_leaf_updates_per_s": leaf_updates / (cnt["transport_ms"] * 1e-3),
        "mass_final": sum(st["mass"] for st in stats),
    }
    if state0 is not None:
        out["cpu_baseline"] = cpu_baseline(items[big][0], state0[0], state0[1], args.cpu_seconds)
        if sim.B > 1:
            out["cpu_baseline"]["sample"] += " (instance %d of %d, levels %d..%d)" % (
                big, sim.B, items[big][0]["jmin"], items[big][0]["jmax"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
