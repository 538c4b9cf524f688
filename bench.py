"""Benchmark of the MR-LBM hot path on one MI355X.

A step is one full pass of Algorithm 1 (mesh adaptation + transfer, MR
transport, collision) over the whole synthetic state, replayed from a HIP
graph. The default workload is the largest one: 96 independent D2Q9 double
shear layers (finest levels 7..10) advanced together in FP32. Prints one JSON
line: leaf updates per second over the timed steps; the roofline of the
dominant kernel (transport + collision, HBM-bound), timed with HIP events on
the library's stream inside the timed region; the same batch in FP64, the
single 1024^2 shear layer in FP64 and FP32, the adjoint, and the method's
variants (walls, gamma = 2 and 3, the l2 metric, the Euler scheme), measured on
the same GPU next to it; and the FP64 oracle timed on the host on a bounded
sample.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision 8|4]
  python bench.py --copy-calibration     (plain copy kernel of known size only)
  python bench.py --adjoint-only 4       (the adjoint leg only, 4 or 8: for a kernel trace)
  python bench.py --scope-only [NAME]    (the walls, gamma, l2, Euler and 3D workloads only)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leaf updates/s + HBM GB/s (% peak) at 1 GPU; FP32/batched/adjoint vs plain FP64"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
COPY_BYTES = 1 << 30


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
               "eps drawn in {1e-2,1e-3,1e-4}, Re uniform in [1e3,3e4], seeded perturbations; one graph " \
               "replay per step for all instances"
        prec = 4
    elif name == "d2q9_vortex_256":
        items = [W.random_vortex_d2q9()]
        desc = "D2Q9 MRT, periodic unit square, levels 3..8 (256^2 finest), eps=1e-3, seeded smooth " \
               "solenoidal velocity from 16 Fourier modes"
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


def measured_traffic(workload_name: str, precision: int, kernel: str):
    """HBM bytes per transport launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source and transport variant (else None)."""
    path = os.path.join(ROOT, "profiles", "transport_collide_%s_fp%d_counters.json" % (workload_name, 8 * precision))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    from paper_2103_02903_amd.profiling import kernel_source_hash

    if d.get("kernel_source_hash") != kernel_source_hash() or not d.get("kernel", "").startswith(kernel):
        return None
    return d.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, tree, values, seconds: float):
    """The FP64 oracle stepping from the GPU's state, timed on the host: with
    all the threads OpenMP gets here (its parallel per-cell loops; the value
    reported) and single-threaded, each for about `seconds` of host time."""
    import numpy as np

    import oracle

    o = oracle.Oracle(cfg)
    n_all = oracle.threads()

    def run(nthreads, secs):
        oracle.threads(nthreads)
        t, v = tree.copy(), values.astype(np.float64)
        updates, steps = 0, 0
        t0 = time.perf_counter()
        while True:
            o.step(t, v)
            updates += int(o.leaf_counts(t).sum())
            steps += 1
            if time.perf_counter() - t0 >= secs:
                break
        return updates / (time.perf_counter() - t0), steps, time.perf_counter() - t0

    rate_all, steps_all, dt_all = run(n_all, seconds)
    rate_one, steps_one, dt_one = run(1, seconds)
    oracle.threads(n_all)
    host = dict(cpu_model=_cpu_model(), nproc=os.cpu_count(), affinity=len(os.sched_getaffinity(0)),
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"))
    return dict(value=rate_all, unit="leaf updates/s", cores=n_all, kind="oracle",
                sample="%d oracle steps (%.1f s, %d threads) from the GPU state at the start of the measured "
                       "window" % (steps_all, dt_all, n_all),
                single_thread=dict(value=rate_one, cores=1,
                                   sample="%d oracle steps (%.1f s, one thread), same start" % (steps_one, dt_one)),
                host=host)


def copy_bandwidth(nbytes: int = COPY_BYTES, reps: int = 5):
    """GB/s (read + write) of the library's plain copy kernel."""
    import torch

    from paper_2103_02903_amd import mrlbm

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream()
    mrlbm.copy(dst, src, nbytes, stream)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        mrlbm.copy(dst, src, nbytes, stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return dict(bytes_per_launch=2 * nbytes, avg_launch_ms=ms, gbs=2 * nbytes / (ms * 1e-3) / 1e9)


def timed_run(items, precision, steps, warmup, keep_state_of=None, tune=True, schedule=None, markers=False):
    """Warm up, pick the launch schedule with the library's autotuner, then run
    two windows of `steps` graph-replayed steps each:
      A (the measurement of `value` and ms_per_step): no timing inside the steps;
      B (the roofline): HIP events inside every step graph bracket the transport
        kernel, on the library's stream, so every launch of the window is timed
        (each bracket costs the step a few microseconds, which is why A is kept
        free of them).
    Returns (result dict, sim, state of instance `keep_state_of` at the start of
    window A or None). `schedule` (transport variant, all-level cap, per-level
    cap) replaces the autotuner; `markers` puts a 256-byte launch of the copy
    kernel before A, between A and B and after B, which profiles use to find
    the dispatches of each window."""
    import torch

    from paper_2103_02903_amd import mrlbm

    sim = mrlbm.Batch([c for c, _ in items], precision=precision)
    for i, (_, m0) in enumerate(items):
        sim.init_equilibrium(i, m0)
    sim.step(warmup)
    sim.synchronize()
    if schedule is not None:
        sim.set_tuning(*schedule)
        tuning = sim.tuning()
    else:
        tuning = sim.autotune(reps=5) if tune else sim.tuning()
    mark = None
    if markers:
        mark = (torch.zeros(256, dtype=torch.uint8, device=sim.device),
                torch.zeros(256, dtype=torch.uint8, device=sim.device))
    state0 = sim.get_state(keep_state_of) if keep_state_of is not None else None
    stream = sim.stream

    def marker():
        if mark is not None:
            mrlbm.copy(mark[1], mark[0], 256, stream)

    # window A
    sim.profile(0)  # counters reset, no timing events
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    marker()
    t_start.record(stream)
    sim.step(steps)
    t_end.record(stream)
    marker()
    torch.cuda.synchronize()
    elapsed_ms = t_start.elapsed_time(t_end)
    cnt_a = sim.counters()
    leaf_updates = int(cnt_a["leaf_updates"])
    stats = [sim.stats(i) for i in range(sim.B)]
    # window B
    sim.profile(2)
    sim.step(steps)
    marker()
    torch.cuda.synchronize()
    cnt = sim.counters()
    sim.profile(0)
    q, rs, d = sim.q, precision, sim.dim
    launches = max(1, int(cnt["timed_launches"]))
    avg_ms = cnt["transport_ms"] / launches
    bytes_per_leaf = 2 * q * rs  # read q populations, write q (neighbour reads are cache reuse)
    bytes_per_launch = int(cnt["leaf_updates"]) * bytes_per_leaf / max(1, int(cnt["transport_launches"]))
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # whole step: the minimum fused step moves (2 + 2^d / (2^d - 1)) q s bytes per leaf
    step_bytes_per_leaf = (2.0 + 2.0 ** d / (2.0 ** d - 1.0)) * q * rs
    step_gbs = step_bytes_per_leaf * leaf_updates / (elapsed_ms * 1e-3) / 1e9
    finest = sum(1 << (sim.dim * int(c["jmax"])) for c, _ in items)
    leaves_now = sum(int(st["leaves"].sum()) for st in stats)
    by_n = {}
    for (c, _), st in zip(items, stats):
        J = int(c["jmax"])
        for l, k in enumerate(st["leaves"]):
            if k:
                by_n[J - l] = by_n.get(J - l, 0) + int(k)
    res = dict(value=leaf_updates / (elapsed_ms * 1e-3), ms_per_step=elapsed_ms / steps, steps=steps,
               warmup=warmup, leaf_updates=leaf_updates, transport_avg_launch_ms=avg_ms,
               transport_bytes_per_launch=bytes_per_launch, transport_gbs=achieved,
               transport_frac=achieved / HBM_PEAK_GBS,
               transport_leaf_updates_per_s=bytes_per_launch / bytes_per_leaf / (avg_ms * 1e-3),
               transport_launches=int(cnt["transport_launches"]), timed_launches=int(cnt["timed_launches"]),
               step_bytes_per_leaf=step_bytes_per_leaf, step_gbs=step_gbs, step_frac=step_gbs / HBM_PEAK_GBS,
               mean_leaves_per_step=leaf_updates / max(1, steps),
               compression_rate_final=1.0 - leaves_now / finest,
               compression_rate_mean=1.0 - leaf_updates / max(1, steps) / finest,
               mass_final=sum(st["mass"] for st in stats),
               tuning=tuning,
               transport_kernel=("k3_transport_collide" if d == 3 else
                                 "k_transport_collide_%s" % ("leaf" if tuning["transport_variant"] == 1 else "pop")),
               final_leaves_by_levels_above_finest={str(k): by_n[k] for k in sorted(by_n)})
    return res, sim, state0


def phase_breakdown(sim, steps):
    """Per-phase ms/step from kernel-by-kernel launches between HIP events
    (diagnostic; the graph-replayed timing above is the measurement)."""
    from paper_2103_02903_amd import mrlbm

    eager = mrlbm.Batch(sim.cfgs, precision=sim.precision)
    t = sim.tuning()
    eager.set_tuning(t["transport_variant"], t["list_grid_all"], t["list_grid_level"], graph=0)
    for i in range(sim.B):
        t, v = sim.get_state(i)
        eager.set_state(i, t, v)
    eager.profile(True)
    eager.step(steps)
    cnt = eager.counters()
    eager.close()
    return {"adapt": cnt["adapt_ms"] / steps, "reconstruct": cnt["reconstruct_ms"] / steps,
            "transport_collide": cnt["transport_ms"] / steps}


def ke_gradient(sim, region=(0.375, 0.625)):
    """Kinetic energy sum over leaves centred in region^2 of |C|/|C_J| |q|^2/(2 rho)
    (D2Q9, lambda = 1) and its gradient in the library's values layout."""
    import torch

    cells, vals = sim.leaves()
    cfg = sim.cfgs[0]
    jmin, J = int(cfg["jmin"]), int(cfg["jmax"])
    lv = (cells >> 26).long()
    c = (cells & ((1 << 26) - 1)).long()
    n = torch.ones_like(lv) << lv
    x, y = c & (n - 1), c >> lv
    cx, cy = (x.double() + 0.5) / n.double(), (y.double() + 0.5) / n.double()
    inside = ((cx >= region[0]) & (cx < region[1]) & (cy >= region[0]) & (cy < region[1])).double()
    vol = (torch.ones_like(lv) << (2 * (J - lv))).double() * inside
    ex = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=torch.float64, device=vals.device)
    ey = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=torch.float64, device=vals.device)
    f = vals.double()
    rho, qx, qy = f.sum(1), f @ ex, f @ ey
    q2 = qx * qx + qy * qy
    Jval = float(torch.sum(vol * 0.5 * q2 / rho))
    g = vol[:, None] * (-0.5 * (q2 / (rho * rho))[:, None] + (qx[:, None] * ex + qy[:, None] * ey) / rho[:, None])
    loff = [0] * (J + 2)
    for l in range(jmin, J + 1):
        loff[l + 1] = loff[l] + (1 << (2 * l))
    loff_t = torch.tensor(loff, dtype=torch.long, device=vals.device)
    idx = 9 * loff_t[lv][:, None] + torch.arange(9, device=vals.device)[None, :] * (n * n)[:, None] + c[:, None]
    abar = torch.zeros(9 * loff[J + 1], dtype=torch.float64, device=vals.device)
    abar[idx.reshape(-1)] = g.reshape(-1)
    return Jval, abar


def adjoint_run(nsteps: int, ckpt: int, precision: int):
    """Forward steps alone, then a recorded forward + checkpointed adjoint, of the
    256^2 vortex workload. Returns timings and the gradient."""
    import torch

    from paper_2103_02903_amd import mrlbm

    (cfg, m0), = workload("d2q9_vortex_256")[0]
    sim = mrlbm.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(nsteps)
    sim.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.init_equilibrium(m0)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.forward_record(nsteps, ckpt)
    sim.synchronize()
    t_rec = time.perf_counter() - t0
    Jval, abar = ke_gradient(sim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mbar, sbar = sim.adjoint(abar)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    sim.profile(True)  # leaf updates of one plain forward run for the rate
    sim.init_equilibrium(m0)
    sim.step(nsteps)
    leaf_updates = int(sim.counters()["leaf_updates"])
    sim.close()
    from paper_2103_02903_amd import workloads as W

    da = W.vortex_amplitude_gradient(cfg, mbar.double().cpu().numpy())
    return dict(t_forward=t_fwd, t_record=t_rec, t_adjoint=t_adj, J=Jval, mbar=mbar.double(), sbar=sbar,
                dJda=da.tolist(), leaf_updates=leaf_updates)


def finest_moments(sim, i):
    """Conserved moments (first nc rows of M f) of the finest-level reconstruction
    of instance i, float64 numpy [nc][N_J^d]."""
    f = sim.fields(i, "finest").double()
    if sim.q == 9:
        import torch

        ex = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=torch.float64, device=f.device)
        ey = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=torch.float64, device=f.device)
        lam = float(sim.cfgs[i].get("lam", 1.0))
        m = torch.stack([f.sum(0), lam * (ex @ f), lam * (ey @ f)])
    else:
        m = f.sum(0)[None]
    return m.cpu().numpy()


def field_errors(a, b, names):
    out = {}
    for k, n in enumerate(names):
        d = abs(a[k] - b[k])
        out[n] = dict(l1_rel=float(d.sum() / abs(b[k]).sum()), linf=float(d.max()))
    return out


def sample_instances(items):
    """One instance of each finest level of a batch (the first one)."""
    seen, out = set(), []
    for i, (c, _) in enumerate(items):
        if c["jmax"] not in seen:
            seen.add(c["jmax"])
            out.append(i)
    return out


def scope_row_workloads():
    """The method's variants beyond the periodic D2Q9 batch, each at a size that
    fills the GPU: (name, items, description, precision)."""
    from paper_2103_02903_amd import workloads as W

    def batch(**kw):
        items = W.shear_layer_batch(96)
        for c, _ in items:
            c.update(kw)
        return items

    walled = batch(bc=(0, 0, 2, 2))
    return [
        ("walls_bounce_back_batch96_fp32", walled,
         "the 96-instance shear-layer batch with bounce-back walls on the y sides (x periodic)", 4),
        ("gamma2_batch96_fp32", batch(gamma=2, mu_bar=1.0),
         "the 96-instance shear-layer batch with the prediction of half-width gamma = 2 (Table 1)", 4),
        ("gamma3_batch96_fp32", batch(gamma=3, mu_bar=1.0),
         "the 96-instance shear-layer batch with the prediction of half-width gamma = 3 (Table 1)", 4),
        ("l2_metric_batch96_fp32", batch(metric="l2"),
         "the 96-instance shear-layer batch with the l2 sibling metric", 4),
        ("euler_d2q4_riemann_1024_fp32", [W.riemann_d2q4e(jmin=3, jmax=10, eps=1e-3, seed=0)],
         "vectorial D2Q4 Euler scheme (lambda 5, copy walls), seeded two-dimensional Riemann problem, levels "
         "3..10 (1024^2 finest), eps 1e-3", 4),
        ("euler_d2q4_riemann_1024_fp64", [W.riemann_d2q4e(jmin=3, jmax=10, eps=1e-3, seed=0)],
         "the same Euler run in FP64", 8),
        ("d3q6_ball_256_fp32", [W.ball_d3q6()],
         "D3Q6 advection of a ball indicator (radius 0.15, periodic [-1, 1]^3, V = (0.3, 0.2, 0.1)), levels "
         "1..8 (256^3 finest), mu_bar 2, eps 1e-3, s = (1.4, 1)", 4),
        ("d3q6_ball_256_fp64", [W.ball_d3q6()], "the same 3D run in FP64", 8),
    ]


def scope_rows(args, only=None):
    """Leaf updates/s and the transport kernel's roofline fraction of each
    workload of scope_row_workloads (windows A and B as for the headline), or
    of the one named `only`."""
    out = {}
    for name, items, desc, prec in scope_row_workloads():
        if only is not None and name != only:
            continue
        # (alone, the windows get the copy-kernel markers the profile summaries use)
        r, sim, _ = timed_run(items, prec, args.scope_steps, args.scope_warmup, markers=only is not None)
        sim.close()
        out[name] = dict(workload=desc, value=r["value"], unit="leaf updates/s", ms_per_step=r["ms_per_step"],
                         mean_leaves_per_step=r["mean_leaves_per_step"],
                         compression_rate_mean=r["compression_rate_mean"],
                         transport_avg_launch_ms=r["transport_avg_launch_ms"],
                         transport_gbs=r["transport_gbs"], transport_frac=r["transport_frac"],
                         step_frac=r["step_frac"], launch_schedule=r["tuning"])
    return out


def variants(args, head):
    """The same batch in FP64, the single 1024^2 shear layer (plain FP64 and
    FP32), and the adjoint in both precisions, each measured on this GPU."""
    import torch

    out = {}
    items, desc, _ = workload("d2q9_shear_batch96")
    r64, s64, _ = timed_run(items, 8, args.steps, args.warmup)
    fin64 = {i: finest_moments(s64, i) for i in head.get("finest_check", {})}
    s64.close()
    r64["workload"] = desc
    r64["fp32_vs_fp64"] = head["value"] / r64["value"]
    r64["accuracy"] = dict(
        mass_rel=abs(head["mass_final"] - r64["mass_final"]) / abs(r64["mass_final"]),
        per_field_fp32_vs_fp64={"instance %d (J=%d)" % (i, items[i][0]["jmax"]):
                                field_errors(head["finest_check"][i], fin64[i], ("rho", "q_x", "q_y"))
                                for i in fin64},
        basis="finest-level reconstruction of the FP32 batch (the measured run) and of this FP64 batch after the "
              "same steps, one instance of each finest level; each precision decides its own meshes")
    out["batched_fp64"] = r64
    items, desc, _ = workload("d2q9_shear_1024")
    single, fin = {}, {}
    for prec in (8, 4):
        r, sm, _ = timed_run(items, prec, args.single_steps, args.single_warmup)
        fin[prec] = finest_moments(sm, 0)
        sm.close()
        r["workload"] = desc
        single[prec] = r
    single[8]["batched_fp32_vs_this"] = head["value"] / single[8]["value"]
    single[4]["fp32_vs_fp64"] = single[4]["value"] / single[8]["value"]
    single[4]["accuracy"] = dict(
        per_field_fp32_vs_fp64=field_errors(fin[4], fin[8], ("rho", "q_x", "q_y")),
        mass_rel=abs(single[4]["mass_final"] - single[8]["mass_final"]) / abs(single[8]["mass_final"]),
        basis="finest-level reconstruction of both runs after the same steps; each precision decides its own "
              "meshes; the FP64 path is the one the GPU tests replay against the FP64 oracle")
    out["single_fp64"] = single[8]
    out["single_fp32"] = single[4]
    a32 = adjoint_run(args.adjoint_steps, args.adjoint_ckpt, 4)
    a64 = adjoint_run(args.adjoint_steps, args.adjoint_ckpt, 8)
    for name, a in (("adjoint_fp32", a32), ("adjoint_fp64", a64)):
        grad_ms = (a["t_record"] + a["t_adjoint"]) * 1e3
        out[name] = dict(
            workload=workload("d2q9_vortex_256")[1] + "; %d steps, checkpoint every %d, gradient of the kinetic "
                     "energy in [3/8,5/8]^2 w.r.t. the initial moments, the relaxation rates and the 16 mode "
                     "amplitudes" %
                     (args.adjoint_steps, args.adjoint_ckpt),
            value=a["leaf_updates"] / ((a["t_record"] + a["t_adjoint"])),
            unit="forward leaf updates/s of the gradient computation (record + adjoint)",
            gradient_ms=grad_ms, forward_ms=a["t_forward"] * 1e3,
            gradient_over_forward=grad_ms / (a["t_forward"] * 1e3), J=a["J"],
            dJ_ds2=float(a["sbar"][7] + a["sbar"][8]), dJ_da=a["dJda"])
    rel = float(torch.max(torch.abs(a32["mbar"] - a64["mbar"])) / torch.max(torch.abs(a64["mbar"])))
    out["adjoint_fp32"]["accuracy"] = ("max |dJ/dm0 (FP32) - dJ/dm0 (FP64)| / max |dJ/dm0 (FP64)| = %.2e, each "
                                       "precision on the meshes it chose itself" % rel)
    out["adjoint_fp32"]["fp32_vs_fp64"] = out["adjoint_fp32"]["value"] / out["adjoint_fp64"]["value"]
    # the same gradient with one segment: the recorded forward tapes every step
    # (about 4.3 MB per step here) and the adjoint recomputes nothing
    at = adjoint_run(args.adjoint_steps, args.adjoint_steps, 4)
    grad_ms = (at["t_record"] + at["t_adjoint"]) * 1e3
    out["adjoint_fp32_taped"] = dict(
        workload="as adjoint_fp32, with one checkpoint: every step taped during the recorded forward",
        value=at["leaf_updates"] / (at["t_record"] + at["t_adjoint"]),
        unit="forward leaf updates/s of the gradient computation (record + adjoint)",
        gradient_ms=grad_ms, forward_ms=at["t_forward"] * 1e3, gradient_over_forward=grad_ms / (at["t_forward"] * 1e3),
        vs_checkpointed=float(torch.max(torch.abs(at["mbar"] - a32["mbar"])) / torch.max(torch.abs(a32["mbar"]))))
    out["scope_rows"] = scope_rows(args)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="d2q9_shear_batch96")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 4, 8], help="0: the workload's default")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--single-steps", type=int, default=1000)
    ap.add_argument("--single-warmup", type=int, default=100)
    ap.add_argument("--adjoint-steps", type=int, default=800)
    ap.add_argument("--adjoint-ckpt", type=int, default=50)
    ap.add_argument("--scope-steps", type=int, default=100)
    ap.add_argument("--scope-warmup", type=int, default=30)
    ap.add_argument("--scope-only", nargs="?", const="all", default="",
                    help="only the walls, gamma, l2-metric and Euler workloads, or the one named (kernel traces)")
    ap.add_argument("--schedule", default="",
                    help="transport variant,all-level cap,per-level cap[,graph 1|0[,pair links 0|1]] (skips "
                         "autotuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy kernel on %d bytes (counter calibration)" % COPY_BYTES)
    ap.add_argument("--adjoint-only", type=int, default=0, choices=[0, 4, 8],
                    help="only the adjoint leg in this precision (for a kernel trace of the adjoint kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single GPU (instances of a batch are "
              "independent; a multi-GPU run would give each GPU its own batch); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2103_02903_amd import mrlbm

    if not os.path.exists(mrlbm.LIB_PATH):
        from paper_2103_02903_amd import build as hip_build

        hip_build.build(force=False)
    if args.copy_calibration:
        print(json.dumps({"copy_kernel": "k_copy_u4", **copy_bandwidth()}))
        return
    if args.scope_only:
        print(json.dumps(scope_rows(args, None if args.scope_only == "all" else args.scope_only)))
        return
    if args.adjoint_only:
        a = adjoint_run(args.adjoint_steps, args.adjoint_ckpt, args.adjoint_only)
        print(json.dumps({k: a[k] for k in ("t_forward", "t_record", "t_adjoint", "J", "leaf_updates")}))
        return
    items, desc, prec = workload(args.workload)
    precision = args.precision or prec
    # the CPU baseline steps the largest instance from its state at the start of the timed region
    big = max(range(len(items)), key=lambda i: items[i][0]["jmax"])
    schedule = tuple(int(v) for v in args.schedule.split(",")) if args.schedule else None
    head, sim, state0 = timed_run(items, precision, args.steps, args.warmup,
                                  None if args.no_cpu_baseline else big, schedule=schedule, markers=True)
    check = sample_instances(items)
    head["finest_check"] = {i: finest_moments(sim, i) for i in check}
    phases = phase_breakdown(sim, min(args.steps, 100))
    sim.close()
    copy = copy_bandwidth()
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "leaf updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "precision": "fp%d" % (8 * precision),
                   "instances": len(items)},
        "roofline": {
            "kernel": head["transport_kernel"],
            "bound": "hbm",
            "achieved": head["transport_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": head["transport_frac"],
            "traffic": measured_traffic(args.workload, precision, head["transport_kernel"]),
            "algorithmic_bytes_per_launch": head["transport_bytes_per_launch"],
            "avg_launch_ms": head["transport_avg_launch_ms"],
            "launches": head["transport_launches"],
            "event_timed_launches": head["timed_launches"],
            "window": "second window of --steps graph steps after the measured one, every transport launch "
                      "bracketed by HIP events in the step graph",
            "step": {"bytes_per_leaf": head["step_bytes_per_leaf"], "achieved": head["step_gbs"],
                     "frac": head["step_frac"], "unit": "GB/s",
                     "basis": "minimum fused step (2 + 2^d/(2^d-1)) q s bytes per leaf update, times the leaf "
                              "updates of the measured window, over its wall time"},
        },
        "copy_reference": {"kernel": "k_copy_u4", "gbs": copy["gbs"], "frac": copy["gbs"] / HBM_PEAK_GBS},
        "mean_leaves_per_step": head["mean_leaves_per_step"],
        "compression_rate_final": head["compression_rate_final"],
        "compression_rate_mean": head["compression_rate_mean"],
        "transport_kernel_leaf_updates_per_s": head["transport_leaf_updates_per_s"],
        "phase_ms_per_step_eager": phases,
        "mass_final": head["mass_final"],
        "launch_schedule": head["tuning"],
        "final_leaves_by_levels_above_finest": head["final_leaves_by_levels_above_finest"],
    }
    if not args.no_variants and args.workload == "d2q9_shear_batch96" and precision == 4:
        out["variants"] = variants(args, head)
    if state0 is not None:
        out["cpu_baseline"] = cpu_baseline(items[big][0], state0[0], state0[1], args.cpu_seconds)
        if len(items) > 1:
            out["cpu_baseline"]["sample"] += " (instance %d of %d, levels %d..%d)" % (
                big, len(items), items[big][0]["jmin"], items[big][0]["jmax"])
    head.pop("finest_check", None)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
