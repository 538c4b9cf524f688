"""Per-field error of the GPU paths against the FP64 oracle's own free-running
trajectory, at the full sizes of the workloads (a measurement script, not
collected by pytest).

The fields are the conserved moments (D2Q9: rho, q_x, q_y; D1Q3: all three
moments u, m1, m2) of the finest-level reconstruction (the double-hat operator
of section "Mesh coarsening") after the same number of steps. Each run decides
its own meshes. Errors: L1-relative sum |a - b| / sum |b| over the finest grid
(the error metric of the numerical experiments), and the max norm |a - b|.

  python tests/fullsize_accuracy.py gpu CONFIG OUT.npz       (on a GPU)
  python tests/fullsize_accuracy.py oracle CONFIG OUT.npz    (on the host)
  python tests/fullsize_accuracy.py compare CONFIG GPU.npz ORACLE.npz

CONFIG: c2 (D1Q3 Burgers, levels 2..14, 4000 steps), c3 (D2Q9 double shear
layer, levels 3..10, 5000 steps) or c4 (the 96-instance batch, 1000 steps; one
instance of each finest level is compared).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2103_02903_amd import workloads as W  # noqa: E402


def _items(config):
    """(list of (cfg, m0), steps, indices compared, field names)."""
    if config == "c2":
        return [W.burgers_d1q3()], 4000, [0], ("u", "m1", "m2")
    if config == "c3":
        return [W.shear_layer_d2q9()], 5000, [0], ("rho", "q_x", "q_y")
    if config == "c4":
        items = W.shear_layer_batch(96)
        seen, idx = set(), []
        for i, (c, _) in enumerate(items):
            if c["jmax"] not in seen:
                seen.add(c["jmax"])
                idx.append(i)
        return items, 1000, idx, ("rho", "q_x", "q_y")
    raise SystemExit("unknown config %s" % config)


def gpu_fields(config, out):
    import torch

    from paper_2103_02903_amd import mrlbm

    items, steps, idx, names = _items(config)
    res = {}
    for prec in (4, 8):
        b = mrlbm.Batch([c for c, _ in items], precision=prec)
        for i, (_, m0) in enumerate(items):
            b.init_equilibrium(i, m0)
        t0 = time.time()
        b.step(steps)
        b.synchronize()
        print("%s fp%d: %d steps in %.2f s" % (config, 8 * prec, steps, time.time() - t0), flush=True)
        nc = len(names)
        for i in idx:
            f = b.fields(i, "finest").double()
            M = torch.as_tensor(_moment_matrix(items[i][0]), dtype=torch.float64, device=f.device)
            m = (M[:nc] @ f).cpu().numpy()
            res["fp%d_%d" % (8 * prec, i)] = m.astype(np.float32 if prec == 4 else np.float64)
            res["leaves_fp%d_%d" % (8 * prec, i)] = np.int64(b.stats(i)["leaves"].sum())
        b.close()
    np.savez(out, **res)


def _moment_matrix(cfg):
    """The scheme's moment matrix, from the oracle (the same M the library uses)."""
    import oracle

    return oracle.Oracle(cfg).moment_matrix()


def oracle_fields(config, out):
    import oracle

    items, steps, idx, names = _items(config)
    res = {}
    nc = len(names)
    for i in idx:
        cfg, m0 = items[i]
        o = oracle.Oracle(cfg)
        t, v = o.init(m0)
        t0 = time.time()
        o.step(t, v, steps)
        print("%s oracle instance %d: %d steps in %.1f s (%d threads)" % (config, i, steps, time.time() - t0,
                                                                          oracle.threads()), flush=True)
        f = o.finest(t, v).reshape(o.q, -1)
        res["fp64_%d" % i] = (o.moment_matrix()[:nc] @ f)
        res["leaves_%d" % i] = np.int64(o.leaf_counts(t).sum())
        np.savez(out, **res)


def compare(config, gpu_npz, oracle_npz):
    items, steps, idx, names = _items(config)
    g, o = np.load(gpu_npz), np.load(oracle_npz)
    table = []
    for i in idx:
        ref = o["fp64_%d" % i]
        cfg = items[i][0]
        for prec in ("fp32", "fp64"):
            a = g["%s_%d" % (prec, i)].astype(np.float64)
            row = dict(config=config, instance=i, jmax=int(cfg["jmax"]), eps=float(cfg["eps"]), steps=steps,
                       precision=prec, leaves_gpu=int(g["leaves_%s_%d" % (prec, i)]),
                       leaves_oracle=int(o["leaves_%d" % i]))
            for k, n in enumerate(names):
                d = np.abs(a[k] - ref[k])
                row[n] = dict(l1_rel=float(d.sum() / np.abs(ref[k]).sum()), linf=float(d.max()))
            table.append(row)
    print(json.dumps(table, indent=1))
    return table


if __name__ == "__main__":
    mode, config = sys.argv[1], sys.argv[2]
    if mode == "gpu":
        gpu_fields(config, sys.argv[3])
    elif mode == "oracle":
        oracle_fields(config, sys.argv[3])
    elif mode == "compare":
        compare(config, sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
