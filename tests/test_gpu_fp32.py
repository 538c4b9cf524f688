"""FP32 path of the HIP library against the oracle.

The mesh is decided by floating-point comparisons, so both sides take it in the
kernel's precision: the oracle's single-precision decision (same expressions,
same order, thresholds rounded to float) must give the GPU's mesh bit for bit.
Fields are compared with the FP64 oracle step taken from the same (upcast)
state on that mesh, to a tolerance derived from float rounding; the FP32
decisions are also compared with the FP64 ones (epsilon-consistency), and the
per-field error of free FP32 runs against FP64 runs is reported.
"""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

from test_gpu_parity import _cfg, leaf_err

pytestmark = pytest.mark.gpu

# One FP32 step: the E - A transport sum has at most 25 + 32 terms whose weights
# are at most a few times 2^{(d-1) n}, scaled back by 2^{-d n}, and the collision
# some twenty operations, each rounding at 2^-24 relative: well below 1e-5.
TOL32 = 1e-5


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


CASES = [("D1Q2", 2, 10, 1e-4, 0), ("D1Q3", 2, 10, 1e-4, 1), ("D2Q9", 2, 7, 1e-3, 3), ("D2Q9", 3, 8, 1e-4, 4)]


@pytest.mark.parametrize("scheme,jmin,jmax,eps,seed", CASES)
def test_fp32_step_replay(mr, scheme, jmin, jmax, eps, seed):
    cfg = _cfg(scheme, jmin, jmax, eps)
    m0 = W.random_field(cfg, seed, "jump")
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=4)
    sim.init_equilibrium(m0)
    for k in range(10):
        tg, vg = sim.get_state()
        tnew = o.new_tree_f32(tg, vg)
        t_o, v_o = tg.copy(), vg.astype(np.float64)
        o.step_frozen(t_o, tnew, v_o)
        sim.step(1)
        tg2, vg2 = sim.get_state()
        assert np.array_equal(tg2, tnew), "FP32 mesh differs at step %d" % k
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= TOL32, "FP32 field error %g at step %d" % (e, k)


def test_fp32_decisions_epsilon_consistent(mr):
    """FP32 versus FP64 mesh decisions on the same state: every group whose keep
    or refine decision differs has its FP64 metric within a few float ulps of the
    threshold (tau = 64 * 2^-24 * max|f|)."""
    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=8, eps=1e-4, re=1000.0, width=1.0 / 40)
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=4)
    sim.init_equilibrium(m0)
    mism, worst = 0, 0.0
    d = o.dim
    for k in range(30):
        tg, vg = sim.get_state()
        _, D32 = o.new_tree_f32(tg, vg, return_details=True)
        D64 = o.details(tg, o.reconstruct(tg, vg.astype(np.float64)))
        tau = 64 * 2.0 ** -24 * float(np.max(np.abs(vg)))
        for l in range(o.jmin + 1, o.jmax + 1):
            sl = slice(o.level_offset(l - 1), o.level_offset(l - 1) + o.ncells(l - 1))
            a, b = D32[sl], D64[sl]
            has = b >= 0
            epsl = np.ldexp(cfg["eps"], d * (l - o.jmax))
            refl = np.ldexp(epsl, d) * 2.0 ** cfg["mu_bar"]
            for thr in (epsl, refl):
                diff = has & ((a >= np.float32(thr)) != (b >= thr))
                mism += int(diff.sum())
                if diff.any():
                    margin = np.abs(b[diff] - thr)
                    worst = max(worst, float(margin.max()) / tau)
                    assert np.all(margin <= tau)
        sim.step(1)
    print("FP32/FP64 decision mismatches over 30 steps: %d, worst margin %.3g tau" % (mism, worst))


def _moments_finest(o, tree, values):
    recon = o.finest(tree, values.astype(np.float64)).reshape(o.q, -1)
    return o.moment_matrix() @ recon


@pytest.mark.parametrize("case", ["d1q3_burgers", "d2q9_shear"])
def test_fp32_vs_fp64_per_field_error(mr, case):
    """Free FP32 and FP64 GPU runs from the same initial data: relative L1 and
    max errors of each conserved field of the finest reconstruction."""
    if case == "d1q3_burgers":
        cfg, m0 = W.burgers_d1q3(jmax=12)
        steps, names = 1500, ["u"]
    else:
        cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=8, eps=1e-3, re=2000.0, width=1.0 / 40)
        steps, names = 400, ["rho", "q_x", "q_y"]
    o = oracle.Oracle(cfg)
    runs = {}
    for prec in (8, 4):
        sim = mr.Sim(cfg, precision=prec)
        sim.init_equilibrium(m0)
        sim.step(steps)
        runs[prec] = _moments_finest(o, *sim.get_state())
    report = {}
    for k, name in enumerate(names):
        a, b = runs[4][k], runs[8][k]
        l1 = float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))
        linf = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        report[name] = (l1, linf)
        assert l1 < 1e-3 and linf < 1e-2, (name, l1, linf)
    print(case, "FP32 vs FP64 (L1 rel, Linf rel):", report)
