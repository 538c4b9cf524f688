"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (graph-replayed steps with the autotuned schedule).

After free GPU steps, the GPU state of selected instances is handed to the
oracle, both advance one step, and the meshes must agree bit for bit and the
leaf values to the tolerance of the precision (1e-12 in FP64; in FP32 the
oracle takes the mesh decision in float and the FP64 step from the upcast
state, tolerance 1e-5). The adjoint is checked on the 256^2 workload against
the oracle's frozen-mesh gradient on the GPU's own mesh sequence.
"""
import numpy as np
import pytest

import oracle
from adjoint_helpers import ke_functional
from ghost_sets import ghost_sets
from paper_2103_02903_amd import workloads as W

from test_gpu_parity import TOL64, leaf_err

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


def test_batch96_fp32_step_replay(mr):
    """96 D2Q9 shear layers (finest levels 7..10) in FP32, as benchmarked: two
    instances of each finest level replayed on the oracle."""
    items = W.shear_layer_batch(96)
    b = mr.Batch([c for c, _ in items], precision=4)
    for i, (_, m0) in enumerate(items):
        b.init_equilibrium(i, m0)
    b.step(40)
    b.autotune(reps=2)
    b.step(10)
    chosen = []
    for J in (7, 8, 9, 10):
        chosen += [i for i, (c, _) in enumerate(items) if c["jmax"] == J][:2]
    expect = {}
    for i in chosen:
        cfg = items[i][0]
        o = oracle.Oracle(cfg)
        tg, vg = b.get_state(i)
        tnew = o.new_tree_f32(tg, vg)
        t_o, v_o = tg.copy(), vg.astype(np.float64)
        o.step_frozen(t_o, tnew, v_o)
        expect[i] = (o, tnew, t_o, v_o)
    b.step(1)
    for i in chosen:
        o, tnew, t_o, v_o = expect[i]
        tg2, vg2 = b.get_state(i)
        print("instance", i, "J", items[i][0]["jmax"], "leaves", int(o.leaf_counts(tg2).sum()), flush=True)
        assert np.array_equal(tg2, tnew), "FP32 mesh of instance %d differs" % i
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= TOL32, "FP32 field error %g on instance %d" % (e, i)
        G = ghost_sets(o, tg2)
        want = np.array([int(G[l].sum()) if l in G else 0 for l in range(o.jmax + 1)])
        assert np.array_equal(b.stats(i)["ghosts"], want), "ghost counts of instance %d" % i
    b.close()


def test_shear_1024_fp64_step_replay(mr):
    """The 1024^2 double shear layer (levels 3..10) in FP64."""
    cfg, m0 = W.shear_layer_d2q9()
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=8)
    sim.init_equilibrium(m0)
    sim.step(80)
    sim.autotune(reps=2)
    sim.step(20)
    for k in range(2):
        tg, vg = sim.get_state()
        t_o, v_o = tg.copy(), vg.copy()
        o.step(t_o, v_o)
        sim.step(1)
        tg2, vg2 = sim.get_state()
        assert np.array_equal(tg2, t_o), "mesh differs at replay %d" % k
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= TOL64, "field error %g at replay %d" % (e, k)
    sim.close()


def test_burgers_16384_fp64_4000_steps(mr):
    """D1Q3 Burgers on levels 2..14 (16384 finest cells) for 4000 steps, with a
    one-step replay every 500 steps (shocks form along the way)."""
    cfg, m0 = W.burgers_d1q3()
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=8)
    sim.init_equilibrium(m0)
    sim.step(10)
    sim.autotune(reps=2)
    done = 10
    while done < 4000:
        sim.step(499)
        done += 499
        tg, vg = sim.get_state()
        t_o, v_o = tg.copy(), vg.copy()
        o.step(t_o, v_o)
        sim.step(1)
        done += 1
        tg2, vg2 = sim.get_state()
        assert np.array_equal(tg2, t_o), "mesh differs at step %d" % done
        assert leaf_err(o, t_o, vg2, v_o) <= TOL64
    st = sim.stats()  # the datum has zero mean: mass conserved to round-off in absolute terms
    assert abs(st["mass"] - o.mass(*o.init(m0))) <= 1e-10
    sim.close()


def test_vortex_256_fp32_adjoint_vs_oracle(mr):
    """The adjoint workload (D2Q9 on levels 3..8, 256^2 finest) in FP32 with a
    checkpoint every 50 steps: 120 steps (three segments, the last one ragged)
    against the oracle's FP64 frozen-mesh gradient on the GPU's meshes."""
    import torch

    cfg, m0 = W.random_vortex_d2q9()
    nsteps, K = 120, 50
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=4)
    sim.init_equilibrium(m0)
    trees = [sim.get_state()[0]]
    for _ in range(nsteps):
        sim.step(1)
        trees.append(sim.get_state()[0])
    sim.close()
    sim = mr.Sim(cfg, precision=4)
    sim.init_equilibrium(m0)
    sim.forward_record(nsteps, K)
    t_fin, v_fin = sim.get_state()
    assert np.array_equal(t_fin, trees[-1])
    _, abar = ke_functional(o, t_fin, v_fin.astype(np.float64))
    mbar_g, sbar_g = sim.adjoint(torch.from_numpy(abar).to(sim.device))
    mbar_o, sbar_o = o.gradient_frozen(m0, trees, abar)
    mbar_g = mbar_g.double().cpu().numpy()
    rel = float(np.max(np.abs(mbar_g - mbar_o))) / float(np.max(np.abs(mbar_o)))
    print("adjoint FP32 vs FP64 oracle, max-norm relative", rel, flush=True)
    assert rel <= 1e-3
    rs = abs(sbar_g[7] + sbar_g[8] - sbar_o[7] - sbar_o[8]) / abs(sbar_o[7] + sbar_o[8])
    assert rs <= 1e-3
    sim.close()
