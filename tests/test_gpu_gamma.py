"""Predictions of half-width gamma = 2 and 3 (Table 1) and the l2 sibling metric
(footnote of section "Mesh coarsening") on the GPU, through the C-ABI, against
the oracle.

One-step replays as in test_gpu_parity: from the GPU state before a step, the
oracle's step (FP64; FP32: the oracle's float mesh decision, then its FP64 step
from the upcast state) must give the GPU's mesh bit for bit and its leaf values
within 1e-12 (FP64) or 1e-5 (FP32) relative. gamma > 1 runs every leaf through
the library's general transport path (tables over the box of half-width
2 gamma); the l2 metric with gamma = 1 keeps the fast kernels. The finest-level
reconstruction (the gamma-wide prediction applied level by level) equals the
oracle's.
"""
import numpy as np
import pytest

import oracle
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


def _cfg(scheme, jmin, jmax, eps, bc, gamma, metric, mu_bar=1.0):
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=mu_bar, eq_param=0.5 if scheme == "D1Q3" else 1.0, bc=bc,
                    gamma=gamma, metric=metric)


CASES = [
    # scheme, jmin, jmax, eps, sides, gamma, metric, seed, steps
    ("D1Q2", 2, 10, 1e-4, ("periodic",) * 2, 2, "linf", 1, 24),
    ("D1Q3", 2, 10, 1e-4, ("periodic",) * 2, 3, "l2", 2, 24),
    ("D1Q3", 3, 10, 1e-4, ("bounce_back", "anti_bounce_back"), 3, "linf", 3, 20),
    ("D1Q2", 2, 9, 1e-4, ("copy", "copy"), 2, "l2", 4, 20),
    ("D2Q9", 3, 7, 1e-3, ("periodic",) * 4, 2, "linf", 5, 10),
    ("D2Q9", 3, 7, 1e-3, ("periodic",) * 4, 3, "l2", 6, 8),
    ("D2Q9", 3, 7, 1e-3, ("bounce_back",) * 4, 2, "l2", 7, 10),
    ("D2Q9", 3, 7, 1e-3, ("copy", "copy", "bounce_back", "bounce_back"), 3, "linf", 8, 8),
    ("D2Q9", 3, 7, 3e-3, ("periodic",) * 4, 1, "l2", 9, 12),
    ("D1Q3", 2, 10, 1e-4, ("copy", "bounce_back"), 1, "l2", 10, 20),
]


@pytest.mark.parametrize("scheme,jmin,jmax,eps,sides,gamma,metric,seed,steps", CASES)
@pytest.mark.parametrize("precision", [8, 4])
def test_gamma_step_replay(mr, scheme, jmin, jmax, eps, sides, gamma, metric, seed, steps, precision):
    cfg = _cfg(scheme, jmin, jmax, eps, sides, gamma, metric)
    print("gamma", gamma, metric, scheme, jmin, jmax, sides, "precision", precision, flush=True)
    o = oracle.Oracle(cfg)
    m0 = W.random_field(cfg, seed, "jump")
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    t0, v0 = o.init(m0) if precision == 8 else (None, None)
    if precision == 8:
        tg, vg = sim.get_state()
        assert np.array_equal(tg, t0) and leaf_err(o, t0, vg, v0) <= TOL64
    levels = set()
    for k in range(steps):
        tg, vg = sim.get_state()
        t_o, v_o = tg.copy(), vg.astype(np.float64)
        if precision == 8:
            o.step(t_o, v_o)
        else:
            o.step_frozen(t_o, o.new_tree_f32(tg, vg), v_o)
        sim.step(1)
        tg2, vg2 = sim.get_state()
        assert np.array_equal(tg2, t_o), "mesh differs at step %d" % (k + 1)
        assert o.check_tree(tg2) == 0
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= (TOL64 if precision == 8 else TOL32), "field error %g at step %d" % (e, k + 1)
        levels |= {l for l, c in enumerate(o.leaf_counts(tg2)) if c}
    assert len(levels) >= 3
    if precision == 8:
        fin = sim.fields("finest").cpu().numpy()
        tg, vg = sim.get_state()
        assert np.array_equal(fin, o.finest(tg, vg).reshape(o.q, -1))
    sim.close()


@pytest.mark.parametrize("gamma", [2, 3])
@pytest.mark.parametrize("precision", [8, 4])
def test_gamma_euler_step_replay(mr, gamma, precision):
    cfg, m0 = W.riemann_d2q4e(jmin=3, jmax=7, eps=1e-3, seed=gamma, bc="copy", gamma=gamma, metric="l2")
    print("gamma euler", gamma, "precision", precision, flush=True)
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    for k in range(6):
        tg, vg = sim.get_state()
        t_o, v_o = tg.copy(), vg.astype(np.float64)
        if precision == 8:
            o.step(t_o, v_o)
        else:
            o.step_frozen(t_o, o.new_tree_f32(tg, vg), v_o)
        sim.step(1)
        tg2, vg2 = sim.get_state()
        assert np.array_equal(tg2, t_o), "mesh differs at step %d" % (k + 1)
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= (TOL64 if precision == 8 else TOL32), "field error %g at step %d" % (e, k + 1)
    sim.close()


def test_gamma_batch_of_instances(mr):
    """A batch shares gamma; each instance keeps its own metric, threshold and
    walls, and every instance's step replays on the oracle."""
    cfgs = [_cfg("D2Q9", 3, 7, 1e-3, ("periodic",) * 4, 2, "linf"),
            _cfg("D2Q9", 3, 6, 3e-3, ("bounce_back",) * 4, 2, "l2"),
            _cfg("D2Q9", 3, 7, 1e-3, ("copy", "copy", "periodic", "periodic"), 2, "l2")]
    bat = mr.Batch(cfgs, precision=8)
    for i, c in enumerate(cfgs):
        bat.init_equilibrium(i, W.random_field(c, 20 + i, "jump"))
    oracles = [oracle.Oracle(c) for c in cfgs]
    for k in range(5):
        pre = [bat.get_state(i) for i in range(len(cfgs))]
        bat.step(1)
        for i, o in enumerate(oracles):
            t_o, v_o = pre[i][0].copy(), pre[i][1].astype(np.float64)
            o.step(t_o, v_o)
            tg, vg = bat.get_state(i)
            assert np.array_equal(tg, t_o), "instance %d mesh differs at step %d" % (i, k)
            assert leaf_err(o, t_o, vg, v_o) <= TOL64
    bat.close()


@pytest.mark.parametrize("gamma", [2, 3])
def test_gamma_ghost_sets_match_definition(mr, gamma):
    """Per-level ghost counts of the wide classification equal the host sets
    built from the definition with the boxes of half-width 2 gamma and gamma."""
    from ghost_sets import ghost_sets

    cfgs = [_cfg("D2Q9", 3, 7, 1e-3, ("periodic",) * 4, gamma, "linf"),
            _cfg("D2Q9", 3, 8, 1e-3, ("periodic",) * 4, gamma, "l2"),
            _cfg("D2Q9", 3, 6, 1e-2, ("periodic",) * 4, gamma, "linf")]
    bat = mr.Batch(cfgs, precision=8)
    for i, c in enumerate(cfgs):
        bat.init_equilibrium(i, W.random_field(c, 40 + i, "jump"))
    oracles = [oracle.Oracle(c) for c in cfgs]
    seen = 0
    for k in range(3):
        bat.step(2)
        for i, o in enumerate(oracles):
            tree, _ = bat.get_state(i)
            G = ghost_sets(o, tree, gamma)
            want = np.array([int(G[l].sum()) if l in G else 0 for l in range(o.jmax + 1)])
            got = bat.stats(i)["ghosts"]
            assert np.array_equal(got, want), "instance %d after %d steps: %s vs %s" % (i, 2 * k + 2, got, want)
            seen += int(want.sum())
    assert seen > 0
    bat.close()


def test_gamma_refuses_adjoint(mr):
    cfg = _cfg("D2Q9", 2, 5, 1e-3, ("periodic",) * 4, 2, "linf")
    sim = mr.Sim(cfg)
    sim.init_equilibrium(W.random_field(cfg, 1))
    with pytest.raises(mr.MrlbmError) as e:
        sim.forward_record(4, 2)
    assert e.value.status == -1
    sim.close()
