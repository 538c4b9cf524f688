"""The vectorial D2Q4 scheme of the Euler system on the GPU (through the
C-ABI) against the oracle: one-step replays on a seeded two-dimensional
Riemann problem with the paper's copy walls and on the periodic box, FP64
(mesh bit for bit, leaf values within 1e-12 relative) and FP32 (the oracle's
float mesh decision, then its FP64 step from the upcast state); the leaf
moments and the finest-level reconstruction; the uniform limit; the adjoint
refuses the scheme.
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


CASES = [(2, 7, 1e-3, "copy", 0, 12), (3, 8, 1e-3, "copy", 1, 8), (2, 7, 1e-2, "periodic", 2, 12)]


@pytest.mark.parametrize("jmin,jmax,eps,bc,seed,steps", CASES)
@pytest.mark.parametrize("precision", [8, 4])
def test_euler_step_replay(mr, jmin, jmax, eps, bc, seed, steps, precision):
    cfg, m0 = W.riemann_d2q4e(jmin=jmin, jmax=jmax, eps=eps, seed=seed, bc=bc)
    print("euler", jmin, jmax, eps, bc, "precision", precision, flush=True)
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    t0, v0 = o.init(m0)
    tg, vg = sim.get_state()
    assert np.array_equal(tg, t0) and leaf_err(o, t0, vg, v0) <= (TOL64 if precision == 8 else TOL32)
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
        e = leaf_err(o, t_o, vg2, v_o)
        assert e <= (TOL64 if precision == 8 else TOL32), "field error %g at step %d" % (e, k + 1)
        levels |= {l for l, c in enumerate(o.leaf_counts(tg2)) if c}
    assert len(levels) >= 3
    tg, vg = sim.get_state()
    v64 = vg.astype(np.float64)
    # leaf moments m = M f (block D2Q4 matrix) and the finest-level reconstruction
    pops = sim.fields("populations").cpu().numpy().astype(np.float64)
    mom = sim.fields("moments").cpu().numpy().astype(np.float64)
    want = pops @ o.moment_matrix().T
    assert np.max(np.abs(mom - want) / np.maximum(1.0, np.abs(want))) <= (1e-13 if precision == 8 else 2e-6)
    if precision == 8:
        assert np.array_equal(sim.fields("finest").cpu().numpy(), o.finest(tg, v64).reshape(o.q, -1))
    sim.close()


def test_euler_uniform_limit(mr):
    J = 6
    cfg, m0 = W.riemann_d2q4e(jmin=J, jmax=J, eps=1e-3, seed=4)
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=8)
    sim.init_equilibrium(m0)
    t, v = o.init(m0)
    fJ = o.values_level(v, J).reshape(-1).copy()
    for _ in range(20):
        sim.step(1)
        o.uniform_step(fJ)
    _, vg = sim.get_state()
    g = o.values_level(vg, J).reshape(-1)
    # the GPU applies M^-1 in the closed form of the orthogonal D2Q4 rows, the
    # oracle a Gauss-Jordan inverse: equal in exact arithmetic
    assert np.max(np.abs(g - fJ) / np.maximum(1.0, np.abs(fJ))) <= 1e-13
    sim.close()


def test_euler_refuses_adjoint(mr):
    cfg, m0 = W.riemann_d2q4e(jmin=2, jmax=5, bc="periodic")
    sim = mr.Sim(cfg)
    sim.init_equilibrium(m0)
    with pytest.raises(mr.MrlbmError) as e:
        sim.forward_record(4, 2)
    assert e.value.status == -1
    sim.close()
