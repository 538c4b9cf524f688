"""C-ABI outputs and replay mode on the GPU, against the oracle.

* ``mrlbm_fields``: the leaf table and leaf populations equal the state; the
  leaf moments equal M f of the oracle's moment matrix; the finest-level
  reconstruction (double-hat operator of section "Mesh coarsening") equals the
  oracle's dense reconstruction bit for bit (both evaluate the same projection
  and prediction expressions in the same order).
* ``mrlbm_step_frozen``: a run that replays a recorded mesh sequence gives the
  recorded run's bits, and one frozen step matches the oracle's frozen step.
* Failure flags: a non-finite leaf is reported by ``mrlbm_stats``; a paired
  launch whose wait is made to give up (test hook: tiny spin budget and a
  counter that cannot be reached) is reported as MRLBM_ERR_SYNC by the next
  synchronising call, while every kernel runs to its end.
"""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

from test_gpu_parity import TOL64, _cfg, _leaf_entries, leaf_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


FIELD_CASES = [("D1Q3", 2, 10, 1e-4, 1, 8), ("D2Q9", 2, 7, 1e-3, 3, 8), ("D2Q9", 3, 8, 1e-4, 4, 4),
               ("D1Q2", 2, 9, 1e-4, 0, 4)]


@pytest.mark.parametrize("scheme,jmin,jmax,eps,seed,precision", FIELD_CASES)
def test_fields_match_oracle(mr, scheme, jmin, jmax, eps, seed, precision):
    cfg = _cfg(scheme, jmin, jmax, eps)
    m0 = W.random_field(cfg, seed, "jump")
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    sim.step(7)
    tree, vals = sim.get_state()
    v64 = vals.astype(np.float64)
    print(scheme, "precision", precision, "leaves", int(o.leaf_counts(tree).sum()), flush=True)
    # leaf table and populations, in (level, cell) order
    table = sim.fields("leaf_table").cpu().numpy().astype(np.uint32)
    pops = sim.fields("populations").cpu().numpy()
    lv, cell = table >> 26, table & ((1 << 26) - 1)
    want_l, want_c = [], []
    for l in range(o.jmin, o.jmax + 1):
        idx = np.flatnonzero(o.leaf_mask(tree, l).ravel())
        want_l.append(np.full(idx.size, l))
        want_c.append(idx)
    assert np.array_equal(lv, np.concatenate(want_l)) and np.array_equal(cell, np.concatenate(want_c))
    for l in range(o.jmin, o.jmax + 1):
        sel = lv == l
        want = o.values_level(vals, l).reshape(o.q, -1)[:, cell[sel]].T
        assert np.array_equal(pops[sel], want)
    # moments m = M f on every leaf
    mom = sim.fields("moments").cpu().numpy().astype(np.float64)
    want = pops.astype(np.float64) @ o.moment_matrix().T
    tol = 1e-13 if precision == 8 else 2e-6
    assert np.max(np.abs(mom - want) / np.maximum(1.0, np.abs(want))) <= tol
    # finest-level reconstruction
    fin = sim.fields("finest").cpu().numpy()
    if precision == 8:
        ref = o.finest(tree, v64).reshape(o.q, -1)
        print("finest max |gpu - oracle|", float(np.max(np.abs(fin - ref))), flush=True)
        assert np.array_equal(fin, ref)
    else:
        ref = o.finest(tree, v64).reshape(o.q, -1)
        # float evaluation of the same operators: a few roundings per level
        err = float(np.max(np.abs(fin.astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))))
        print("finest FP32 vs FP64 oracle", err, flush=True)
        assert err <= 1e-5
    # the finest reconstruction leaves the state untouched and stepping goes on as before
    t2, v2 = sim.get_state()
    keep = _leaf_entries(o, tree)
    assert np.array_equal(t2, tree) and np.array_equal(v2[keep], vals[keep])
    t_o, v_o = tree.copy(), v64.copy()
    if precision == 8:
        o.step(t_o, v_o)
        sim.step(1)
        tg, vg = sim.get_state()
        assert np.array_equal(tg, t_o) and leaf_err(o, t_o, vg, v_o) <= TOL64
    sim.close()


def test_fields_capacity_and_sizes(mr):
    import ctypes

    cfg = _cfg("D2Q9", 2, 6, 1e-3)
    sim = mr.Sim(cfg)
    n = ctypes.c_int64(0)
    assert mr.lib().mrlbm_fields(sim._ctx, 0, 4, None, 0, ctypes.byref(n)) == -5  # before initialisation
    sim.init_equilibrium(W.random_field(cfg, 2, "smooth"))
    assert mr.lib().mrlbm_fields(sim._ctx, 0, 4, None, 0, ctypes.byref(n)) == -2
    assert n.value == 9 * 64 * 64
    assert mr.lib().mrlbm_fields(sim._ctx, 0, 1, None, 0, ctypes.byref(n)) == -2
    assert n.value == 64 * 64
    assert mr.lib().mrlbm_fields(sim._ctx, 0, 3, None, 0, ctypes.byref(n)) == -2
    assert n.value == 9 * 64 * 64
    assert mr.lib().mrlbm_fields(sim._ctx, 0, 5, None, 0, ctypes.byref(n)) == -1
    assert mr.lib().mrlbm_fields(sim._ctx, 1, 1, None, 0, ctypes.byref(n)) == -1
    sim.close()


@pytest.mark.parametrize("precision", [8, 4])
def test_frozen_replay_equals_recorded_run(mr, precision):
    """Replaying a run's own mesh sequence through mrlbm_step_frozen gives the
    run's meshes and bits; one frozen step matches the oracle's frozen step."""
    cfg, m0 = W.shear_layer_d2q9(jmin=2, jmax=7, eps=1e-3, re=1000.0, width=1.0 / 20)
    o = oracle.Oracle(cfg)
    a = mr.Sim(cfg, precision=precision)
    a.init_equilibrium(m0)
    meshes = []
    for _ in range(15):
        a.step(1)
        meshes.append(a.get_mesh())
    ta, va = a.get_state()
    a.close()
    b = mr.Sim(cfg, precision=precision)
    b.init_equilibrium(m0)
    for k, t in enumerate(meshes):
        if k == 9:
            tg, vg = b.get_state()
            t_o, v_o = tg.copy(), vg.astype(np.float64)
            o.step_frozen(t_o, t, v_o)
        b.step_frozen(t)
        if k == 9:
            tg2, vg2 = b.get_state()
            assert np.array_equal(tg2, t)
            e = leaf_err(o, t_o, vg2, v_o)
            print("frozen step vs oracle", e, flush=True)
            assert e <= (TOL64 if precision == 8 else 1e-5)
    tb, vb = b.get_state()
    assert np.array_equal(ta, tb)
    keep = _leaf_entries(o, ta)
    assert np.array_equal(va[keep], vb[keep])
    # a mesh that refines a leaf by two levels in one step is rejected, state unchanged
    bad = tb.copy()
    lvl_leaves = [l for l in range(o.jmin, o.jmax - 1) if o.leaf_mask(tb, l).any()]
    l = lvl_leaves[0]
    k = int(np.flatnonzero(o.leaf_mask(tb, l).ravel())[0])
    x, y = k % (1 << l), k // (1 << l)
    for dl in (1, 2):
        n = 1 << (l + dl)
        for yy in range(y << dl, (y + 1) << dl):
            for xx in range(x << dl, (x + 1) << dl):
                bad[o.level_offset(l + dl) + xx + n * yy] = 1
    with pytest.raises(mr.MrlbmError) as ei:
        b.step_frozen(bad)
    assert ei.value.status == -1
    tc, vc = b.get_state()
    assert np.array_equal(tc, tb) and np.array_equal(vc[keep], vb[keep])
    b.close()


def test_nonfinite_leaf_reported(mr):
    cfg = _cfg("D2Q9", 2, 6, 1e-3)
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg)
    t, v = o.init(W.random_field(cfg, 3, "smooth"))
    sim.set_state(t, v)
    assert sim.stats()["leaves"].sum() == 64 * 64
    v = v.copy()
    v[o.q * o.level_offset(6) + 3 * 64 * 64 + 100] = np.nan  # population 3 of one finest leaf
    sim.set_state(t, v)
    with pytest.raises(mr.MrlbmError) as ei:
        sim.stats()
    assert ei.value.status == -3
    sim.close()
    # the flag is per instance: a batch reports it for the instance that holds the value
    bat = mr.Batch([cfg, cfg])
    bat.set_state(0, t, o.init(W.random_field(cfg, 3, "smooth"))[1])
    bat.set_state(1, t, v)
    assert bat.stats(0)["leaves"].sum() == 64 * 64
    with pytest.raises(mr.MrlbmError) as ei:
        bat.stats(1)
    assert ei.value.status == -3
    bat.close()


def test_pair_wait_timeout_is_reported(mr):
    """Full finest mesh on levels 3..8: the finest two links of the projection
    and ancestor chains both have work, so their paired launches wait. With the
    test hook the waits give up after 64 spins; the step completes, and the
    sticky flag is reported by every synchronising call."""
    cfg = _cfg("D2Q9", 3, 8, 0.0)
    m0 = W.random_field(cfg, 4, "smooth")
    sim = mr.Sim(cfg)
    sim.init_equilibrium(m0)
    t = sim.tuning()  # the paired launches (tuning pair_links)
    sim.set_tuning(t["transport_variant"], t["list_grid_all"], t["list_grid_level"], graph=t["graph"], pair_links=1)
    sim.step(2)
    assert sim.stats()["leaves"][8] == 256 * 256  # no flag after ordered waits that succeed
    sim.debug_pair_wait(64, -(1 << 30))
    sim.step(1)
    for call in (sim.stats, sim.get_state, sim.get_mesh):
        with pytest.raises(mr.MrlbmError) as ei:
            call()
        assert ei.value.status == -6
    sim.debug_pair_wait(0, 0)
    sim.step(1)  # kernels still run to their end; the flag stays
    with pytest.raises(mr.MrlbmError) as ei:
        sim.stats()
    assert ei.value.status == -6
    sim.close()
    fresh = mr.Sim(cfg)
    fresh.init_equilibrium(m0)
    fresh.step(2)
    assert fresh.stats()["leaves"][8] == 256 * 256
    fresh.close()
