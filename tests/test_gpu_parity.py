"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

One-step replay: the GPU state (tree and leaf values) before a step is handed to
the oracle, both advance one step, and the meshes must agree bit for bit and
the leaf values within 1e-12 * max(1, |f|) (FP64). Replaying every step keeps
the check exact although free-running trajectories drift apart at round-off.
"""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


def _s(scheme):
    return {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]


def _cfg(scheme, jmin, jmax, eps, mu_bar=1.0):
    return W.params(scheme, jmin, jmax, eps, _s(scheme), mu_bar=mu_bar, eq_param=0.5 if scheme == "D1Q3" else 1.0)


def leaf_err(o, tree, a, b):
    """max over complete leaves of |a - b| / max(1, |b|)."""
    err = 0.0
    for l in range(o.jmin, o.jmax + 1):
        mask = o.leaf_mask(tree, l)
        va = o.values_level(a, l)[:, mask].astype(np.float64)
        vb = o.values_level(b, l)[:, mask].astype(np.float64)
        if va.size:
            err = max(err, float(np.max(np.abs(va - vb) / np.maximum(1.0, np.abs(vb)))))
    return err


def replay(mr, cfg, m0, nsteps, check_every=1, precision=8):
    """Run nsteps on the GPU; every `check_every` steps replay one step on the
    oracle from the GPU state. Returns the worst field error and the GPU sim."""
    o = oracle.Oracle(cfg)
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    t0, v0 = o.init(m0)
    tg, vg = sim.get_state()
    assert np.array_equal(tg, t0)
    worst = leaf_err(o, t0, vg, v0)
    assert worst <= TOL64
    for k in range(nsteps):
        if k % check_every == 0:
            tg, vg = sim.get_state()
            t_o, v_o = tg.copy(), vg.astype(np.float64)
            o.step(t_o, v_o)
            sim.step(1)
            tg2, vg2 = sim.get_state()
            assert np.array_equal(tg2, t_o), "mesh differs at step %d (%d cells)" % (k, int((tg2 != t_o).sum()))
            e = leaf_err(o, t_o, vg2, v_o)
            assert e <= TOL64, "field error %g at step %d" % (e, k)
            worst = max(worst, e)
        else:
            sim.step(1)
    return worst, sim, o


@pytest.mark.parametrize("scheme,jmin,jmax,eps,seed", [
    ("D1Q2", 2, 10, 1e-4, 0), ("D1Q3", 2, 10, 1e-4, 1), ("D1Q3", 1, 9, 1e-3, 2),
    ("D2Q9", 2, 6, 1e-3, 3), ("D2Q9", 3, 7, 1e-4, 4), ("D2Q9", 1, 5, 1e-2, 5),
    # coarsest level at and above the largest level the one-block-per-instance
    # kernels walk (2D: 5, 1D: 10): those kernels then cover one level or none
    ("D2Q9", 5, 8, 1e-3, 6), ("D2Q9", 6, 8, 1e-3, 7), ("D1Q3", 10, 13, 1e-3, 8), ("D1Q3", 11, 13, 1e-3, 9)])
def test_step_replay_random_fields(mr, scheme, jmin, jmax, eps, seed):
    cfg = _cfg(scheme, jmin, jmax, eps)
    m0 = W.random_field(cfg, seed, "jump")
    worst, sim, o = replay(mr, cfg, m0, 12)
    print(scheme, "worst rel err", worst, "leaves", sim.stats()["leaves"][jmin:])


def test_step_replay_shear_layer_several_levels(mr):
    cfg, m0 = W.shear_layer_d2q9(jmin=2, jmax=8, eps=1e-3, re=1000.0, width=1.0 / 40)
    worst, sim, o = replay(mr, cfg, m0, 8)
    counts = sim.stats()["leaves"]
    assert (counts[2:8] > 0).sum() >= 3  # several levels of leaves present


def test_d1q2_advection_config_1000_steps(mr):
    """The D1Q2 workload (levels 2..10, eps 1e-4, 1000 steps), replayed every 10 steps."""
    cfg, m0 = W.advection_d1q2()
    worst, sim, o = replay(mr, cfg, m0, 1000, check_every=10)
    st = sim.stats()
    assert st["leaves"].sum() < 1024


def test_uniform_limits_match_oracle_uniform(mr):
    """jmin = J and eps = 0: the adaptive GPU path reduces to the uniform scheme,
    bit for bit in 1D. In D2Q9 the GPU's collision applies M^-1 in the closed
    form M^T diag(1/|row|^2) of the orthogonal moment basis and the oracle a
    Gauss-Jordan inverse: equal in exact arithmetic, a few roundings apart."""
    for scheme, J in [("D1Q2", 8), ("D1Q3", 8), ("D2Q9", 5)]:
        for cfg in (_cfg(scheme, J, J, 1e-3), _cfg(scheme, 2, J, 0.0)):
            o = oracle.Oracle(cfg)
            m0 = W.random_field(cfg, 1, "jump")
            sim = mr.Sim(cfg)
            sim.init_equilibrium(m0)
            t, v = o.init(m0)
            fJ = o.values_level(v, J).reshape(o.q, -1).copy()
            o.uniform_step(fJ, 10)
            sim.step(10)
            tg, vg = sim.get_state()
            assert tg.all()
            g = o.values_level(vg, J).reshape(o.q, -1)
            if scheme == "D2Q9":
                assert np.max(np.abs(g - fJ)) <= 1e-13
            else:
                assert np.array_equal(g, fJ)


def test_d1q2_courant_one_exact_shift_on_gpu(mr):
    cfg, m0 = W.advection_d1q2()
    cfg = dict(cfg, jmin=cfg["jmax"])
    sim = mr.Sim(cfg)
    sim.init_equilibrium(m0)
    sim.step(1000)
    _, vg = sim.get_state()
    f = vg.reshape(2, -1)
    assert np.array_equal(f[0] + f[1], np.roll(m0[0], 1000))


def test_huge_eps_coarsest_mesh(mr):
    cfg = _cfg("D2Q9", 2, 6, 1e300)
    sim = mr.Sim(cfg)
    sim.init_equilibrium(W.random_field(cfg, 0, "jump"))
    sim.step(2)
    st = sim.stats()
    assert st["leaves"][2] == 16 and st["leaves"].sum() == 16


def test_mass_conserved_on_gpu(mr):
    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=8, eps=1e-3, re=1000.0, width=1.0 / 40)
    sim = mr.Sim(cfg)
    sim.init_equilibrium(m0)
    m_prev = sim.stats()["mass"]
    for _ in range(10):
        sim.step(5)
        m = sim.stats()["mass"]
        assert abs(m - m_prev) <= 1e-13 * abs(m_prev)
        m_prev = m


@pytest.mark.parametrize("precision", [8, 4])
def test_mass_is_compensated_sum(mr, precision):
    """The reported mass equals the exactly rounded sum (math.fsum) of the
    volume-weighted leaf populations to a few ulps: on the full 1024^2 finest
    mesh right after the initialisation (9.4 M terms, where plain summation
    drifts by far more) and after adaptive steps."""
    import math

    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=10, eps=1e-3, re=1e4, width=1.0 / 80)
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    for k in range(2):
        cells, vals = sim.leaves()
        lev = (cells.cpu().numpy().astype(np.int64) >> 26)
        w = np.ldexp(1.0, 2 * (cfg["jmax"] - lev))
        terms = (vals.double().cpu().numpy() * w[:, None]).ravel()  # exact: power-of-two scaling
        exact = math.fsum(terms.tolist())
        got = sim.stats()["mass"]
        assert abs(got - exact) <= 4 * np.spacing(exact), (k, got, exact, got - exact)
        sim.step(20)
    sim.close()


def test_gpu_run_is_deterministic(mr):
    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=8, eps=1e-3, re=1000.0, width=1.0 / 40)
    out = []
    for _ in range(2):
        sim = mr.Sim(cfg)
        sim.init_equilibrium(m0)
        sim.step(20)
        out.append(sim.get_state())
    leaves = _leaf_entries(oracle.Oracle(cfg), out[0][0])
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1][leaves], out[1][1][leaves])


def test_set_state_rejects_ungraded_tree(mr):
    cfg = _cfg("D1Q3", 2, 6, 1e-3)
    sim = mr.Sim(cfg)
    o = oracle.Oracle(cfg)
    tree, v = o.new_state()
    tree[:] = 0
    o.tree_level(tree, 2)[:] = 1
    o.tree_level(tree, 6)[:2] = 1  # a finest group without ancestors
    with pytest.raises(mr.MrlbmError) as ei:
        sim.set_state(tree, v)
    assert ei.value.status == -1


def test_leaf_export_matches_state(mr):
    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=7, eps=1e-3, re=1000.0, width=1.0 / 40)
    sim = mr.Sim(cfg)
    sim.init_equilibrium(m0)
    sim.step(3)
    cells, vals = sim.leaves()
    tree, v = sim.get_state()
    o = oracle.Oracle(cfg)
    cells = cells.cpu().numpy().astype(np.uint32)
    vals = vals.cpu().numpy()
    lv = cells >> 26
    cc = cells & ((1 << 26) - 1)
    assert len(cells) == sum(int(o.leaf_mask(tree, l).sum()) for l in range(3, 8))
    for i in range(0, len(cells), 97):
        lvl = o.values_level(v, int(lv[i])).reshape(o.q, -1)
        assert np.array_equal(vals[i], lvl[:, cc[i]])


# ------------------------------------------------------------ batches

def _batch_cfgs(scheme):
    if scheme == "D2Q9":
        out = []
        for k, (J, eps, re) in enumerate([(6, 1e-3, 800.0), (8, 1e-4, 2000.0), (7, 1e-2, 5000.0), (5, 1e-3, 300.0)]):
            cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=J, eps=eps, re=re, width=1.0 / 30, seed=k)
            out.append((cfg, m0))
        return out
    out = []
    for k, (J, eps) in enumerate([(9, 1e-4), (7, 1e-3), (10, 1e-5)]):
        cfg = _cfg("D1Q3", 2, J, eps)
        out.append((cfg, W.random_field(cfg, 10 + k, "jump")))
    return out


@pytest.mark.parametrize("scheme", ["D1Q3", "D2Q9"])
def test_batch_replay_each_instance(mr, scheme):
    """Uneven instances advanced together: every instance's step replays exactly
    on the oracle (mesh bit-exact, fields within 1e-12)."""
    items = _batch_cfgs(scheme)
    bat = mr.Batch([c for c, _ in items])
    for i, (_, m0) in enumerate(items):
        bat.init_equilibrium(i, m0)
    oracles = [oracle.Oracle(c) for c, _ in items]
    for k in range(6):
        pre = [bat.get_state(i) for i in range(len(items))]
        bat.step(1)
        for i, o in enumerate(oracles):
            t_o, v_o = pre[i][0].copy(), pre[i][1].astype(np.float64)
            o.step(t_o, v_o)
            tg, vg = bat.get_state(i)
            assert np.array_equal(tg, t_o), "instance %d mesh differs at step %d" % (i, k)
            assert leaf_err(o, t_o, vg, v_o) <= TOL64


@pytest.mark.parametrize("scheme,precision", [("D1Q3", 8), ("D2Q9", 4), ("D2Q9", 8)])
def test_ghost_sets_match_definition(mr, scheme, precision):
    """Per-level ghost counts of the GPU classification (16-cell runs and
    4-cell runs) equal the ghost sets built on the host from their definition,
    on the meshes of several steps of uneven instances."""
    from ghost_sets import ghost_sets

    items = _batch_cfgs(scheme)
    bat = mr.Batch([c for c, _ in items], precision=precision)
    for i, (_, m0) in enumerate(items):
        bat.init_equilibrium(i, m0)
    oracles = [oracle.Oracle(c) for c, _ in items]
    seen = 0
    for k in range(5):
        bat.step(2)
        for i, o in enumerate(oracles):
            tree, _ = bat.get_state(i)
            G = ghost_sets(o, tree)
            want = np.array([int(G[l].sum()) if l in G else 0 for l in range(o.jmax + 1)])
            got = bat.stats(i)["ghosts"]
            assert np.array_equal(got, want), "instance %d after %d steps: %s vs %s" % (i, 2 * k + 2, got, want)
            seen += int(want.sum())
    assert seen > 0
    bat.close()


@pytest.mark.parametrize("jmin", [3, 6, 7])
def test_batch32_replay_coarse_levels(mr, jmin):
    """Batches of 32 instances (the one-block-per-instance kernels then walk
    the 2D levels up to 6) with coarsest level below, at and above that level
    and uneven finest levels: every instance's step replayed on the oracle
    (mesh bit-exact, fields within 1e-12)."""
    items = []
    for k in range(32):
        jmax = max(jmin + 1, [7, 8][k % 2])
        cfg = _cfg("D2Q9", jmin, jmax, [1e-3, 1e-2][(k // 2) % 2])
        items.append((cfg, W.random_field(cfg, 100 + k, "jump" if k % 3 else "smooth")))
    bat = mr.Batch([c for c, _ in items])
    for i, (_, m0) in enumerate(items):
        bat.init_equilibrium(i, m0)
    bat.step(3)
    oracles = [oracle.Oracle(c) for c, _ in items]
    for k in range(2):
        pre = [bat.get_state(i) for i in range(len(items))]
        bat.step(1)
        for i, o in enumerate(oracles):
            t_o, v_o = pre[i][0].copy(), pre[i][1].copy()
            o.step(t_o, v_o)
            tg, vg = bat.get_state(i)
            assert np.array_equal(tg, t_o), "instance %d mesh differs at replay %d" % (i, k)
            assert leaf_err(o, t_o, vg, v_o) <= TOL64
    bat.close()


def test_batch_instance_equals_single_run(mr):
    """An instance advanced inside a batch is bit-identical to the same instance
    advanced alone."""
    items = _batch_cfgs("D2Q9")
    bat = mr.Batch([c for c, _ in items])
    for i, (_, m0) in enumerate(items):
        bat.init_equilibrium(i, m0)
    bat.step(15)
    for i, (cfg, m0) in enumerate(items):
        sim = mr.Sim(cfg)
        sim.init_equilibrium(m0)
        sim.step(15)
        a, b = bat.get_state(i), sim.get_state()
        leaves = _leaf_entries(oracle.Oracle(cfg), a[0])
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1][leaves], b[1][leaves])


def test_set_state_to_a_finer_mesh_midrun(mr):
    """After some steps (the dense passes then skip the levels no mesh
    reaches), one instance of a batch is set to its full finest mesh. Every
    level must be processed again: the batch instance stays bit-identical to
    the same state advanced in a fresh context, and the others to a batch run
    without the change."""
    items = _batch_cfgs("D2Q9")
    cfgs = [c for c, _ in items]
    runs = []
    for change in (True, False):
        bat = mr.Batch(cfgs)
        for i, (_, m0) in enumerate(items):
            bat.init_equilibrium(i, m0)
        bat.step(20)
        if change:
            o = oracle.Oracle(cfgs[0])
            t0, v0 = o.init(items[0][1])
            bat.set_state(0, t0, v0)
        bat.step(12)
        runs.append([bat.get_state(i) for i in range(bat.B)])
        bat.close()
    sim = mr.Sim(cfgs[0])
    o = oracle.Oracle(cfgs[0])
    sim.init_equilibrium(items[0][1])  # any state, then replaced
    sim.set_state(*o.init(items[0][1]))
    sim.step(12)
    a, b = runs[0][0], sim.get_state()
    print("instance 0 leaves", int(o.leaf_counts(a[0]).sum()), flush=True)
    leaves = _leaf_entries(o, a[0])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1][leaves], b[1][leaves])
    for i in range(1, len(cfgs)):
        (ta, va), (tb, vb) = runs[0][i], runs[1][i]
        assert np.array_equal(ta, tb)
        assert np.array_equal(va[_leaf_entries(oracle.Oracle(cfgs[i]), ta)],
                              vb[_leaf_entries(oracle.Oracle(cfgs[i]), tb)])
    sim.close()


def test_transport_variants_bit_identical(mr):
    """The per-item and per-population variants of the transport and details
    kernels compute the same meshes and the same bits."""
    cfg, m0 = W.shear_layer_d2q9(jmin=3, jmax=8, eps=1e-4, re=1000.0, width=1.0 / 40)
    out = {}
    for v in ("leaf", "pop"):
        for prec in (8, 4):
            sim = mr.Sim(cfg, precision=prec)
            t = sim.tuning()
            sim.set_tuning(1 if v == "leaf" else 2, t["list_grid_all"], t["list_grid_level"])
            sim.init_equilibrium(m0)
            sim.step(12)
            out[(v, prec)] = sim.get_state()
    for prec in (8, 4):
        a, b = out[("leaf", prec)], out[("pop", prec)]
        leaves = _leaf_entries(oracle.Oracle(cfg), a[0])
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1][leaves], b[1][leaves])


@pytest.mark.parametrize("prec", [8, 4])
def test_paired_links_bit_identical(mr, prec):
    """The finest two links of the level chains in one paired launch (tuning
    pair_links = 1) or in one launch each: the same meshes and bits, with the
    finest level holding cells (the pairs then wait) and with a batch whose
    instances reach it unevenly."""
    cfgs = [_cfg("D2Q9", 3, 8, 0.0), _cfg("D2Q9", 3, 8, 1e-3), _cfg("D2Q9", 3, 7, 1e-3)]
    m0s = [W.random_field(c, 70 + k, "jump") for k, c in enumerate(cfgs)]
    out = {}
    for pl in (0, 1):
        b = mr.Batch(cfgs, precision=prec)
        t = b.tuning()
        b.set_tuning(t["transport_variant"], t["list_grid_all"], t["list_grid_level"], graph=t["graph"], pair_links=pl)
        assert b.tuning()["pair_links"] == pl
        for i, m in enumerate(m0s):
            b.init_equilibrium(i, m)
        b.step(6)
        out[pl] = [b.get_state(i) for i in range(len(cfgs))]
        b.close()
    for i, c in enumerate(cfgs):
        a, p = out[0][i], out[1][i]
        leaves = _leaf_entries(oracle.Oracle(c), a[0])
        assert np.array_equal(a[0], p[0]) and np.array_equal(a[1][leaves], p[1][leaves])


def test_graph_steps_match_eager_launches(mr):
    """Steps replayed from HIP graphs (plain and with the timed transport launched
    outside the graph) compute the same bits as kernel-by-kernel launches, also
    after single adapt / transport calls change the buffer assignment."""
    cfgs = [it[0] for it in W.shear_layer_batch(3, jmax_choices=(6, 7))]
    m0s = [it[1] for it in W.shear_layer_batch(3, jmax_choices=(6, 7))]
    out = {}
    for mode in ("0", "1"):
        for prec in (8, 4):
            b = mr.Batch(cfgs, precision=prec)
            t = b.tuning()
            b.set_tuning(t["transport_variant"], t["list_grid_all"], t["list_grid_level"], graph=int(mode))
            assert b.tuning()["graph"] == int(mode)
            for i, m in enumerate(m0s):
                b.init_equilibrium(i, m)
            b.step(3)
            b.profile(True)
            b.step(2)
            b.profile(False)
            b.adapt()
            b.transport_collide()
            b.transport_collide()
            b.step(3)
            out[(mode, prec)] = [b.get_state(i) for i in range(b.B)]
            cnt = b.counters()
            b.close()
    for prec in (8, 4):
        for cfg, sa, sb in zip(cfgs, out[("0", prec)], out[("1", prec)]):
            assert np.array_equal(sa[0], sb[0])
            leaves = _leaf_entries(oracle.Oracle(cfg), sa[0])
            assert np.array_equal(sa[1][leaves], sb[1][leaves])


def test_reconstruction_after_adaptation_equals_full_one(mr):
    """Right after an adaptation the reconstruction recomputes only the
    projections above cells the adaptation changed. Handing the adapted state
    back through set_state, which forces the full reconstruction, must give the
    same bits in every cell, step after step."""
    items = W.shear_layer_batch(3, jmax_choices=(6, 7))
    cfgs = [c for c, _ in items]
    for prec in (8, 4):
        runs = []
        for full in (False, True):
            b = mr.Batch(cfgs, precision=prec)
            for i, (_, m) in enumerate(items):
                b.init_equilibrium(i, m)
            b.step(5)
            for _ in range(4):
                b.adapt()
                if full:
                    for i in range(b.B):
                        b.set_state(i, *b.get_state(i))
                b.transport_collide()
            runs.append([b.get_state(i) for i in range(b.B)])
            b.close()
        for i, ((ta, va), (tb, vb)) in enumerate(zip(*runs)):
            print("precision", prec, "instance", i, flush=True)
            assert np.array_equal(ta, tb)
            assert np.array_equal(va, vb)


def test_profiled_graph_steps_time_every_eighth_transport(mr):
    """With profiling on, graph-replayed steps count every transport launch and
    bracket the kernel of steps 0, 8, 16, ... with HIP events; the timed steps
    compute the same results as untimed ones."""
    items = _batch_cfgs("D2Q9")
    cfgs = [c for c, _ in items]
    states = {}
    for prof in (False, True):
        b = mr.Batch(cfgs, precision=4)
        for i, (_, m0) in enumerate(items):
            b.init_equilibrium(i, m0)
        b.step(2)
        b.profile(prof)
        b.step(17)
        cnt = b.counters()
        b.profile(False)
        if prof:
            assert cnt["transport_launches"] == 17 and cnt["timed_launches"] == 3
            assert 0.0 < cnt["transport_ms"] < 1e3
        states[prof] = [b.get_state(i) for i in range(b.B)]
        b.close()
    for cfg, sa, sb in zip(cfgs, states[False], states[True]):
        leaves = _leaf_entries(oracle.Oracle(cfg), sa[0])
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1][leaves], sb[1][leaves])


def _leaf_entries(o, tree):
    """Boolean mask of the complete-leaf entries of a values array (the other
    entries hold reconstruction scratch, which the state does not define)."""
    m = np.zeros(o.q * o.total, bool)
    for l in range(o.jmin, o.jmax + 1):
        lm = o.leaf_mask(tree, l).ravel()
        off = o.q * o.level_offset(l)
        for h in range(o.q):
            m[off + h * o.ncells(l): off + (h + 1) * o.ncells(l)] = lm
    return m


def test_autotune_keeps_state_and_results(mr):
    """The autotuner leaves the state and the leaf counters unchanged, the
    schedule it picks computes the same bits, and a second context with the
    same key takes the schedule from the cache."""
    items = W.shear_layer_batch(4, jmax_choices=(6, 7))
    cfgs = [c for c, _ in items]

    def fresh():
        b = mr.Batch(cfgs, precision=4)
        for i, (_, m0) in enumerate(items):
            b.init_equilibrium(i, m0)
        b.step(5)
        return b

    ref = fresh()
    ref.step(6)
    want = [ref.get_state(i) for i in range(ref.B)]
    ref.close()

    b = fresh()
    before = [b.get_state(i) for i in range(b.B)]
    b.profile(True)
    b.step(1)
    n1 = b.counters()["leaf_updates"]
    t = b.autotune(reps=2)
    assert t["transport_variant"] in (1, 2) and t["ms_per_step"] > 0 and t["from_cache"] == 0
    assert b.counters()["leaf_updates"] == n1
    assert b.tuning()["list_grid_all"] == t["list_grid_all"]
    b.step(5)
    got = [b.get_state(i) for i in range(b.B)]
    for cfg, sa, sb in zip(cfgs, want, got):
        leaves = _leaf_entries(oracle.Oracle(cfg), sa[0])
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1][leaves], sb[1][leaves])
    del before

    c2 = fresh()
    t2 = c2.autotune(reps=2)
    assert t2["from_cache"] == 1 and t2["list_grid_all"] == t["list_grid_all"]
    c2.set_tuning(2, 1024, 256)
    assert c2.tuning()["transport_variant"] == 2
    c2.step(2)
    c2.close()
    b.close()
