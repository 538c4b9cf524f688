"""Pins of the oracle's mesh adaptation G o H_eps o T_eps (no GPU): special
cases, invariants, and a brute-force fixed-point construction on tiny meshes."""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W


def _cfg(scheme, jmin, jmax, eps, mu_bar=1.0):
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=mu_bar, eq_param=0.5 if scheme == "D1Q3" else 1.0)


@pytest.mark.parametrize("scheme,jmin,jmax", [("D1Q2", 2, 8), ("D1Q3", 2, 8), ("D2Q9", 2, 5)])
def test_eps_zero_keeps_full_finest_mesh(scheme, jmin, jmax):
    cfg = _cfg(scheme, jmin, jmax, 0.0)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 0, "jump"))
    o.step(tree, v, 3)
    assert tree.all()


@pytest.mark.parametrize("scheme,jmin,jmax", [("D1Q3", 2, 8), ("D2Q9", 2, 5)])
def test_huge_eps_gives_uniform_coarsest_mesh(scheme, jmin, jmax):
    cfg = _cfg(scheme, jmin, jmax, 1e300)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 0, "jump"))
    o.step(tree, v, 1)
    counts = o.leaf_counts(tree)
    assert counts[jmin] == o.ncells(jmin) and counts.sum() == o.ncells(jmin)


@pytest.mark.parametrize("scheme,jmin,jmax,eps", [("D1Q2", 2, 10, 1e-4), ("D1Q3", 2, 10, 1e-4),
                                                  ("D2Q9", 3, 6, 1e-3), ("D2Q9", 2, 6, 1e-4)])
def test_adapted_tree_invariants(scheme, jmin, jmax, eps):
    """Graded complete tree whose complete leaves partition the domain."""
    cfg = _cfg(scheme, jmin, jmax, eps)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 7, "jump"))
    for _ in range(6):
        o.step(tree, v)
        assert o.check_tree(tree) == 0
        counts = o.leaf_counts(tree)
        vol = sum(int(counts[l]) << (o.dim * (jmax - l)) for l in range(jmin, jmax + 1))
        assert vol == o.ncells(jmax)


def _random_graded_tree(o, rng, steps=2):
    tree = np.ones(o.total, np.uint8)
    for _ in range(steps):
        D = 10.0 ** rng.uniform(-4, 0, o.total)
        tree = o.adapt_tree(tree, D)
    return tree


def _brute_adapt(o, cfg, told, D):
    """The mesh G(H_eps(T_eps(told))) built from the definitions with naive
    fixed-point closures on sets of (level, coords)."""
    jmin, J, d = o.jmin, o.jmax, o.dim
    eta = [tuple(e[:d]) for e in o.velocities()]

    def N(l):
        return 1 << l

    def cells(l):
        if d == 1:
            return [(x,) for x in range(N(l))]
        return [(x, y) for y in range(N(l)) for x in range(N(l))]

    def idx(l, c):
        return o.level_offset(l) + (c[0] if d == 1 else c[0] + N(l) * c[1])

    def parent(c):
        return tuple(v >> 1 for v in c)

    def children(c):
        if d == 1:
            return [(2 * c[0] + s,) for s in (0, 1)]
        return [(2 * c[0] + sx, 2 * c[1] + sy) for sy in (0, 1) for sx in (0, 1)]

    walls = [cfg.get("bc", (0, 0, 0, 0))[2 * a] != 0 for a in range(d)]

    def wrap(l, c):  # periodic axes wrap; beyond a wall the cell does not exist (None)
        if any(walls[a] and not 0 <= c[a] < N(l) for a in range(d)):
            return None
        return tuple(v % N(l) for v in c)

    def D_of(l, c):  # metric of the group of (l, c), stored at the parent's slot
        return D[idx(l - 1, parent(c))]

    sq = cfg.get("metric", "linf") == "l2"  # the l2 metric is compared squared
    g = int(cfg.get("gamma", 1))

    def eps_l(l):
        e = np.ldexp(cfg["eps"], d * (l - J))
        return e * e if sq else e

    def ref_l(l):
        r = np.ldexp(np.ldexp(cfg["eps"], d * (l - J)), d) * 2.0 ** cfg["mu_bar"]
        return r * r if sq else r

    old = {(l, c) for l in range(jmin, J + 1) for c in cells(l) if told[idx(l, c)]}
    K = {(jmin, c) for c in cells(jmin)}
    K |= {(l, c) for (l, c) in old if l > jmin and D_of(l, c) >= eps_l(l)}
    changed = True
    while changed:  # smallest tree (parents and siblings) containing K
        changed = False
        for (l, c) in list(K):
            if l > jmin:
                for s in children(parent(c)) + [None]:
                    item = (l - 1, parent(c)) if s is None else (l, s)
                    if item not in K:
                        K.add(item)
                        changed = True
    H = set(K)
    for (l, c) in K:
        for e in eta:
            nb = wrap(l, tuple(ci - ei for ci, ei in zip(c, e)))
            if nb is not None:
                H.add((l, nb))
        if jmin < l < J and D_of(l, c) >= ref_l(l):
            for ch in children(c):
                H.add((l + 1, ch))
    changed = True
    while changed:  # smallest graded complete tree containing H
        changed = False
        for (l, c) in list(H):
            if l == jmin:
                continue
            p = parent(c)
            need = [(l, s) for s in children(p)]
            rng_ = range(-g, g + 1)
            if d == 1:
                need += [(l - 1, wrap(l - 1, (p[0] + a,))) for a in rng_]
            else:
                need += [(l - 1, wrap(l - 1, (p[0] + a, p[1] + b))) for b in rng_ for a in rng_]
            for item in need:
                if item[1] is not None and item not in H:
                    H.add(item)
                    changed = True
    H |= {(jmin, c) for c in cells(jmin)}
    out = np.zeros(o.total, np.uint8)
    for (l, c) in H:
        out[idx(l, c)] = 1
    return out


@pytest.mark.parametrize("scheme,jmin,jmax,mu_bar,seed", [("D1Q2", 2, 6, 0.0, 0), ("D1Q3", 1, 6, 1.0, 1),
                                                          ("D1Q3", 2, 6, 2.0, 2), ("D2Q9", 1, 4, 1.0, 3),
                                                          ("D2Q9", 2, 4, 0.0, 4)])
@pytest.mark.parametrize("walls", [False, True])
def test_adapt_equals_brute_force_fixed_point(scheme, jmin, jmax, mu_bar, seed, walls):
    cfg = _cfg(scheme, jmin, jmax, 1e-2, mu_bar)
    if walls:  # the set operations ignore cells beyond a wall
        cfg = dict(cfg, bc=(2, 1, 3, 2) if cfg["dim"] == 2 else (1, 2, 0, 0))
    o = oracle.Oracle(cfg)
    rng = np.random.default_rng(seed)
    for trial in range(4):
        told = _random_graded_tree(o, rng, steps=trial % 3 + 1)
        assert o.check_tree(told) == 0
        D = 10.0 ** rng.uniform(-5, 0, o.total)
        assert np.array_equal(o.adapt_tree(told, D), _brute_adapt(o, cfg, told, D))


def test_enlargement_keeps_upwind_neighbours_and_refines():
    """eq. AdditionNeigh and the refinement rule, checked on the result."""
    cfg = _cfg("D2Q9", 2, 5, 1e-2, 1.0)
    o = oracle.Oracle(cfg)
    rng = np.random.default_rng(11)
    told = _random_graded_tree(o, rng, 2)
    D = 10.0 ** rng.uniform(-5, 0, o.total)
    tnew = o.adapt_tree(told, D)
    eta = o.velocities()
    for l in range(o.jmin + 1, o.jmax + 1):
        t_old, t_new = o.tree_level(told, l), o.tree_level(tnew, l)
        Dp = D[o.level_offset(l - 1):o.level_offset(l - 1) + o.ncells(l - 1)].reshape(1 << (l - 1), -1)
        epsl = np.ldexp(1e-2, 2 * (l - o.jmax))
        n = 1 << l
        for y in range(n):
            for x in range(n):
                if t_old[y, x] and Dp[y >> 1, x >> 1] >= epsl:
                    for ex, ey in eta:
                        assert t_new[(y - ey) % n, (x - ex) % n]
                    if l < o.jmax and Dp[y >> 1, x >> 1] >= np.ldexp(epsl, 2) * 2.0:
                        assert o.tree_level(tnew, l + 1)[2 * y, 2 * x]


@pytest.mark.parametrize("scheme,jmin,jmax", [("D1Q3", 2, 8), ("D2Q9", 2, 6)])
def test_float_decision_matches_double_on_exact_data(scheme, jmin, jmax):
    """With leaf values that are small dyadic rationals, every projection,
    prediction and detail is exact in float and double, so the single-precision
    mesh decision must equal the double one."""
    cfg = _cfg(scheme, jmin, jmax, 2.0 ** -6)
    o = oracle.Oracle(cfg)
    rng = np.random.default_rng(5)
    tree = o.adapt_tree(np.ones(o.total, np.uint8), 10.0 ** rng.uniform(-4, 0, o.total))
    _, v = o.new_state()
    v[:] = rng.integers(-64, 64, v.size) / 64.0
    assert np.array_equal(o.new_tree_f32(tree, v.astype(np.float32)), o.new_tree_from_state(tree, v))


def test_step_frozen_equals_step_on_own_mesh():
    cfg = _cfg("D2Q9", 2, 6, 1e-3)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 3, "jump"))
    o.step(tree, v, 2)
    tnew = o.new_tree_from_state(tree, v)
    t1, v1 = tree.copy(), v.copy()
    o.step(t1, v1)
    t2, v2 = tree.copy(), v.copy()
    o.step_frozen(t2, tnew, v2)
    assert np.array_equal(t1, t2) and np.array_equal(v1, v2)


@pytest.mark.parametrize("scheme,jmin,jmax,eps,kind", [("D1Q3", 2, 10, 1e-4, "jump"), ("D2Q9", 3, 7, 1e-3, "smooth"),
                                                       ("D2Q9", 2, 6, 1e-3, "jump")])
def test_ghosts_lie_next_to_coarser_internal_cells(scheme, jmin, jmax, eps, kind):
    """Every ghost of level l has an internal cell of level l-1 within one cell
    of its parent, on adapted meshes and on random graded trees. The GPU ghost
    classification skips runs of cells that fail this necessary condition."""
    from ghost_sets import ghost_near_internal, ghost_sets

    cfg = _cfg(scheme, jmin, jmax, eps)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 3, kind))
    n_ghosts = 0
    for _ in range(4):
        o.step(tree, v)
        assert ghost_near_internal(o, tree) == []
        n_ghosts += sum(int(g.sum()) for g in ghost_sets(o, tree).values())
    rng = np.random.default_rng(5)
    for _ in range(3):
        t = _random_graded_tree(o, rng)
        assert o.check_tree(t) == 0
        assert ghost_near_internal(o, t) == []
        n_ghosts += sum(int(g.sum()) for g in ghost_sets(o, t).values())
    assert n_ghosts > 0


def test_ghost_condition_check_catches_a_violation():
    """The check itself: a ghost planted away from every internal cell fails it."""
    from ghost_sets import _children, _dilate, tree_sets

    cfg = _cfg("D2Q9", 2, 5, 1e-3)
    o = oracle.Oracle(cfg)
    tree = np.zeros(o.total, np.uint8)
    tree[o.level_offset(2):o.level_offset(2) + o.ncells(2)] = 1  # uniform coarsest mesh
    assert o.check_tree(tree) == 0
    _, _, I = tree_sets(o, tree)
    assert not I[2].any()
    g = np.zeros((8, 8), bool)
    g[3, 3] = True
    assert np.any(g & ~_children(_dilate(I[2], 1)))


@pytest.mark.parametrize("scheme,jmin,jmax,eps,kind", [("D1Q3", 2, 10, 1e-4, "jump"), ("D2Q9", 3, 7, 1e-3, "smooth"),
                                                       ("D2Q9", 2, 6, 1e-3, "jump")])
def test_kept_and_refined_cells_belong_to_the_new_tree(scheme, jmin, jmax, eps, kind):
    """Every cell kept by the thresholding (with the sibling groups of its
    ancestors) and every parent flagged for refinement is a cell of the new
    tree: the GPU zeroes these flags only where the new tree has cells."""
    cfg = _cfg(scheme, jmin, jmax, eps)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 4, kind))
    d, mu = o.dim, float(cfg.get("mu_bar", 0.0))
    checked = 0
    for _ in range(5):
        D = o.details(tree, o.reconstruct(tree, v))
        tnew = o.adapt_tree(tree, D)
        for l in range(jmin + 1, jmax + 1):
            eps_l = np.ldexp(eps, d * (l - jmax))
            ref_l = np.ldexp(eps_l, d) * 2.0 ** mu
            Dp = o.tree_level(D, l - 1) if d == 2 else D[o.level_offset(l - 1):o.level_offset(l - 1) + o.ncells(l - 1)]
            told_l = o.tree_level(tree, l).astype(bool)
            kept_groups = Dp >= eps_l  # parents whose children are kept
            kept = told_l & (np.repeat(np.repeat(kept_groups, 2, 0), 2, 1) if d == 2 else np.repeat(kept_groups, 2))
            tn_l = o.tree_level(tnew, l).astype(bool)
            assert not np.any(kept & ~tn_l), "kept cell outside the new tree at level %d" % l
            # the sibling group of a kept cell's parent (ancestor closure)
            if l - 1 > jmin:
                par = (kept.reshape(kept.shape[0] // 2, 2, kept.shape[1] // 2, 2).any(axis=(1, 3)) if d == 2
                       else kept.reshape(-1, 2).any(axis=1))
                grp = (par.reshape(par.shape[0] // 2, 2, par.shape[1] // 2, 2).any(axis=(1, 3)) if d == 2
                       else par.reshape(-1, 2).any(axis=1))
                sib = np.repeat(np.repeat(grp, 2, 0), 2, 1) if d == 2 else np.repeat(grp, 2)
                assert not np.any(sib & ~o.tree_level(tnew, l - 1).astype(bool))
            if jmin < l < jmax:
                refined = (Dp >= ref_l) & (Dp >= 0)
                assert not np.any(refined & ~o.tree_level(tnew, l - 1).astype(bool))
            checked += int(kept.sum())
        o.step(tree, v)
    assert checked > 0


def _change_marks(o, told, tnew, propagate=True):
    """Marks of the reconstruction that follows an adaptation: the new leaves
    outside the old tree and (with propagate) every internal cell of the new
    tree with a marked child, finest level first."""
    from ghost_sets import _parents, tree_sets

    To, _, Io = tree_sets(o, told)
    _, Sn, In = tree_sets(o, tnew)
    M = {l: Sn[l] & ~To[l] for l in Sn}
    if propagate:
        for l in range(o.jmax - 1, o.jmin - 1, -1):
            M[l] = M[l] | (In[l] & _parents(M[l + 1]))
    return M, Io, In


def _unmarked_violations(o, told, dense_old, tnew, dense_new, M, Io, In):
    """Unmarked internal cells of the new tree that were not internal before
    or whose projection changed (bitwise), and the number of unmarked ones."""
    bad, n = 0, 0
    for l in range(o.jmin, o.jmax):
        keep = In[l] & ~M[l]
        n += int(keep.sum())
        bad += int(np.sum(keep & ~Io[l]))
        a, b = o.values_level(dense_old, l)[:, keep], o.values_level(dense_new, l)[:, keep]
        bad += int(np.sum(np.any(a != b, axis=0)))
    return bad, n


@pytest.mark.parametrize("scheme,jmin,jmax,eps,kind", [("D1Q3", 2, 10, 1e-4, "jump"), ("D2Q9", 3, 7, 1e-3, "jump"),
                                                       ("D2Q9", 2, 6, 1e-3, "jump")])
def test_unmarked_projections_survive_the_adaptation(scheme, jmin, jmax, eps, kind):
    """The reconstruction after an adaptation recomputes only the projections
    of marked cells (new leaves outside the old tree, then internal cells with
    a marked child): every unmarked internal cell of the new tree was internal
    in the old one and its reconstructed value is bit for bit the old one."""
    cfg = _cfg(scheme, jmin, jmax, eps)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 6, kind))
    skipped = marked = 0
    for _ in range(5):
        o.step(tree, v)
        dense_old = o.reconstruct(tree, v)
        tnew = o.adapt_tree(tree, o.details(tree, dense_old))
        dense_new = o.reconstruct(tnew, o.transfer(tree, dense_old, tnew))
        M, Io, In = _change_marks(o, tree, tnew)
        bad, n = _unmarked_violations(o, tree, dense_old, tnew, dense_new, M, Io, In)
        assert bad == 0
        skipped += n
        marked += sum(int(m.sum()) for m in M.values())
    assert skipped > 0 and marked > 0


def test_change_marks_need_the_upward_pass():
    """The check has teeth: marking only the new leaves, without the upward
    pass, leaves changed projections unmarked."""
    cfg = _cfg("D2Q9", 2, 6, 1e-3)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 6, "jump"))
    found = 0
    for _ in range(5):
        o.step(tree, v)
        dense_old = o.reconstruct(tree, v)
        tnew = o.adapt_tree(tree, o.details(tree, dense_old))
        dense_new = o.reconstruct(tnew, o.transfer(tree, dense_old, tnew))
        M, Io, In = _change_marks(o, tree, tnew, propagate=False)
        found += _unmarked_violations(o, tree, dense_old, tnew, dense_new, M, Io, In)[0]
    assert found > 0


def _codes(o, tree):
    """Dense codes of a mesh per level: 3 leaf, 2 internal, 1 ghost, 0 none."""
    from ghost_sets import ghost_sets, tree_sets

    _, S, I = tree_sets(o, tree)
    G = ghost_sets(o, tree)
    return {l: (3 * S[l] + 2 * I[l] + (G[l] if l in G else 0)).astype(np.uint8) for l in S}


def _finest(o, tree):
    return max(l for l in range(o.jmin, o.jmax + 1) if o.tree_level(tree, l).any())


def _refine_reach(o, cfg, tree, values):
    """Finest level the refinement flags of the next adaptation reach (the
    grandchildren of flagged parents), 0 if there are none."""
    D = o.details(tree, o.reconstruct(tree, values))
    d, mu, eps = o.dim, float(cfg.get("mu_bar", 0.0)), float(cfg["eps"])
    reach = 0
    for l in range(o.jmin + 1, o.jmax):
        ref_l = np.ldexp(np.ldexp(eps, d * (l - o.jmax)), d) * 2.0 ** mu
        Dp = o.tree_level(D, l - 1) if d == 2 else D[o.level_offset(l - 1):o.level_offset(l - 1) + o.ncells(l - 1)]
        inner = o.tree_level(tree, l - 1).astype(bool) & ~o.leaf_mask(tree, l - 1)
        if np.any(inner & (Dp >= ref_l)):
            reach = max(reach, l + 1)
    return reach


def _activity_run(o, cfg, tree, v, steps, keep_history=True, use_reach=True):
    """Replays the GPU's level skipping on the two code buffers and the
    membership array: each adaptation writes only levels up to
    max(finest of the old mesh, refinement reach, finest of the mesh before),
    starting from all levels active. Returns the number of (step, level)
    pairs where a buffer then differs from the true mesh, and of skipped ones."""
    code = [_codes(o, tree), {l: np.zeros_like(c) for l, c in _codes(o, tree).items()}]
    tnew = {l: np.zeros_like(c) for l, c in code[0].items()}
    hist = [o.jmax, 64]  # the compaction of the initial mesh, after a reset
    cur, bad, skipped = 0, 0, 0
    for _ in range(steps):
        reach = _refine_reach(o, cfg, tree, v) if use_reach else 0
        top = min(o.jmax, max(hist[0], reach, hist[1] if keep_history else 0))
        o.step(tree, v)
        want, memb = _codes(o, tree), {l: o.tree_level(tree, l).astype(np.uint8) for l in code[0]}
        for l in want:
            if l <= top:
                code[1 - cur][l] = want[l].copy()
                tnew[l] = memb[l].copy()
            else:
                skipped += 1
            bad += int(not np.array_equal(code[1 - cur][l], want[l])) + int(not np.array_equal(tnew[l], memb[l]))
        cur = 1 - cur
        hist = [_finest(o, tree), hist[0]]
    return bad, skipped


def _activity_case(name):
    if name == "burgers":  # a shock forms: the mesh refines into new levels
        cfg, m0 = W.burgers_d1q3(jmin=2, jmax=9, eps=3e-3, mu_bar=1.0, nmodes=3)
        return cfg, m0, 150
    scheme, jmin, jmax, eps, seed = {"d1q2": ("D1Q2", 2, 10, 1e-3, 3), "d2q9": ("D2Q9", 2, 7, 1e-2, 1)}[name]
    cfg = _cfg(scheme, jmin, jmax, eps)
    return cfg, W.random_field(cfg, seed, "smooth"), 12


@pytest.mark.parametrize("name", ["burgers", "d1q2", "d2q9"])
def test_dense_passes_may_skip_inactive_levels(name):
    """Levels above max(finest level of the old mesh, reach of its refinement
    flags, finest level of the mesh before) hold only zeros in the code buffer
    an adaptation rewrites and in the membership array: writing only the levels
    below keeps both equal to the true meshes, step after step."""
    cfg, m0, steps = _activity_case(name)
    o = oracle.Oracle(cfg)
    tree, v = o.init(m0)
    bad, skipped = _activity_run(o, cfg, tree, v, steps)
    assert bad == 0 and skipped > 0


@pytest.mark.parametrize("name,keep_history,use_reach", [("d2q9", False, True), ("burgers", True, False)])
def test_level_skipping_needs_both_terms(name, keep_history, use_reach):
    """The check has teeth: without the mesh before the old one (coarsening
    leaves its codes in the buffer being rewritten), or without the reach of
    the refinement (new levels), some buffer goes stale."""
    cfg, m0, steps = _activity_case(name)
    o = oracle.Oracle(cfg)
    tree, v = o.init(m0)
    bad, _ = _activity_run(o, cfg, tree, v, steps, keep_history, use_reach)
    assert bad > 0
