"""Pins of the oracle's walls (section "Boundary conditions"; no GPU).

* Uniform limit: with jmin = J, or eps = 0, the adapted scheme with walls is
  bit for bit the uniform scheme with the same conditions (whose boundary cells
  take their own value of the population, or of its opposite, eq.
  refBoundaryConditions), in both evaluations of the wall values.
* D1Q2 at Courant 1 with copy conditions: the uniform solution is the datum
  shifted by one cell per step, the inflow cell repeating its own value: exact.
* Bounce back with the wall values taken on the reconstruction conserves the
  mass of the adapted scheme to round-off (the incoming finest values are the
  outgoing ones of the opposite velocity); copy does not.
* Direct evaluation on the leaf (the paper's choice) equals the evaluation on
  the reconstruction wherever the reconstruction of a wall leaf is its own
  value: one step from data that are constant near the walls.
* Even reflection: the reconstruction and the details with walls equal those
  of the periodic problem on the mirrored domain twice as large (one level
  more per axis), restricted to the original cells; bit for bit in 1D, to
  round-off in 2D (the 2D cross term sums its four values in another order
  after the mirror).
"""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

KINDS = {"copy": 1, "bounce_back": 2, "anti_bounce_back": 3}


def _cfg(scheme, jmin, jmax, eps, bc, bc_eval=0, mu_bar=1.0):
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=mu_bar, eq_param=0.5 if scheme == "D1Q3" else 1.0, bc=bc,
                    bc_eval=bc_eval)


def _walls(scheme, kind, other=None):
    k = KINDS[kind]
    o = KINDS[other] if other else k
    return (k, o, 0, 0) if scheme != "D2Q9" else (k, o, o, k)


def _leaf_fJ(o, tree, values):
    """Values of the finest level as [q][N_J^d] (every finest cell a leaf)."""
    return o.values_level(values, o.jmax).reshape(o.q, -1).copy()


@pytest.mark.parametrize("scheme,J", [("D1Q2", 8), ("D1Q3", 8), ("D2Q9", 5)])
@pytest.mark.parametrize("kind", ["copy", "bounce_back", "anti_bounce_back"])
@pytest.mark.parametrize("mode", ["jmin=J", "eps=0"])
@pytest.mark.parametrize("bc_eval", [0, 1])
def test_walls_reduce_bitwise_to_uniform(scheme, J, kind, mode, bc_eval):
    jmin, eps = (J, 1e-3) if mode == "jmin=J" else (2, 0.0)
    cfg = _cfg(scheme, jmin, J, eps, _walls(scheme, kind, "copy" if kind != "copy" else "bounce_back"), bc_eval)
    o = oracle.Oracle(cfg)
    m0 = W.random_field(cfg, 3, "jump")
    tree, v = o.init(m0)
    fJ = _leaf_fJ(o, tree, v).ravel()
    for _ in range(12):
        o.step(tree, v)
        o.uniform_step(fJ)
        assert tree.all() if mode == "eps=0" else True
        assert np.array_equal(_leaf_fJ(o, tree, v).ravel(), fJ)


def test_d1q2_copy_courant_one_is_exact_shift():
    J = 7
    cfg = _cfg("D1Q2", J, J, 1e-3, _walls("D1Q2", "copy"))
    o = oracle.Oracle(cfg)
    u0 = np.random.default_rng(5).uniform(-1, 1, 1 << J)
    fJ = np.concatenate([u0, np.zeros_like(u0)])  # f+ = u, f- = 0: the equilibrium of V = lambda = 1
    tree, v = o.init(u0[None, :])
    assert np.array_equal(_leaf_fJ(o, tree, v).ravel(), fJ)
    for n in range(1, 200):
        o.step(tree, v)
        o.uniform_step(fJ)
        want = u0[np.maximum(np.arange(1 << J) - n, 0)]
        assert np.array_equal(fJ[: 1 << J], want) and not fJ[1 << J:].any()
        assert np.array_equal(_leaf_fJ(o, tree, v)[0], want)


@pytest.mark.parametrize("scheme,jmin,jmax,eps", [("D1Q2", 2, 9, 1e-3), ("D1Q3", 2, 9, 1e-3),
                                                  ("D2Q9", 2, 6, 1e-3), ("D2Q9", 3, 7, 1e-4)])
def test_bounce_back_on_reconstruction_conserves_mass(scheme, jmin, jmax, eps):
    cfg = _cfg(scheme, jmin, jmax, eps, _walls(scheme, "bounce_back"), bc_eval=1)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 11, "jump"))
    m0 = o.mass(tree, v)
    levels = set()
    for _ in range(30):
        o.step(tree, v)
        assert o.check_tree(tree) == 0
        levels |= {l for l, k in enumerate(o.leaf_counts(tree)) if k}
        assert abs(o.mass(tree, v) - m0) <= 1e-13 * max(1.0, abs(m0)) * o.ncells(jmax) ** 0.5
    assert len(levels) >= 2  # the mesh is adapted, not uniform
    # the copy condition lets mass in and out
    cfg_c = _cfg(scheme, jmin, jmax, eps, _walls(scheme, "copy"), bc_eval=1)
    oc = oracle.Oracle(cfg_c)
    tree, v = oc.init(W.random_field(cfg, 11, "jump"))
    oc.step(tree, v, 30)
    assert abs(oc.mass(tree, v) - m0) > 1e-9 * max(1.0, abs(m0))


def _constant_near_walls(cfg, seed):
    """A datum equal to a constant state except in the middle fifth of each axis."""
    m = W.random_field(cfg, seed, "smooth")
    n = 1 << cfg["jmax"]
    xc = (np.arange(n) + 0.5) / n
    inside = (xc > 0.4) & (xc < 0.6)
    if cfg["dim"] == 2:
        inside = inside[None, :] & inside[:, None]
    const = m[:, :1].copy()
    return np.where(inside.ravel()[None, :], m, const)


@pytest.mark.parametrize("scheme,jmin,jmax", [("D1Q2", 3, 9), ("D1Q3", 3, 9), ("D2Q9", 3, 6)])
@pytest.mark.parametrize("kind", ["copy", "bounce_back", "anti_bounce_back"])
def test_direct_evaluation_equals_reconstruction_on_constant_walls(scheme, jmin, jmax, kind):
    m0 = None
    out = []
    for bc_eval in (0, 1):
        cfg = _cfg(scheme, jmin, jmax, 1e-3, _walls(scheme, kind), bc_eval)
        if m0 is None:
            m0 = _constant_near_walls(cfg, 4)
        o = oracle.Oracle(cfg)
        tree, v = o.init(m0)
        o.step(tree, v)
        out.append((tree, v))
        counts = o.leaf_counts(tree)
    assert np.array_equal(out[0][0], out[1][0])
    mask = np.concatenate([np.repeat(o.leaf_mask(out[0][0], l).ravel()[None, :], o.q, 0).ravel()
                           for l in range(jmin, jmax + 1)])
    assert np.array_equal(out[0][1][mask], out[1][1][mask])
    assert counts[jmin] > 0 and counts[jmax] > 0  # walls on coarse leaves, fine cells in the middle


def _mirror_level(a, dim):
    """Level array [..., N] or [..., N, N] extended to 2N by even reflection."""
    if dim == 1:
        return np.concatenate([a, a[..., ::-1]], axis=-1)
    a = np.concatenate([a, a[..., ::-1]], axis=-1)
    return np.concatenate([a, a[..., ::-1, :]], axis=-2)


@pytest.mark.parametrize("scheme,jmin,jmax,eps", [("D1Q3", 2, 8, 1e-3), ("D2Q9", 2, 5, 1e-3),
                                                  ("D2Q9", 3, 6, 1e-4)])
def test_reflection_equals_mirrored_periodic_problem(scheme, jmin, jmax, eps):
    cfg = _cfg(scheme, jmin, jmax, eps, _walls(scheme, "bounce_back"))
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 2, "jump"))
    o.step(tree, v, 3)
    cfg2 = _cfg(scheme, jmin + 1, jmax + 1, eps, None)
    o2 = oracle.Oracle(cfg2)
    t2, v2 = o2.new_state()
    for l in range(jmin, jmax + 1):
        o2.tree_level(t2, l + 1)[...] = _mirror_level(o.tree_level(tree, l), o.dim)
        o2.values_level(v2, l + 1)[...] = _mirror_level(o.values_level(v, l), o.dim)
    assert o2.check_tree(t2) == 0
    dense = o.reconstruct(tree, v)
    dense2 = o2.reconstruct(t2, v2)
    D = o.details(tree, dense)
    D2 = o2.details(t2, dense2)
    tol = 0.0 if o.dim == 1 else 4e-16
    for l in range(jmin, jmax + 1):
        n = 1 << l
        a = o.values_level(dense, l)
        b = o2.values_level(dense2, l + 1)
        b = b[..., :n] if o.dim == 1 else b[..., :n, :n]
        assert np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(a)))
        da = D[o.level_offset(l):o.level_offset(l) + o.ncells(l)].reshape(a.shape[1:])
        db = D2[o2.level_offset(l + 1):o2.level_offset(l + 1) + o2.ncells(l + 1)]
        db = db.reshape((2 * n, 2 * n) if o.dim == 2 else (2 * n,))
        db = db[:n] if o.dim == 1 else db[:n, :n]
        assert np.max(np.abs(da - db)) <= tol * 10


def test_wall_parameters_are_checked():
    cfg = _cfg("D1Q3", 2, 6, 1e-3, (1, 0, 0, 0))  # one side periodic, the other a wall
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 1))
    with pytest.raises(RuntimeError):
        o.step(tree, v)
    cfg = _cfg("D2Q9", 2, 4, 1e-3, (2, 2, 2, 2))
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 1))
    with pytest.raises(RuntimeError):  # the adjoint covers periodic boundaries only
        o.adjoint_step(tree, tree, v, np.zeros_like(v))
