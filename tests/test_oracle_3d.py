"""Pins of the oracle's three-dimensional path (section "Three dimensional
advection equation": the D3Q6 scheme; section "Projection and prediction
operators": the d = 3 prediction) against what the paper and mathematics fix,
with no GPU: the printed D3Q6 matrix and velocities, the Kronecker product of
three 1D predictions of Table 1, exactness on tensor products of quadratics,
the reduction to the 2D prediction, the transport against sums of an
independently built finest-level reconstruction, the uniform limit against a
numpy stream-and-collide, grading and mass conservation."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
V = (0.3, 0.2, 0.1)


def _cfg(jmin=2, jmax=5, eps=1e-3, mu_bar=1.0, s1=1.4, s2=1.0, gamma=1, metric="linf", vel=V):
    return W.params("D3Q6", jmin, jmax, eps, W.d3q6_s(s1, s2), mu_bar=mu_bar, lam=1.0, gamma=gamma,
                    metric=metric, velocity=vel)


def _c1d(gamma):
    with open(os.path.join(GOLD, "table1_prediction_coefficients.json")) as f:
        return [float(Fr(v)) for v in json.load(f)["coefficients"][str(gamma)]]


def _p1(n, gamma):
    """1D periodic prediction matrix (2n x n) of Table 1: child 2k + d of parent k
    is f_k + (-1)^d sum_a c_a (f_{k+a} - f_{k-a})."""
    c = _c1d(gamma)
    P = np.zeros((2 * n, n))
    for k in range(n):
        for d in (0, 1):
            s = 1.0 if d == 0 else -1.0
            P[2 * k + d, k] += 1.0
            for a in range(1, gamma + 1):
                P[2 * k + d, (k + a) % n] += s * c[a - 1]
                P[2 * k + d, (k - a) % n] -= s * c[a - 1]
    return P


def _p3(n, gamma):
    """Three-dimensional prediction as the Kronecker product of three 1D ones, for
    the cell index x + n (y + n z) (z outermost)."""
    P = _p1(n, gamma)
    return np.kron(P, np.kron(P, P))


# ------------------------------------------------------------ D3Q6 scheme

def test_d3q6_matrix_and_velocities_as_printed():
    o = oracle.Oracle(_cfg())
    L = 1.0
    M = np.array([[1, 1, 1, 1, 1, 1],
                  [L, -L, 0, 0, 0, 0],
                  [0, 0, L, -L, 0, 0],
                  [0, 0, 0, 0, L, -L],
                  [L * L, L * L, -L * L, -L * L, 0, 0],
                  [L * L, L * L, 0, 0, -L * L, -L * L]], float)
    assert np.array_equal(o.moment_matrix(), M)
    assert np.allclose(o.moment_matrix_inverse() @ M, np.eye(6), atol=1e-15)
    eta = o.velocities()
    want = np.array([[round(np.cos(np.pi * h)) if h // 2 == a else 0 for a in range(3)] for h in range(6)])
    assert np.array_equal(eta, want)


def test_d3q6_lambda_scales_the_matrix():
    cfg = _cfg()
    cfg["lam"] = 2.0
    o = oracle.Oracle(cfg)
    M = o.moment_matrix()
    assert np.array_equal(M[1], [2, -2, 0, 0, 0, 0]) and np.array_equal(M[4], [4, 4, -4, -4, 0, 0])


def test_d3q6_equilibrium_and_collision():
    o = oracle.Oracle(_cfg())
    u = 0.7
    assert np.allclose(o.equilibrium([u, 9, 9, 9, 9, 9]), [u, V[0] * u, V[1] * u, V[2] * u, 0, 0], rtol=0, atol=0)
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, 6)
    M = o.moment_matrix()
    m = M @ f
    g = o.collide_cell(f)
    mg = M @ g
    s = np.array(W.d3q6_s())
    meq = np.array([m[0], V[0] * m[0], V[1] * m[0], V[2] * m[0], 0, 0])
    assert np.allclose(mg, m + s * (meq - m), atol=1e-14)
    assert abs(mg[0] - m[0]) <= 1e-15


# ------------------------------------------------------------ 3D prediction

@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_prediction_is_kronecker_product_of_1d(gamma):
    o = oracle.Oracle(_cfg(jmin=2, jmax=5, gamma=gamma))
    n = 8  # parent level 3, children at level 4
    F = np.random.default_rng(gamma).normal(size=n ** 3)
    want = _p3(n, gamma) @ F
    N = 2 * n
    got = np.array([o.predict(F, 4, x, y, z) for z in range(N) for y in range(N) for x in range(N)])
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_prediction_exact_on_tensor_products_of_quadratics():
    """Table 1's gamma = 1 operator is exact on quadratics (cell averages); the
    tensor product is exact on every x^a y^b z^c with a, b, c <= 2. A wrong sign
    of a pair term fails x y, of the triple term x y z."""
    o = oracle.Oracle(_cfg(jmin=2, jmax=5))
    n = 8

    def avg(p, lo, w):  # average of x^p over [lo, lo + w]
        return ((lo + w) ** (p + 1) - lo ** (p + 1)) / ((p + 1) * w)

    for (a, b, c) in [(1, 0, 0), (2, 0, 0), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1), (2, 1, 1), (2, 2, 2)]:
        F = np.array([avg(a, x, 1.0) * avg(b, y, 1.0) * avg(c, z, 1.0)
                      for z in range(n) for y in range(n) for x in range(n)])
        worst = 0.0
        for cz in range(2, 2 * n - 2):
            for cy in range(2, 2 * n - 2):
                for cx in range(2, 2 * n - 2):
                    exact = avg(a, cx / 2, 0.5) * avg(b, cy / 2, 0.5) * avg(c, cz / 2, 0.5)
                    worst = max(worst, abs(o.predict(F, 4, cx, cy, cz) - exact) / (1 + abs(exact)))
        assert worst <= 1e-13, (a, b, c, worst)


def test_prediction_of_z_constant_data_is_the_2d_prediction():
    o3 = oracle.Oracle(_cfg(jmin=2, jmax=5))
    o2 = oracle.Oracle(W.params("D2Q9", 2, 5, 1e-3, W.d2q9_s(1.5, 1.8), mu_bar=1.0))
    n = 8
    F2 = np.random.default_rng(5).normal(size=n * n)
    F3 = np.tile(F2, n)
    for cz in (0, 5, 15):
        for cy in range(0, 16, 3):
            for cx in range(0, 16, 5):
                assert abs(o3.predict(F3, 4, cx, cy, cz) - o2.predict(F2, 4, cx, cy)) <= 1e-15


def test_projection_of_prediction_is_identity():
    o = oracle.Oracle(_cfg(jmin=2, jmax=4, eps=1e30))
    cfg = _cfg(jmin=2, jmax=4, eps=1e30)
    m0 = W.random_field(cfg, 4)
    tree, v = o.init(m0)
    dense = o.reconstruct(tree, v)
    # predictions of level 3 from level 2, averaged over the eight children, give level 2 back
    F2 = o.values_level(dense, 2)[0].ravel()
    kids = np.array([o.predict(F2, 3, x, y, z) for z in range(8) for y in range(8) for x in range(8)])
    avg = kids.reshape(4, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5)).ravel()
    assert np.max(np.abs(avg - F2)) <= 1e-15 * np.max(np.abs(F2))


# ------------------------------------------------------------ reconstruction and transport

def _coarse_tree(o, level):
    """Graded tree whose leaves are all the cells of `level`."""
    tree = np.zeros(o.total, np.uint8)
    for l in range(o.jmin, level + 1):
        tree[o.level_offset(l):o.level_offset(l) + o.ncells(l)] = 1
    return tree


@pytest.mark.parametrize("level", [2, 3])
def test_finest_reconstruction_is_repeated_kronecker_prediction(level):
    cfg = _cfg(jmin=2, jmax=5)
    o = oracle.Oracle(cfg)
    tree = _coarse_tree(o, level)
    assert o.check_tree(tree) == 0
    rng = np.random.default_rng(level)
    v = np.zeros(o.q * o.total)
    for l in range(o.jmin, level + 1):
        o.values_level(v, l)[...] = rng.normal(size=o.values_level(v, l).shape)
    fin = o.finest(tree, v).reshape(o.q, -1)
    for h in range(o.q):
        f = o.values_level(v, level)[h].ravel()
        for l in range(level, o.jmax):
            f = _p3(1 << l, 1) @ f
        assert np.max(np.abs(fin[h] - f)) <= 1e-13 * np.max(np.abs(f))


def test_transport_on_a_coarse_mesh_against_finest_sums():
    """eq. AdaptiveAdvectionPhase: a leaf's new value is f + 2^{-3n}(sum over E -
    sum over A) of the finest-level reconstruction; here that reconstruction is
    the repeated Kronecker prediction and the sums are taken with numpy."""
    cfg = _cfg(jmin=2, jmax=5)
    o = oracle.Oracle(cfg)
    level = 3
    tree = _coarse_tree(o, level)
    v = np.zeros(o.q * o.total)
    o.values_level(v, level)[...] = np.random.default_rng(11).normal(size=o.values_level(v, level).shape)
    dense = o.reconstruct(tree, v)
    out = o.transport(tree, dense)
    n = o.jmax - level
    w = 1 << n
    N = 1 << o.jmax
    eta = o.velocities()
    for h in range(o.q):
        f = o.values_level(v, level)[h].ravel()
        for l in range(level, o.jmax):
            f = _p3(1 << l, 1) @ f
        fJ = f.reshape(N, N, N)  # [z][y][x]
        ex, ey, ez = (int(e) for e in eta[h])
        # streamed field: g(k) = fJ(k - eta); the new leaf value is the block mean of g
        g = np.roll(fJ, shift=(ez, ey, ex), axis=(0, 1, 2))
        want = g.reshape(N // w, w, N // w, w, N // w, w).mean(axis=(1, 3, 5)).ravel()
        got = o.values_level(out, level)[h].ravel()
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # the E/A form equals the definition form on an adapted mesh as well
    cfg2, m0 = W.ball_d3q6(jmin=2, jmax=5)
    o2 = oracle.Oracle(cfg2)
    t, vv = o2.init(m0)
    o2.step(t, vv, 2)
    d2 = o2.reconstruct(t, vv)
    a, b = o2.transport(t, d2), o2.transport(t, d2, definition_form=True)
    assert np.max(np.abs(a - b)) <= 1e-14


def _numpy_uniform_step(o, fJ):
    """Stream f_h(k) <- f_h(k - eta_h) (periodic) and collide with the printed M,
    S = diag(0, s1, s1, s1, s2, s2) and m_eq = (u, V u, 0, 0)."""
    N = 1 << o.jmax
    eta = o.velocities()
    f = fJ.reshape(o.q, N, N, N)
    g = np.stack([np.roll(f[h], shift=(int(eta[h][2]), int(eta[h][1]), int(eta[h][0])), axis=(0, 1, 2))
                  for h in range(o.q)]).reshape(o.q, -1)
    M = o.moment_matrix()
    m = M @ g
    s = np.array(W.d3q6_s())[:, None]
    meq = np.stack([m[0], V[0] * m[0], V[1] * m[0], V[2] * m[0], 0 * m[0], 0 * m[0]])
    return np.linalg.solve(M, m + s * (meq - m))


def test_uniform_limit_eps_zero_is_the_reference_scheme():
    """With eps = 0 every detail passes the threshold: the mesh stays full at J
    and the adaptive step is the reference scheme on level J."""
    cfg = _cfg(jmin=2, jmax=4, eps=0.0)
    o = oracle.Oracle(cfg)
    m0 = W.random_field(cfg, 7, "jump")
    tree, v = o.init(m0)
    fJ = o.values_level(v, o.jmax).reshape(o.q, -1).copy()
    ref = fJ.copy()
    for _ in range(5):
        o.step(tree, v)
        ref = _numpy_uniform_step(o, ref)
        o.uniform_step(fJ)
    assert o.leaf_counts(tree)[o.jmax] == o.ncells(o.jmax)
    got = o.values_level(v, o.jmax).reshape(o.q, -1)
    assert np.array_equal(got, fJ)
    assert np.max(np.abs(got - ref)) <= 1e-13


# ------------------------------------------------------------ mesh

def _graded(o, tree):
    """Independent check of a 3D complete graded tree: jmin full, sibling groups
    complete, every tree cell's parent's 3^3 box (periodic) in the tree."""
    if not o.tree_level(tree, o.jmin).all():
        return False
    for l in range(o.jmin + 1, o.jmax + 1):
        t = o.tree_level(tree, l).astype(bool)
        n = 1 << (l - 1)
        groups = t.reshape(n, 2, n, 2, n, 2)
        cnt = groups.sum(axis=(1, 3, 5))
        if not np.all((cnt == 0) | (cnt == 8)):
            return False
        need = cnt > 0
        box = np.zeros_like(need)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    box |= np.roll(need, shift=(dz, dy, dx), axis=(0, 1, 2))
        if np.any(box & ~o.tree_level(tree, l - 1).astype(bool)):
            return False
    return True


@pytest.mark.parametrize("metric", ["linf", "l2"])
def test_ball_meshes_graded_and_mass_conserved(metric):
    cfg, m0 = W.ball_d3q6(jmin=2, jmax=5, metric=metric)
    o = oracle.Oracle(cfg)
    tree, v = o.init(m0)
    mass0 = o.mass(tree, v)
    seen = set()
    for _ in range(6):
        o.step(tree, v)
        assert _graded(o, tree) and o.check_tree(tree) == 0
        assert abs(o.mass(tree, v) - mass0) <= 1e-12 * abs(mass0)
        seen |= {l for l, c in enumerate(o.leaf_counts(tree)) if c}
    assert len(seen) >= 3


def test_constant_data_coarsens_to_jmin():
    """Details vanish where the prediction is exact: a periodic field that is
    constant coarsens to level jmin in one adaptation, whatever eps > 0."""
    cfg = _cfg(jmin=2, jmax=5, eps=1e-12)
    o = oracle.Oracle(cfg)
    m0 = np.full((1, 1 << 15), 0.25)
    tree, v = o.init(m0)
    tnew = o.new_tree_from_state(tree, v)
    counts = o.leaf_counts(tnew)
    # the initial full mesh keeps its finest level (T_eps on the old tree; the
    # neighbour addition and grading add no finer cells), then coarsens a level per step
    for _ in range(4):
        o.step(tree, v)
    assert o.leaf_counts(tree)[o.jmin] == o.ncells(o.jmin), (counts, o.leaf_counts(tree))


def test_float_decision_matches_double_away_from_thresholds():
    cfg, m0 = W.ball_d3q6(jmin=2, jmax=5)
    o = oracle.Oracle(cfg)
    tree, v = o.init(m0)
    for _ in range(3):
        o.step(tree, v)
        t64 = o.new_tree_from_state(tree, v)
        t32 = o.new_tree_f32(tree, v.astype(np.float32))
        assert np.array_equal(t64, t32)


def test_3d_refuses_walls_and_adjoint():
    cfg = _cfg(jmin=2, jmax=4)
    cfg["bc"] = (2, 2, 0, 0)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 1))
    with pytest.raises(RuntimeError):
        o.step(tree, v)
    o = oracle.Oracle(_cfg(jmin=2, jmax=4))
    tree, v = o.init(W.random_field(_cfg(jmin=2, jmax=4), 1))
    with pytest.raises(RuntimeError):
        o.adjoint_step(tree, tree, v, np.zeros_like(v))
