"""Pins of the oracle adjoint (frozen meshes): every transpose passes the
dot-product test against its forward map, the linearised collision and the
initial-datum map match central differences of the forward, and the whole
adjoint gradient matches central finite differences of the frozen-mesh run."""
import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W
from adjoint_helpers import ke_functional as _ke_functional


def _cfg(scheme, jmin, jmax, eps):
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=1.0, eq_param=0.5 if scheme == "D1Q3" else 1.0)


def _leafmask_flat(o, tree):
    m = np.zeros(o.q * o.total, bool)
    for l in range(o.jmin, o.jmax + 1):
        lm = o.leaf_mask(tree, l).ravel()
        off = o.q * o.level_offset(l)
        for h in range(o.q):
            m[off + h * o.ncells(l): off + (h + 1) * o.ncells(l)] = lm
    return m


SCHEMES = [("D1Q3", 2, 8), ("D2Q9", 2, 5)]


@pytest.mark.parametrize("scheme,jmin,jmax", SCHEMES)
def test_predict_stencil_reproduces_prediction(scheme, jmin, jmax):
    o = oracle.Oracle(_cfg(scheme, jmin, jmax, 1e-3))
    rng = np.random.default_rng(0)
    l = jmax
    F = rng.normal(size=o.ncells(l - 1))
    for _ in range(20):
        cx, cy = (int(v) for v in rng.integers(0, 1 << l, 2))
        idx, w = o.predict_stencil(l, cx, cy if o.dim == 2 else 0)
        assert abs(np.dot(w, F[idx]) - o.predict(F, l, cx, cy if o.dim == 2 else 0)) <= 1e-14


@pytest.mark.parametrize("scheme,jmin,jmax", SCHEMES)
def test_dot_product_reconstruct_transport_transfer(scheme, jmin, jmax):
    o = oracle.Oracle(_cfg(scheme, jmin, jmax, 1e-3))
    rng = np.random.default_rng(1)
    # a new mesh must have every cell's parent in the old one: take a step's mesh
    m0 = W.random_field(_cfg(scheme, jmin, jmax, 1e-3), 3, "jump")
    t0, v0 = o.init(m0)
    o.step(t0, v0, 2)
    told = t0.copy()
    tnew = o.new_tree_from_state(told, v0)
    L_old, L_new = _leafmask_flat(o, told), _leafmask_flat(o, tnew)
    # reconstruction R: leaf values -> dense
    x = np.where(L_old, rng.normal(size=o.q * o.total), 0.0)
    y = rng.normal(size=o.q * o.total)
    lhs = np.dot(o.reconstruct(told, x), y)
    rhs = np.dot(x, o.reconstruct_T(told, y))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # transport T: dense -> leaves of tnew
    G = rng.normal(size=o.q * o.total)
    ob = np.where(L_new, rng.normal(size=o.q * o.total), 0.0)
    lhs = np.dot(np.where(L_new, o.transport(tnew, G), 0.0), ob)
    rhs = np.dot(G, o.transport_T(tnew, ob))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # transfer X: dense (old) -> leaves of tnew
    g = np.where(L_new, rng.normal(size=o.q * o.total), 0.0)
    lhs = np.dot(np.where(L_new, o.transfer(told, G, tnew), 0.0), g)
    rhs = np.dot(G, o.transfer_T(tnew, g))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("scheme", ["D1Q2", "D1Q3", "D2Q9"])
def test_equilibrium_jacobian_and_collision_adjoint_vs_differences(scheme):
    o = oracle.Oracle(_cfg(scheme, 2, 4, 1e-3))
    rng = np.random.default_rng(2)
    M = o.moment_matrix()
    feq = o.moment_matrix_inverse() @ o.equilibrium(np.r_[1.0, 0.05, -0.03, np.zeros(6)][:o.q] if o.q == 9
                                                    else np.r_[0.3, np.zeros(o.q - 1)])
    f = feq + 0.01 * rng.normal(size=o.q)
    m = M @ f
    Je = o.equilibrium_jacobian(m)
    h = 1e-6
    for j in range(o.q):
        dm = np.zeros(o.q)
        dm[j] = h
        fd = (o.equilibrium(m + dm) - o.equilibrium(m - dm)) / (2 * h)
        assert np.allclose(Je[:, j], fd, atol=1e-8)
    # collision adjoint on a one-leaf tree: <J_C df, a> = <df, J_C^T a>, J_C df by differences
    cfg = _cfg(scheme, 2, 2, 1e-3)
    o1 = oracle.Oracle(cfg)
    tree = np.ones(o1.total, np.uint8)
    H = np.tile(f[:, None], (1, o1.total)).ravel()
    a = rng.normal(size=o1.q * o1.total)
    hb, sb = o1.collide_T(tree, H, a)
    df = rng.normal(size=o1.q * o1.total)
    jv = (o1.collide(tree, H + h * df) - o1.collide(tree, H - h * df)) / (2 * h)
    assert abs(np.dot(jv, a) - np.dot(df, hb)) <= 1e-7 * (1 + abs(np.dot(df, hb)))
    # derivative with respect to each relaxation rate
    for k in range(o1.q):
        if cfg["s"][k] == 0:
            continue
        cp, cm = dict(cfg), dict(cfg)
        cp["s"] = list(cfg["s"]); cm["s"] = list(cfg["s"])
        cp["s"][k] += h; cm["s"][k] -= h
        fd = (np.dot(oracle.Oracle(cp).collide(tree, H), a) - np.dot(oracle.Oracle(cm).collide(tree, H), a)) / (2 * h)
        assert abs(fd - sb[k]) <= 1e-7 * (1 + abs(fd))


@pytest.mark.parametrize("scheme,jmin,jmax,steps", [("D1Q3", 2, 7, 12), ("D2Q9", 2, 5, 8)])
def test_adjoint_gradient_vs_central_differences(scheme, jmin, jmax, steps):
    cfg = _cfg(scheme, jmin, jmax, 1e-3)
    o = oracle.Oracle(cfg)
    m0 = W.random_field(cfg, 4, "smooth")
    # the mesh sequence of a normal adaptive run, then frozen
    t, v = o.init(m0)
    trees = [t.copy()]
    for _ in range(steps):
        o.step(t, v)
        trees.append(t.copy())
    states = o.run_frozen(m0, trees)
    J0, dJdf = _ke_functional(o, *states[-1])
    mbar, sbar = o.gradient_frozen(m0, trees, dJdf)
    rng = np.random.default_rng(6)
    h = 1e-6
    for trial in range(2):
        dm = rng.normal(size=m0.shape) * (0.01 if o.q == 9 else 0.05)
        Jp = _ke_functional(o, *o.run_frozen(m0 + h * dm, trees)[-1])[0]
        Jm = _ke_functional(o, *o.run_frozen(m0 - h * dm, trees)[-1])[0]
        fd = (Jp - Jm) / (2 * h)
        ad = float(np.sum(mbar * dm))
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-10), (fd, ad)
    # relaxation rate of the last non-conserved moments (s2 for D2Q9)
    k = o.q - 1
    cp, cm = dict(cfg), dict(cfg)
    cp["s"] = list(cfg["s"]); cm["s"] = list(cfg["s"])
    idx = [7, 8] if o.q == 9 else [k]
    for i in idx:
        cp["s"][i] += h
        cm["s"][i] -= h
    Jp = _ke_functional(o, *oracle.Oracle(cp).run_frozen(m0, trees)[-1])[0]
    Jm = _ke_functional(o, *oracle.Oracle(cm).run_frozen(m0, trees)[-1])[0]
    fd = (Jp - Jm) / (2 * h)
    ad = float(sum(sbar[i] for i in idx))
    assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-10), (fd, ad)
