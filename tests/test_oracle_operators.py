"""Pins of the oracle's multiresolution operators against what the paper and
mathematics fix (no GPU). Each test names the passage it checks."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_2103_02903_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _cfg(scheme="D1Q3", jmin=2, jmax=6, eps=1e-3):
    dim, q, _ = W.SCHEME_DIMS[scheme]
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=1.0, eq_param=0.5 if scheme == "D1Q3" else 1.0)


# ------------------------------------------------------------ Table 1 / Appendix 2

def _solve_exact(A, b):
    n = len(A)
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def appendix2_coefficients(gamma):
    """Appendix 2: fit the degree-2*gamma polynomial whose averages on the cells
    k-gamma..k+gamma are the data, average it on the left child; return c_alpha."""
    offs = list(range(-gamma, gamma + 1))
    deg = 2 * gamma
    T = [[(Fr(2 * d + 1, 2) ** (m + 1) - Fr(2 * d - 1, 2) ** (m + 1)) / (m + 1) for m in range(deg + 1)]
         for d in offs]
    # weight of each datum f_{k+d} in the left-child average 2 * int_{-1/2}^{0} pi
    weights = []
    for j in range(len(offs)):
        e = [Fr(int(i == j)) for i in range(len(offs))]
        A = _solve_exact(T, e)
        weights.append(sum(2 * A[m] * (Fr(0) - Fr(-1, 2) ** (m + 1)) / (m + 1) for m in range(deg + 1)))
    w = dict(zip(offs, weights))
    assert w[0] == 1
    for a in range(1, gamma + 1):
        assert w[a] == -w[-a]
    return [w[a] for a in range(1, gamma + 1)]


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_table1_regenerated_by_appendix2(gamma):
    printed = [Fr(s) for s in _gold("table1_prediction_coefficients.json")["coefficients"][str(gamma)]]
    assert appendix2_coefficients(gamma) == printed


def test_oracle_prediction_uses_table1_gamma1():
    c1 = float(Fr(_gold("table1_prediction_coefficients.json")["coefficients"]["1"][0]))
    o = oracle.Oracle(_cfg("D1Q3", 2, 6))
    for p in [0, 3, 7]:
        F = np.zeros(8)
        F[(p + 1) % 8] = 1.0
        assert o.predict(F, 4, 2 * p) == c1            # left child
        assert o.predict(F, 4, 2 * p + 1) == -c1       # right child
        F = np.zeros(8)
        F[p] = 1.0
        assert o.predict(F, 4, 2 * p) == 1.0


def test_prediction_2d_weights_against_figure():
    g = _gold("prediction_weights_2d.json")["printed"]
    pos = {"C": (0, 0), "E": (1, 0), "W": (-1, 0), "N": (0, 1), "S": (0, -1),
           "NE": (1, 1), "SW": (-1, -1), "NW": (-1, 1), "SE": (1, -1)}
    o = oracle.Oracle(_cfg("D2Q9", 3, 6))
    n = 8
    px, py = 3, 4
    for key, (ax, ay) in pos.items():
        F = np.zeros((n, n))
        F[py + ay, px + ax] = 1.0
        w = o.predict(F, 4, 2 * px, 2 * py)  # lower-left child
        printed = float(Fr(g[key]))
        if len(key) == 2:  # diagonal: magnitude as printed, sign of the tensor product
            assert abs(w) == abs(printed) == 1.0 / 64
            assert w == -printed
        else:
            assert w == printed


# ------------------------------------------------------------ polynomial exactness

def _avg1d(coefs, a, b):
    """Exact average of sum_m coefs[m] x^m over [a, b]."""
    return sum(c * (b ** (m + 1) - a ** (m + 1)) / (m + 1) for m, c in enumerate(coefs)) / (b - a)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_prediction_1d_exact_on_degree_2gamma(deg):
    """Section 'Projection and prediction operators': exact for degree <= 2 gamma."""
    rng = np.random.default_rng(deg)
    coefs = [Fr(int(v), 7) for v in rng.integers(-20, 20, deg + 1)]
    o = oracle.Oracle(_cfg("D1Q3", 2, 7))
    n = 32
    F = np.array([float(_avg1d(coefs, Fr(k, n), Fr(k + 1, n))) for k in range(n)])
    for p in range(1, n - 1):
        for dlt in (0, 1):
            exact = float(_avg1d(coefs, Fr(2 * p + dlt, 2 * n), Fr(2 * p + dlt + 1, 2 * n)))
            assert abs(o.predict(F, 6, 2 * p + dlt) - exact) <= 1e-13 * (1 + abs(exact))


def test_prediction_1d_not_exact_on_cubic():
    o = oracle.Oracle(_cfg("D1Q3", 2, 7))
    n = 32
    coefs = [Fr(0), Fr(0), Fr(0), Fr(1)]
    F = np.array([float(_avg1d(coefs, Fr(k, n), Fr(k + 1, n))) for k in range(n)])
    p = 10
    exact = float(_avg1d(coefs, Fr(2 * p, 2 * n), Fr(2 * p + 1, 2 * n)))
    assert abs(o.predict(F, 6, 2 * p) - exact) > 1e-9


@pytest.mark.parametrize("a,b", [(a, b) for a in range(3) for b in range(3)])
def test_prediction_2d_exact_on_q2_monomials(a, b):
    """Tensor-product prediction is exact on x^a y^b, a, b <= 2 (this fixes the
    sign of the cross term)."""
    o = oracle.Oracle(_cfg("D2Q9", 3, 6))
    n = 16
    ca = [Fr(0)] * a + [Fr(1)]
    cb = [Fr(0)] * b + [Fr(1)]
    ax = [_avg1d(ca, Fr(k, n), Fr(k + 1, n)) for k in range(n)]
    by = [_avg1d(cb, Fr(k, n), Fr(k + 1, n)) for k in range(n)]
    F = np.array([[float(ax[i] * by[j]) for i in range(n)] for j in range(n)])
    for py in range(1, n - 1, 3):
        for px in range(1, n - 1, 3):
            for dx in (0, 1):
                for dy in (0, 1):
                    cx, cy = 2 * px + dx, 2 * py + dy
                    ex = _avg1d(ca, Fr(cx, 2 * n), Fr(cx + 1, 2 * n)) * _avg1d(cb, Fr(cy, 2 * n), Fr(cy + 1, 2 * n))
                    assert abs(o.predict(F, 5, cx, cy) - float(ex)) <= 1e-14


# ------------------------------------------------------------ consistency and details

@pytest.mark.parametrize("scheme", ["D1Q3", "D2Q9"])
def test_projection_of_prediction_is_identity(scheme):
    """eq. ConsistencyPrediction: P_nabla(P_delta(f)) = f, to round-off."""
    o = oracle.Oracle(_cfg(scheme, 2, 6))
    rng = np.random.default_rng(1)
    n = 16
    F = rng.normal(size=(n,) if o.dim == 1 else (n, n))
    for p in range(n):
        if o.dim == 1:
            avg = 0.5 * (o.predict(F, 5, 2 * p) + o.predict(F, 5, 2 * p + 1))
            assert abs(avg - F[p]) <= 4e-16 * 8
        else:
            for py in range(n):
                kids = [o.predict(F, 5, 2 * p + dx, 2 * py + dy) for dy in (0, 1) for dx in (0, 1)]
                assert abs(0.25 * sum(kids) - F[py, p]) <= 4e-16 * 16


@pytest.mark.parametrize("scheme", ["D1Q3", "D2Q9"])
def test_sibling_details_sum_to_zero(scheme):
    """eq. DetailRedundancy on a full tree reconstructed by the oracle."""
    cfg = _cfg(scheme, 2 if scheme == "D1Q3" else 3, 7 if scheme == "D1Q3" else 5)
    o = oracle.Oracle(cfg)
    tree, v = o.init(W.random_field(cfg, 3, "jump"))
    dense = o.reconstruct(tree, v)
    l = o.jmax
    Fc = o.values_level(dense, l)[1]
    Fp = o.values_level(dense, l - 1)[1]
    npar = 1 << (l - 1)
    for p in range(0, npar, 3):
        if o.dim == 1:
            d = [Fc[2 * p + s] - o.predict(Fp, l, 2 * p + s) for s in (0, 1)]
        else:
            d = [Fc[2 * p + sy, 2 * p + sx] - o.predict(Fp, l, 2 * p + sx, 2 * p + sy)
                 for sy in (0, 1) for sx in (0, 1)]
        assert abs(sum(d)) <= 1e-14 * (1 + np.max(np.abs(Fc)))


def test_reconstruction_equals_matrix_powers():
    """eq. PredictionWithMatrix: n recursive predictions from a uniform level-l
    patch equal the n-th power of the printed 4x4 matrix (exact arithmetic)."""
    Mg = [[Fr(s) for s in row] for row in _gold("prediction_matrix_1d.json")["matrix"]]
    l = 4
    rng = np.random.default_rng(5)
    data = rng.integers(-1000, 1000, 1 << l)
    for n in range(1, 7):
        cfg = _cfg("D1Q3", 2, l + n)
        o = oracle.Oracle(cfg)
        tree, v = o.new_state()
        for m in range(o.jmin, l + 1):
            o.tree_level(tree, m)[:] = 1
        o.values_level(v, l)[0][:] = data
        FJ = o.values_level(o.reconstruct(tree, v), o.jmax)[0]
        P = [[Fr(int(i == j)) for j in range(4)] for i in range(4)]
        for _ in range(n):
            P = [[sum(P[i][k] * Mg[k][j] for k in range(4)) for j in range(4)] for i in range(4)]
        N = 1 << l
        for k in range(3, N - 2):
            win = [Fr(int(data[(k + a) % N])) for a in (-2, -1, 0, 1)]
            want = [sum(P[i][j] * win[j] for j in range(4)) for i in range(4)]
            got = [FJ[(2 ** n) * k + a] for a in (-2, -1, 0, 1)]
            assert [Fr(g) for g in got] == want


def test_detail_decay_rates():
    """eq. DetailsDecayEstimate: details of a smooth function fall by 2^{2 gamma + 1}
    per level; across a jump they keep their size."""
    for kind, lo, hi in [("smooth", 6.5, 9.0), ("jump", 0.7, 1.4)]:
        cfg = _cfg("D1Q3", 2, 12)
        o = oracle.Oracle(cfg)
        n = 1 << 12
        x = (np.arange(n) + 0.5) / n
        if kind == "smooth":
            u = (np.cos(2 * np.pi * (x - 0.5 / n)) - np.cos(2 * np.pi * (x + 0.5 / n))) / (2 * np.pi / n)
        else:
            u = (x > 0.3001).astype(float)
        tree, v = o.init((0.3 * u)[None, :])
        D = o.details(tree, o.reconstruct(tree, v))
        dmax = [D[o.level_offset(l - 1):o.level_offset(l - 1) + (1 << (l - 1))].max() for l in range(5, 13)]
        ratios = [a / b for a, b in zip(dmax[:-1], dmax[1:])]
        # geometric mean over the last four level pairs (a jump's detail size
        # depends on where it sits inside the dyadic cell of each level)
        gmean = float(np.prod(ratios[-4:])) ** 0.25
        assert lo < gmean < hi, (kind, ratios)
