"""Host-side ghost sets of a complete tree, written from their definition, for
checking the GPU classification.

A cell of level l > jmin outside the tree is a ghost if a leaf of level l lies
in its box of half-width 2 gamma (5^d for gamma = 1: the transport and
transfer stencils of that leaf) or if it lies in the box of half-width gamma of
the parent of a ghost of level l+1 (the prediction stencil of that ghost,
section "Projection and prediction operators"). The sets are built from the
finest level down; all boxes wrap periodically (with walls this is the superset
the library classifies).
"""
import numpy as np


def _dilate(m: np.ndarray, r: int) -> np.ndarray:
    out = m.copy()
    axes = tuple(range(m.ndim))
    for off in np.ndindex(*([2 * r + 1] * m.ndim)):
        sh = tuple(o - r for o in off)
        if any(sh):
            out |= np.roll(m, sh, axis=axes)
    return out


def _parents(m: np.ndarray) -> np.ndarray:
    """Cells of the coarser level with at least one child in m."""
    out = np.zeros(tuple(n // 2 for n in m.shape), bool)
    for off in np.ndindex(*([2] * m.ndim)):
        out |= m[tuple(slice(o, None, 2) for o in off)]
    return out


def _children(m: np.ndarray) -> np.ndarray:
    """Children (one level finer) of the cells in m."""
    out = m
    for ax in range(m.ndim):
        out = np.repeat(out, 2, axis=ax)
    return out


def tree_sets(o, tree):
    """Per level: (tree mask, leaf mask, internal mask)."""
    T = {l: o.tree_level(tree, l).astype(bool) for l in range(o.jmin, o.jmax + 1)}
    S, I = {}, {}
    for l in T:
        S[l] = o.leaf_mask(tree, l)
        I[l] = T[l] & ~S[l]
    return T, S, I


def ghost_sets(o, tree, gamma=1):
    """Per level l > jmin: the ghost mask (level jmin holds every cell in the tree)."""
    T, S, _ = tree_sets(o, tree)
    G = {}
    for l in range(o.jmax, o.jmin, -1):
        need = _dilate(S[l], 2 * gamma)
        if l < o.jmax:
            need |= _dilate(_parents(G[l + 1]), gamma)
        G[l] = need & ~T[l]
    return G


def _axis_rows(m: np.ndarray, r: int) -> np.ndarray:
    """m and its shifts by up to r cells along each axis separately."""
    out = m.copy()
    for ax in range(m.ndim):
        for d in range(1, r + 1):
            out |= np.roll(m, d, axis=ax) | np.roll(m, -d, axis=ax)
    return out


def ghost_sets_3d(o, tree):
    """The ghosts of the three-dimensional (D3Q6) path, per level l > jmin: the
    cells outside the tree in the 3^3 box of a leaf of level l (the parent
    stencil of a child the next adaptation may create there) or in its rows
    of +-2 cells along the axes (its transport: each velocity lies along one
    axis), or in the 3^3 box of the parent of a ghost of level l+1."""
    T, S, _ = tree_sets(o, tree)
    G = {}
    for l in range(o.jmax, o.jmin, -1):
        need = _dilate(S[l], 1) | _axis_rows(S[l], 2)
        if l < o.jmax:
            need |= _dilate(_parents(G[l + 1]), 1)
        G[l] = need & ~T[l]
    return G


def ghost_near_internal(o, tree):
    """Levels where some ghost has no internal cell of the coarser level within
    one cell of its parent (empty if the property holds everywhere)."""
    _, _, I = tree_sets(o, tree)
    G = ghost_sets(o, tree)
    bad = []
    for l, g in G.items():
        allowed = _children(_dilate(I[l - 1], 1))
        if np.any(g & ~allowed):
            bad.append(l)
    return bad
