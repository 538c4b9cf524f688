"""Shared pieces of the adjoint tests: the kinetic-energy functional of the
final leaf values and its gradient (test glue, evaluated with the oracle's
layout helpers)."""
import numpy as np


def ke_functional(o, tree, values, region=(0.25, 0.75)):
    """J = sum over leaves whose centre lies in the region (each axis) of
    |C|/|C_J| * |q|^2 / (2 rho) (D2Q9) or of |C|/|C_J| * u^2 / 2 (1D); returns
    (J, dJ/dvalues)."""
    J = 0.0
    g = np.zeros_like(values)
    M = o.moment_matrix()
    for l in range(o.jmin, o.jmax + 1):
        mask = o.leaf_mask(tree, l)
        n = 1 << l
        cen = (np.arange(n) + 0.5) / n
        inside = (cen >= region[0]) & (cen < region[1])
        if o.dim == 2:
            mask = mask & inside[:, None] & inside[None, :]
        else:
            mask = mask & inside
        vol = float(1 << (o.dim * (o.jmax - l)))
        vl = o.values_level(values, l)
        gl = o.values_level(g, l)
        f = vl[:, mask]
        m = M @ f
        if o.q == 9:
            rho, q2 = m[0], m[1] ** 2 + m[2] ** 2
            J += vol * float(np.sum(0.5 * q2 / rho))
            dm = np.zeros_like(m)
            dm[0] = -0.5 * q2 / rho ** 2
            dm[1] = m[1] / rho
            dm[2] = m[2] / rho
        else:
            J += vol * float(np.sum(0.5 * m[0] ** 2))
            dm = np.zeros_like(m)
            dm[0] = m[0]
        gl[:, mask] = vol * (M.T @ dm)
    return J, g


def final_frozen(o, m0, trees):
    """Final leaf values of the oracle run from m0 on the mesh sequence trees
    (trees[0] the full initial mesh), without keeping the intermediate states."""
    t, v = o.init(m0)
    assert np.array_equal(t, trees[0])
    for tn in trees[1:]:
        o.step_frozen(t, tn, v)
    return t, v


from paper_2103_02903_amd.workloads import vortex_amplitude_gradient  # noqa: E402,F401
