"""The oracle's parallel loops (per cell, or per population for the adjoint's
scatters) give the same bits for any number of host threads."""
import numpy as np

import oracle
from paper_2103_02903_amd import workloads as W


def _run(cfg, m0, nthreads):
    oracle.threads(nthreads)
    o = oracle.Oracle(cfg)
    t, v = o.init(m0)
    o.step(t, v, 3)
    told, vold = t.copy(), v.copy()
    o.step(t, v, 1)
    rng = np.random.default_rng(0)
    anew = rng.standard_normal(v.size)
    aold, sb = o.adjoint_step(told, t, vold, anew)
    tf = o.new_tree_f32(told, vold.astype(np.float32))
    return t, v, aold, sb, tf


def test_thread_count_does_not_change_results():
    n0 = oracle.threads()
    try:
        for cfg, m0 in [W.shear_layer_d2q9(jmin=2, jmax=7, eps=1e-3, re=1000.0, width=1.0 / 20),
                        (W.params("D1Q3", 2, 10, 1e-4, [0, 1.5, 1.5], eq_param=0.5), None)]:
            if m0 is None:
                m0 = W.random_field(cfg, 1, "jump")
            a = _run(cfg, m0, 1)
            b = _run(cfg, m0, 4)
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
    finally:
        oracle.threads(n0)
