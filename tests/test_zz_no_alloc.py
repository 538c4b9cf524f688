"""The context whose workspace is the library's own device array
(mrlbm_create_static), against an ordinary context on a caller-allocated
workspace (mrlbm_create): the same steps give the same meshes and the same
bits in every output, on two contexts in a row (the second smaller, in the
array the first one left behind). Also the limits: a configuration beyond the
array's size, a second live static context on the device, and graph replay
are refused.
"""
import numpy as np
import pytest

from paper_2103_02903_amd import workloads as W

from test_gpu_parity import _cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


def _outputs(sim):
    """Everything a caller can read back, as host arrays."""
    sim.synchronize()
    tree, _ = sim.get_state()
    st = sim.stats()
    out = dict(tree=tree, leaves=st["leaves"], internal=st["internal"], ghosts=st["ghosts"],
               mass=np.float64(st["mass"]))
    for what in ("leaf_table", "populations", "moments", "finest"):
        out[what] = sim.fields(what).cpu().numpy()
    return out


CASES = [  # the first fills most of the 16 MiB array, the second is smaller
    ("D2Q9", 3, 8, 1e-3, 5, 8, 12),
    ("D1Q3", 2, 10, 1e-4, 6, 4, 20),
]


@pytest.mark.parametrize("scheme,jmin,jmax,eps,seed,precision,steps", CASES)
def test_static_context_matches_ordinary(mr, scheme, jmin, jmax, eps, seed, precision, steps):
    cfg = _cfg(scheme, jmin, jmax, eps)
    m0 = W.random_field(cfg, seed, "jump")
    print("static vs ordinary:", scheme, "levels %d..%d" % (jmin, jmax), "precision", precision, flush=True)
    ref = mr.Sim(cfg, precision=precision)
    ref.init_equilibrium(m0)
    ref.step(steps)
    want = _outputs(ref)
    ref.close()
    sim = mr.Sim(cfg, precision=precision, static=True)
    try:
        assert sim.workspace is None and sim.workspace_bytes <= 16 << 20
        assert sim.tuning()["graph"] == 0
        sim.init_equilibrium(m0)
        sim.step(steps)
        got = _outputs(sim)
    finally:
        sim.close()
    assert int(want["leaves"].sum()) > 0
    for k in want:
        assert np.array_equal(got[k], want[k]), "static context differs in %s" % k


def test_static_context_limits(mr):
    import torch

    big = W.shear_layer_d2q9()[0]  # levels 3..10: far beyond the array
    with pytest.raises(mr.MrlbmError) as e:
        mr.Sim(big, precision=8, static=True)
    assert e.value.status == -2
    cfg = _cfg("D1Q2", 2, 9, 1e-4)
    m0 = W.random_field(cfg, 1, "jump")
    a = mr.Sim(cfg, precision=8, static=True)
    try:
        with pytest.raises(mr.MrlbmError) as e:
            mr.Sim(cfg, precision=8, static=True)  # the array is in use
        assert e.value.status == -5
        with pytest.raises(mr.MrlbmError) as e:
            a.set_tuning(1, 1024, 256, graph=1)  # graph capture would need a capture stream
        assert e.value.status == -5
        a.init_equilibrium(m0)
        a.step(3)
        a.synchronize()
        assert a.stats()["leaves"].sum() > 0
    finally:
        a.close()
    b = mr.Sim(cfg, precision=8, static=True)  # free again after destroy
    b.close()
    torch.cuda.synchronize()
