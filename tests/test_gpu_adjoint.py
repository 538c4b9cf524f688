"""GPU adjoint on frozen meshes (through the C-ABI) against the oracle adjoint.

The GPU run's own mesh sequence (read back step by step) is handed to the
oracle, whose frozen-mesh gradient is pinned by dot-product tests and central
differences on the CPU. The checkpointed GPU backward must reproduce it: FP64
within 1e-10 of the gradient's max norm (the scatters add in a run-dependent
order), FP32 within 5e-4. The autograd wrapper is checked the same way and
against central differences of GPU forward runs whose mesh sequences are
verified to be unchanged by the perturbation.
"""
import numpy as np
import pytest

import oracle
from adjoint_helpers import ke_functional
from paper_2103_02903_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_02903_amd import mrlbm

    mrlbm.lib()
    return mrlbm


def _cfg(scheme, jmin, jmax, eps):
    s = {"D1Q2": [0, 1.9], "D1Q3": [0, 1.5, 1.5], "D2Q9": W.d2q9_s(1.5, 1.8)}[scheme]
    return W.params(scheme, jmin, jmax, eps, s, mu_bar=1.0, eq_param=0.5 if scheme == "D1Q3" else 1.0)


def _gpu_mesh_sequence(mr, cfg, m0, nsteps, precision):
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    trees, states = [], []
    t, v = sim.get_state()
    trees.append(t)
    for _ in range(nsteps):
        sim.step(1)
        t, v = sim.get_state()
        trees.append(t)
    sim.close()
    return trees, v


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / max(float(np.max(np.abs(b))), 1e-300)


CASES = [("D1Q2", 2, 9, 20, 6, 5), ("D1Q3", 2, 9, 16, 5, 3), ("D2Q9", 2, 6, 10, 4, 7), ("D2Q9", 3, 7, 9, 9, 8)]


@pytest.mark.parametrize("scheme,jmin,jmax,nsteps,K,seed", CASES)
@pytest.mark.parametrize("precision", [8, 4])
def test_gpu_adjoint_matches_oracle(mr, scheme, jmin, jmax, nsteps, K, seed, precision):
    import torch

    print("adjoint case", scheme, jmin, jmax, nsteps, K, seed, precision, flush=True)
    cfg = _cfg(scheme, jmin, jmax, 1e-3)
    o = oracle.Oracle(cfg)
    m0 = W.random_field(cfg, seed, "smooth" if scheme != "D1Q2" else "jump")
    trees, v_steps = _gpu_mesh_sequence(mr, cfg, m0, nsteps, precision)
    for t in trees:
        assert o.check_tree(t) == 0
    sim = mr.Sim(cfg, precision=precision)
    sim.init_equilibrium(m0)
    sim.forward_record(nsteps, K)
    t_fin, v_fin = sim.get_state()
    # the recording run is the same computation as plain stepping
    assert np.array_equal(t_fin, trees[-1])
    assert np.array_equal(v_fin, v_steps)
    _, abar = ke_functional(o, t_fin, v_fin.astype(np.float64))
    mbar_g, sbar_g = sim.adjoint(torch.from_numpy(abar).to(sim.device))
    mbar_g = mbar_g.double().cpu().numpy()
    mbar_o, sbar_o = o.gradient_frozen(m0, trees, abar)
    tol = 1e-10 if precision == 8 else 5e-4
    assert mbar_g.shape == mbar_o.shape
    assert _rel(mbar_g, mbar_o) <= tol, _rel(mbar_g, mbar_o)
    nz = [k for k in range(o.q) if cfg["s"][k] != 0]
    assert _rel(sbar_g[nz], sbar_o[nz]) <= tol, (sbar_g, sbar_o)
    sim.close()


@pytest.mark.parametrize("K", [3, 4])
def test_adjoint_graph_replay_matches_eager_launches(mr, K):
    """The adjoint's full segments run as captured graphs (a recomputation and a
    sweep per tape, the sweep also per buffer holding the running adjoint); with
    the launch schedule's graph switch off every launch is eager. Both orders of
    the two streams give the same gradient (up to the order of atomic adds):
    odd and even K, four full segments and a partial one."""
    import torch

    cfg = _cfg("D2Q9", 2, 6, 1e-3)
    m0 = W.random_field(cfg, 11, "smooth")
    nsteps = 4 * K + 2
    out = []
    for graph in (1, 0):
        sim = mr.Sim(cfg, precision=8)
        t = sim.tuning()
        sim.set_tuning(t["transport_variant"], t["list_grid_all"], t["list_grid_level"], graph=graph,
                       pair_links=t["pair_links"])
        sim.init_equilibrium(m0)
        sim.forward_record(nsteps, K)
        t_fin, v_fin = sim.get_state()
        _, abar = ke_functional(oracle.Oracle(cfg), t_fin, v_fin.astype(np.float64))
        mbar, sbar = sim.adjoint(torch.from_numpy(abar).to(sim.device))
        out.append((mbar.double().cpu().numpy(), np.array(sbar)))
        sim.close()
    assert _rel(out[0][0], out[1][0]) <= 1e-12
    assert _rel(out[0][1], out[1][1]) <= 1e-12


def test_adjoint_rejects_batches_and_unrecorded_runs(mr):
    import torch

    cfg = _cfg("D1Q3", 2, 6, 1e-3)
    b = mr.Batch([cfg, cfg])
    with pytest.raises(mr.MrlbmError):
        b.forward_record(4, 2)
    b.close()
    sim = mr.Sim(cfg)
    sim.init_equilibrium(W.random_field(cfg, 1))
    with pytest.raises(mr.MrlbmError):
        sim.adjoint(torch.zeros(3 * sim.total_cells[0], dtype=torch.float64, device=sim.device))
    sim.close()


def _ke_torch(o, tree_np, values, region=(0.25, 0.75)):
    """The kinetic-energy functional of ke_functional, evaluated with torch on
    the device values so that autograd carries it."""
    import torch

    M = torch.as_tensor(o.moment_matrix(), dtype=values.dtype, device=values.device)
    J = values.new_zeros(())
    for l in range(o.jmin, o.jmax + 1):
        mask = o.leaf_mask(tree_np, l)
        n = 1 << l
        cen = (np.arange(n) + 0.5) / n
        inside = (cen >= region[0]) & (cen < region[1])
        mask = mask & inside[:, None] & inside[None, :] if o.dim == 2 else mask & inside
        cells = np.flatnonzero(mask.ravel())
        if cells.size == 0:
            continue
        off = o.q * o.level_offset(l)
        idx = off + np.arange(o.q)[:, None] * o.ncells(l) + cells[None, :]
        f = values[torch.as_tensor(idx, device=values.device)]
        m = M @ f
        vol = float(1 << (o.dim * (o.jmax - l)))
        if o.q == 9:
            J = J + vol * torch.sum(0.5 * (m[1] ** 2 + m[2] ** 2) / m[0])
        else:
            J = J + vol * torch.sum(0.5 * m[0] ** 2)
    return J


def test_autograd_gradient_vs_oracle_and_differences(mr):
    import torch

    from paper_2103_02903_amd import adjoint

    scheme, jmin, jmax, nsteps, seed = "D2Q9", 2, 6, 10, 7
    cfg = _cfg(scheme, jmin, jmax, 1e-3)
    o = oracle.Oracle(cfg)
    m0_np = W.random_field(cfg, seed, "smooth")
    dev = torch.device("cuda:0")
    m0 = torch.tensor(m0_np, dtype=torch.float64, device=dev, requires_grad=True)
    s = torch.tensor(cfg["s"], dtype=torch.float64, requires_grad=True)
    values, tree = adjoint.run(m0, s, cfg, nsteps, ckpt_every=3)
    tree_np = tree.cpu().numpy()
    J = _ke_torch(o, tree_np, values)
    J.backward()
    trees, _ = _gpu_mesh_sequence(mr, cfg, m0_np, nsteps, 8)
    assert np.array_equal(trees[-1], tree_np)
    _, abar = ke_functional(o, tree_np, values.detach().cpu().numpy())
    mbar_o, sbar_o = o.gradient_frozen(m0_np, trees, abar)
    assert _rel(m0.grad.cpu().numpy(), mbar_o) <= 1e-10
    assert _rel(s.grad.numpy()[3:], sbar_o[3:9]) <= 1e-10
    # directional central differences of GPU forward runs on unchanged meshes
    rng = np.random.default_rng(11)
    dm = rng.normal(size=m0_np.shape) * 0.01
    h = 1e-6
    Js = []
    for sgn in (1, -1):
        mp = m0_np + sgn * h * dm
        tp, _ = _gpu_mesh_sequence(mr, cfg, mp, nsteps, 8)
        assert all(np.array_equal(a, b) for a, b in zip(tp, trees)), "perturbation changed the meshes"
        with torch.no_grad():
            vp, _ = adjoint.run(torch.tensor(mp, device=dev), s.detach(), cfg, nsteps)
            Js.append(float(_ke_torch(o, tree_np, vp)))
    fd = (Js[0] - Js[1]) / (2 * h)
    ad = float(np.sum(m0.grad.cpu().numpy() * dm))
    assert abs(fd - ad) <= 1e-6 * abs(fd), (fd, ad)
