"""Differentiable MR-LBM run on frozen meshes (``torch.autograd``).

``run(m0, s, cfg, nsteps)`` advances the adaptive scheme from the equilibrium
initial datum of the conserved moments ``m0`` with relaxation rates ``s`` and
returns the final leaf values. Its backward pass is the discrete adjoint of the
run with every step's mesh held at the one the forward pass chose (the
thresholding is piecewise constant, so this is the derivative wherever the
mesh sequence does not change under the perturbation). Forward checkpoints
every ``ckpt_every`` steps; the backward recomputes each segment and sweeps it
in reverse, all in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from .mrlbm import Sim


class _FrozenMeshRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, s, cfg, nsteps, ckpt_every, precision):
        c = dict(cfg)
        c["s"] = [float(v) for v in s.detach().cpu().double().tolist()]
        sim = Sim(c, precision=precision, device=m0.device)
        sim.init_equilibrium(m0.detach())
        sim.forward_record(nsteps, ckpt_every)
        tree, values = sim.state_tensor(0)
        ctx.sim = sim
        ctx.s_meta = (s.dtype, s.device)
        ctx.m_meta = (m0.dtype, m0.shape)
        ctx.mark_non_differentiable(tree)
        return values, tree

    @staticmethod
    def backward(ctx, gvalues, gtree):
        sim = ctx.sim
        mbar, sbar = sim.adjoint(gvalues)
        ctx.sim = None
        sim.close()
        dtype, device = ctx.s_meta
        mdtype, mshape = ctx.m_meta
        mbar = mbar.to(mdtype).reshape(mshape)
        return mbar, torch.as_tensor(np.asarray(sbar), dtype=dtype, device=device), None, None, None, None


def run(m0: torch.Tensor, s: torch.Tensor, cfg: dict, nsteps: int, ckpt_every: int = 16, precision: int = 8):
    """Final (values, tree) of an ``nsteps`` run; differentiable in ``m0``
    ([nc][N_J^d], device) and ``s`` ([q] relaxation rates). ``values`` is in the
    values layout of the library (levels jmin..J, population-major per level);
    only complete-leaf entries (tree == leaf) are meaningful, and a functional
    must read only those."""
    return _FrozenMeshRun.apply(m0, s, cfg, int(nsteps), int(ckpt_every), int(precision))
