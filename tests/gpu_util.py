"""Shared set-up for the GPU parity tests: build one HIP context and the
matching oracle objects from the same seeded workload recipe.  Each side uses
its own mesh coordinates and overlap; nothing computed by one side is fed to
the other."""
import numpy as np

import workloads as W
from oracle.mesh import Mesh


def gpu_context(cfg, n_orb=None, k_max=None, precision=0):
    import torch
    from paper_1810_13130_amd import tdfe
    n_orb = cfg.n_orb if n_orb is None else n_orb
    ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=n_orb,
                       k_max=cfg.k_max if k_max is None else k_max, precision=precision)
    xq = ctx.quad_coords().cpu().numpy()
    ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
    return ctx


def gpu_initial_state(ctx, cfg, n_orb=None):
    import torch
    psi = W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(), ctx.mass_diag().cpu().numpy())
    if n_orb is not None:
        psi = psi[:, :n_orb]
    return torch.from_numpy(np.ascontiguousarray(psi)).cuda()


def oracle_mesh(cfg):
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    return m, vq


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
