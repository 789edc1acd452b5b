"""Run-to-run reproducibility.

The operator kernels scatter a cell's contributions with hardware atomics,
whose order changes between launches, so two launches on the same input agree
to the order of summation, not bit for bit: each output is a sum of at most
eight cells' contributions, each formed in FP64 from terms no larger than the
largest output times the condition of the local sum, which bounds the
difference by a few hundred units of FP64 roundoff of the largest output
(written here as 1e-13).  Every reduction that decides control flow (alpha,
beta, norms, the stop test) sums block partials in a fixed order, so the
Krylov dimensions the adaptive stop picks must agree exactly between runs.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["box", "graded"])
def test_operator_repeats_to_summation_order(which):
    cfg = (W.scaled(W.CONFIGS[2], ncell=(6, 6, 6), p=5, n_orb=8) if which == "box"
           else W.scaled(W.CONFIGS[3], ncell=(4, 4, 4), p=6, n_orb=8))
    ctx = gpu_context(cfg, n_orb=8)
    x = torch.from_numpy(W.random_block(ctx.n_dof, 8, 17)).cuda()
    ys = [ctx.apply_H(x).cpu().numpy() for _ in range(5)]
    d = max(rel(y, ys[0]) for y in ys[1:])
    print(f"[determinism] {which}: largest run-to-run difference {d:.2e} of max |y|", flush=True)
    assert d <= 1e-13
    ctx.close()


def test_lanczos_dimensions_repeat_exactly():
    cfg = W.scaled(W.CONFIGS[3], ncell=(4, 4, 4), p=6, n_orb=4)
    ctx = gpu_context(cfg, n_orb=4)
    x = W.random_block(ctx.n_dof, 4, 23)
    x /= np.linalg.norm(x, axis=0)
    runs = []
    for _ in range(3):
        g = torch.from_numpy(x).cuda()
        k, _ = ctx.lanczos_expm(g, 0.05, 1e-10)
        runs.append((list(k), g.cpu().numpy()))
    print(f"[determinism] Krylov dimensions {[r[0] for r in runs]}", flush=True)
    for k, z in runs[1:]:
        assert k == runs[0][0]
        assert rel(z, runs[0][1]) <= 1e-12
    ctx.close()
