"""Writes tests/golden/hartree_<case>.json: the oracle's Hartree potential on
box meshes whose one-dimensional interior sizes select each tile width of the
GPU's fast-diagonalisation solver (and its line-tiled form above 128 nodes),
and on the full graded molecule mesh (curved cells), sampled at seeded nodes
and Gauss points.

Only oracle/ and workloads/ are used.  Each case: the pseudopotential-like
molecule recipe (Gaussian wells, seeded smooth orbitals, kick) on a uniform
box mesh; rho from the recipe's orbitals (Sec. "Time-dependent Kohn-Sham
Equations"); phi from the discrete Poisson problem K phi = 4 pi c with the
boundary values f = sum Z/|r - R| (Eqs. Poisson, VHDiscretePoisson), solved by
the oracle's Jacobi-PCG from a zero start to a relative residual of 1e-13 and
then, warm-started, to 1e-14; W = V_H + V_xc at the Gauss points (LDA
exchange on the box meshes, exchange + PZ81 correlation on the graded one).
The change between the two solves is stored as the oracle's own accuracy
estimate.

Run: python tests/golden/make_hartree_golden.py [case ...]   (minutes per case;
the 26^3 case about half an hour on one core, the graded case hours)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import scf  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402

# name: (cells per axis, order p, orbitals); interior nodes per axis = nc p - 1
CASES = {
    "box8_p5": (8, 5, 2),     # 39  -> 3 modes per lane group
    "box13_p4": (13, 4, 2),   # 51  -> 4
    "box16_p5": (16, 5, 8),   # 79  -> 5 (the benchmark mesh and orbitals)
    "box17_p5": (17, 5, 2),   # 84  -> 6
    "box22_p5": (22, 5, 2),   # 109 -> 8
    "box26_p5": (26, 5, 1),   # 129 -> line-tiled kernel
}
# curved cells: the graded molecule recipe (31^3 trilinear cells, p = 6,
# exchange + correlation) with its first two orbitals
CURVED_CASES = {
    "graded31_p6": (31, 6, 2),
}
N_SAMPLES = 2048


def case_config(name):
    if name in CURVED_CASES:
        nc, p, n_orb = CURVED_CASES[name]
        return W.scaled(W.CONFIGS[3], ncell=(nc, nc, nc), p=p, n_orb=n_orb)
    nc, p, n_orb = CASES[name]
    return W.scaled(W.CONFIGS[2], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


def run(name):
    cfg = case_config(name)
    t0 = time.time()
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    psi = W.initial_psibar(cfg, m.dof_xyz, m.M)
    rho = scf.density(m, psi)
    Z, R = W.atoms(cfg)
    h = scf.Hartree(m, Z, R, tol=1e-13, maxit=20000)
    phi13, _ = h.solve(rho)
    it13 = h.last_iters
    h.tol = 1e-14
    try:
        phi, vq = h.solve(rho)
        tol = 1e-14
    except RuntimeError:
        h.tol = 1e-13
        phi, vq = h.solve(rho)
        tol = 1e-13
    change = float(np.abs(phi - phi13).max() / np.abs(phi).max())
    w = vq + scf.xc_potential(rho, cfg.xc)
    rng = np.random.default_rng(77)
    nodes = np.sort(rng.choice(m.n_nodes, N_SAMPLES, replace=False))
    quad = np.sort(rng.choice(w.size, N_SAMPLES, replace=False))
    out = {
        "what": "oracle Hartree potential phi (all nodes, boundary included) and W = V_H + V_xc at the Gauss points",
        "recipe": (f"workloads.CONFIGS[{3 if name in CURVED_CASES else 2}] scaled to ncell=(nc, nc, nc), order p, "
                   "n_orb orbitals (initial_psibar)"),
        "xc": cfg.xc,
        "case": name, "ncell": cfg.ncell[0], "p": cfg.p, "n_orb": cfg.n_orb,
        "n_nodes": int(m.n_nodes), "n_dof": int(m.n_dof), "n_cell": int(m.n_cell),
        "pcg_iters_1e-13": int(it13), "pcg_tol_final": tol, "max_change_1e-13_to_final": change,
        "phi_max_abs": float(np.abs(phi).max()), "w_max_abs": float(np.abs(w).max()),
        "node_index": nodes.tolist(), "phi": [float(v) for v in phi[nodes]],
        "quad_index": quad.tolist(), "w": [float(v) for v in w.reshape(-1)[quad]],
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, f"hartree_{name}.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: {m.n_nodes} nodes, PCG {it13} its, change {change:.2e}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES) + list(CURVED_CASES):
        run(name)
