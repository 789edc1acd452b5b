"""Benchmark: second-order Magnus steps per second on one MI355X.

Workload (default): 16^3 box cells on [-10,10]^3, order p = 5 (493,039 DoFs),
8 complex orbitals, 4 Gaussian-well atoms, Hartree + LDA exchange, kick 1e-3
along z, dt = 0.05, Lanczos tolerance 1e-10 -- the pseudopotential-like
molecule workload.  One step = the whole hot path: predictor Lanczos
exp(-i dt/2 Hbar), density, Hartree, XC, corrector Lanczos exp(-i dt Hbar),
density, Hartree, XC, dipole.  Inputs are resident on the GPU before timing.

Prints ONE JSON line (rank 0).  Besides the contract fields it reports the
operator kernel's roofline position (per-launch duration measured with HIP
events on the library's stream), its throughput in GDoF-orbitals/s, and a
bounded CPU-oracle baseline measured on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3


def apply_work(n, nq, n_cell, n_dof, n_orb, elem_bytes=8):
    """Algorithmic work of one Hbar apply on n_orb complex orbitals.

    bytes: read psibar and write Hbar psibar once (2 x 2 real numbers per
    DoF-orbital), the weighted potential once per Gauss point, M^-1/2 once
    per DoF.  flops: per cell and real column 12 one-dimensional passes of
    n^4 multiply-adds (3 interpolations, 3 collocation derivatives, their 6
    transposes) plus ~7 n^3 pointwise.
    """
    bytes_ = n_dof * n_orb * 2 * elem_bytes * 2 + n_cell * nq ** 3 * elem_bytes + n_dof * 8
    flops = n_cell * 2 * n_orb * (24 * n ** 4 + 7 * n ** 3)
    return bytes_, flops


# sources of the box-cell operator kernels (the lane-pair FP64 kernel and the
# plane FP32 kernel) whose counters profiles/ holds
OPERATOR_SOURCES = ("tdfe_apply_box.hip", "tdfe_apply_pair.hip", "tdfe_fold.h", "tdfe_rule1d.h")


def operator_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in OPERATOR_SOURCES:
        with open(os.path.join(ROOT, "paper_1810_13130_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(label):
    """HBM bytes per operator launch from the committed rocprofv3 counter summary,
    or None when the operator sources have changed since the counters were taken."""
    prof = os.path.join(ROOT, "profiles", "operator_16x16x16_p5_8orb_hbm_bytes.md")
    try:
        text = open(prof).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if "=" in line and not line.startswith("|"):
            k, v = (x.strip() for x in line.split("=", 1))
            vals[k] = v
    if vals.get("source_sha256_prefix") != operator_source_hash():
        return None
    v = vals.get(f"traffic_bytes_per_launch.{label}")
    return float(v) if v is not None else None


def adjoint_rate(n_steps=20):
    """Field gradient dmu_z(t_N)/dE_n on the adjoint workload (16^3 p=5, 8 orbitals,
    Hartree + exchange, no kick): forward sweep + checkpointed reverse sweep."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[5]
    ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=cfg.n_orb, k_max=cfg.k_max)
    xq = ctx.quad_coords().cpu().numpy()
    ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=cfg.n_orb)
    psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                            ctx.mass_diag().cpu().numpy())).cuda()
    E = W.field_amplitudes(n_steps)
    ctx.dipole_gradient(psi, E[:2], cfg.dt, cfg.tol)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    L, g = ctx.dipole_gradient(psi, E, cfg.dt, cfg.tol, checkpoint_every=n_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ctx.close()
    return {"workload": cfg.name, "steps": n_steps, "value": n_steps / wall,
            "unit": "Magnus steps/s (forward + reverse, gradient w.r.t. every E_n)",
            "wall_s": wall, "L": L, "grad_norm": float(np.linalg.norm(g))}


def graded_apply(reps=3):
    """Operator on curved (trilinear) cells: the graded workload (31^3 cells, p = 6,
    6,331,625 DoFs, 32 orbitals), FP64 and FP32 launches."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[3]
    out = {"workload": cfg.name}
    for prec, name in ((tdfe.FP64, "f64"), (tdfe.MIXED_FP32, "f32")):
        ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=cfg.n_orb, k_max=4, precision=prec)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
        dt_ = torch.complex128 if prec == tdfe.FP64 else torch.complex64
        f = ctx.apply_H_add if prec == tdfe.FP64 else ctx.apply_H_add_f32
        x = torch.randn(ctx.n_dof, cfg.n_orb, dtype=dt_, device="cuda")
        y = torch.zeros_like(x)
        f(x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            f(x, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_launch_ms"] = ms
        out[name + "_gdof_orb_per_s"] = ctx.n_dof * cfg.n_orb / (ms * 1e-3) / 1e9
        del x, y
        ctx.close()
        torch.cuda.empty_cache()
    return out


def nonlocal_term(n_steps=30, reps=50):
    """Kleinman-Bylander term (Eq. VPSP) on the benchmark workload: 4 atoms x
    (s, p_x, p_y, p_z) Gaussian projectors from the workload recipe.  Magnus
    steps/s with the term, the operator launch with and without it, and the
    streaming bytes of its passes (Cbar read by both passes, x over the boxes,
    the output read and written over the crossed lines) against HBM."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[2]
    out = {"workload": cfg.name + " + Kleinman-Bylander projectors (4 atoms x s, p)"}
    for prec, name, eb in ((tdfe.FP64, "f64", 8), (tdfe.MIXED_FP32, "mixed", 4)):
        ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=cfg.n_orb, k_max=cfg.k_max, precision=prec)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
        Z, R = W.atoms(cfg)
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=cfg.n_orb)
        dt_ = torch.complex128 if prec == tdfe.FP64 else torch.complex64
        f = ctx.apply_H_add if prec == tdfe.FP64 else ctx.apply_H_add_f32
        x = torch.randn(ctx.n_dof, cfg.n_orb, dtype=dt_, device="cuda")
        y = torch.zeros_like(x)

        def launch_us():
            for _ in range(3):
                f(x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                f(x, y)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / reps

        t_local = launch_us()
        u, dv = W.kb_projector_values(cfg, xq)
        ctx.set_projectors(torch.from_numpy(np.ascontiguousarray(u.reshape(u.shape[0], -1))).cuda(),
                           torch.from_numpy(np.ascontiguousarray(dv.reshape(dv.shape[0], -1))).cuda())
        groups, stored, box_dofs, line_dofs = ctx.projector_info()
        t_nl = launch_us()
        cols = 2 * cfg.n_orb
        nl_bytes = 2 * stored * eb + box_dofs * cols * eb + 2 * line_dofs * cols * eb
        psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        for _ in range(3):
            ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n_steps):
            ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        extra = t_nl - t_local
        out.update({"n_proj": int(u.shape[0]), "groups": groups, "stored_entries": stored, "box_dofs": box_dofs,
                    "line_dofs": line_dofs})
        out[name] = {"steps_per_s": n_steps / wall, "launch_us_local": t_local, "launch_us_with_term": t_nl,
                     "term_us": extra, "term_bytes": nl_bytes,
                     "term_hbm_frac": nl_bytes / (extra * 1e-6) / (HBM_PEAK_GBS * 1e9) if extra > 0 else None}
        del x, y, psi
        ctx.close()
        torch.cuda.empty_cache()
    return out


def field_and_spectra(n_steps=30, n_t=20000, n_omega=2000):
    """Time-dependent excitation and observables: FP64 Magnus steps on the
    benchmark workload under the weak Gaussian pulse (kappa 2e-5, t0 3, w 0.2,
    along x, held at each step's midpoint), then the absorption spectrum of
    a 20,000-sample dipole record (1000 a.u. at dt = 0.05) on 2,000
    frequencies, and the dipole power spectrum of the same record."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[2]
    ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=cfg.n_orb, k_max=cfg.k_max)
    xq = ctx.quad_coords().cpu().numpy()
    ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=cfg.n_orb)
    ctx.set_field_direction((1.0, 0.0, 0.0))
    psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                            ctx.mass_diag().cpu().numpy())).cuda()
    tm = cfg.dt * (np.arange(n_steps + 3) + 0.5)
    E = tdfe.field_samples(tdfe.FIELD_GAUSSIAN, (2e-5, 3.0, 0.2), tm)
    for k in range(3):
        ctx.magnus_step(psi, cfg.dt, float(E[k]), cfg.tol)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(3, n_steps + 3):
        ctx.magnus_step(psi, cfg.dt, float(E[k]), cfg.tol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ctx.close()
    tt = 0.05 * np.arange(n_t)
    mu = torch.from_numpy(np.stack([1e-5 * np.sin(w0 * tt) * np.exp(-1e-3 * tt) for w0 in (0.3, 0.5, 0.7)])).cuda()
    om = torch.linspace(0.0, 1.5, n_omega, dtype=torch.float64, device="cuda")

    def ms(f, reps=5):
        f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_abs = ms(lambda: tdfe.absorption_spectrum(mu, 0.05, om, 0.005, kappa=1e-3))
    t_pow = ms(lambda: tdfe.power_spectrum(mu[0].contiguous(), 0.05, om))
    return {"workload": cfg.name + " under a Gaussian pulse along x; spectra of a 20,000-sample record",
            "pulse_steps_per_s": n_steps / wall,
            "absorption_ms": t_abs, "power_ms": t_pow,
            "absorption_sample_freq_per_s": 3 * n_t * n_omega / (t_abs * 1e-3),
            "power_sample_freq_per_s": n_t * n_omega / (t_pow * 1e-3)}


def midpoint_modes(n_steps=20):
    """The midpoint Hamiltonian options on the benchmark workload (FP64):
    predictor-corrector with linear and quadratic predictors and the fully
    self-consistent iteration (sc_tol 1e-10 Hartree), from the same state;
    steps/s, propagations per step and the dipole gap to the self-consistent
    trajectory."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[2]
    out = {"workload": cfg.name, "steps": n_steps}
    mus = {}
    for name, mode, order in (("pc_linear", tdfe.MIDPOINT_PC, 1), ("pc_quadratic", tdfe.MIDPOINT_PC, 2),
                              ("self_consistent", tdfe.MIDPOINT_SC, 1)):
        ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=cfg.n_orb, k_max=cfg.k_max)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
        Z, R = W.atoms(cfg)
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=cfg.n_orb)
        ctx.set_midpoint(mode, order=order, sc_tol=1e-10, sc_maxit=50)
        psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        mu, its = [], 0
        for _ in range(n_steps):
            rep = ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
            mu.append(rep["mu"])
            its += rep["sc_iters"] if mode == tdfe.MIDPOINT_SC else 2
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        mus[name] = np.array(mu)
        out[name] = {"steps_per_s": n_steps / wall, "propagations_per_step": its / n_steps}
        ctx.close()
        torch.cuda.empty_cache()
    ref = mus["self_consistent"]
    dmu = np.abs(ref - ref[0]).max()
    for name in ("pc_linear", "pc_quadratic"):
        out[name]["dipole_gap_to_sc_rel_induced"] = float(np.abs(mus[name] - ref).max() / max(dmu, 1e-300))
    return out


def adaptive_mesh(n_elem=1728, n_steps=10):
    """A priori graded mesh against a uniform one with the same element count:
    the induced dipole of the benchmark workload's recipe (4 atoms, 8
    orbitals, Hartree + exchange, kick, p = 5) over 10 steps, each against a
    32^3-cell uniform reference."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    base = W.CONFIGS[2]
    Z, R = W.atoms(base)

    def run(verts, ncell):
        ctx = tdfe.Context(base.p, ncell, verts, n_orb_max=base.n_orb, k_max=base.k_max)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(base, xq).reshape(ctx.n_cell, -1)).cuda())
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=base.n_orb)
        psi = torch.from_numpy(W.initial_psibar(base, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        mu = [ctx.dipole(psi)[0][2]]
        for _ in range(n_steps):
            mu.append(ctx.magnus_step(psi, base.dt, 0.0, base.tol)["mu"][2])
        n_dof = ctx.n_dof
        ctx.close()
        torch.cuda.empty_cache()
        mu = np.array(mu)
        return mu - mu[0], n_dof

    n1 = int(round(n_elem ** (1 / 3)))
    uni = W.box_vertices(base.lo, base.hi, (n1, n1, n1))
    axes, E = tdfe.adaptive_axes(base.p, base.lo, base.hi, R, Z, [1.0] * len(Z), [0.5] * len(Z), n_elem, samples=129)
    ncell = tuple(len(a) - 1 for a in axes)
    t = time.perf_counter()
    ref, nd_ref = run(W.box_vertices(base.lo, base.hi, (32, 32, 32)), (32, 32, 32))
    d_uni, nd_uni = run(uni, (n1, n1, n1))
    d_ada, nd_ada = run(tdfe.rectilinear_vertices(*axes), ncell)
    scale = np.abs(ref).max()
    return {"workload": base.name + f" recipe, {n_steps} steps, p = {base.p}",
            "reference": {"cells": [32, 32, 32], "n_dof": nd_ref},
            "uniform": {"cells": [n1] * 3, "n_dof": nd_uni, "induced_dipole_rel_err": float(np.abs(d_uni - ref).max() / scale)},
            "adaptive": {"cells": list(ncell), "n_dof": nd_ada, "E": E,
                         "spacing_min_max": [float(min(np.diff(a).min() for a in axes)),
                                             float(max(np.diff(a).max() for a in axes))],
                         "induced_dipole_rel_err": float(np.abs(d_ada - ref).max() / scale)},
            "wall_s": time.perf_counter() - t}


def cpu_oracle_baseline(cfg, ks_total):
    """Bounded sample of the CPU oracle on this host, scaled to steps/s."""
    import threadpoolctl
    import workloads as W
    from oracle import lanczos, operators as op, scf
    from oracle.mesh import Mesh
    t0 = time.perf_counter()
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    psi = W.initial_psibar(cfg, m.dof_xyz, m.M)
    # (a) Lanczos propagations of two orbitals, one at a time: cost per Krylov iteration
    t = time.perf_counter()
    ks = []
    for o in range(2):
        _, k_o, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), psi[:, o:o + 1], cfg.dt, cfg.tol)
        ks.append(k_o[0])
    t_it = (time.perf_counter() - t) / sum(ks)
    # (b) 20 iterations of the oracle's Hartree PCG: cost per PCG iteration
    Z, R = W.atoms(cfg)
    h = scf.Hartree(m, Z, R, tol=1e-13, maxit=20)
    rho = scf.density(m, psi)
    t = time.perf_counter()
    try:
        h.solve(rho)
    except RuntimeError:
        pass
    t_cg = (time.perf_counter() - t) / 20
    # (c) one density evaluation
    t = time.perf_counter()
    scf.density(m, psi)
    t_rho = time.perf_counter() - t
    # the oracle's own warm-started config-2 Hartree solves take ~357 iterations
    # to reach 1e-13 (measured with the oracle on this workload)
    pcg_its = 357
    step = ks_total * t_it + 2 * pcg_its * t_cg + 2 * t_rho
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    return {
        "value": 1.0 / step, "unit": "Magnus steps/s", "cores": threads, "kind": "oracle",
        "apply_H_gdof_orb_per_s": m.n_dof / t_it / 1e9,
        "sample": (f"oracle on this host: Lanczos propagations of 2 orbitals ({sum(ks)} its, {t_it*1e3:.0f} ms/it), "
                   f"20 Hartree PCG its ({t_cg*1e3:.0f} ms/it), 1 density ({t_rho:.2f} s); step = "
                   f"{ks_total} Krylov its + 2x{pcg_its} PCG its + 2 densities = {step:.1f} s; "
                   f"sample wall {time.perf_counter()-t0:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-graded", action="store_true")
    ap.add_argument("--no-nonlocal", action="store_true")
    ap.add_argument("--no-spectra", action="store_true")
    ap.add_argument("--no-midpoint", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU: the orbital-sharded multi-GPU layout is described, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
    cfg = W.CONFIGS[args.config]
    n_orb = cfg.n_orb

    def make(precision):
        ctx = tdfe.Context(cfg.p, cfg.ncell, W.vertices(cfg), n_orb_max=n_orb, k_max=cfg.k_max,
                           precision=precision)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
        if cfg.hartree or cfg.xc != "none":
            Z, R = W.atoms(cfg)
            ctx.set_scf(hartree=cfg.hartree, xc={"none": 0, "x": 1, "xc": 2}[cfg.xc], Z=Z, R=R, n_orb=n_orb)
        psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        return ctx, psi

    def run(precision):
        """warm-up steps one call each, then the timed steps in one
        tdfe_propagate call (no host synchronisation between steps); the
        per-step dipoles come back from the device record"""
        ctx, psi = make(precision)
        mus = []
        for _ in range(args.warmup):
            mus.append(ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)["mu"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec, tot = ctx.propagate(psi, args.steps, cfg.dt, None, cfg.tol)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mus.extend(rec[:, 1:].cpu().numpy())
        return ctx, wall, tot["k_corr_sum"], np.array(mus)

    def per_call_rate(ctx, n=None):
        """the same steps driven by one magnus_step call each (a host
        synchronisation at the end of every step)"""
        n = n or args.steps
        psi = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol, report=False)
        torch.cuda.synchronize()
        return n / (time.perf_counter() - t0)

    def time_apply(ctx, fp32):
        dt_ = torch.complex64 if fp32 else torch.complex128
        x = torch.randn(ctx.n_dof, n_orb, dtype=dt_, device="cuda")
        y = torch.zeros_like(x)
        f = ctx.apply_H_add_f32 if fp32 else ctx.apply_H_add
        for _ in range(5):
            f(x, y)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.apply_reps):
            f(x, y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / args.apply_reps

    def roofline(ctx, t_apply, elem_bytes, alu_peak, label):
        by, fl = apply_work(cfg.p + 1, cfg.nq, ctx.n_cell, ctx.n_dof, n_orb, elem_bytes)
        t_hbm = by / (HBM_PEAK_GBS * 1e9)
        t_alu = fl / (alu_peak * 1e12)
        if t_alu >= t_hbm:
            roof = {"bound": "alu", "achieved": fl / t_apply / 1e12, "peak": alu_peak, "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": by / t_apply / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = profiled_traffic("fp64" if elem_bytes == 8 else "fp32")
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
        roof["kernel"] = label
        roof["launch_us"] = t_apply * 1e6
        roof["algorithmic_bytes"] = by
        roof["algorithmic_flops"] = fl
        roof["hbm_frac"] = (by / t_apply / 1e9) / HBM_PEAK_GBS
        roof["alu_frac"] = (fl / t_apply / 1e12) / alu_peak
        return roof

    ctx, dt_wall, ks_total, mu64 = run(tdfe.FP64)
    steps_per_s = args.steps / dt_wall
    per_call = per_call_rate(ctx)
    # the paper's production Krylov tolerance (1e-8) on the same workload, FP64
    prod = None
    if cfg.tol != 1e-8:
        psi_p = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                  ctx.mass_diag().cpu().numpy())).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, tot_p = ctx.propagate(psi_p, args.steps, cfg.dt, None, 1e-8, record=False)
        torch.cuda.synchronize()
        prod = {"tol": 1e-8, "steps_per_s": args.steps / (time.perf_counter() - t0),
                "krylov_its_per_step": tot_p["k_corr_sum"] / args.steps}
    t_apply = time_apply(ctx, False)
    roof = roofline(ctx, t_apply, 8, FP64_VECTOR_PEAK_TFLOPS, "pair_kernel<double,6,16,1> (Hbar, 16^3 p=5, 8 orbitals)")
    gdof = ctx.n_dof * n_orb / t_apply / 1e9
    n_dof, n_cell = ctx.n_dof, ctx.n_cell
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    mixed = None
    if not args.no_mixed:
        ctxm, wall_m, ks_m, mu32 = run(tdfe.MIXED_FP32)
        per_call_m = per_call_rate(ctxm)
        t_apply_m = time_apply(ctxm, True)
        err = float(np.abs(mu32 - mu64).max() / np.abs(mu64).max())
        dmu = mu64 - mu64[0]
        err_induced = float(np.abs(mu32 - mu64).max() / max(np.abs(dmu).max(), 1e-300))
        mixed = {"value": args.steps / wall_m, "unit": "Magnus steps/s", "ms_per_step": 1e3 * wall_m / args.steps,
                 "dtype": "f32 operator + Krylov storage, f64 scalars/orbitals",
                 "lanczos_tol": f"max({cfg.tol:g}, 16 * 2^-24 * ||psibar_alpha||) per orbital (FP32 storage floor)",
                 "speedup_vs_f64": (args.steps / wall_m) / steps_per_s,
                 "per_call_steps_per_s": per_call_m,
                 "dipole_rel_err": err, "dipole_err_rel_induced": err_induced,
                 "steps_compared": len(mu64), "krylov_its_per_step": ks_m / args.steps,
                 "apply_H_gdof_orb_per_s": ctxm.n_dof * n_orb / t_apply_m / 1e9,
                 "roofline": roofline(ctxm, t_apply_m, 4, FP32_VECTOR_PEAK_TFLOPS,
                                      "plane_kernel<float,6,16,2> (Hbar, 16^3 p=5, 8 orbitals)")}
        ctxm.close()

    out = {
        "metric": "Magnus steps/sec and apply_H GDoF-orbitals/s, FP64 vs mixed at dipole err<=1e-5",
        "value": steps_per_s, "unit": "Magnus steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt_wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "n_dof": n_dof, "n_cell": n_cell, "p": cfg.p,
                   "n_orb": n_orb, "dt": cfg.dt, "tol": cfg.tol, "krylov_its_per_step": ks_total / args.steps,
                   "hartree": "fast diagonalisation (exact)", "xc": cfg.xc},
        "apply_H_gdof_orb_per_s": gdof,
        "per_call_steps_per_s": per_call,
        "production_tolerance": prod,
        "timed_region": "one tdfe_propagate call of the timed steps (per_call_steps_per_s: one magnus_step call per step)",
        "roofline": roof,
        "mixed": mixed,
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_rate()
    if not args.no_graded:
        out["graded_apply"] = graded_apply()
    if not args.no_nonlocal:
        out["nonlocal"] = nonlocal_term()
    if not args.no_spectra:
        out["field_and_spectra"] = field_and_spectra()
    if not args.no_midpoint:
        out["midpoint"] = midpoint_modes()
    if not args.no_adaptive:
        out["adaptive_mesh"] = adaptive_mesh()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_baseline(cfg, int(round(ks_total / args.steps)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
