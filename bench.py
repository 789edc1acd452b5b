"""Benchmark: second-order Magnus steps per second on one MI355X.

Headline workload: the graded molecule -- 31^3 trilinear cells on
[-16,16]^3 graded towards 16 Gaussian-well atoms (cells 0.25 to 2 bohr),
order p = 6 (6,331,625 DoFs), 32 complex orbitals, Hartree + LDA exchange and
PZ81 correlation, kick 1e-3 along z, dt = 0.05, Lanczos tolerance 1e-10.  One
step = the whole hot path: predictor Lanczos exp(-i dt/2 Hbar), density,
Hartree, XC, corrector Lanczos exp(-i dt Hbar), density, Hartree, XC, dipole.
Inputs are resident on the GPU before timing; the timed steps run in one
tdfe_propagate call.

Prints ONE JSON line.  Besides the contract fields: the mixed-precision path
(FP32 operator and Krylov storage, FP64 scalars) with its dipole error against
the FP64 trajectory and its speedup both at equal nominal tolerance and
against FP64 run at the mixed path's effective stop tolerance; the operator
kernel's position on the HBM roofline (launch duration from HIP events on the
library's stream, in the step's own launch shape); the pseudopotential-like
box workload (16^3 cells, p = 5, 8 orbitals) and two mixed steps of the
all-electron-like workload (39^3 cells, p = 7, 20 M DoFs, 24 orbitals) as
extras; and the CPU oracle timed on this host (a subprocess that runs beside
the GPU legs).
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3
MIXED_TOL_FLOOR = 16.0 * 2.0 ** -24  # the mixed path's stop floor per unit ||psibar_alpha||


def apply_bytes(n_dof, n_cell, n_quad, n_orb, elem_bytes, curved):
    """Algorithmic HBM bytes of one Hbar launch on n_orb complex orbitals:
    read psibar and write Hbar psibar once (2 reals each per DoF-orbital), the
    weighted potential once per Gauss point, M^-1/2 once per DoF (all in the
    kernel's precision), and on curved cells the 8 corner vertices per cell
    (FP64) from which the metric is recomputed."""
    b = n_dof * n_orb * 2 * elem_bytes * 2 + n_quad * elem_bytes + n_dof * elem_bytes
    if curved:
        b += n_cell * 24 * 8
    return b


def apply_flops(n, n_cell, n_orb):
    """Flops of one launch as the kernels execute them: per cell and real
    column 12 one-dimensional passes with even/odd folded tables (n^4 / 2
    multiply-adds each) plus ~7 n^3 pointwise; the per-point metric of curved
    cells is not counted."""
    return n_cell * 2 * n_orb * (12 * n ** 4 + 7 * n ** 3)


# the operator sources of the kernels the committed counter summaries cover
OPERATOR_SOURCES = {"curved": ("tdfe_apply_curved.hip", "tdfe_fold.h", "tdfe_rule1d.h"),
                    "box": ("tdfe_apply_box.hip", "tdfe_apply_pair.hip", "tdfe_fold.h", "tdfe_rule1d.h")}
TRAFFIC_PROFILES = {"curved": "operator_graded_31x31x31_p6_hbm_bytes.md",
                    "box": "operator_16x16x16_p5_8orb_hbm_bytes.md"}


def operator_source_hash(kind):
    h = hashlib.sha256()
    for name in OPERATOR_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1810_13130_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(kind, label):
    """HBM bytes per operator launch from the committed rocprofv3 counter
    summary, or None when the operator sources have changed since the
    counters were taken."""
    try:
        text = open(os.path.join(ROOT, "profiles", TRAFFIC_PROFILES[kind])).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if "=" in line and not line.startswith("|"):
            k, v = (x.strip() for x in line.split("=", 1))
            vals[k] = v
    if vals.get("source_sha256_prefix") != operator_source_hash(kind):
        return None
    v = vals.get(f"traffic_bytes_per_launch.{label}")
    return float(v) if v is not None else None


def cpu_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_worker(cfg_id):
    """The CPU oracle on this host (run in a subprocess beside the GPU legs):
    (1) real oracle Magnus steps of the harmonic trap, all 20 steps, with the
    BLAS pool's threads and with one thread; (2) a bounded sample of the
    headline workload on its full mesh: two Krylov iterations of one orbital's
    propagation, two iterations of the Hartree Jacobi-PCG, the density of two
    orbitals and the XC potential -- per-unit times that the parent scales by
    the iteration counts it measures."""
    import threadpoolctl
    import workloads as W
    from oracle import lanczos, operators as op, scf
    from oracle.magnus import State, System, magnus_step
    from oracle.mesh import Mesh
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    out = {"threads": threads, **cpu_info()}
    c1 = W.CONFIGS[1]

    def trap_steps():
        m1 = Mesh(c1.p, c1.ncell, W.vertices(c1), c1.nq)
        s1 = System(m1, W.external_potential(c1, m1.quad_xyz), tol=c1.tol)
        st = State(s1, W.initial_psibar(c1, m1.dof_xyz, m1.M))
        t = time.perf_counter()
        for _ in range(c1.steps):
            magnus_step(s1, st, c1.dt)
        return c1.steps / (time.perf_counter() - t)

    out["trap_steps_per_s"] = trap_steps()
    with threadpoolctl.threadpool_limits(1):
        out["trap_steps_per_s_1thread"] = trap_steps()

    def apply_rate(c, n_orb, reps):
        # oracle H-bar applications on n_orb orbitals, DoF-orbitals per second
        mc = Mesh(c.p, c.ncell, W.vertices(c), c.nq)
        vc = W.external_potential(c, mc.quad_xyz)
        xc = W.random_block(mc.n_dof, n_orb, 3)
        op.apply_Hbar(mc, vc, xc)  # first call builds the mesh's cached tables
        t0 = time.perf_counter()
        for _ in range(reps):
            op.apply_Hbar(mc, vc, xc)
        return mc.n_dof * n_orb * reps / (time.perf_counter() - t0)

    out["apply_dof_orb_per_s_cfg1"] = apply_rate(c1, 1, 20)
    out["apply_dof_orb_per_s_cfg2"] = apply_rate(W.CONFIGS[2], 8, 1)
    cfg = W.CONFIGS[cfg_id]
    t = time.perf_counter()
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    psi = W.initial_psibar(W.scaled(cfg, n_orb=2), m.dof_xyz, m.M)
    out["setup_s"] = time.perf_counter() - t

    def krylov_its(n):
        t0 = time.perf_counter()
        try:
            lanczos.lanczos_expm_vec(lambda v: op.apply_Hbar(m, vq, v), psi[:, 0], cfg.dt, 1e-300, k_max=n)
        except lanczos.NotConverged:
            pass
        return (time.perf_counter() - t0) / n

    out["krylov_it_s"] = krylov_its(2)
    with threadpoolctl.threadpool_limits(1):
        out["krylov_it_s_1thread"] = krylov_its(1)
    t0 = time.perf_counter()
    rho = scf.density(m, psi)
    out["density_per_orbital_s"] = (time.perf_counter() - t0) / psi.shape[1]
    t0 = time.perf_counter()
    scf.xc_potential(rho, cfg.xc)
    out["xc_s"] = time.perf_counter() - t0
    if cfg.hartree:
        # one PCG iteration: the difference of a 3-iteration and a 1-iteration
        # solve (each also forms the load vector, the initial residual and the
        # interpolation to the Gauss points)
        Z, R = W.atoms(cfg)
        h = scf.Hartree(m, Z, R, tol=1e-300, maxit=1)
        ts = []
        for its in (1, 3):
            h.maxit = its
            h.phi0[:] = 0.0
            t0 = time.perf_counter()
            try:
                h.solve(rho)
            except RuntimeError:
                pass
            ts.append(time.perf_counter() - t0)
        out["pcg_it_s"] = max(ts[1] - ts[0], 0.0) / 2
    out["n_dof"] = int(m.n_dof)
    out["wall_s"] = time.perf_counter() - t
    print(json.dumps(out), flush=True)


def start_cpu_worker(cfg_id):
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", "--config", str(cfg_id)],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def cpu_baseline(proc, cfg, counts, timeout_s=900):
    """Oracle Magnus steps/s on the headline workload from the worker's sample,
    scaled by the counts of the GPU's FP64 run of the same steps (Krylov
    iterations per step over all orbitals; Jacobi-PCG iterations per step, the
    oracle's own solver run on the GPU from the same states)."""
    try:
        so, se = proc.communicate(timeout=timeout_s)
        w = json.loads(so.strip().splitlines()[-1])
    except Exception as e:  # the baseline is reported, never required
        proc.kill()
        return {"error": f"oracle sample failed: {e}"}
    K, P, N = counts["krylov_its_per_step"], counts.get("jacobi_pcg_its_per_step", 0.0), cfg.n_orb
    step = (K * w["krylov_it_s"] + P * w.get("pcg_it_s", 0.0) + 2 * N * w["density_per_orbital_s"] + 2 * w["xc_s"])
    step1 = step * w["krylov_it_s_1thread"] / w["krylov_it_s"]
    return {
        "value": 1.0 / step, "unit": "Magnus steps/s", "cores": w["threads"], "kind": "oracle",
        "os_cpu_count": w["os_cpu_count"], "cpu_model": w["cpu_model"],
        "value_1thread_est": 1.0 / step1,
        "apply_H_gdof_orb_per_s": w["n_dof"] / w["krylov_it_s"] / 1e9,
        "apply_H_gdof_orb_per_s_trap": w.get("apply_dof_orb_per_s_cfg1", 0.0) / 1e9,
        "apply_H_gdof_orb_per_s_box_8orb": w.get("apply_dof_orb_per_s_cfg2", 0.0) / 1e9,
        "trap_steps_per_s": w["trap_steps_per_s"], "trap_steps_per_s_1thread": w["trap_steps_per_s_1thread"],
        "sample": (f"oracle (numpy/scipy FP64) on this host, {w['threads']} BLAS threads: timed pieces of a "
                   f"{cfg.name} step on its full mesh -- 2 Krylov iterations of one orbital "
                   f"({w['krylov_it_s']:.2f} s/it; 1 thread {w['krylov_it_s_1thread']:.2f} s/it), "
                   f"Hartree Jacobi-PCG iterations ({w.get('pcg_it_s', 0.0):.2f} s/it), the density of 2 "
                   f"orbitals ({w['density_per_orbital_s']:.2f} s/orbital), XC ({w['xc_s']:.2f} s) -- scaled "
                   f"by this run's counts per step: {K:.0f} Krylov its (GPU FP64, same recurrence), {P:.0f} "
                   f"Jacobi-PCG its (the oracle's solver and tolerance, run on the GPU from the same states), "
                   f"{2 * N} orbital densities: {step:.0f} s per step.  Also real oracle steps: the harmonic trap's "
                   f"20 Magnus steps at {w['trap_steps_per_s']:.2f} steps/s ({w['trap_steps_per_s_1thread']:.2f} "
                   f"on 1 thread).  Mesh set-up ({w['setup_s']:.0f} s) not counted."),
    }


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


def octree_mesh(n_elem=1728.0, n_steps=10, n0=4, max_level=3):
    """Octree mesh with hanging nodes from the a priori element size against
    a uniform mesh with about the same DoF count: the induced dipole of the
    benchmark workload's recipe with its potential held fixed (4 atoms, 8
    orbitals, kick, p = 5; octree contexts take no Hartree term) over 10
    steps, each against a 32^3-cell uniform reference; and the octree
    operator's rate."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    base = W.CONFIGS[2]
    Z, R = W.atoms(base)

    def run(ctx):
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(base, xq).reshape(ctx.n_cell, -1)).cuda())
        psi = torch.from_numpy(W.initial_psibar(base, ctx.dof_coords().cpu().numpy(),
                                                ctx.mass_diag().cpu().numpy())).cuda()
        mu = [ctx.dipole(psi)[0][2]]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n_steps):
            mu.append(ctx.magnus_step(psi, base.dt, 0.0, base.tol)["mu"][2])
        torch.cuda.synchronize()
        mu = np.array(mu)
        return mu - mu[0], time.perf_counter() - t

    t0 = time.perf_counter()
    leaves, E = tdfe.octree_leaves(base.p, base.lo, base.hi, R, Z, [1.0] * len(Z), [0.5] * len(Z), n_elem, n0,
                                   max_level, samples=129)
    t_leaves = time.perf_counter() - t0
    t0 = time.perf_counter()
    oc = tdfe.Context.octree(base.p, base.lo, base.hi, n0, max_level, leaves, n_orb_max=base.n_orb, k_max=base.k_max)
    t_setup = time.perf_counter() - t0
    d_oct, w_oct = run(oc)
    t_apply = time_apply(oc, base.n_orb, False, 20)
    res_oct = {"leaves": int(len(leaves)), "levels": np.bincount(leaves[:, 0]).tolist(), "n_dof": oc.n_dof,
               "hanging_nodes": oc.n_hanging, "constraint_nnz": oc.constraint_nnz, "E": E,
               "leaves_s": t_leaves, "setup_s": t_setup, "steps_per_s": n_steps / w_oct,
               "apply_us": t_apply * 1e6, "apply_H_gdof_orb_per_s": oc.n_dof * base.n_orb / t_apply / 1e9}
    nd_oct = oc.n_dof
    oc.close()
    torch.cuda.empty_cache()
    n1 = max(2, int(round((nd_oct ** (1.0 / 3.0) + 1.0) / base.p)))

    def uniform(nc):
        return tdfe.Context(base.p, (nc, nc, nc), W.box_vertices(base.lo, base.hi, (nc, nc, nc)),
                            n_orb_max=base.n_orb, k_max=base.k_max)

    ref_ctx = uniform(32)
    ref, _ = run(ref_ctx)
    nd_ref = ref_ctx.n_dof
    ref_ctx.close()
    torch.cuda.empty_cache()
    uc = uniform(n1)
    d_uni, w_uni = run(uc)
    nd_uni = uc.n_dof
    uc.close()
    torch.cuda.empty_cache()
    scale = np.abs(ref).max()
    res_oct["induced_dipole_rel_err"] = float(np.abs(d_oct - ref).max() / scale)
    return {"workload": base.name + f" recipe with a fixed potential, {n_steps} steps, p = {base.p}",
            "reference": {"cells": [32, 32, 32], "n_dof": nd_ref},
            "uniform": {"cells": [n1] * 3, "n_dof": nd_uni, "steps_per_s": n_steps / w_uni,
                        "induced_dipole_rel_err": float(np.abs(d_uni - ref).max() / scale)},
            "octree": res_oct}


class Workload:
    """One seeded workload on the GPU: the host-side inputs (vertices, V_ext at
    the Gauss points, the initial psibar) are formed once and shared by every
    context of the run (FP64 and mixed contexts have the same nodes and M)."""

    def __init__(self, cfg):
        import workloads as W
        self.W = W
        self.cfg = cfg
        self.V = W.vertices(cfg)
        self.vq = None
        self.psi0 = None

    def context(self, precision, pcg_precond=None, state=True):
        import torch
        from paper_1810_13130_amd import tdfe
        cfg, W = self.cfg, self.W
        ctx = tdfe.Context(cfg.p, cfg.ncell, self.V, n_orb_max=cfg.n_orb, k_max=cfg.k_max, precision=precision)
        if self.vq is None:
            xq = ctx.quad_coords().cpu().numpy()
            self.vq = torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1))
        if state and self.psi0 is None:
            self.psi0 = torch.from_numpy(W.initial_psibar(cfg, ctx.dof_coords().cpu().numpy(),
                                                          ctx.mass_diag().cpu().numpy()))
        ctx.set_potential(self.vq.cuda())
        if cfg.hartree or cfg.xc != "none":
            Z, R = W.atoms(cfg)
            ctx.set_scf(hartree=cfg.hartree, xc={"none": 0, "x": 1, "xc": 2}[cfg.xc], Z=Z, R=R, n_orb=cfg.n_orb,
                        pcg_tol=cfg.pcg_tol, pcg_precond=pcg_precond)
        return ctx, (self.psi0.cuda() if state else None)


def close(ctx):
    import torch
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def run_steps(ctx, psi, cfg, tol, steps, warmup):
    """warm-up steps one call each, then the timed steps in one tdfe_propagate
    call (no host synchronisation between steps); per-step dipoles of all
    steps from the reports and the device record"""
    import torch
    mus, kw = [], 0
    for _ in range(warmup):
        rep = ctx.magnus_step(psi, cfg.dt, 0.0, tol)
        mus.append(rep["mu"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec, tot = ctx.propagate(psi, steps, cfg.dt, None, tol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mus.extend(rec[:, 1:].cpu().numpy())
    return {"wall": wall, "steps_per_s": steps / wall, "krylov_its_per_step": tot["k_corr_sum"] / steps,
            "poisson_its_last_solve": tot["poisson_iters"], "mu": np.array(mus)}


def time_apply(ctx, n_orb, fp32, reps):
    """average duration of one operator launch on n_orb orbitals, from HIP
    events recorded on the library's stream (the current torch stream)"""
    import torch
    dt_ = torch.complex64 if fp32 else torch.complex128
    x = torch.randn(ctx.n_dof, n_orb, dtype=dt_, device="cuda")
    y = torch.zeros_like(x)
    f = ctx.apply_H_add_f32 if fp32 else ctx.apply_H_add
    # warm up for at least 50 ms of launches (clocks settle; a propagation
    # runs thousands of launches back to back)
    t_w = time.perf_counter()
    for i in range(1000):
        f(x, y)
        if i >= 2 and i % 4 == 3:
            torch.cuda.synchronize()
            if time.perf_counter() - t_w > 0.05:
                break
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        f(x, y)
    e1.record()
    torch.cuda.synchronize()
    del x, y
    return e0.elapsed_time(e1) / 1e3 / reps


def roofline(ctx, cfg, n_orb, t_launch, fp32, kernel, curved):
    eb = 4 if fp32 else 8
    by = apply_bytes(ctx.n_dof, ctx.n_cell, ctx.n_quad, n_orb, eb, curved)
    fl = apply_flops(cfg.p + 1, ctx.n_cell, n_orb)
    kind = "curved" if curved else "box"
    alu_peak = FP32_VECTOR_PEAK_TFLOPS if fp32 else FP64_VECTOR_PEAK_TFLOPS
    return {"bound": "hbm", "achieved": by / t_launch / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": by / t_launch / 1e9 / HBM_PEAK_GBS,
            "traffic": profiled_traffic(kind, ("fp32" if fp32 else "fp64") + f"_{n_orb}orb"),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated)",
            "kernel": kernel, "launch_orbitals": n_orb, "launch_us": t_launch * 1e6,
            "algorithmic_bytes": by, "bytes_per_dof_orb": by / (ctx.n_dof * n_orb),
            "executed_flops": fl, "alu_frac": fl / t_launch / 1e12 / alu_peak,
            "alu_peak_tflops": alu_peak}


def dipole_errors(mu, ref):
    n = min(len(mu), len(ref))
    d = np.abs(mu[:n] - ref[:n]).max()
    induced = np.abs(ref[:n] - ref[0]).max()
    return float(d / np.abs(ref[:n]).max()), float(d / max(induced, 1e-300)), n


def hartree_solves(reps=3):
    """The Hartree solve of the graded workload on its own (31^3 trilinear
    cells, p = 6, 6.5 M nodes): CG to relative residual 1e-13, preconditioned
    by the fast diagonalisation of the axis-averaged rectilinear stand-in
    (rocBLAS DGEMM passes) and by Jacobi, from a cold start and then warm
    started from the previous solution; time per solve and iterations."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.scaled(W.CONFIGS[3], n_orb=2)
    wl = Workload(cfg)
    out = {"workload": cfg.name + " (density of 2 orbitals)"}
    for name, pc in (("fdm", tdfe.PCG_FDM), ("jacobi", tdfe.PCG_JACOBI)):
        ctx, psi = wl.context(tdfe.FP64, pcg_precond=pc)
        res = []
        for r in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.scf_fields(psi, phi=False)
            torch.cuda.synchronize()
            res.append(time.perf_counter() - t)
        rep = ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        out[name] = {"cold_solve_s": res[0], "warm_solve_s": float(np.median(res[1:])),
                     "its_per_solve_in_a_step": rep["poisson_iters"]}
        close(ctx)
    return out


def ae_steps(n_steps=3):
    """The all-electron-like workload at full size (39^3 graded trilinear
    cells down to ~0.02 bohr at the nuclei, p = 7, 20,123,648 DoFs, 24
    orbitals, smoothed Coulomb wells Z in {6,7,8}, Hartree + exchange +
    correlation, kick 1e-3, dt 0.005, k_max 512) on the mixed path: the
    Krylov basis in FP32, chunked to the device memory (k_max + 2 vectors
    per orbital), recurrence scalars and the small exponential in FP64.  The
    first step also forms W_0 and runs at k_max; later steps may run wider
    chunks under a soft cap on the Krylov dimension (the chunk and cap in
    effect are recorded per step).  Step times, Krylov dimensions, charge."""
    import torch
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[4]
    t0 = time.perf_counter()
    wl = Workload(cfg)
    ctx, psi = wl.context(tdfe.MIXED_FP32)
    out = {"workload": cfg.name, "n_dof": ctx.n_dof, "n_orb": cfg.n_orb, "k_max": cfg.k_max, "dt": cfg.dt,
           "tol": cfg.tol, "krylov_chunk_orbitals": ctx.krylov_chunk(cfg.n_orb), "setup_s": None, "steps": []}
    torch.cuda.synchronize()
    out["setup_s"] = time.perf_counter() - t0
    for _ in range(n_steps):
        chunk, kcap = ctx.krylov_soft_chunk(cfg.n_orb)
        t = time.perf_counter()
        try:
            rep = ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        except tdfe.TdfeError as e:
            out["steps"].append({"error": str(e), "wall_s": time.perf_counter() - t})
            break
        torch.cuda.synchronize()
        out["steps"].append({"wall_s": time.perf_counter() - t, "chunk_orbitals": chunk, "k_cap": kcap,
                             "k_pred_max": rep["k_pred_max"],
                             "k_corr_max": rep["k_corr_max"], "k_pred_sum": rep["k_pred_sum"],
                             "k_corr_sum": rep["k_corr_sum"], "err_max": rep["err_max"],
                             "hartree_its": rep["poisson_iters"], "charge": rep["charge"], "mu": list(rep["mu"])})
    # the FP32 operator at the step's launch shape (the Krylov chunk) and at 8
    # orbitals, against the HBM roof
    out["operator"] = []
    for norb in sorted({out["krylov_chunk_orbitals"], 8} | {st.get("chunk_orbitals", 8) for st in out["steps"]}):
        t = time_apply(ctx, norb, True, 10)
        by = apply_bytes(ctx.n_dof, ctx.n_cell, ctx.n_quad, norb, 4, True)
        out["operator"].append({"orbitals": norb, "launch_us": t * 1e6, "algorithmic_bytes": by,
                                "hbm_frac": by / t / 1e9 / HBM_PEAK_GBS})
    close(ctx)
    return out


def matrix_core_engines(steps=100, warmup=5, reps=100):
    """The box-cell workload (16^3 cells, p = 5, 8 orbitals, Hartree + LDA x)
    with the cell operator's 1D contractions on each engine: the VALU kernels
    of the FP64 and mixed paths and the matrix-core variants (FP64, FP32 and
    split BF16 products): operator launch time in the step's shape, Magnus
    steps/s and the dipole error against the FP64 VALU trajectory."""
    import workloads as W
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[2]
    wl = Workload(cfg)
    out = {"workload": cfg.name, "steps": steps}
    ref = None
    engines = (("f64_valu", tdfe.FP64, False, "pair_kernel<double,6,16,1>"),
               ("f64_mfma", tdfe.FP64_MFMA, False, "mfma_box_kernel<FP64,6> (v_mfma_f64_16x16x4)"),
               ("f32_valu", tdfe.MIXED_FP32, True, "plane_kernel<float,6,16,2>"),
               ("f32_mfma", tdfe.FP32_MFMA, True, "mfma_box_kernel<FP32,6> (v_mfma_f32_16x16x4)"),
               ("bf16x3_mfma", tdfe.BF16_MFMA, True, "mfma_box_kernel<BF16x3,6> (v_mfma_f32_16x16x16_bf16)"))
    for name, prec, fp32, kernel in engines:
        ctx, psi = wl.context(prec)
        n = ctx.krylov_chunk(cfg.n_orb)
        r = run_steps(ctx, psi, cfg, cfg.tol, steps, warmup)
        t = time_apply(ctx, n, fp32, reps)
        rec = {"kernel": kernel, "launch_us": t * 1e6, "launch_orbitals": n, "steps_per_s": r["steps_per_s"],
               "krylov_its_per_step": r["krylov_its_per_step"],
               "hbm_frac": apply_bytes(ctx.n_dof, ctx.n_cell, ctx.n_quad, n, 4 if fp32 else 8, False) / t / 1e9
               / HBM_PEAK_GBS}
        if ref is None:
            ref = r["mu"]
        else:
            e, e_ind, m = dipole_errors(r["mu"], ref)
            rec.update({"dipole_rel_err": e, "dipole_err_rel_induced": e_ind, "steps_compared": m})
        out[name] = rec
        close(ctx)
    return out


def curved_kernel_name(p, cols, fp32):
    """Name of the trilinear-cell operator kernel a launch of `cols` real
    columns runs (the library's default choice: lane pairs for FP64 and for
    FP32 at p = 7, plane ownership for FP32 below; columns per block the next
    power of two up to 16, at least 2 for lane pairs, or 32 for FP32 plane
    launches of more than 16)."""
    n = p + 1
    pw = 1
    while pw < cols:
        pw *= 2
    if not fp32 or n == 8:
        t = "float" if fp32 else "double"
        return f"cpair_kernel<{t},{n},{max(2, min(pw, 16))},CPB> (trilinear cells, lane pairs)"
    return f"cplane_kernel<float,{n},{32 if cols > 16 else pw},CPB> (trilinear cells)"


def workload_legs(cfg, steps, warmup, apply_reps, curved, matched=True, jacobi_count=False):
    """FP64, mixed and (optionally) FP64 at the mixed path's effective stop
    tolerance on one workload; operator launches in the step's shape."""
    from paper_1810_13130_amd import tdfe
    wl = Workload(cfg)
    res = {}
    ctx, psi = wl.context(tdfe.FP64)
    chunk64 = ctx.krylov_chunk(cfg.n_orb)
    r64 = run_steps(ctx, psi, cfg, cfg.tol, steps, warmup)
    t_chunk = time_apply(ctx, chunk64, False, apply_reps)
    t_full = time_apply(ctx, cfg.n_orb, False, max(3, apply_reps // 4))
    kname = curved_kernel_name(cfg.p, 2 * chunk64, False) if curved else "pair_kernel<double,6,16,1> (box cells)"
    res["f64"] = {**{k: v for k, v in r64.items() if k != "mu"}, "chunk_orbitals": chunk64,
                  "roofline": roofline(ctx, cfg, chunk64, t_chunk, False, kname, curved),
                  "apply_H_gdof_orb_per_s": ctx.n_dof * cfg.n_orb / t_full / 1e9, "apply_full_ms": t_full * 1e3}
    res["n_dof"], res["n_cell"] = ctx.n_dof, ctx.n_cell
    if jacobi_count:
        # the oracle's Hartree solver (Jacobi-PCG at the same tolerance) from the
        # same states: one step to restart the history, then one step counted
        Z, R = wl.W.atoms(cfg)
        ctx.set_scf(hartree=cfg.hartree, xc={"none": 0, "x": 1, "xc": 2}[cfg.xc], Z=Z, R=R, n_orb=cfg.n_orb,
                    pcg_tol=cfg.pcg_tol, pcg_precond=tdfe.PCG_JACOBI)
        ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        rj = ctx.magnus_step(psi, cfg.dt, 0.0, cfg.tol)
        res["jacobi_pcg_its_per_solve"] = rj["poisson_iters"]
    close(ctx)
    ctx, psi = wl.context(tdfe.MIXED_FP32)
    chunk32 = ctx.krylov_chunk(cfg.n_orb)
    r32 = run_steps(ctx, psi, cfg, cfg.tol, steps, warmup)
    t_chunk32 = time_apply(ctx, chunk32, True, apply_reps)
    t_full32 = time_apply(ctx, cfg.n_orb, True, max(3, apply_reps // 4))
    kname32 = curved_kernel_name(cfg.p, 2 * chunk32, True) if curved else None
    e, e_ind, n = dipole_errors(r32["mu"], r64["mu"])
    res["mixed"] = {**{k: v for k, v in r32.items() if k != "mu"}, "chunk_orbitals": chunk32,
                    "dipole_rel_err": e, "dipole_err_rel_induced": e_ind, "steps_compared": n,
                    "speedup_vs_f64_same_tol": r32["steps_per_s"] / r64["steps_per_s"],
                    "roofline": roofline(ctx, cfg, chunk32, t_chunk32, True,
                                         kname32 if curved else "plane_kernel<float,6,16,2> (box cells)", curved),
                    "apply_H_gdof_orb_per_s": ctx.n_dof * cfg.n_orb / t_full32 / 1e9, "apply_full_ms": t_full32 * 1e3}
    close(ctx)
    if matched:
        tol_m = max(cfg.tol, MIXED_TOL_FLOOR)  # ||psibar_alpha|| = 1 (orthonormal orbitals)
        ctx, psi = wl.context(tdfe.FP64)
        rm = run_steps(ctx, psi, cfg, tol_m, steps, warmup)
        em, em_ind, _ = dipole_errors(rm["mu"], r64["mu"])
        res["f64_matched_tol"] = {**{k: v for k, v in rm.items() if k != "mu"}, "tol": tol_m,
                                  "dipole_rel_err": em, "dipole_err_rel_induced": em_ind}
        res["mixed"]["speedup_vs_f64_matched_tol"] = r32["steps_per_s"] / rm["steps_per_s"]
        close(ctx)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-matched", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the box workload and the extension legs")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the operator launches of the headline workload (for counter runs)")
    ap.add_argument("--engines", default="f64,mixed",
                    help="with --apply-only: comma list of f64, mixed, f64_mfma, f32_mfma, bf16_mfma (the matrix-core "
                         "variants need a box-cell workload, --config 2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference kernel for HBM byte counters)")
    ap.add_argument("--legs", default=None,
                    help="comma list of extra legs to run alone (ae, box, hartree, adjoint, nonlocal, spectra, midpoint, "
                         "adaptive, octree, mfma)")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.config)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU: the orbital-sharded multi-GPU layout is described, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import workloads as W
    cfg = W.CONFIGS[args.config]
    curved = cfg.graded
    cpu = None if (args.no_cpu_baseline or args.apply_only or args.legs) else start_cpu_worker(args.config)

    import torch
    from paper_1810_13130_amd import tdfe
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    legs = {"ae": ae_steps, "hartree": hartree_solves, "adjoint": adjoint_rate, "nonlocal": nonlocal_term, "spectra": field_and_spectra,
            "midpoint": midpoint_modes, "adaptive": adaptive_mesh, "octree": octree_mesh, "mfma": matrix_core_engines,
            "box": lambda: {"workload": W.CONFIGS[2].name, **workload_legs(W.CONFIGS[2], 100, 5, 100, False)}}
    if args.legs:
        print(json.dumps({name: legs[name]() for name in args.legs.split(",")}), flush=True)
        return
    if args.apply_only:
        wl = Workload(cfg)
        engines = {"f64": (tdfe.FP64, False), "mixed": (tdfe.MIXED_FP32, True), "f64_mfma": (tdfe.FP64_MFMA, False),
                   "f32_mfma": (tdfe.FP32_MFMA, True), "bf16_mfma": (tdfe.BF16_MFMA, True)}
        for name in args.engines.split(","):
            prec, fp32 = engines[name]
            ctx, _ = wl.context(prec, state=False)
            n = ctx.krylov_chunk(cfg.n_orb)
            t = time_apply(ctx, n, fp32, args.apply_reps)
            print(json.dumps({"precision": name, "launch_orbitals": n, "launch_us": t * 1e6}), flush=True)
            close(ctx)
        return

    res = workload_legs(cfg, args.steps, args.warmup, args.apply_reps, curved, matched=not args.no_matched,
                        jacobi_count=curved and cfg.hartree)
    f64 = res["f64"]
    counts = {"krylov_its_per_step": f64["krylov_its_per_step"]}
    if "jacobi_pcg_its_per_solve" in res:
        counts["jacobi_pcg_its_per_step"] = 2.0 * res["jacobi_pcg_its_per_solve"]
    hartree = ("none" if not cfg.hartree else
               ("CG with the fast diagonalisation of the axis-averaged rectilinear mesh as preconditioner, "
                f"relative residual {cfg.pcg_tol:g}" if curved else "fast diagonalisation (exact)"))
    out = {
        "metric": "Magnus steps/sec and apply_H GDoF-orbitals/s, FP64 vs mixed at dipole err<=1e-5",
        "value": f64["steps_per_s"], "unit": "Magnus steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * f64["wall"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "n_dof": res["n_dof"], "n_cell": res["n_cell"], "p": cfg.p,
                   "n_orb": cfg.n_orb, "dt": cfg.dt, "tol": cfg.tol, "krylov_its_per_step": f64["krylov_its_per_step"],
                   "krylov_chunk_orbitals": f64["chunk_orbitals"], "hartree": hartree,
                   "hartree_its_last_solve": f64["poisson_its_last_solve"],
                   "jacobi_pcg_its_per_solve": res.get("jacobi_pcg_its_per_solve"), "xc": cfg.xc},
        "apply_H_gdof_orb_per_s": f64["apply_H_gdof_orb_per_s"],
        "apply_H_gdof_orb_per_s_mixed": res["mixed"]["apply_H_gdof_orb_per_s"],
        "timed_region": "one tdfe_propagate call of the timed steps; warm-up steps one magnus_step call each",
        "roofline": f64["roofline"],
        "mixed": {"value": res["mixed"]["steps_per_s"], "unit": "Magnus steps/s",
                  "dtype": "f32 operator + Krylov storage, f64 recurrence scalars / small exponential / orbitals",
                  "lanczos_tol": f"max({cfg.tol:g}, 16 * 2^-24 * ||psibar_alpha||) per orbital (FP32 storage floor)",
                  **{k: v for k, v in res["mixed"].items() if k not in ("steps_per_s", "wall")}},
        "f64_matched_tol": res.get("f64_matched_tol"),
    }
    if not args.no_extras:
        c2 = W.CONFIGS[2]
        r2 = workload_legs(c2, 100, 5, 100, False, matched=True)
        out["box_workload"] = {"workload": c2.name, **r2}
        out["ae_workload"] = ae_steps()
        out["hartree_graded"] = hartree_solves()
        for name, fn in (("adjoint", adjoint_rate), ("nonlocal", nonlocal_term), ("field_and_spectra", field_and_spectra),
                         ("midpoint", midpoint_modes), ("adaptive_mesh", adaptive_mesh),
                         ("octree_mesh", octree_mesh), ("matrix_cores", matrix_core_engines)):
            out[name] = fn()
    if cpu is not None:
        out["cpu_baseline"] = cpu_baseline(cpu, cfg, counts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
