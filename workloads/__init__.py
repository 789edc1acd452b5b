"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds none of the method's arithmetic: it draws atoms, builds
vertex arrays, evaluates the synthetic potential and orbital recipes at
coordinates handed in by the caller, and orthonormalises sampled columns in
a caller-given weighted inner product.  Each side passes its OWN node and
quadrature coordinates and its OWN overlap diagonal, so the two paths share
no computed quantity.

The molecule-like systems stand in for the paper's molecules (which need
pseudopotential tables and ground-state solutions that are not available):
Gaussian-well local potentials or smoothed Coulomb wells at seeded atom
positions, and smooth random orbitals.  Atomic units throughout.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Config:
    name: str
    lo: float
    hi: float
    ncell: tuple
    p: int
    nq: int
    n_orb: int
    dt: float
    steps: int
    tol: float
    k_max: int = 128
    hartree: bool = False
    xc: str = "none"
    kick: float = 0.0
    graded: bool = False
    atoms: dict = field(default_factory=dict)
    orbitals: dict = field(default_factory=dict)
    vmap: dict = field(default_factory=dict)
    potential: str = "gauss"
    pcg_tol: float = 1e-13


CONFIGS = {
    1: Config("harmonic-trap-1orb-p4-4^3", -8.0, 8.0, (4, 4, 4), 4, 5, 1, 0.05, 20, 1e-10,
              potential="harmonic"),
    2: Config("psp-like-4atoms-p5-16^3-8orb", -10.0, 10.0, (16, 16, 16), 5, 6, 8, 0.05, 200, 1e-10,
              hartree=True, xc="x", kick=1e-3,
              atoms=dict(seed=2, count=4, box=4.0, min_dist=2.0, Z=(1, 4)),
              orbitals=dict(seed=1000, sigma=2.5)),
    3: Config("graded-16atoms-p6-31^3-32orb", -16.0, 16.0, (31, 31, 31), 6, 7, 32, 0.05, 500, 1e-10,
              k_max=192, hartree=True, xc="xc", kick=1e-3, graded=True,
              atoms=dict(seed=3, count=16, box=5.0, min_dist=1.8, Z=(1, 4, 6)),
              orbitals=dict(seed=2000, sigma=3.5), vmap=dict(s=1.5, h_min=0.25)),
    4: Config("ae-like-6atoms-p7-39^3-24orb", -16.0, 16.0, (39, 39, 39), 7, 8, 24, 0.005, 1000, 1e-10,
              k_max=512, hartree=True, xc="xc", kick=1e-3, graded=True,
              atoms=dict(seed=4, count=6, box=3.0, min_dist=2.2, Z=(6, 7, 8)),
              orbitals=dict(seed=4000, sigma=2.0), vmap=dict(s=1.0, h_min=0.02),
              potential="coulomb"),
    5: Config("adjoint-field-p5-16^3-8orb", -10.0, 10.0, (16, 16, 16), 5, 6, 8, 0.05, 200, 1e-10,
              hartree=True, xc="x", kick=0.0,
              atoms=dict(seed=2, count=4, box=4.0, min_dist=2.0, Z=(1, 4)),
              orbitals=dict(seed=1000, sigma=2.5)),
}


def scaled(cfg, ncell=None, p=None, n_orb=None, steps=None, **kw):
    """A copy of ``cfg`` with a reduced mesh / orbital count for fast tests."""
    import dataclasses
    c = dataclasses.replace(cfg)
    if ncell is not None:
        c.ncell = tuple(ncell)
    if p is not None:
        c.p = p
        c.nq = p + 1
    if n_orb is not None:
        c.n_orb = n_orb
    if steps is not None:
        c.steps = steps
    for k, v in kw.items():
        setattr(c, k, v)
    return c


# ---------------------------------------------------------------------------
# atoms and meshes
# ---------------------------------------------------------------------------
def atoms(cfg):
    """Seeded atom positions (rejection sampling with a minimum distance) and charges."""
    a = cfg.atoms
    if not a:
        return np.zeros(0), np.zeros((0, 3))
    rng = np.random.default_rng(a["seed"])
    R = []
    while len(R) < a["count"]:
        x = rng.uniform(-a["box"], a["box"], 3)
        if all(np.linalg.norm(x - y) >= a["min_dist"] for y in R):
            R.append(x)
    Z = rng.choice(np.asarray(a["Z"], dtype=np.float64), size=a["count"])
    return Z, np.array(R)


def box_vertices(lo, hi, ncell):
    """Uniform box: vertices (ncz+1, ncy+1, ncx+1, 3), x fastest."""
    ncx, ncy, ncz = ncell
    xs = np.linspace(lo, hi, ncx + 1)
    ys = np.linspace(lo, hi, ncy + 1)
    zs = np.linspace(lo, hi, ncz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _corner_volumes_ok(V):
    """Every cell corner has a positively oriented edge triple."""
    e = {}
    for ax in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[2 - ax] = slice(0, -1)
        sl_hi[2 - ax] = slice(1, None)
        e[ax] = V[tuple(sl_hi)] - V[tuple(sl_lo)]
    ex, ey, ez = e[0][:-1, :-1, :], e[1][:-1, :, :-1], e[2][:, :-1, :-1]
    # corner (0,0,0) of every cell; the map is smooth, so this plus the
    # Jacobian checks done by each side at the quadrature points suffices
    return np.all(np.einsum("...i,...i->...", np.cross(ex, ey), ez) > 0)


def graded_vertices(cfg, Z, R):
    """Box vertices moved by x -> x - sum_I a (x - R_I) exp(-|x - R_I|^2 / s^2).

    ``a`` is chosen so that a cell at a nucleus shrinks to about h_min, and is
    reduced until every cell stays positively oriented.
    """
    V = box_vertices(cfg.lo, cfg.hi, cfg.ncell)
    if not cfg.graded:
        return V
    s = cfg.vmap["s"]
    h = (cfg.hi - cfg.lo) / cfg.ncell[0]
    a = 1.0 - cfg.vmap["h_min"] / h
    X = V.copy()
    while True:
        d = np.zeros_like(X)
        for r in R:
            dx = X - r
            d += a * dx * np.exp(-np.sum(dx * dx, axis=-1, keepdims=True) / s ** 2)
        W = X - d
        if _corner_volumes_ok(W):
            return W
        a *= 0.98


def vertices(cfg):
    Z, R = atoms(cfg)
    return graded_vertices(cfg, Z, R)


# ---------------------------------------------------------------------------
# potentials and orbitals evaluated at caller-given coordinates
# ---------------------------------------------------------------------------
def external_potential(cfg, xyz):
    """V_ext at points xyz (..., 3)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    if cfg.potential == "harmonic":
        return 0.5 * np.sum(xyz * xyz, axis=-1)
    Z, R = atoms(cfg)
    v = np.zeros(xyz.shape[:-1])
    for z, r in zip(Z, R):
        d2 = np.sum((xyz - r) ** 2, axis=-1)
        if cfg.potential == "gauss":
            v -= z * np.exp(-d2 / (2.0 * 0.5 ** 2))
        elif cfg.potential == "coulomb":
            v -= z / np.sqrt(d2 + 0.01 ** 2)
        else:
            raise ValueError(cfg.potential)
    return v


def orbital_samples(cfg, xyz):
    """Raw orbital values at points xyz: (npts, n_orb), complex."""
    xyz = np.asarray(xyz, dtype=np.float64)
    if cfg.potential == "harmonic":
        r2 = np.sum(xyz * xyz, axis=-1)
        psi = np.pi ** -0.75 * np.exp(-0.5 * r2) * np.exp(0.1j * xyz[:, 2])
        return psi[:, None]
    o = cfg.orbitals
    out = np.empty((len(xyz), cfg.n_orb))
    env = np.exp(-np.sum(xyz * xyz, axis=-1) / (2.0 * o["sigma"] ** 2))
    for al in range(cfg.n_orb):
        rng = np.random.default_rng(o["seed"] + al)
        amp = rng.normal(size=6)
        ks = []
        while len(ks) < 6:
            k = rng.uniform(-1.0, 1.0, 3)
            if np.linalg.norm(k) <= 1.0:
                ks.append(k)
        ph = rng.uniform(0.0, 2.0 * np.pi, 6)
        f = np.zeros(len(xyz))
        for m in range(6):
            f += amp[m] * np.cos(xyz @ ks[m] + ph[m])
        out[:, al] = env * f
    return out.astype(np.complex128)


def orthonormalize(X):
    """Cholesky-QR, twice, in the Euclidean inner product."""
    for _ in range(2):
        G = X.conj().T @ X
        Lc = np.linalg.cholesky(G)
        X = np.linalg.solve(Lc.conj(), X.T).T  # X L^-H
    return X


def initial_psibar(cfg, dof_xyz, mass_diag):
    """Initial Loewdin coefficients psibar = M^1/2 psi(x_j), orthonormalised, kicked.

    dof_xyz and mass_diag come from the side that will propagate the state.
    """
    f = orbital_samples(cfg, dof_xyz)
    X = np.sqrt(np.asarray(mass_diag))[:, None] * f
    if cfg.potential == "harmonic":
        X = X / np.linalg.norm(X)
    else:
        X = orthonormalize(X)
    if cfg.kick:
        X = X * np.exp(-1j * cfg.kick * np.asarray(dof_xyz)[:, 2])[:, None]
    return np.ascontiguousarray(X)


def field_amplitudes(n=200, seed=5):
    """Per-step field amplitudes E_n ~ U(-1e-3, 1e-3)."""
    return np.random.default_rng(seed).uniform(-1e-3, 1e-3, n)


def fd_indices(n=200, count=10, seed=55):
    return np.random.default_rng(seed).choice(n, count, replace=False)


# Kleinman-Bylander projector recipe (nonlocal pseudopotential term, Eq.
# VPSP): per atom an s and three p channels, u_lm = Y_lm-like polynomial times
# a Gaussian, dV_l a short-range Gaussian well of the channel's strength.  The
# values stand in for pseudo-atomic tables that are not available here.
KB_DEFAULT = dict(sigma_u=0.9, rc=0.75, A=(-1.5, 0.8))


def kb_projector_values(cfg, xyz, kb=None):
    """(u, dV) at the points xyz (..., 3): arrays (n_proj, ...) with n_proj =
    4 per atom, ordered atom-major, channels s, p_x, p_y, p_z."""
    kb = dict(KB_DEFAULT, **(kb or {}))
    _, R = atoms(cfg)
    xyz = np.asarray(xyz)
    us, dvs = [], []
    for Ra in R:
        d = xyz - Ra
        r2 = np.sum(d * d, axis=-1)
        env = np.exp(-r2 / (2.0 * kb["sigma_u"] ** 2))
        well = np.exp(-r2 / (2.0 * kb["rc"] ** 2))
        us.append(env)
        dvs.append(kb["A"][0] * well)
        for ax in range(3):
            us.append(d[..., ax] * env)
            dvs.append(kb["A"][1] * well)
    return np.array(us), np.array(dvs)


def random_block(n_dof, n_orb, seed):
    """A seeded random complex block (n_dof, n_orb) for operator tests."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n_dof, n_orb)) + 1j * rng.normal(size=(n_dof, n_orb))


def random_potential(n_cell, nq3, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.normal(size=(n_cell, nq3))
