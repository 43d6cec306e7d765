"""Seeded synthetic inputs and the named workloads.

This module only manufactures inputs: grids, initial distributions, random
occupation fields, random proposal tables and random network weights.  It holds
none of the collision-term arithmetic, so both the GPU path and the CPU oracle
can be fed from it.

Initial conditions follow the paper's own formulas where it gives them: the
step function of Eq. CGC (Sec. IV E), the Bose-Einstein / Fermi-Dirac forms of
Eq. fg / Eq. fq, and a Gaussian transverse profile or Gaussian blobs for the
spatially inhomogeneous runs (the paper's Eq. ini_f_test_spread is linear in x;
the profiles here are smooth and periodic-friendly stand-ins of the same kind).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SPECIES = ("u", "d", "s", "ubar", "dbar", "sbar", "g")
GLUON = 6
ALL_SPECIES = 0x7F
ALL_ROWS = 0x7F
PHILOX_SEED = 0x5EED2019
BLOB_SEED = 12345


@dataclass(frozen=True)
class Workload:
    name: str
    n_x: tuple
    n_p: tuple
    x_half: tuple
    p_half: tuple
    species_mask: int
    n_samples: int
    precision: str          # "f64" or "f32"
    steps: int
    dt_fm: float
    drift: str = "upwind"
    sampler: str = "uniform"
    alpha_s: float = 0.3
    row_mask: int = ALL_ROWS
    init: dict = field(default_factory=dict)
    symmetric: bool = True

    @property
    def cells(self) -> int:
        return int(np.prod(self.n_x))

    @property
    def nodes(self) -> int:
        return int(np.prod(self.n_p))

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads of the measurement plan.
C1 = Workload("gg_1cell_10cube_f64", (1, 1, 1), (10, 10, 10), (3.0, 3.0, 3.0), (2.0, 2.0, 2.0),
              1 << GLUON, 1000, "f64", 1, 0.01, init=dict(kind="cgc", f0=0.5, Qs=1.0))
C2 = Workload("gg_16x16x1_20cube_f32", (16, 16, 1), (20, 20, 20), (6.0, 6.0, 0.375), (3.0, 3.0, 3.0),
              1 << GLUON, 2048, "f32", 20, 0.01,
              init=dict(kind="gauss_transverse", f0=0.5, Qs=1.0, width_fm=2.0))
C3 = Workload("qg7_1cell_20cube_f32", (1, 1, 1), (20, 20, 20), (3.0, 3.0, 3.0), (3.0, 3.0, 3.0),
              ALL_SPECIES, 4096, "f32", 1, 0.01,
              init=dict(kind="cgc_fd", f0=1.0, Qs=1.0, T=0.3))
C4 = replace(C3, name="qg7_1cell_20cube_learned", sampler="learned")
C5 = Workload("qg7_12cube_16cube_learned", (12, 12, 12), (16, 16, 16), (6.0, 6.0, 6.0),
              (3.0, 3.0, 3.0), ALL_SPECIES, 256, "f32", 50, 0.01, sampler="learned",
              init=dict(kind="blobs_fd", Qs=1.0, T=0.3, n_blobs=3, seed=BLOB_SEED))
# The stability test of Sec. IV A: f uniform in [0, 1] on 40^3 nodes, 100
# samples per node, one step of the direct estimator, with the paper's root
# parameterisation (and its alternative elimination).
ROOTS = Workload("g_1cell_40cube_roots", (1, 1, 1), (40, 40, 40), (3.0, 3.0, 3.0), (2.0, 2.0, 2.0),
                 1 << GLUON, 100, "f64", 1, 0.01, sampler="roots", symmetric=False,
                 init=dict(kind="uniform", seed=7))
ROOTS_ALT = replace(ROOTS, name="g_1cell_40cube_roots_alt", sampler="roots_alt")
WORKLOADS = {w.name: w for w in (C1, C2, C3, C4, C5, ROOTS, ROOTS_ALT)}


def node_momenta(n_p, p_half) -> np.ndarray:
    """Cell-centred momentum nodes, shape (nodes, 3), pz fastest."""
    axes = [-ph + (np.arange(n) + 0.5) * 2.0 * ph / n for n, ph in zip(n_p, p_half)]
    return np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)


def cell_centres(n_x, x_half) -> np.ndarray:
    axes = [-xh + (np.arange(n) + 0.5) * 2.0 * xh / n for n, xh in zip(n_x, x_half)]
    return np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)


def bose_einstein(E, T, mu=0.0):
    return 1.0 / np.expm1((E - mu) / T)


def fermi_dirac(E, T, mu=0.0):
    return 1.0 / (np.exp((E - mu) / T) + 1.0)


def initial_f(wl: Workload) -> np.ndarray:
    """Initial occupation, float64 of shape (7, cells, nodes)."""
    P = node_momenta(wl.n_p, wl.p_half)
    X = cell_centres(wl.n_x, wl.x_half)
    absp = np.linalg.norm(P, axis=1)
    f = np.zeros((7, wl.cells, wl.nodes))
    ini = wl.init
    kind = ini.get("kind", "cgc")
    step = (absp < ini.get("Qs", 1.0)).astype(np.float64)
    if kind == "cgc":
        f[GLUON] = ini["f0"] * step[None, :]
    elif kind == "gauss_transverse":
        r2 = X[:, 0] ** 2 + X[:, 1] ** 2
        prof = np.exp(-r2 / (2.0 * ini["width_fm"] ** 2))
        f[GLUON] = ini["f0"] * prof[:, None] * step[None, :]
    elif kind in ("cgc_fd", "blobs_fd"):
        fq = fermi_dirac(absp, ini["T"])
        for sp in range(6):
            f[sp] = fq[None, :]
        if kind == "cgc_fd":
            f[GLUON] = ini["f0"] * step[None, :]
        else:
            f0 = blob_profile(wl, X, ini)
            f[GLUON] = f0[:, None] * step[None, :]
    elif kind == "uniform":
        rng = np.random.Generator(np.random.PCG64(ini.get("seed", 7)))
        f[GLUON] = rng.uniform(0.0, 1.0, size=(wl.cells, wl.nodes))
    else:
        raise ValueError(f"unknown initial condition {kind}")
    for sp in range(7):
        if not (wl.species_mask >> sp) & 1:
            f[sp] = 0.0
    return f


def blob_profile(wl: Workload, X: np.ndarray, ini: dict) -> np.ndarray:
    """f0(x) = 0.2 + 0.8 G/max G with G a sum of Gaussian blobs (seeded)."""
    rng = np.random.Generator(np.random.PCG64(ini.get("seed", BLOB_SEED)))
    half = np.asarray(wl.x_half)
    G = np.zeros(len(X))
    for _ in range(ini.get("n_blobs", 3)):
        c = rng.uniform(-half, half)
        s = rng.uniform(1.0, 2.0)
        G += np.exp(-np.sum((X - c) ** 2, axis=1) / (2.0 * s * s))
    return 0.2 + 0.8 * G / G.max()


def random_f(seed: int, cells: int, nodes: int, species_mask: int = ALL_SPECIES,
             quark_max: float = 0.6, gluon_max: float = 1.2) -> np.ndarray:
    """Uniform random occupations (quarks in [0, quark_max], gluons in [0, gluon_max])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((7, cells, nodes))
    for sp in range(7):
        if (species_mask >> sp) & 1:
            top = gluon_max if sp == GLUON else quark_max
            f[sp] = rng.uniform(0.0, top, size=(cells, nodes))
    return f


def smooth_f(cells: int, n_p, p_half, species_mask: int = ALL_SPECIES, amp_g: float = 0.8,
             T: float = 0.4) -> np.ndarray:
    """Smooth occupations: a Gaussian bump for gluons, Fermi-Dirac for quarks."""
    P = node_momenta(n_p, p_half)
    absp = np.linalg.norm(P, axis=1)
    f = np.zeros((7, cells, len(P)))
    for sp in range(7):
        if not (species_mask >> sp) & 1:
            continue
        if sp == GLUON:
            f[sp] = amp_g * np.exp(-absp ** 2 / 2.0)[None, :]
        else:
            f[sp] = fermi_dirac(absp, T, 0.05 * (sp % 3) * (1 if sp < 3 else -1))[None, :]
    return f


def cell_varied_f(seed: int, n_x, n_p, p_half, x_half, species_mask: int = ALL_SPECIES) -> np.ndarray:
    """Smooth momentum profiles (smooth_f) whose amplitude varies from cell to
    cell: a seeded random factor in [0.4, 1.2] per (species, cell) times a
    gradient along x, so that neighbouring cells differ in f and in their
    thermal masses (a spatial force in the drift)."""
    cells = int(np.prod(n_x))
    f = smooth_f(cells, n_p, p_half, species_mask=species_mask)
    rng = np.random.Generator(np.random.PCG64(seed))
    X = cell_centres(n_x, x_half)
    tilt = 1.0 + 0.3 * X[:, 0] / max(x_half[0], 1e-300)
    f *= rng.uniform(0.4, 1.2, size=(7, cells))[:, :, None] * tilt[None, :, None]
    return f


def random_mog_table(seed: int, rows: int, K: int = 8, alpha: float = 0.1,
                     mu_scale: float = 1.5, log_sigma=(-1.0, 0.7)):
    """Random mixture table in the proposal-table format.

    Returns (thr u32 [rows, K], mu f32 [rows, K, 5], sigma f32 [rows, K, 5]).
    thr[:, 0] is the defensive-uniform boundary alpha * 2^32, thr[:, k] the
    cumulative lower boundary of component k.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.dirichlet(np.ones(K), size=rows)
    cum = np.concatenate([np.zeros((rows, 1)), np.cumsum(w, axis=1)[:, :-1]], axis=1)
    lo = alpha + (1.0 - alpha) * cum
    thr = np.floor(lo * 4294967296.0).astype(np.uint64)
    thr = np.minimum(thr, 4294967295).astype(np.uint32)
    mu = rng.normal(0.0, mu_scale, size=(rows, K, 5)).astype(np.float32)
    sigma = np.exp(rng.uniform(log_sigma[0], log_sigma[1], size=(rows, K, 5))).astype(np.float32)
    return thr, mu, sigma


def random_mlp_params(seed: int, n_in: int = 8, hidden: int = 128, n_out: int = 88,
                      head_scale: float = 0.1) -> np.ndarray:
    """Flat FP32 parameter vector W1, b1, W2, b2, W3, b3 (row-major [in][out]),
    He-style initialisation with a small head."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0.0, np.sqrt(2.0 / n_in), (n_in, hidden))
    b1 = rng.normal(0.0, 0.05, hidden)
    W2 = rng.normal(0.0, np.sqrt(2.0 / hidden), (hidden, hidden))
    b2 = rng.normal(0.0, 0.05, hidden)
    W3 = rng.normal(0.0, head_scale * np.sqrt(1.0 / hidden), (hidden, n_out))
    b3 = rng.normal(0.0, 0.05, n_out)
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)
