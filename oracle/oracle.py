"""FP64 CPU oracle for the Monte Carlo collision term (arXiv:1912.04457).

TEST INFRASTRUCTURE ONLY.  This module and the C library it drives are the
plain, slow reference the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it.  It shares no code with the GPU library and imports nothing from it.

Arrays follow the layout of the C oracle: ``f`` and ``A`` are float64 arrays of
shape ``(7, cells, nodes)`` (species u, d, s, ubar, dbar, sbar, g), ``mass2`` is
``(7, cells)``.

The time step (``step``) composes the C primitives the way Sec. III of the
paper states it: thermal masses (Eq. mg, Eq. mq, with E = |p| on the first
step and the lagged masses afterwards), the collision term, the drift in flux
form (Eq. left handside), and a forward-Euler update.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_qgbe.so")
SRC = os.path.join(HERE, "qgbe_oracle.c")

HBARC = 0.1973269804  # GeV fm
SPECIES = ("u", "d", "s", "ubar", "dbar", "sbar", "g")
GLUON = 6
DEGENERACY = np.array([6.0] * 6 + [16.0])  # N_q = 2*3, N_g = 2*8

REF_B_ONE, REF_NO_BOXCUT, REF_MASSLESS, REF_ANALYTIC_F = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "qgbe_oracle.h"))
    ):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-o", LIB_PATH + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


OPCOUNT_SRC = os.path.join(HERE, "opcount.cpp")
OPCOUNT_BIN = os.path.join(HERE, "opcount")


def build_opcount(force: bool = False) -> str:
    """Compile the op-count build of the oracle (the same C source with a
    counting number type; see opcount.cpp) with g++."""
    deps = [OPCOUNT_SRC, SRC, os.path.join(HERE, "qgbe_oracle.h")]
    if force or not os.path.exists(OPCOUNT_BIN) or os.path.getmtime(OPCOUNT_BIN) < max(map(os.path.getmtime, deps)):
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-o", OPCOUNT_BIN + ".tmp", OPCOUNT_SRC, "-lm"])
        os.replace(OPCOUNT_BIN + ".tmp", OPCOUNT_BIN)
    return OPCOUNT_BIN


def op_counts() -> dict:
    """Per-sample operation counts of the oracle's estimators, by class (the
    JSON object opcount.cpp prints)."""
    import json
    return json.loads(subprocess.check_output([build_opcount()], text=True))


class _Grid(C.Structure):
    _fields_ = [("n_x", C.c_int32 * 3), ("n_p", C.c_int32 * 3),
                ("x_half", C.c_double * 3), ("p_half", C.c_double * 3),
                ("species_mask", C.c_uint32), ("row_mask", C.c_uint32),
                ("alpha_s", C.c_double)]


class _Channel(C.Structure):
    _fields_ = [("row", C.c_int32), ("sp", C.c_int32 * 4), ("code", C.c_int32),
                ("w", C.c_double), ("sigma", C.c_double)]


class _Eq(C.Structure):
    _fields_ = [("T", C.c_double), ("mu", C.c_double * 7)]


class _Point(C.Structure):
    _fields_ = [("valid", C.c_int32), ("k", (C.c_double * 4) * 4),
                ("s", C.c_double), ("t", C.c_double), ("u", C.c_double),
                ("pstar", C.c_double), ("msq", C.c_double), ("f", C.c_double * 4),
                ("B", C.c_double), ("GL", C.c_double), ("g", C.c_double),
                ("gscale", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i32, u32, u64, p = C.c_double, C.c_int32, C.c_uint32, C.c_uint64, C.c_void_p
        _lib.ref_philox4x32_10.argtypes = [p, p, p]
        _lib.ref_msq.restype = d
        _lib.ref_msq.argtypes = [i32, d, d, d, d, d]
        _lib.ref_channels.restype = i32
        _lib.ref_channels.argtypes = [p, p, i32]
        _lib.ref_masses.restype = i32
        _lib.ref_masses.argtypes = [p, p, p, p]
        _lib.ref_eval_cm.restype = i32
        _lib.ref_eval_cm.argtypes = [p, p, p, p, i32, p, i32, p, d, d, i32, p, p]
        _lib.ref_collision.restype = i32
        _lib.ref_collision.argtypes = [p, p, p, u64, u32, i32, i32, i32, i32, p, p, p, p, i32]
        _lib.ref_collision_learned.restype = i32
        _lib.ref_collision_learned.argtypes = [p, p, p, u64, u32, i32, i32, p, p, p, i32, p,
                                               p, p, p, i32]
        _lib.ref_item_sums.restype = i32
        _lib.ref_item_sums.argtypes = [p, p, p, u64, u32, i32, i32, C.c_int64, p, p, p, i32]
        _lib.ref_set_matrix_element.restype = i32
        _lib.ref_set_matrix_element.argtypes = [i32, i32, p, p]
        _lib.ref_item_sums_learned.restype = i32
        _lib.ref_item_sums_learned.argtypes = [p, p, p, u64, u32, i32, i32, p, p, p, i32, p, C.c_int64, p, p, p,
                                               i32]
        _lib.ref_item_sums_est.restype = i32
        _lib.ref_item_sums_est.argtypes = [p, p, p, u64, u32, i32, i32, i32, C.c_int64, p, p, p, i32]
        _lib.ref_collision_points.restype = i32
        _lib.ref_collision_points.argtypes = [p, p, p, C.c_int64, p, p, i32, i32, p, i32]
        _lib.ref_drift.restype = i32
        _lib.ref_drift.argtypes = [p, p, p, i32, p]
        _lib.ref_observables.restype = i32
        _lib.ref_observables.argtypes = [p, p, p, p, p, p]
        _lib.ref_stencil.restype = i32
        _lib.ref_stencil.argtypes = [p, C.c_int64, p, p, p]
        _lib.ref_sample_uniforms.restype = None
        _lib.ref_sample_uniforms.argtypes = [u64, u32, u32, u32, u32, u32, p]
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class Grid:
    """Phase-space grid and physics switches (cell-centred momentum nodes)."""
    n_x: tuple = (1, 1, 1)
    n_p: tuple = (10, 10, 10)
    x_half: tuple = (3.0, 3.0, 3.0)
    p_half: tuple = (2.0, 2.0, 2.0)
    species_mask: int = 1 << GLUON
    row_mask: int = 0x7F
    alpha_s: float = 0.3

    @property
    def cells(self) -> int:
        return int(np.prod(self.n_x))

    @property
    def nodes(self) -> int:
        return int(np.prod(self.n_p))

    def c(self) -> _Grid:
        g = _Grid()
        g.n_x[:] = list(self.n_x)
        g.n_p[:] = list(self.n_p)
        g.x_half[:] = [float(v) for v in self.x_half]
        g.p_half[:] = [float(v) for v in self.p_half]
        g.species_mask = self.species_mask
        g.row_mask = self.row_mask
        g.alpha_s = self.alpha_s
        return g

    def momenta(self) -> np.ndarray:
        """Node momenta, shape (nodes, 3), pz fastest."""
        axes = [-ph + (np.arange(n) + 0.5) * 2 * ph / n for n, ph in zip(self.n_p, self.p_half)]
        P = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
        return P.reshape(-1, 3)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample_uniforms(seed: int, step: int, s: int, p1_lin: int, cell: int, code: int) -> np.ndarray:
    """The five unit-cube variables of one sample of the uniform sampler."""
    out = np.zeros(5)
    lib().ref_sample_uniforms(seed, step, s, p1_lin, cell, code, _ptr(out))
    return out


def msq(row: int, s: float, t: float, u: float, mg2: float, alpha_s: float) -> float:
    return lib().ref_msq(row, s, t, u, mg2, alpha_s)


def set_matrix_element(row: int, terms) -> None:
    """Replace Table I row `row` by g^4 sum_k c_k s^a t^b u^c / ((t - m_g^2)^d
    (u - m_g^2)^e s^f); terms = [(c, (a, b, c, d, e, f)), ...]; [] restores it.
    Process-wide (call with [] when done)."""
    coef = np.ascontiguousarray([t[0] for t in terms], dtype=np.float64)
    powers = np.ascontiguousarray([t[1] for t in terms], dtype=np.int32).reshape(-1, 6)
    if lib().ref_set_matrix_element(row, len(terms), _ptr(coef) if len(terms) else None,
                                    powers.ctypes.data_as(C.c_void_p) if len(terms) else None) < 0:
        raise ValueError("bad matrix element terms")


def channels(grid: Grid) -> list[dict]:
    buf = (_Channel * 128)()
    g = grid.c()
    n = lib().ref_channels(C.byref(g), buf, 128)
    if n < 0:
        raise RuntimeError("channel table overflow")
    return [dict(row=buf[i].row, sp=tuple(buf[i].sp), code=buf[i].code, w=buf[i].w,
                 sigma=buf[i].sigma) for i in range(n)]


def _field(grid: Grid, a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (7, grid.cells, grid.nodes):
        raise ValueError(f"expected f of shape {(7, grid.cells, grid.nodes)}, got {a.shape}")
    return a


def _mass(grid: Grid, m) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.float64)
    if m.shape != (7, grid.cells):
        raise ValueError(f"expected mass2 of shape {(7, grid.cells)}, got {m.shape}")
    return m


def masses(grid: Grid, f, mass2_lag=None) -> np.ndarray:
    """Eq. mg / Eq. mq; ``mass2_lag=None`` uses E = |p| (first time step)."""
    f = _field(grid, f)
    lag = None if mass2_lag is None else _mass(grid, mass2_lag)
    out = np.zeros((7, grid.cells))
    g = grid.c()
    if lib().ref_masses(C.byref(g), _ptr(f), _ptr(lag), _ptr(out)) != 0:
        raise ValueError("bad grid")
    return out


def constant_masses(grid: Grid, m2_by_species) -> np.ndarray:
    m = np.asarray(m2_by_species, dtype=np.float64).reshape(7, 1)
    return np.repeat(m, grid.cells, axis=1)


def eval_cm(grid: Grid, chan: dict, f, mass2, cell: int, p1, p2, cos_th: float, phi: float,
            flags: int = 0, eq: dict | None = None, p1_lin: int = -1) -> dict:
    """Evaluate the CM-angle parameterisation at one configuration."""
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    ch = _Channel(chan["row"], (C.c_int32 * 4)(*chan["sp"]), chan["code"], chan["w"], chan["sigma"])
    e = _make_eq(eq)
    pt = _Point()
    g = grid.c()
    a1 = np.asarray(p1, dtype=np.float64)
    a2 = np.asarray(p2, dtype=np.float64)
    lib().ref_eval_cm(C.byref(g), C.byref(ch), _ptr(f), _ptr(mass2), cell, _ptr(a1), p1_lin,
                      _ptr(a2), cos_th, phi, flags, None if e is None else C.byref(e), C.byref(pt))
    return dict(valid=bool(pt.valid), k=np.array([[pt.k[i][j] for j in range(4)] for i in range(4)]),
                s=pt.s, t=pt.t, u=pt.u, pstar=pt.pstar, msq=pt.msq, f=np.array(pt.f[:]),
                B=pt.B, GL=pt.GL, g=pt.g, gscale=pt.gscale)


def _make_eq(eq):
    if eq is None:
        return None
    e = _Eq()
    e.T = eq["T"]
    e.mu[:] = list(eq.get("mu", [0.0] * 7))
    return e


def collision(grid: Grid, f, mass2, seed: int, step: int, n_samples: int, *, estimator: str = "cm",
              symmetric: bool = True, flags: int = 0, eq: dict | None = None,
              want_scale: bool = True, want_items: bool = False, threads: int = 0):
    """Monte Carlo collision term A = N_Y C_Y with the uniform sampler.

    Returns (A, S, items): S is the gain+loss scale (or None), items the
    per-(cell, channel, p1) sums of the direct part (or None).
    """
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    A = np.zeros_like(f)
    S = np.zeros_like(f) if want_scale else None
    nch = len(channels(grid))
    items = np.zeros((grid.cells, nch, grid.nodes)) if want_items else None
    e = _make_eq(eq)
    g = grid.c()
    est = {"cm": 0, "root": 1, "root_k3": 2}[estimator]
    r = lib().ref_collision(C.byref(g), _ptr(f), _ptr(mass2), seed, step, n_samples, est,
                            int(symmetric), flags, None if e is None else C.byref(e),
                            _ptr(A), _ptr(S), _ptr(items), threads)
    if r < 0:
        raise ValueError("oracle rejected the arguments")
    return A, S, items


def collision_learned(grid: Grid, f, mass2, seed: int, step: int, n_samples: int, thr, mu, sigma, *,
                      table_per_cell: bool = False, chan_learned=None, want_scale: bool = True,
                      want_items: bool = False, threads: int = 0):
    """Collision term with the mixture proposal given as a table (see header).
    chan_learned: per-channel 0/1 (0 = that channel falls back to the uniform
    sampler), None = every channel uses the mixture."""
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    mu = np.ascontiguousarray(mu, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    K = thr.shape[-1]
    nch = len(channels(grid))
    rows = (grid.cells if table_per_cell else 1) * nch * grid.nodes
    if thr.size != rows * K or mu.size != rows * K * 5 or sigma.size != rows * K * 5:
        raise ValueError("table shape does not match the grid")
    if chan_learned is not None:
        chan_learned = np.ascontiguousarray(chan_learned, dtype=np.uint8)
        if chan_learned.size != nch:
            raise ValueError("chan_learned needs one entry per channel")
    A = np.zeros_like(f)
    S = np.zeros_like(f) if want_scale else None
    items = np.zeros((grid.cells, nch, grid.nodes)) if want_items else None
    g = grid.c()
    r = lib().ref_collision_learned(C.byref(g), _ptr(f), _ptr(mass2), seed, step, n_samples, K,
                                    _ptr(thr), _ptr(mu), _ptr(sigma), int(table_per_cell),
                                    _ptr(chan_learned), _ptr(A), _ptr(S), _ptr(items), threads)
    if r < 0:
        raise ValueError("oracle rejected the arguments")
    return A, S, items


def item_sums_learned(grid: Grid, f, mass2, seed: int, step: int, n_samples: int, thr, mu, sigma, items, *,
                      table_per_cell: bool = False, chan_learned=None, threads: int = 0,
                      want_scale: bool = False):
    """Direct sums of selected (cell, channel, node) items with the mixture
    proposal (the table as in collision_learned); with want_scale also the
    sum of the samples' gain+loss magnitudes."""
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    mu = np.ascontiguousarray(mu, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    K = thr.shape[-1]
    nch = len(channels(grid))
    rows = (grid.cells if table_per_cell else 1) * nch * grid.nodes
    if thr.size != rows * K or mu.size != rows * K * 5 or sigma.size != rows * K * 5:
        raise ValueError("table shape does not match the grid")
    if chan_learned is not None:
        chan_learned = np.ascontiguousarray(chan_learned, dtype=np.uint8)
    items = np.ascontiguousarray(items, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(len(items))
    scale = np.zeros(len(items)) if want_scale else None
    g = grid.c()
    if lib().ref_item_sums_learned(C.byref(g), _ptr(f), _ptr(mass2), seed, step, n_samples, K, _ptr(thr),
                                   _ptr(mu), _ptr(sigma), int(table_per_cell), _ptr(chan_learned),
                                   len(items), _ptr(items), _ptr(out), _ptr(scale), threads) < 0:
        raise ValueError("oracle rejected the arguments")
    return (out, scale) if want_scale else out


def item_sums(grid: Grid, f, mass2, seed: int, step: int, n_samples: int, items, *,
              symmetric: bool = True, want_scale: bool = False, threads: int = 0,
              estimator: str = "cm"):
    """Sum of the sample values of each selected (cell, channel, node) item;
    with want_scale also the sum of the samples' gain+loss magnitudes."""
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    items = np.ascontiguousarray(items, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(len(items))
    scale = np.zeros(len(items)) if want_scale else None
    g = grid.c()
    est = {"cm": 0, "root": 1, "root_k3": 2}[estimator]
    if lib().ref_item_sums_est(C.byref(g), _ptr(f), _ptr(mass2), seed, step, n_samples, est, int(symmetric),
                               len(items), _ptr(items), _ptr(out), _ptr(scale), threads) < 0:
        raise ValueError("oracle rejected the arguments")
    return (out, scale) if want_scale else out


def collision_points(grid: Grid, f, mass2, pts, wts, *, symmetric: bool = True,
                     flags: int = 0, threads: int = 0) -> np.ndarray:
    """The collision operator by quadrature over (p2, cos theta, phi) nodes."""
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 5)
    wts = np.ascontiguousarray(wts, dtype=np.float64).reshape(-1)
    if pts.shape[0] != wts.shape[0]:
        raise ValueError("points and weights differ in length")
    A = np.zeros_like(f)
    g = grid.c()
    if lib().ref_collision_points(C.byref(g), _ptr(f), _ptr(mass2), pts.shape[0], _ptr(pts),
                                  _ptr(wts), int(symmetric), flags, _ptr(A), threads) < 0:
        raise ValueError("oracle rejected the arguments")
    return A


def drift(grid: Grid, f, mass2, scheme: str = "upwind") -> np.ndarray:
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    D = np.zeros_like(f)
    g = grid.c()
    if lib().ref_drift(C.byref(g), _ptr(f), _ptr(mass2), {"upwind": 0, "central": 1}[scheme], _ptr(D)):
        raise ValueError("bad grid")
    return D


def stencil(grid: Grid, pts) -> tuple:
    """The trilinear stencil of the collision term (reading R2: per axis the
    stencil coordinate is clamped to the outermost node centres) for momenta
    pts [n, 3]: node indices [n, 8] and weights [n, 8]."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    idx = np.zeros((len(pts), 8), dtype=np.int64)
    w = np.zeros((len(pts), 8))
    g = grid.c()
    if lib().ref_stencil(C.byref(g), len(pts), _ptr(pts), _ptr(idx), _ptr(w)):
        raise ValueError("bad grid")
    return idx, w


def interpolate(grid: Grid, f_cell, pts) -> np.ndarray:
    """f of one (species, cell) row [nodes] at momenta pts [n, 3]."""
    idx, w = stencil(grid, pts)
    return (w * np.asarray(f_cell, dtype=np.float64)[idx]).sum(1)


def observables(grid: Grid, f, mass2) -> dict:
    f = _field(grid, f)
    mass2 = _mass(grid, mass2)
    N = np.zeros(7)
    E = np.zeros(7)
    P = np.zeros((7, 3))
    g = grid.c()
    lib().ref_observables(C.byref(g), _ptr(f), _ptr(mass2), _ptr(N), _ptr(E), _ptr(P))
    return dict(N=N, E=E, P=P, N_total=float(N.sum()), E_total=float(E.sum()))


def _cell_measure(grid: Grid) -> float:
    """dV_x dV_p / (2 pi)^3 of one phase-space cell."""
    dx = np.prod([2.0 * h / n for n, h in zip(grid.n_x, grid.x_half)])
    dp = np.prod([2.0 * h / n for n, h in zip(grid.n_p, grid.p_half)])
    return float(dx * dp / (2.0 * np.pi) ** 3)


def _energies(grid: Grid, mass2) -> np.ndarray:
    """E = sqrt(p^2 + m^2) on every (species, cell, node), shape (7, cells, nodes)."""
    p2 = (grid.momenta() ** 2).sum(axis=1)
    return np.sqrt(p2[None, None, :] + _mass(grid, mass2)[:, :, None])


def energy_budget(grid: Grid, f, A, mass2, mass2_prev, dt_fm: float) -> dict:
    """Energy bookkeeping of one step taken from f with masses mass2.

    Eq. current conservation gives the kinetic tensor a source S_ex^0 from the
    time dependence of the masses; over one step, at fixed f, its integral is
    the change of sum N dV E f when E = sqrt(p^2 + m^2) moves from the previous
    masses to the current ones (``E_source``; 0 without previous masses).  The
    collision term changes f by dt A / (N hbar c), i.e. the energy by
    ``E_collide`` = dt / (hbar c) sum dV E A over evolved species, which the
    paper shows is not exactly zero on a grid (Sec. IV, energy test).
    """
    f = _field(grid, f)
    A = _field(grid, A)
    meas = _cell_measure(grid)
    E = _energies(grid, mass2)
    if mass2_prev is None:
        src = 0.0
    else:
        dE = E - _energies(grid, mass2_prev)
        src = float((DEGENERACY[:, None, None] * f * dE).sum() * meas)
    evolve = np.array([(grid.species_mask >> sp) & 1 for sp in range(7)], dtype=bool)
    col = float((E * A)[evolve].sum() * meas * dt_fm / HBARC)
    return dict(E_source=src, E_collide=col)


def modified_energy(grid: Grid, f, mass2) -> float:
    """T^00 of the modified tensor of Sec. IV: T_kin^00 - 1/4 sum N dV m^2 f / E
    (a massless p = 0 node contributes nothing)."""
    f = _field(grid, f)
    m2 = _mass(grid, mass2)[:, :, None]
    E = _energies(grid, mass2)
    meas = _cell_measure(grid)
    with np.errstate(divide="ignore", invalid="ignore"):
        term = np.where(E > 0.0, m2 * f / np.where(E > 0.0, E, 1.0), 0.0)
    T = (DEGENERACY[:, None, None] * E * f).sum() * meas
    return float(T - 0.25 * (DEGENERACY[:, None, None] * term).sum() * meas)


def thermo(grid: Grid, f, mass2) -> dict:
    """Entropy and the diagonal of Eq. energy momentum tensor.

    entropy = sum N dV [(1 + s f) ln(1 + s f)/s - f ln f], s = +1 for gluons
    and -1 for quarks, over the nodes with f > 0 and 1 + s f > 0 (the others
    add nothing); T_ii = sum N dV p_i^2 f / E over nodes with E > 0.
    """
    f = _field(grid, f)
    meas = _cell_measure(grid)
    E = _energies(grid, mass2)
    S = 0.0
    for sp in range(7):
        s = 1.0 if sp == GLUON else -1.0
        fv = f[sp]
        one = 1.0 + s * fv
        ok = (fv > 0.0) & (one > 0.0)
        term = one[ok] * np.log(one[ok]) / s - fv[ok] * np.log(fv[ok])
        S += DEGENERACY[sp] * term.sum()
    P = grid.momenta()
    T = np.zeros(3)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(E > 0.0, f / np.where(E > 0.0, E, 1.0), 0.0)
        T[a] = (DEGENERACY[:, None, None] * w * (P[:, a] ** 2)[None, None, :]).sum()
    return dict(entropy=float(S * meas), T_ii=T * meas)


@dataclass
class State:
    """Evolving state of the oracle's time stepper."""
    f: np.ndarray
    step: int = 0
    mass2_lag: np.ndarray | None = None
    history: list = field(default_factory=list)


def step(grid: Grid, state: State, dt_fm: float, n_samples: int, seed: int, *,
         scheme: str = "upwind", symmetric: bool = True, const_mass2=None,
         threads: int = 0) -> dict:
    """One forward-Euler step f <- f + dt (A/(N_Y hbar c) - D[f]) (Sec. III)."""
    if const_mass2 is not None:
        m2 = constant_masses(grid, const_mass2)
    else:
        m2 = masses(grid, state.f, state.mass2_lag)
    A, _, _ = collision(grid, state.f, m2, seed, state.step, n_samples, symmetric=symmetric,
                        want_scale=False, threads=threads)
    budget = energy_budget(grid, state.f, A, m2, state.mass2_lag, dt_fm)
    D = drift(grid, state.f, m2, scheme)
    evolve = np.array([(grid.species_mask >> sp) & 1 for sp in range(7)], dtype=bool)
    upd = dt_fm * (A / (DEGENERACY[:, None, None] * HBARC) - D)
    upd[~evolve] = 0.0
    state.f = state.f + upd
    state.mass2_lag = m2
    state.step += 1
    obs = observables(grid, state.f, m2)
    obs["mass2"] = m2
    obs.update(budget)
    obs["E_total_mod"] = modified_energy(grid, state.f, m2)
    obs.update(thermo(grid, state.f, m2))
    state.history.append(obs)
    return obs
