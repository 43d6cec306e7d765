"""Long runs of the collision path toward equilibrium (Sec. IV C and D).

One homogeneous cell of pure gluons, pure quarks (u and ubar) or the
quark-gluon mixture, started from the step occupation of Eq. CGC,
f0 theta(Qs - |p|_xi) with |p|_xi^2 = px^2 + py^2 + (xi pz)^2 (xi = 1 is the
paper's isotropic step; xi > 1 squeezes it along z), and evolved with
``qgbe_step`` (dynamic thermal masses, symmetric sampling).  Every ``every``
steps a record is taken from the step's own statistics: particle number and
energy (conserved by the collision term up to the grid's energy residue), the
entropy (non-decreasing), the pressure ratio T_zz / T_xx (-> 1 as the system
isotropises), the thermal masses, the energy budget of the step, and the
occupation of the softest nodes (the soft-gluon accumulation the paper
reports for overpopulated initial states).

    python -m paper_1912_04457_amd.thermalize --kind gluon --steps 2000 --every 100

prints one JSON object per record.  Everything that evolves runs in the
library's kernels; the host only reads back the statistics and, for the
soft-node occupation, the few values of f at the nodes nearest p = 0.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import qgbe
from . import workloads as W

KINDS = {"gluon": 1 << W.GLUON, "quark": (1 << 0) | (1 << 3), "u": 1 << 0, "mixture": W.ALL_SPECIES,
         "mixture_g": W.ALL_SPECIES}
# Species that start from the step; the others start empty.  "u" is the
# paper's pure-quark system (u quarks only, Sec. IV D); "mixture_g" its
# quark-gluon run, all species evolving from gluons alone (Sec. IV E).
STARTS = {"mixture_g": 1 << W.GLUON}


def initial_step(n_p, p_half, mask: int, f0: float, Qs: float, xi: float = 1.0) -> np.ndarray:
    """f0 theta(Qs - |p|_xi) for every evolving species, shape (7, 1, nodes)."""
    P = W.node_momenta(n_p, p_half)
    r = np.sqrt(P[:, 0] ** 2 + P[:, 1] ** 2 + (xi * P[:, 2]) ** 2)
    f = np.zeros((7, 1, len(P)))
    for sp in range(7):
        if (mask >> sp) & 1:
            f[sp, 0] = f0 * (r < Qs)
    return f


def soft_nodes(n_p, p_half, k: int = 8) -> np.ndarray:
    """Indices of the k nodes nearest p = 0."""
    P = W.node_momenta(n_p, p_half)
    return np.argsort((P ** 2).sum(1), kind="stable")[:k]


def evolve(kind: str = "gluon", n_p=(20, 20, 20), p_half=(2.0, 2.0, 2.0), f0: float = 0.5, Qs: float = 1.5,
           xi: float = 1.0, alpha_s: float = 0.3, dt_fm: float = 0.005, steps: int = 1000, every: int = 100,
           samples: int = 256, precision: int = qgbe.FP32, seed: int = W.PHILOX_SEED, device: int = 0,
           const_mass2=None):
    """Evolve, yielding a record (dict) every ``every`` steps as it is taken.
    const_mass2: None for the dynamic masses of Eq. mg / mq, else the 7
    constant squared masses (GeV^2) of the energy test of Sec. IV."""
    if steps < 1 or every < 1:
        raise ValueError("steps and every must be >= 1")
    mask = KINDS[kind]
    f = initial_step(n_p, p_half, STARTS.get(kind, mask), f0, Qs, xi)
    soft = soft_nodes(n_p, p_half)
    masses = {} if const_mass2 is None else dict(mass_mode=qgbe.MASS_CONSTANT, const_mass2=tuple(const_mass2))
    with qgbe.Solver(n_x=(1, 1, 1), n_p=tuple(n_p), p_half=tuple(p_half), species_mask=mask, alpha_s=alpha_s,
                     precision=precision, seed=seed, device=device, **masses) as s:
        s.set_f(f)
        def record(done, st):
            fs = s.get_f()[:, 0, soft]
            T = st["T_ii"]
            return dict(
                step=done, t_fm=done * dt_fm, N_total=st["N_total"], E_total=st["E_total"],
                E_total_mod=st["E_total_mod"], entropy=st["entropy"], Tzz_over_Txx=T[2] / T[0] if T[0] else None,
                mass2_g=st["mass2_avg"][W.GLUON], mass2_q=st["mass2_avg"][0], E_source=st["E_source"],
                E_collide=st["E_collide"], min_f=st["min_f"], f_soft_g=float(fs[W.GLUON].mean()),
                f_soft_q=float(fs[0].mean()), flags=st["flags"], t_step_ms=st["t_step_ms"])

        yield record(0, s.observables())   # the initial state (masses with E = |p|)
        done = 0
        while done < steps:
            k = min(every, steps - done)
            st = s.step(dt_fm, samples, n_steps=k, last_only=True)[0]
            done += k
            yield record(done, st)


def run(*args, **kw) -> list:
    """evolve() collected into a list."""
    return list(evolve(*args, **kw))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kind", choices=sorted(KINDS), default="gluon")
    ap.add_argument("--n", type=int, default=20, help="momentum nodes per axis")
    ap.add_argument("--p-half", type=float, default=2.0, help="momentum box half-width, GeV")
    ap.add_argument("--f0", type=float, default=0.5)
    ap.add_argument("--qs", type=float, default=1.5, help="saturation scale Qs, GeV")
    ap.add_argument("--xi", type=float, default=1.0, help="anisotropy of the initial step")
    ap.add_argument("--alpha-s", type=float, default=0.3)
    ap.add_argument("--dt", type=float, default=0.005, help="time step, fm/c")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--samples", type=int, default=256, help="samples per (channel, node)")
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--const-mg2", type=float, default=None,
                    help="constant gluon mass^2 (GeV^2; quarks get a third of it) instead of Eq. mg / mq")
    a = ap.parse_args(argv)
    cm = None if a.const_mg2 is None else (a.const_mg2 / 3.0,) * 6 + (a.const_mg2,)
    for rec in evolve(a.kind, (a.n,) * 3, (a.p_half,) * 3, a.f0, a.qs, a.xi, a.alpha_s, a.dt, a.steps, a.every,
                      a.samples, qgbe.FP64 if a.fp64 else qgbe.FP32, const_mass2=cm):
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
