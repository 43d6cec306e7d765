#!/usr/bin/env python3
"""Benchmark of the Monte Carlo collision-term step on one MI355X.

A step is one pass of the whole hot path over the workload: thermal masses,
the collision term with symmetric sampling, the drift + forward-Euler update,
and the FP64 bookkeeping.  The default workload is the pure-gluon spatial run:
16 x 16 x 1 cells, 20^3 momentum nodes on [-3,3]^3 GeV, 2048 samples per
(cell, node), FP32 integrand with FP64 geometry and accumulation, upwind drift,
dt = 0.01 fm/c.  Inputs are synthetic (a Gaussian transverse profile of a
step-function gluon distribution) and resident in HBM when timing starts.

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1912_04457_amd import qgbe  # noqa: E402
from paper_1912_04457_amd import workloads as W  # noqa: E402

METRIC = "collision integrand evals/s + time/step at fixed MC error, plain vs learned"

# Algorithmic VALU work per evaluation, in lane-issue slots (full-rate op = 1,
# quarter-rate transcendental or 32-bit integer product = 4):
#   Philox4x32-10 block 120 (10 rounds x (2 products x 4 + 4 xor)),
#   five 23-bit uniforms 20, FP64 sample geometry up to the box cut 130
#   (4 square roots, 3 reciprocals, sin/cos, two boosts, the frame), then for
#   accepted samples: t and u 16, |M|^2 27 (3 reciprocals), three trilinear
#   interpolations 123, bracket and value 17, three trilinear deposits 66.
SLOTS_REJECTED = 120 + 20 + 130
SLOTS_ACCEPTED = SLOTS_REJECTED + 16 + 27 + 123 + 17 + 66
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = one full-rate lane op per slot
ALU_PEAK_SLOTS = 256 * 64 * 2.4e9
# LDS: 128 B/clk/CU -> 32 four-byte lane accesses per clock per CU
LDS_PEAK = 256 * 32 * 2.4e9
LDS_PER_ACCEPTED = 24 + 24     # 3 x 8 gathers, 3 x 8 atomic adds


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=W.C2.name, choices=sorted(W.WORKLOADS))
    ap.add_argument("--samples", type=int, default=0, help="override samples per point")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB before timing (counter calibration)")
    return ap.parse_args()


def cpu_baseline(wl, f, n_samples, budget_s):
    """The FP64 oracle on the first cells of the same workload (collision term)."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    total_evals, total_t, cells_done = 0.0, 0.0, 0
    nch = len(O.channels(O.Grid(species_mask=wl.species_mask)))
    k = 1
    while cells_done < wl.cells:
        k = min(k, wl.cells - cells_done)
        g = O.Grid(n_x=(k, 1, 1), n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                   species_mask=wl.species_mask, alpha_s=wl.alpha_s)
        fs = np.ascontiguousarray(f[:, cells_done:cells_done + k])
        t0 = time.perf_counter()
        m = O.masses(g, fs)
        O.collision(g, fs, m, W.PHILOX_SEED, 0, n_samples, want_scale=False, threads=threads)
        dt = time.perf_counter() - t0
        total_t += dt
        total_evals += k * nch * wl.nodes * n_samples
        cells_done += k
        if total_t >= budget_s:
            break
        per_cell = total_t / cells_done
        k = max(1, int((budget_s - total_t) / per_cell))
    return dict(value=total_evals / total_t, unit="evals/s", cores=threads, kind="oracle",
                sample=f"collision term of {cells_done} of {wl.cells} cells x {wl.nodes} nodes x "
                       f"{nch} channel(s) x {n_samples} samples ({total_evals:.3g} evals, "
                       f"{total_t:.1f} s, FP64, OpenMP)")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if a.copy_mib:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the byte counts read for the collision kernel
        src = torch.ones(a.copy_mib * 2**18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = W.WORKLOADS[a.workload]
    N = a.samples or wl.n_samples
    f0 = W.initial_f(wl)
    prec = qgbe.FP64 if wl.precision == "f64" else qgbe.FP32
    drift = qgbe.DRIFT_UPWIND if wl.drift == "upwind" else qgbe.DRIFT_CENTRAL
    solver = qgbe.Solver(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                         species_mask=wl.species_mask, alpha_s=wl.alpha_s, precision=prec,
                         drift=drift, seed=W.PHILOX_SEED, device=0)
    solver.set_f(f0)
    if a.warmup:
        solver.step(wl.dt_fm, N, n_steps=a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = solver.step(wl.dt_fm, N, n_steps=a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solver.close()

    evals = sum(s["n_evals"] for s in stats)
    accepted = sum(s["n_accepted"] for s in stats)
    t_coll = np.array([s["t_collide_ms"] for s in stats]) * 1e-3
    value = evals / elapsed
    slots = SLOTS_ACCEPTED * accepted + SLOTS_REJECTED * (evals - accepted)
    achieved = slots / t_coll.sum()
    roof = dict(bound="alu", achieved=achieved, peak=ALU_PEAK_SLOTS, unit="lane-op slots/s",
                frac=achieved / ALU_PEAK_SLOTS, traffic=None,
                kernel="collide_f32_kernel" if prec == qgbe.FP32 else "collide_f64_kernel",
                kernel_ms_avg=float(t_coll.mean() * 1e3),
                lds_frac=(LDS_PER_ACCEPTED * accepted / t_coll.sum()) / LDS_PEAK)
    N0 = stats[0]["N_total"]
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == qgbe.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": wl.cells, "momentum_nodes": wl.nodes,
                   "species_mask": wl.species_mask, "channels": solver.n_channels,
                   "samples_per_point": N, "sampler": "uniform", "symmetric": True,
                   "precision": "fp32 integrand, fp64 geometry + accumulation" if prec == qgbe.FP32
                   else "fp64", "drift": wl.drift, "dt_fm": wl.dt_fm},
        "roofline": roof,
        "accepted_fraction": accepted / evals,
        "collide_ms_per_step": float(t_coll.mean() * 1e3),
        "N_total_rel_drift": abs(stats[-1]["N_total"] - N0) / N0,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, f0, N, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
