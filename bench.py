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

# Algorithmic work per evaluation in lane-op issue slots.  The floating-point
# part is the oracle's per-sample arithmetic as its op-count build counts it
# (oracle/opcount.cpp: the operations that depend on the sample, each distinct
# operation once per sample, a multiplication whose only use is an addition
# fused with it), weighted by issue cost on gfx950: 1 for add, mul, fma,
# compare and conversion, 4 for a division by a sample-dependent value, a
# square root and exp/log/sin/cos (one quarter-rate hardware instruction).
# The integer part follows the definitions: a Philox4x32-10 block is ten rounds
# of two 32x32->64 products and four xors, 60 slots (the product instruction
# issues at full rate, measured); five 23-bit uniforms from a block 27 (12
# shifts, masks and ors, 5 conversions, 5 additions, 5 scalings).
# tests/test_opcount.py checks these figures against the op-count build.
PHILOX_BLOCK = 60
UNIFORMS_FROM_BLOCK = 27
FP_OUTSIDE_BOX = 179.0      # uniform sampler, sample rejected by the box cut
FP_ACCEPTED = 388.7         # accepted, symmetric deposits
FP_DEPOSITS = 21.2          # of which the three symmetric deposits (direct estimator: without)
FP_MIXTURE = 519.0          # mixture draw (three Box-Muller pairs, five logistic maps) and density
MIXTURE_INT = 24 + 14       # six more 23-bit uniforms; the component choice (7 compares, 7 selects)
FP_ROOTS_SAMPLE = 47.3      # root parameterisation: the quadratic and its two candidates
FP_ROOTS_PER_ROOT = 180.3   # per valid root (direct); with symmetric deposits FP_DEPOSITS more
SLOTS_REJECTED = PHILOX_BLOCK + UNIFORMS_FROM_BLOCK + FP_OUTSIDE_BOX
SLOTS_ACCEPTED = PHILOX_BLOCK + UNIFORMS_FROM_BLOCK + FP_ACCEPTED
SLOTS_DEPOSITS = FP_DEPOSITS
# the learned sampler: a second Philox block and the mixture draw and density
# in place of the five uniforms of the plain map
SLOTS_LEARNED_EXTRA = PHILOX_BLOCK + MIXTURE_INT + FP_MIXTURE - UNIFORMS_FROM_BLOCK
SLOTS_ROOTS_SAMPLE = PHILOX_BLOCK + UNIFORMS_FROM_BLOCK + FP_ROOTS_SAMPLE
SLOTS_ROOTS_ACCEPTED = FP_ROOTS_PER_ROOT
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = one full-rate lane op per slot
ALU_PEAK_SLOTS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12               # bytes/s
# Timed steps by default: about a minute of the GPU for the 7-species spatial
# workload (its 50-step run is reported separately), the configured count for
# the others.
DEFAULT_STEPS = {W.C5.name: 8}


# HBM traffic of the collision kernel from rocprofv3 counters, one summary per
# workload, valid only for the kernel sources it was measured on (see
# kernel_sources_digest).
def traffic_profile(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"collide_f32_{workload}_hbm_counters.md")


KERNEL_SOURCES = ("collide.hip", "collide.h", "qgbe_common.h", "api.hip")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_04457_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed counter summary, or None when
    the summary is for another workload or for other kernel sources."""
    try:
        text = open(traffic_profile(workload)).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("sources_sha256:", "workload:",
                                                                                          "hbm_bytes_per_launch:")))
    if fields.get("workload", "").strip() != workload:
        return None
    if fields.get("sources_sha256", "").strip() != kernel_sources_digest():
        return None
    return float(fields["hbm_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0: the workload's default)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=W.C5.name, choices=sorted(W.WORKLOADS))
    ap.add_argument("--samples", type=int, default=0, help="override samples per point")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB before timing (counter calibration)")
    ap.add_argument("--no-sub", action="store_true", help="skip the pure-gluon spatial sub-record")
    ap.add_argument("--progress", action="store_true", help="print a line per timed step on stderr")
    ap.add_argument("--save-proposal", default="", help="learned sampler: save the trained table (.npz)")
    ap.add_argument("--load-proposal", default="",
                    help="learned sampler: install a table saved by --save-proposal instead of training")
    ap.add_argument("--no-compare", action="store_true",
                    help="learned sampler: skip the learned and plain terms after the timed steps")
    ap.add_argument("--no-fixed-error", action="store_true",
                    help="skip the plain-vs-learned time per step at fixed MC error")
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--train-epochs", type=int, default=4)
    return ap.parse_args()


def mc_error(reps):
    """Relative MC error of replicated collision terms: sqrt(mean Var) / rms(mean)."""
    reps = np.asarray(reps)
    mean = reps.mean(0)
    var = reps.var(0, ddof=1)
    return float(np.sqrt(var.mean()) / np.sqrt((mean ** 2).mean()))


def train_proposal(solver, wl, epochs, target_rows=1_000_000):
    """Record ~10^6 uniform samples of the workload itself (every k-th work
    item), train the network on the GPU, run the fallback judge; the table
    then follows the masses at every learned step."""
    import torch
    items = wl.cells * solver.n_channels * wl.nodes
    per_item = max(1, -(-target_rows // items))
    stride = max(1, items * per_item // target_rows)
    n_sel = -(-items // stride)
    rows = torch.empty((n_sel * per_item, qgbe.RECORD_WIDTH), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_rows = qgbe.qgbe_record_samples(solver.ctx, per_item, stride, rows)
    qgbe.qgbe_proposal_set_weights(solver.ctx, W.random_mlp_params(1))
    cfg = qgbe.TrainCfg(epochs=epochs, batch=4096, lr=2e-3, lr_final=1e-4, alpha=0.1, seed=1)
    losses = np.zeros(epochs)
    qgbe.qgbe_train_proposal(solver.ctx, rows, cfg, losses)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del rows
    flags, _ = qgbe.qgbe_proposal_judge(solver.ctx, 32, 1, solver.n_channels)
    return dict(train_rows=n_rows, train_epochs=epochs, train_s=train_s, train_loss_last=float(losses[-1]),
                learned_channels=int(flags.sum()), channels=solver.n_channels)


def save_proposal(solver, wl, path):
    """The proposal table and per-channel sampler flags as an .npz file."""
    rows = solver.n_channels * wl.nodes
    thr, mu, sg = qgbe.qgbe_get_proposal_table(solver.ctx, rows)
    samplers = qgbe.qgbe_get_channel_samplers(solver.ctx, solver.n_channels)
    np.savez(path, thr=thr, mu=mu, sigma=sg, samplers=samplers)


def load_proposal(solver, wl, path):
    """Install a table saved by save_proposal (no recording, training or judge)."""
    z = np.load(path)
    rows = solver.n_channels * wl.nodes
    if z["thr"].shape[0] != rows or z["samplers"].shape != (solver.n_channels,):
        raise ValueError(f"{path}: table for another grid ({z['thr'].shape[0]} rows, {rows} expected)")
    qgbe.qgbe_set_proposal_table(solver.ctx, z["thr"], z["mu"], z["sigma"])
    qgbe.qgbe_set_channel_samplers(solver.ctx, z["samplers"])
    return dict(loaded=os.path.basename(path), learned_channels=int(z["samplers"].sum()), channels=solver.n_channels)


def fixed_error(R, epochs):
    """Time per step of the 7-species homogeneous workload (20^3 nodes, 70
    channels) with the plain symmetric sampler at 4096 samples per point,
    against the learned proposal at the smallest sample count whose MC error
    is no larger.  The network is trained on the GPU on ~10^6 integrand
    samples of the plain sampler; its time is reported separately.  The
    learned step includes the network evaluation that rebuilds the proposal
    table from the step's masses."""
    wl = W.C3
    n_plain = wl.n_samples
    f0 = W.initial_f(wl)
    out = {"workload": wl.name, "replicas": R, "samples_plain": n_plain}
    solver = qgbe.Solver(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                         species_mask=wl.species_mask, alpha_s=wl.alpha_s, precision=qgbe.FP32,
                         drift=qgbe.DRIFT_UPWIND, seed=W.PHILOX_SEED, device=0)
    with solver:
        solver.set_f(f0)

        def replicas(n, sampler):
            reps = []
            for r in range(R):
                qgbe.qgbe_set_step_index(solver.ctx, 1000 + r)
                reps.append(solver.collision(n, sampler=sampler)[0])
            return reps

        def step_ms(n, sampler, steps=5):
            solver.set_f(f0)
            qgbe.qgbe_set_step_index(solver.ctx, 0)
            st = solver.step(wl.dt_fm, n, n_steps=steps + 1, sampler=sampler)
            return float(np.median([s["t_step_ms"] for s in st[1:]])), float(
                np.median([s["t_collide_ms"] for s in st[1:]]))

        reps_plain = replicas(n_plain, qgbe.SAMPLER_UNIFORM)
        eps_plain = mc_error(reps_plain)
        mean_plain = np.mean(reps_plain, axis=0)
        del reps_plain
        t_plain, c_plain = step_ms(n_plain, qgbe.SAMPLER_UNIFORM)
        out.update(eps_plain=eps_plain, t_step_plain_ms=t_plain, t_collide_plain_ms=c_plain)

        # training data: 2 uniform samples per (channel, node), ~1.1e6 rows
        solver.set_f(f0)
        items = wl.cells * solver.n_channels * wl.nodes
        per_item = max(1, -(-1_000_000 // items))
        import torch
        rows = torch.empty((items * per_item, qgbe.RECORD_WIDTH), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_rows = qgbe.qgbe_record_samples(solver.ctx, per_item, 1, rows)
        qgbe.qgbe_proposal_set_weights(solver.ctx, W.random_mlp_params(1))
        cfg = qgbe.TrainCfg(epochs=epochs, batch=4096, lr=2e-3, lr_final=1e-4, alpha=0.1, seed=1)
        losses = np.zeros(epochs)
        qgbe.qgbe_train_proposal(solver.ctx, rows, cfg, losses)
        torch.cuda.synchronize()
        out.update(train_rows=n_rows, train_epochs=epochs, train_s=time.perf_counter() - t0,
                   train_loss_first=float(losses[0]), train_loss_last=float(losses[-1]))
        del rows
        # fallback judge: channels whose pilot variance x time is not lower
        # with the learned sampler go back to the uniform one
        t0 = time.perf_counter()
        flags, _ = qgbe.qgbe_proposal_judge(solver.ctx, 256, 4, solver.n_channels)
        out.update(judge_s=time.perf_counter() - t0, learned_channels=int(flags.sum()),
                   channels=solver.n_channels)

        cache, means = {}, {}

        def eps_learned(n):
            if n not in cache:
                reps = replicas(n, qgbe.SAMPLER_LEARNED)
                cache[n] = mc_error(reps)
                means[n] = np.mean(reps, axis=0)
            return cache[n]

        # smallest power of two in [64, n_plain] reaching the plain error, then bisect
        hi = 64
        while hi < n_plain and eps_learned(hi) > eps_plain:
            hi *= 2
        if eps_learned(hi) > eps_plain:
            out.update(samples_learned=None, eps_learned=eps_learned(hi),
                       note="learned proposal did not reach the plain MC error at the plain sample count")
            return out
        lo = hi // 2 if hi > 64 else hi
        while hi - lo > max(8, lo // 16):
            mid = (lo + hi) // 2
            if eps_learned(mid) <= eps_plain:
                hi = mid
            else:
                lo = mid
        n_learned = hi
        t_learned, c_learned = step_ms(n_learned, qgbe.SAMPLER_LEARNED)
        out.update(samples_learned=n_learned, eps_learned=eps_learned(n_learned),
                   t_step_learned_ms=t_learned, t_collide_learned_ms=c_learned,
                   time_ratio=t_plain / t_learned,
                   bisection={str(k): v for k, v in sorted(cache.items())})
        # bias check: both replica means against a plain reference of 16 x 65536 samples
        solver.set_f(f0)
        ref_reps = []
        for r in range(16):
            qgbe.qgbe_set_step_index(solver.ctx, 5000 + r)
            ref_reps.append(solver.collision(16 * n_plain)[0])
        ref = np.mean(ref_reps, axis=0)
        eps_ref = mc_error(ref_reps) / np.sqrt(16)
        norm = np.linalg.norm(ref)
        out["bias_check"] = dict(
            reference="16 plain replicas x 65536 samples/point",
            rel_l2_learned=float(np.linalg.norm(means[n_learned] - ref) / norm),
            rel_l2_plain=float(np.linalg.norm(mean_plain - ref) / norm),
            expected_learned=float(np.hypot(eps_learned(n_learned) / np.sqrt(R), eps_ref)),
            expected_plain=float(np.hypot(eps_plain / np.sqrt(R), eps_ref)))
    return out


def cpu_baseline(wl, f, n_samples, budget_s, table=None):
    """The FP64 oracle on the first cells of the same workload (collision term,
    the same sampler: for the learned one, the proposal table and per-channel
    sampler choice the GPU's timed steps started from)."""
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
        if table is not None:
            thr, mu, sg, flags = table
            O.collision_learned(g, fs, m, W.PHILOX_SEED, 0, n_samples, thr, mu, sg, chan_learned=flags,
                                want_scale=False, threads=threads)
        else:
            O.collision(g, fs, m, W.PHILOX_SEED, 0, n_samples, want_scale=False, threads=threads,
                        estimator={"roots": "root", "roots_alt": "root_k3"}.get(wl.sampler, "cm"),
                        symmetric=wl.symmetric)
        dt = time.perf_counter() - t0
        total_t += dt
        total_evals += k * nch * wl.nodes * n_samples
        cells_done += k
        if total_t >= budget_s:
            break
        per_cell = total_t / cells_done
        k = max(1, int((budget_s - total_t) / per_cell))
    return dict(value=total_evals / total_t, unit="evals/s", cores=threads, kind="oracle",
                sample=f"collision term ({wl.sampler} sampler) of {cells_done} of {wl.cells} cells x "
                       f"{wl.nodes} nodes x {nch} channel(s) x {n_samples} samples ({total_evals:.3g} evals, "
                       f"{total_t:.1f} s, FP64, OpenMP)")


def run_workload(wl, N, steps, warmup, train_epochs, progress=False, proposal_in=None, proposal_out=None,
                 compare=True):
    """Time `steps` steps of a workload after `warmup` untimed ones; the learned
    sampler is trained first (outside the timed region), or its table loaded
    from proposal_in.  Returns the fields of a bench record and the solver's
    proposal table (learned runs) for the CPU baseline."""
    import torch
    f0 = W.initial_f(wl)
    prec = qgbe.FP64 if wl.precision == "f64" else qgbe.FP32
    drift = qgbe.DRIFT_UPWIND if wl.drift == "upwind" else qgbe.DRIFT_CENTRAL
    solver = qgbe.Solver(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                         species_mask=wl.species_mask, alpha_s=wl.alpha_s, precision=prec,
                         drift=drift, seed=W.PHILOX_SEED, device=0, symmetric=int(wl.symmetric))
    solver.set_f(f0)
    sampler = {"uniform": qgbe.SAMPLER_UNIFORM, "learned": qgbe.SAMPLER_LEARNED, "roots": qgbe.SAMPLER_ROOTS,
               "roots_alt": qgbe.SAMPLER_ROOTS_ALT}[wl.sampler]
    roots = sampler in (qgbe.SAMPLER_ROOTS, qgbe.SAMPLER_ROOTS_ALT)
    prep, table = None, None
    if sampler == qgbe.SAMPLER_LEARNED:
        prep = load_proposal(solver, wl, proposal_in) if proposal_in else train_proposal(solver, wl, train_epochs)
        if proposal_out:
            save_proposal(solver, wl, proposal_out)
    if warmup:
        solver.step(wl.dt_fm, N, n_steps=warmup, sampler=sampler)
    if sampler == qgbe.SAMPLER_LEARNED:   # the table the timed steps start from (CPU baseline input)
        rows = solver.n_channels * wl.nodes
        table = qgbe.qgbe_get_proposal_table(solver.ctx, rows) + (
            qgbe.qgbe_get_channel_samplers(solver.ctx, solver.n_channels),)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if progress:   # one call per step, a line per step on stderr (long runs)
        stats = []
        for k in range(steps):
            stats += solver.step(wl.dt_fm, N, n_steps=1, sampler=sampler)
            print(f"step {k + 1}/{steps}: {stats[-1]['t_step_ms']:.1f} ms, N {stats[-1]['N_total']:.15g}",
                  file=sys.stderr, flush=True)
    else:
        stats = solver.step(wl.dt_fm, N, n_steps=steps, sampler=sampler)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    want_compare, compare = compare, None
    if sampler == qgbe.SAMPLER_LEARNED and want_compare:
        # after the timed steps, on the same f: one learned and one plain collision
        # term with the same samples per point (the learned one from the proposal
        # table shared by all cells): estimated MC error and kernel time of each
        compare = {}
        for name, smp in (("learned", qgbe.SAMPLER_LEARNED), ("plain", qgbe.SAMPLER_UNIFORM)):
            st = solver.collision(N, sampler=smp)[3]
            compare[name] = dict(mc_err_est=st.mc_err_est, t_collide_ms=st.t_collide_ms)
        compare["error_ratio_plain_over_learned"] = compare["plain"]["mc_err_est"] / compare["learned"]["mc_err_est"]
        compare["variance_time_gain"] = (compare["plain"]["mc_err_est"] ** 2 * compare["plain"]["t_collide_ms"]) / (
            compare["learned"]["mc_err_est"] ** 2 * compare["learned"]["t_collide_ms"])
    solver.close()

    evals = sum(s["n_evals"] for s in stats)
    accepted = sum(s["n_accepted"] for s in stats)
    t_coll = np.array([s["t_collide_ms"] for s in stats]) * 1e-3
    if roots:   # accepted counts the roots that passed
        slots = SLOTS_ROOTS_SAMPLE * evals + (SLOTS_ROOTS_ACCEPTED + SLOTS_DEPOSITS * wl.symmetric) * accepted
    else:
        slots = SLOTS_ACCEPTED * accepted + SLOTS_REJECTED * (evals - accepted)
        if not wl.symmetric:
            slots -= SLOTS_DEPOSITS * accepted
    if sampler == qgbe.SAMPLER_LEARNED:
        slots += SLOTS_LEARNED_EXTRA * evals
    # work over time of all collision launches of the timed steps: the average
    # launch's work over its average duration
    launches = sum(s["n_collide_launches"] for s in stats)
    achieved = slots / t_coll.sum()
    traffic = measured_traffic(wl.name) if N == wl.n_samples else None
    roof = dict(bound="alu", achieved=achieved, peak=ALU_PEAK_SLOTS, unit="lane-op slots/s",
                frac=achieved / ALU_PEAK_SLOTS,
                traffic=traffic,
                kernel="collide_roots_kernel" if roots else
                ("collide_f32_kernel" if prec == qgbe.FP32 else "collide_f64_kernel"),
                kernel_ms_avg=float(t_coll.sum() * 1e3 / launches),
                launches_per_step=launches / len(stats),
                hbm_frac=None if traffic is None else traffic * launches / float(t_coll.sum()) / HBM_PEAK)
    N0, E0 = stats[0]["N_total"], stats[0]["E_total"]
    rec = {
        "value": evals / elapsed, "steps": steps, "warmup": warmup, "ms_per_step": elapsed / steps * 1e3,
        "dtype": "f32" if prec == qgbe.FP32 else "f64",
        "config": {"workload": wl.name, "cells": wl.cells, "momentum_nodes": wl.nodes,
                   "species_mask": wl.species_mask, "channels": solver.n_channels,
                   "samples_per_point": N, "sampler": wl.sampler, "symmetric": wl.symmetric,
                   "precision": "fp32 integrand, fp64 geometry + accumulation" if prec == qgbe.FP32
                   else "fp64", "drift": wl.drift, "dt_fm": wl.dt_fm},
        "roofline": roof,
        "accepted_fraction": accepted / evals,
        "collide_ms_per_step": float(t_coll.mean() * 1e3),
        # particle number over the timed steps (symmetric sampling and the flux-form drift
        # conserve it to rounding); the kinetic energy changes with the dynamic masses
        "N_total_rel_drift": abs(stats[-1]["N_total"] - N0) / N0,
        "E_total_rel_change": (stats[-1]["E_total"] - E0) / E0,
        "mc_err_est": float(np.mean([s["mc_err_est"] for s in stats])),
    }
    if prep is not None:
        rec["proposal"] = prep
    if compare is not None:
        rec["learned_vs_plain_same_samples"] = compare
    return rec, f0, table


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
    steps = a.steps or DEFAULT_STEPS.get(wl.name, wl.steps)
    rec, f0, table = run_workload(wl, N, steps, a.warmup, a.train_epochs, a.progress,
                                  proposal_in=a.load_proposal or None, proposal_out=a.save_proposal or None,
                                  compare=not a.no_compare)
    out = {"metric": METRIC, "value": rec.pop("value"), "unit": "evals/s", "n_gpus": 1,
           "steps": rec.pop("steps"), "warmup": rec.pop("warmup"), "ms_per_step": rec.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": rec.pop("dtype"),
           "data": "synthetic"}
    out.update(rec)
    if not a.no_sub:
        # the pure-gluon spatial workload as a sub-record (its own steps)
        sub, _, _ = run_workload(W.C2, W.C2.n_samples, W.C2.steps, 2, a.train_epochs)
        out["sub_records"] = {W.C2.name: sub}
    if not a.no_fixed_error:
        out["fixed_mc_error"] = fixed_error(a.replicas, a.train_epochs)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, f0, N, a.cpu_seconds, table)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
