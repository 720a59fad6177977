"""Benchmark of the VESIS hot path on one MI355X.

One step = one pass of the whole hot path over the two-globule workload
(two seeded 5,000-atom globules 1.5 nm apart, 256^3 cells of 0.05 nm):
reset positions (device copy), tight initial labels, energy density on every
cell and on the far-field nodes, colour-sweep interface minimisation to
equilibrium, energy, forces, one adaptive-mobility atom step (which itself
re-evaluates the density of each trial; the mobility state carries over
between steps as between iterations of the algorithm).  After the timed
steps, the full alternation runs for --relax-iters outer iterations and is
reported under "relax", and 64 molecules are brought to equilibrium one at a
time and batched, reported under "batch"; the warm-start network is trained
on relaxed molecules and compared with the tight start on held-out ones,
reported under "learned".  All inputs are
resident in device memory before the timed region.

Prints one JSON line.  `value` is atom-gridpoint pairs of one configuration
(N n^3) per second of step time; `ms_per_step` is the step time.  The
roofline object reports the density kernel (the dominant kernel) against
the FP32 vector peak, timed with HIP events on the library's stream; the
cpu_baseline object times the FP64 oracle's density on a bounded sample of
the same grid on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-equilibrium & atom·gridpt/s at 256³; learned-init+batched vs plain"
FP32_PEAK_TFLOPS = 157.3
FLOP_PER_PAIR = 24.0  # 3 sub, r^2 (mul + 2 fma), 1/r^2, 1/r^3, s, s^3 (2), LJ (fma, fma), Q/r^3, E (3 fma)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str = "density_grid_f32"):
    """HBM bytes per launch of the density kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy
    calibration), or None when the kernel source has changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_two_globules_256.md")
    src = os.path.join(ROOT, "paper_2208_05524_amd", "csrc", "density.hip")
    try:
        lines = open(path).read().splitlines()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) > 2 and f[0] == "traffic" and f[1] == kernel:
            kv = dict(x.split("=", 1) for x in f[2:])
            if kv.get("source_sha256") != sha:
                return None
            return float(kv["bytes_per_launch"])
    return None


def measured_flip_traffic(colour_variant: int = 0):
    """HBM traffic of the batched colour-pass launch of the given colour-pass
    variant on the 64-molecule workload, from the committed PMC summary: the
    kernel, bytes per dispatch, average dispatch time and their ratio against
    8 TB/s, or None when the colour-pass source has changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_batch64_flip.md")
    src = os.path.join(ROOT, "paper_2208_05524_amd", "csrc", "labels.hip")
    try:
        lines = open(path).read().splitlines()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) > 2 and f[0] == "traffic" and f[1] == "flip_pass_batch":
            kv = dict(x.split("=", 1) for x in f[2:])
            if int(kv.get("variant", "-1")) != colour_variant:
                continue
            if kv.get("source_sha256") != sha:
                return None
            b, us = float(kv["bytes_per_dispatch"]), float(kv["avg_us"])
            gbs = b / (us * 1e-6) / 1e9
            return {"kernel": kv.get("kernel"), "bytes_per_dispatch": b, "avg_us": us,
                    "GB_per_s": gbs, "frac_of_8TBs": gbs / 8000.0}
    return None


def colour_variant_runs(rounds: int = 3):
    """The 64-molecule batch relaxed from the tight start with each
    colour-pass variant (density tiling 0), rounds times each: the time per
    relaxation and whether the labels agree between the variants."""
    import numpy as np
    import torch

    import synth
    from paper_2208_05524_amd import Batch, Context

    ws = synth.batch_conformations()
    ctxs = []
    for w in ws:
        c = Context(0)
        c.setup(w, precision=32)
        ctxs.append(c)
    b = Batch(ctxs)
    out, labels = {}, []
    for f in range(Batch.FLIP_VARIANTS):
        ms = []
        for r in range(rounds):
            for w, c in zip(ws, ctxs):
                c.set_positions(w.xyz)
                c.init_labels("tight", 1.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.minimize(variant=Batch.DENSITY_VARIANTS * f)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        out[f"colour_variant_{f}_ms"] = ms
        labels.append([c.labels() for c in ctxs])
    out["labels_identical"] = all(all(np.array_equal(a, x) for a, x in zip(labels[0], l))
                                  for l in labels[1:])
    for c in ctxs:
        c.close()
    return out


def batch_comparison(rounds: int = 2):
    """Time to equilibrium of 64 molecules (atom counts log-uniform in [200,
    3000], grids 64^3 to 160^3 at 0.05 nm): each molecule on its own (tight
    labels, density, far field, colour sweeps, one call per molecule) against
    the batched call (one density launch and one launch per colour pass for
    all molecules, groups of sweeps replayed from a captured graph; also
    timed with direct launches).  Both start from the same positions and labels; the
    labels they reach and their energies are compared."""
    import numpy as np
    import torch

    import synth
    from paper_2208_05524_amd import Batch, Context

    ws = synth.batch_conformations()
    ctxs = []
    for w in ws:
        c = Context(0)
        c.setup(w, precision=32)
        ctxs.append(c)
    b = Batch(ctxs)

    def reset():
        for w, c in zip(ws, ctxs):
            c.set_positions(w.xyz)  # marks the density stale
        torch.cuda.synchronize()

    for c in ctxs:
        c.init_labels("tight", 1.0)  # the tuner times colour passes from these labels
    best, tune_ms = b.tune()
    plain_ms, batch_ms, eager_ms = [], [], []
    for r in range(rounds + 1):
        reset()
        t0 = time.perf_counter()
        for c in ctxs:
            c.init_labels("tight", 1.0)
            c.minimize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if r == rounds:
            lab_plain = [c.labels() for c in ctxs]
            e_plain = [c.energy()["total"] for c in ctxs]
        reset()
        t2 = time.perf_counter()
        for c in ctxs:
            c.init_labels("tight", 1.0)
        rc, st = b.minimize(variant=best)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        reset()
        t4 = time.perf_counter()
        for c in ctxs:
            c.init_labels("tight", 1.0)
        b.minimize(variant=best, graph=False)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        if r > 0:  # the first repetition warms up
            plain_ms.append(1e3 * (t1 - t0))
            batch_ms.append(1e3 * (t3 - t2))
            eager_ms.append(1e3 * (t5 - t4))
    reset()  # leave the graph-replayed result in place for the comparison
    for c in ctxs:
        c.init_labels("tight", 1.0)
    rc, st = b.minimize(variant=best)
    same = all(np.array_equal(a, c.labels()) for a, c in zip(lab_plain, ctxs))
    e_batch = [c.energy()["total"] for c in ctxs]
    rel = max(abs(a - e) / abs(a) for a, e in zip(e_plain, e_batch))
    pairs = float(sum(w.natoms * w.n ** 3 for w in ws))
    out = {"molecules": len(ws), "atoms": int(sum(w.natoms for w in ws)),
           "cells": int(sum(w.n ** 3 for w in ws)), "pairs": pairs,
           "plain_ms": min(plain_ms), "batched_ms": min(batch_ms),
           "batched_without_graph_ms": min(eager_ms),
           "speedup": min(plain_ms) / min(batch_ms),
           "batched_atom_gridpt_per_s": pairs / (min(batch_ms) / 1e3),
           "variant": {"code": best, "density_tiling": best % Batch.DENSITY_VARIANTS,
                       "colour_pass": best // Batch.DENSITY_VARIANTS},
           "tune_ms": {"density_tilings": tune_ms[:Batch.DENSITY_VARIANTS],
                       "four_sweeps_per_colour_pass_variant": tune_ms[Batch.DENSITY_VARIANTS:]},
           "flip_pass_hbm": measured_flip_traffic(best // Batch.DENSITY_VARIANTS),
           "sweeps_max": max(x["sweeps"] for x in st), "converged": rc == 0,
           "labels_identical": bool(same), "max_rel_dG": rel}
    for c in ctxs:
        c.close()
    return out


def solute_solute(w, reps: int = 5):
    """The solute-solute terms of Eq. "Gss" beyond bonds (bending, torsion,
    non-bonded LJ + Coulomb) on the same atoms with chain topology: device
    time of their kernels per evaluation (HIP events), and the energies."""
    import torch

    import synth
    from paper_2208_05524_amd import Context
    half = w.natoms // 2
    top = synth.chain_topology([(0, half), (half, w.natoms - half)], seed=3070)
    ctx = Context(0)
    ctx.setup(w, precision=32, with_bonds=True, topology=top)
    ctx.init_labels("tight", 1.0)
    xyz = torch.tensor(w.xyz, dtype=torch.float64, device="cuda").contiguous()
    ctx.energy()
    ctx.profile(True)
    for _ in range(reps):
        ctx.set_positions(xyz)
        e = ctx.energy()
        ctx.forces()
    ms, n = ctx.profile_read("solute")
    ctx.profile(False)
    ctx.close()
    pairs = w.natoms * (w.natoms - 1) // 2 - len(top.exclusions)
    per = ms / max(n, 1)
    return {"angles": len(top.angles), "torsions": len(top.torsions), "pairs": pairs,
            "ms_per_eval": per, "pairs_per_s": pairs / (per / 1000.0),
            "energy": {k: e[k] for k in ("bond", "bend", "torsion", "vdw_ss", "elec_ss")}}


def chain_config(rounds: int = 3):
    """The 1,000-atom chain on 128^3 cells (0.05 nm): time to equilibrium of
    the interface (density, far field and colour sweeps, from fresh
    positions) from the tight and from the loose start, FP32 densities."""
    import torch

    import synth
    from paper_2208_05524_amd import Context
    w = synth.chain_1000()
    ctx = Context(0)
    ctx.setup(w, precision=32, with_bonds=True)
    out = {"atoms": w.natoms, "grid": w.n}
    for mode, param in (("tight", 1.0), ("loose", 2.6)):
        times = []
        for r in range(rounds + 1):
            ctx.set_positions(w.xyz)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.init_labels(mode, param)
            rc, st = ctx.minimize()
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
        ms = 1e3 * sum(times) / len(times)
        out[mode] = {"time_to_equilibrium_ms": ms, "sweeps": st["sweeps"], "flips": st["flips"],
                     "us_per_sweep": 1e3 * ms / max(st["sweeps"], 1), "G": ctx.energy()["total"]}
    ctx.close()
    return out


def cpu_chain_equilibrium():
    """The oracle's full run on the same 1,000-atom chain and start: FP64
    density over the 128^3 grid, far field, colour sweeps to equilibrium."""
    import oracle
    import synth
    w = synth.chain_1000()
    s = oracle.System.from_workload(w)
    t0 = time.perf_counter()
    ulj, ucfa = s.density_grid()
    s.far_field()
    phi = s.init_tight()
    rc, st, _, _ = s.minimize_colour(phi, ulj + ucfa)
    return {"time_to_equilibrium_s": time.perf_counter() - t0, "sweeps": st["sweeps"],
            "start": "tight"}


def cpu_single_atom():
    """The oracle's full run on the single LJ atom (64^3 cells, FP64, loose
    sphere of 1.2 nm): density, far field, colour sweeps to equilibrium."""
    import oracle
    import synth
    w = synth.single_atom()
    s = oracle.System.from_workload(w)
    t0 = time.perf_counter()
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    phi = s.init_loose(1.2)
    rc, st, _, _ = s.minimize_colour(phi, ulj + ucfa)
    e = s.energy(phi, ulj, ucfa, far)
    return {"time_to_equilibrium_s": time.perf_counter() - t0, "sweeps": st["sweeps"],
            "G": e["total"], "start": "loose sphere, R0 = 1.2 nm"}


def cpu_full_two_globules(w):
    """The oracle's full interface relaxation at the benchmark's size: FP64
    density over every cell, far field, tight start, colour sweeps to
    equilibrium (about a minute on 16 host threads; --cpu-full only)."""
    import oracle
    s = oracle.System.from_workload(w)
    t0 = time.perf_counter()
    ulj, ucfa = s.density_grid()
    t1 = time.perf_counter()
    s.far_field()
    phi = s.init_tight()
    rc, st, _, _ = s.minimize_colour(phi, ulj + ucfa)
    t2 = time.perf_counter()
    return {"density_s": t1 - t0, "far_field_and_sweeps_s": t2 - t1,
            "time_to_equilibrium_s": t2 - t0, "sweeps": st["sweeps"], "flips": st["flips"]}


def host_cpu():
    """CPU model name of the host (from /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(w, budget_s: float = 12.0, full: bool = False, relax=None):
    """The FP64 oracle on the host cores, as written (not tuned).  value: its
    density (OpenMP over cells) over whole z-planes of the same grid until
    about budget_s seconds of work, in atom-gridpoint pairs/s; beside it the
    same on one thread (one z-plane), the whole-grid density time both
    imply (extrapolated), full runs of the single-atom and 1,000-atom
    workloads, optionally (full) the full relaxation at this size, and the
    200-iteration alternation extrapolated from the density evaluations the
    GPU run of it made."""
    import numpy as np

    import oracle
    s = oracle.System.from_workload(w)
    n = w.n
    L = n * w.h / 2
    xs = w.center[0] - L + (np.arange(n) + 0.5) * w.h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    planes = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and planes < n:
        z = w.center[2] - L + (n // 2 + planes + 0.5 - n // 4) * w.h
        pts = np.stack([X.ravel(), Y.ravel(), np.full(n * n, z)], axis=1)
        s.density_points(pts)
        planes += 1
    dt = time.perf_counter() - t0
    pairs = planes * n * n * w.natoms
    rate = pairs / dt
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = host_cpu()
    # one thread, one z-plane
    z = w.center[2] - L + (n // 2 + 0.5) * w.h
    pts = np.stack([X.ravel(), Y.ravel(), np.full(n * n, z)], axis=1)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    s.density_points(pts)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    rate1 = n * n * w.natoms / dt1
    grid_pairs = float(n) ** 3 * w.natoms
    single = {"value": rate1, "unit": "atom·gridpt/s", "cores": 1,
              "sample": f"one z-plane ({n * n} cells) x {w.natoms} atoms, {dt1:.1f} s"}
    out = {"value": rate, "unit": "atom·gridpt/s", "cores": cores, "kind": "oracle",
           "host": {"cpu": model, "threads": cores},
           "single_thread": single,
           "density_whole_grid_s_extrapolated": {
               "all_threads": grid_pairs / rate, "one_thread": grid_pairs / rate1,
               "note": "extrapolated from the measured samples (pairs / rate)"},
           "single_atom_64": cpu_single_atom(),
           "chain_1000_128": cpu_chain_equilibrium(),
           "sample": f"FP64 oracle density over {planes} z-planes ({planes * n * n} cells) of "
                     f"the {n}^3 grid x {w.natoms} atoms, {dt:.1f} s on {cores} threads of "
                     f"{model}; the GPU value is a whole hot-path step, whose density work "
                     f"alone is >= 2 such evaluations"}
    if relax is not None:
        evals = relax["iters"] + relax["retries"]
        out["relax_extrapolated_s"] = {
            "all_threads": evals * grid_pairs / rate,
            "note": f"extrapolated: {evals} whole-grid density evaluations (one per outer "
                    f"iteration and per rejected trial of the GPU run of "
                    f"{relax['iters']} iterations) at the measured oracle rate; forces and "
                    f"sweeps not counted"}
    if full:
        out["two_globules_full"] = cpu_full_two_globules(w)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle's full relaxation at the benchmark's size "
                         "(about a minute on 16 host threads)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-molecule batched-vs-one-at-a-time comparison")
    ap.add_argument("--learned-train", type=int, default=2000,
                    help="molecules the warm-start network trains on (0: skip the comparison)")
    ap.add_argument("--learned-test", type=int, default=16)
    ap.add_argument("--relax-iters", type=int, default=200,
                    help="after the timed steps, run this many outer iterations of the full "
                         "alternation (Steps 2-5) from the same start and report them (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 1,000-atom chain and the solute-solute sections (profiling "
                         "runs that should see the two-globule kernels only)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--colour-variants", action="store_true",
                    help="only relax the 64-molecule batch with each colour-pass variant "
                         "(counter runs of the batched colour passes)")
    args = ap.parse_args()
    if args.colour_variants:
        print(json.dumps(colour_variant_runs()), flush=True)
        return
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU kernel set "
              "(the multi-GPU sharding is described, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2208_05524_amd import Context, default_mobility

    w = synth.two_globules()
    log(f"workload {w.name}: n={w.n} atoms={w.natoms}")
    ctx = Context(0)
    ctx.setup(w, precision=32, with_bonds=True)
    xyz0 = torch.tensor(w.xyz, dtype=torch.float64, device="cuda").contiguous()
    torch.cuda.synchronize()

    phases = {"equilibrium": 0.0, "energy": 0.0, "forces": 0.0, "atom_step": 0.0}
    last = {}
    # the mobility state carries over from step to step, as it does from one
    # iteration of the algorithm to the next: warm-up adapts M to the step
    # size this configuration accepts, so the timed steps measure the steady
    # state rather than the start-up shrinking of M
    mob = default_mobility(0.1)

    def step(timed: bool):
        t0 = time.perf_counter()
        ctx.set_positions(xyz0)
        ctx.init_labels("tight", 1.0)
        rc, st = ctx.minimize()
        t1 = time.perf_counter()
        e = ctx.energy()
        t2 = time.perf_counter()
        ctx.forces()
        t3 = time.perf_counter()
        rs, info = ctx.atom_step(mob)
        t4 = time.perf_counter()
        if timed:
            phases["equilibrium"] += t1 - t0
            phases["energy"] += t2 - t1
            phases["forces"] += t3 - t2
            phases["atom_step"] += t4 - t3
        last.update(st=st, e=e, rc=rc, step_rc=rs, accepted=info.accepted, retries=info.retries)

    for i in range(args.warmup):
        step(False)
        log(f"warmup {i} done: {last['st']}")
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dens_ms, dens_n = ctx.profile_read("density")
    kinds = {k: ctx.profile_read(k) for k in ("far_field", "init", "flip", "energy", "force",
                                              "other")}
    ctx.profile(False)

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    pairs = float(w.natoms) * w.n ** 3
    value = pairs / (ms_per_step / 1000.0)
    avg_dens_s = dens_ms / max(dens_n, 1) / 1000.0
    achieved = FLOP_PER_PAIR * pairs / avg_dens_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom·gridpt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two seeded 5,000-atom globules 1.5 nm apart, 256^3 cells, "
                               "h = 0.05 nm, tight start, chain bonds",
                   "grid": w.n, "atoms": w.natoms, "h_nm": w.h, "precision": "fp32 density, "
                   "fp64 totals and near-tie decisions"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "density_grid_f32", "avg_ms": avg_dens_s * 1000.0,
                     "launches": dens_n, "flop_per_pair": FLOP_PER_PAIR},
        "density_atom_gridpt_per_s": pairs / avg_dens_s,
        "time_to_equilibrium_ms": phases["equilibrium"] * 1000.0 / args.steps,
        "phase_ms": {k: v * 1000.0 / args.steps for k, v in phases.items()},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kinds.items()},
        "sweeps": last["st"]["sweeps"],
        "flips": last["st"]["flips"],
        "near_ties": last["st"]["near_ties"],
        "fp64_recomputes": last["st"]["fp64_recomputes"],
        "atom_step": {"accepted": last["accepted"], "retries": last["retries"]},
        "G_total": last["e"]["total"],
    }
    if not args.no_extra:
        log("1,000-atom chain at 128^3 ...")
        out["chain_1000_128"] = chain_config()
        log(f"chain_1000_128: {out['chain_1000_128']}")
        log("solute-solute terms ...")
        out["solute_solute"] = solute_solute(w)
        log(f"solute_solute: {out['solute_solute']}")
    if not args.no_batch:
        log("batch comparison ...")
        out["batch"] = batch_comparison()
        log(f"batch: {out['batch']}")
    if args.learned_train > 0:
        log("learned warm start ...")
        from paper_2208_05524_amd.learned import warm_start_experiment
        res = warm_start_experiment(args.learned_train, args.learned_test, epochs=1, log=log)
        res.pop("rows")
        out["learned"] = res
        log(f"learned: {res}")
    if args.relax_iters > 0:
        ctx.set_positions(xyz0)
        ctx.init_labels("tight", 1.0)
        rmob = default_mobility(0.1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep = ctx.relax(rmob, max_iters=args.relax_iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["relax"] = {"iters": rep.iters, "stop_reason": rep.stop_reason,
                        "ms_per_iter": dt * 1000.0 / max(rep.iters, 1), "total_s": dt,
                        "sweeps": rep.sweeps, "retries": rep.retries,
                        "G_final": rep.G_final, "G_start": last["e"]["total"],
                        "max_grad": rep.max_grad, "dG_rel": rep.dG_rel, "M_final": rmob.M}
        log(f"relax: {out['relax']}")
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, full=args.cpu_full,
                                           relax=out.get("relax"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
