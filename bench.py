#!/usr/bin/env python
"""Benchmark: time-steps/s of the MPFC second-order scheme at 1024^2.

Workload (one GPU): second-order convex-splitting scheme, FP64, periodic
1024 x 1024 grid, h = pi/4, eps = 0.025, beta = 0.9, M = 1, dt = 0.05,
initial data = 0.07 liquid with three seeded one-mode crystallites (seed 2),
FAS V(2,2) cycles to a residual norm of 1e-10, energies computed every step.
A "step" is one whole implicit time step: source, guess, V-cycles to the
tolerance, psi update and energies, all in the library's HIP kernels.

Prints one JSON line.  `roofline` reports the dominant kernel (finest-level
red-black smoothing), timed live with HIP events on the library's stream over
the timed region; `cpu_baseline` times the CPU oracle (test infrastructure)
on a bounded sample of the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-steps/s at 1024² to 1e-10 residual: FP64 MG vs mixed-prec vs learned guess"
HBM_PEAK_GBPS = 8000.0
# Algorithmic bytes per finest cell of the two finest-level launches, FP64,
# scheme 2, V(2,2), per-operation model: one red-black sweep reads u, S, phi^k
# and writes u (80 B); residual + 2x2 restriction of u, R r and phi^k 70 B;
# prolongation + correction 60 B; residual norm 56 B.
#   down = 2 sweeps + residual/restriction, up = prolongation + 2 sweeps + norm.
MODEL_BYTES = {"down": 2 * 80.0 + 70.0, "up": 60.0 + 2 * 80.0 + 56.0}
# Compulsory traffic of the fused launches: down reads u, S, phi^k (56 B),
# writes u (24 B) and the coarse u, v, R r, phi^k (10 quarter fields, 20 B); up
# reads u, S, phi^k (56 B) and the coarse u, v (6 quarter fields, 12 B), writes
# u (24 B).
COMPULSORY_BYTES = {"down": 56.0 + 24.0 + 20.0, "up": 56.0 + 12.0 + 24.0}
# The pinning weight W (8 B per cell) adds one read per sweep and per residual
# pass: down 2 sweeps + residual, up 2 sweeps + norm.
PIN_BYTES = {"down": 3 * 8.0, "up": 3 * 8.0}
# Relaxation factor of the smoother in the relaxed variants (App. B: 1).
RELAXED_OMEGA = 0.9
# One whole V(2,2) cycle, FP64, scheme 2, per finest cell: 468 B on the
# finest level (2 x 2 sweeps of 80 B, residual and restriction 68 B, coarse
# FAS right-hand side 20 B, prolongation 60 B), 4/3 of it over all levels, and
# the stopping test's residual read (56 B).
VCYCLE_MODEL_BYTES = 680.0
# One FP32 correction V(2,2) cycle of the batch, per finest cell (all levels).
BATCH_FP32_VCYCLE_BYTES = 340.0
# HBM bytes per finest-level launch measured with rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by what the counters read for a 128 MiB copy), per tile
# shape "TXxTY/HALO", valid only for the kernel sources they were measured on
# (kernel_source_hash).
MEASURED_TRAFFIC = {
    "src": "a7c916ba31795d62",
    "down": {"64x32/6": 113708059, "32x32/6": 110302851, "32x16/6": 109981065, "16x16/6": 109964685, "64x16/10": 110995883, "32x16/10": 110008707, "16x16/10": 110001541},
    "up": {"64x32/6": 109757846, "32x32/6": 104919287, "32x16/6": 103134588, "16x16/6": 103130493, "64x16/10": 103905108, "32x16/10": 103176563, "16x16/10": 103166325},
}


def kernel_source_hash() -> str:
    """Hash of the sources of the tile kernels (csrc/tiles.hpp and the device
    helpers in csrc/kernels.hpp) with comments and blank space removed, so that
    comment edits and host-side changes keep the measured counters valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("kernels.hpp", "tiles.hpp"):
        f = os.path.join(ROOT, "paper_1208_2643_amd", "csrc", name)
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=1024, help=argparse.SUPPRESS)
    ap.add_argument("--no-energy", action="store_true", help="skip the per-step energies")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 128 MiB device copy (counter calibration)")
    ap.add_argument("--variants", type=int, default=1,
                    help="also time the mixed-precision variant of the workload")
    ap.add_argument("--big-steps", type=int, default=40,
                    help="steps of the 2048^2 FP64-vs-mixed comparison (0 skips it)")
    ap.add_argument("--learned-steps", type=int, default=500,
                    help="steps of the learned-guess comparison (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="steps of the 64-simulation batched variant (0 skips it)")
    ap.add_argument("--bc-steps", type=int, default=100,
                    help="steps of the variant with periodic-x / Neumann-y boundaries (0 skips it)")
    ap.add_argument("--pin-steps", type=int, default=100,
                    help="steps of the variant with the pinning term (0 skips it)")
    ap.add_argument("--shear-steps", type=int, default=100,
                    help="steps of the 512 x 400 sheared-crystal variant of Sec. 4.6 (0 skips it)")
    ap.add_argument("--steps-3d", type=int, default=20,
                    help="steps of the 128^3 three-dimensional variant (0 skips it)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle sample")
    return ap.parse_args()


def host_cores():
    """(logical CPUs this process may use, physical cores among them)."""
    cpus = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    phys = set()
    try:
        for c in cpus:
            base = f"/sys/devices/system/cpu/cpu{c}/topology/"
            with open(base + "physical_package_id") as f1, open(base + "core_id") as f2:
                phys.add((f1.read().strip(), f2.read().strip()))
    except OSError:
        phys = set()
    return len(cpus) or (os.cpu_count() or 1), len(phys) or None


def cpu_baseline(params, phi0, tol, budget_s):
    """The oracle, as it stands, on the same workload from the same initial
    state: whole steps on all usable host threads until about `budget_s`
    seconds have passed; then one V-cycle of the first step on all threads
    and on one thread (a whole step on one core takes minutes), as
    unknowns x V-cycles/s."""
    import numpy as np
    import oracle as O
    p = O.Params(**params)
    logical, physical = host_cores()
    threads = O.num_threads()
    phi, prev, psi = phi0.copy(), phi0.copy(), np.zeros_like(phi0)
    t0 = time.perf_counter()
    steps = 0
    cycles = 0
    while True:
        r = O.step(p, phi, prev, psi, guess=1, tol=tol, max_cycles=100, energy=True)
        steps += 1
        cycles += max(r.cycles, 0)
        prev, phi, psi = phi, r.phi, r.psi
        if time.perf_counter() - t0 >= budget_s or steps >= 20:
            break
    dt = time.perf_counter() - t0
    unknowns = 3.0 * phi0.size
    # one thread: one V-cycle from the completed extrapolated guess of step 1
    S = O.source(p, phi0, phi0, np.zeros_like(phi0))
    u0 = O.complete_guess(p, phi0.copy(), S, phi0 if p.scheme == 2 else None)
    pk = phi0 if p.scheme == 2 else None
    t1 = time.perf_counter()
    O.fas_solve(p, u0, S, phik=pk, tol=1e-30, max_cycles=1)
    t_cycle_all = time.perf_counter() - t1
    O.set_threads(1)
    try:
        t1 = time.perf_counter()
        O.fas_solve(p, u0, S, phik=pk, tol=1e-30, max_cycles=1)
        t_cycle = time.perf_counter() - t1
    finally:
        O.set_threads(threads)
    return {"value": steps / dt, "unit": "time-steps/s", "cores": threads,
            "logical_cpus": logical, "physical_cores": physical,
            "kind": "oracle",
            "sample": f"first {steps} step(s) of the same {phi0.shape[1]}x{phi0.shape[0]} "
                      f"workload from its initial state ({cycles} V-cycles, energies on), "
                      f"{dt:.1f} s wall, {threads} OpenMP threads",
            "vcycle": {"unknowns_x_vcycles_per_s": unknowns / t_cycle_all,
                       "single_thread_unknowns_x_vcycles_per_s": unknowns / t_cycle,
                       "sample": f"one V(2,2) cycle of the first step: {t_cycle_all:.2f} s on "
                                 f"{threads} threads, {t_cycle:.2f} s on one thread (a whole "
                                 "step also solves the -1 norm's Poisson problem to 1e-14 by "
                                 "conjugate gradients, which the whole-step rate above "
                                 "includes)"}}


def bench_big(api, inputs, torch, dev, params, tol, steps, warmup, N=2048, inner=4, nxt=3, nuc=1):
    phi0 = inputs.crystallites(N, N, params["h"], seed=3)
    res = {"workload": f"{N}x{N}, second-order scheme, crystallites seed 3, {steps} steps, "
                       "V(2,2) to 1e-10, energies off; each leg run twice in fresh contexts, "
                       "the faster run reported", "inner_cycles": inner,
           "inner_cycles_next": nxt, "inner_nu_coarse": nuc}
    finals = {}
    # the oracle's trajectory of this workload (FP64, solved to 1e-12 per step),
    # sampled at fixed cells, for the first steps (tests/golden/make_fullsize.py)
    gpath = os.path.join(ROOT, "tests", "golden", f"fullsize_{N}_seed3.npz")
    golden = None
    if os.path.exists(gpath):
        import numpy as np
        with np.load(gpath, allow_pickle=False) as z:
            golden = {"idx": z["idx"], "phi": z["phi"], "steps": int(z["phi"].shape[0])}
        gidx = torch.from_numpy(golden["idx"]).to(dev)
    # each leg twice, interleaved, in fresh contexts; the faster run of each
    # is reported (a context now and then runs slower with identical cycle
    # counts, which would otherwise decide the ratio)
    legs = (("fp64", dict(precision=0)),
            ("mixed", dict(precision=1, inner_cycles=inner, inner_cycles_next=nxt,
                           inner_nu_coarse=nuc)))
    for rep, (name, kw) in [(r, leg) for r in range(2) for leg in legs]:
        st = api.Stepper(N, N, api.Params(**params), tol=tol, nu1=2, nu2=2, energy=0, **kw)
        phi = torch.from_numpy(phi0).to(dev)
        prev = phi.clone()
        psi = torch.zeros_like(phi)
        nxt = torch.empty_like(phi)
        for _ in range(warmup):
            st.step(phi, prev, psi, nxt)
        phi = torch.from_numpy(phi0).to(dev)
        prev = phi.clone()
        psi.zero_()
        gc.collect()  # outside the timed region (the collector is off)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cycles = outer = 0
        sample = None
        for k in range(steps):
            _, info = st.step(phi, prev, psi, nxt)
            cycles += info.n_cycles
            outer += info.outer_iters
            prev, phi, nxt = phi, nxt, prev
            if golden is not None and k + 1 == min(steps, golden["steps"]):
                sample = phi.view(-1)[gidx].clone()  # gathered on the stream, read after timing
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs = res.get(name, {}).get("runs_time_steps_per_s", []) + [steps / el]
        res[name] = {"time_steps_per_s": max(runs), "runs_time_steps_per_s": runs,
                     "vcycles_per_step": cycles / steps}
        if name == "mixed":
            res[name]["outer_per_step"] = outer / steps
        if sample is not None:
            k = min(steps, golden["steps"])
            ref = golden["phi"][k - 1]
            got = sample.cpu().numpy()
            res[name]["rel_l2_vs_oracle"] = {
                "step": k, "value": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                "cells": int(ref.size)}
        finals[name] = phi.cpu()
        st.close()
    d = (finals["mixed"] - finals["fp64"]).norm() / finals["fp64"].norm()
    res["final_state_rel_l2_mixed_vs_fp64"] = float(d)
    res["speedup"] = res["mixed"]["time_steps_per_s"] / res["fp64"]["time_steps_per_s"]
    return res


def bench_learned(api, inputs, torch, dev, params, tol, steps, warmup, N):
    from paper_1208_2643_amd import guess_net
    if not os.path.exists(guess_net.DEFAULT_WEIGHTS):
        return {"skipped": f"no trained network at {guess_net.DEFAULT_WEIGHTS}"}
    blob = guess_net.load()
    phi0 = inputs.crystallites(N, N, params["h"], seed=5)
    res = {"workload": f"{N}x{N}, second-order scheme, crystallites seed 5, {steps} steps, "
                       "V(2,2) to 1e-10 (FP64, and mixed precision with 3 + 2 FP32 cycles "
                       "from the extrapolated guess and 4 + 1 from the learned one, V(1,1) "
                       "below the finest level), energies off",
           "network": guess_net.meta().get("validation_loss") if os.path.exists(
               guess_net.DEFAULT_WEIGHTS + ".json") else None}
    finals = {}
    # FP64, then mixed precision with each guess
    for name, guess, prec in (("extrapolated", 1, 0), ("learned", 2, 0),
                              ("mixed_extrapolated", 1, 1), ("mixed_learned", 2, 1)):
        # mixed precision: 3 + 2 FP32 cycles from the extrapolated guess; the
        # learned guess's smaller defect often reaches 1e-10 in one outer
        # iteration of 4 cycles, so it runs 4 + 1
        st = api.Stepper(N, N, api.Params(**params), tol=tol, nu1=2, nu2=2, energy=0, guess=guess,
                         precision=prec, inner_cycles=4 if guess == 2 else 3,
                         inner_cycles_next=1 if guess == 2 else 2,
                         inner_nu_coarse=1 if prec else 0)
        if guess == 2:
            st.load_cnn(blob)
        phi = torch.from_numpy(phi0).to(dev)
        prev = phi.clone()
        psi = torch.zeros_like(phi)
        nxt = torch.empty_like(phi)
        # warm-up steps restart from the initial state afterwards
        for _ in range(warmup):
            st.step(phi, prev, psi, nxt)
        phi = torch.from_numpy(phi0).to(dev)
        prev = phi.clone()
        psi.zero_()
        if guess == 2:
            st.load_cnn(blob)
        gc.collect()  # outside the timed region (the collector is off)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cycles = 0
        r0 = []
        for _ in range(steps):
            _, info = st.step(phi, prev, psi, nxt)
            cycles += info.n_cycles
            r0.append(info.history[0])
            prev, phi, nxt = phi, nxt, prev
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        entry = {"time_steps_per_s": steps / el,
                 ("fp32_vcycles_per_step" if prec else "vcycles_per_step"): cycles / steps,
                 "median_initial_residual": float(sorted(r0)[len(r0) // 2])}
        if guess == 2:
            used, fb = st.cnn_counts()
            entry["steps_from_learned_guess"] = used
            entry["fallbacks"] = fb
        finals[name] = phi.double().cpu()
        res[name] = entry
        st.close()
    ref = finals["extrapolated"]
    d = (finals["learned"] - ref).norm() / ref.norm()
    res["final_state_rel_l2_difference"] = float(d)
    res["mixed_learned_final_state_rel_l2_vs_fp64"] = float(
        (finals["mixed_learned"] - ref).norm() / ref.norm())
    fp64 = res["extrapolated"]["time_steps_per_s"]
    res["speedup"] = res["learned"]["time_steps_per_s"] / fp64
    res["speedup_mixed_learned"] = res["mixed_learned"]["time_steps_per_s"] / fp64
    return res


def bench_sheared(api, inputs, torch, dev, steps, warmup, energy, nu1, nu2):
    """Sec. 4.6's sheared crystal on its 512 x 400 grid (sides not both powers
    of two: general-index tile kernels, coarsest level 64 x 50 relaxed by one
    red-black sweep per cycle, which converges as fast here as 2 or 4): eps 0.6, M = 15^2, h = 4 pi / (16 sqrt 3), s = 0.025 h^2,
    beta 0.2, scheme 2, FP64, pinning weight 2 in strips of height pi at the
    bottom and top rows of a 20-row crystal band, phi_hat sheared by 4 % of
    2 pi at the bottom; FAS V(nu1, nu2) to 1e-10.  Also the live timing of the
    two finest-level launches."""
    m, n = 512, 400
    h = 4 * math.pi / (16 * math.sqrt(3))
    prm = dict(eps=0.6, beta=0.2, M=225.0, h=h, dt=0.025 * h * h, scheme=2)
    phi0, W, hat = inputs.strained_crystal(m, n, h)
    st = api.Stepper(m, n, api.Params(**prm), tol=1e-10, nu1=nu1, nu2=nu2, energy=energy,
                     coarse_sweeps=1)
    st.set_pinning(torch.from_numpy(W).to(dev), torch.from_numpy(hat).to(dev))
    p_ = torch.from_numpy(phi0).to(dev)
    q_ = p_.clone()
    s_ = torch.zeros_like(p_)
    n_ = torch.empty_like(p_)
    for _ in range(warmup):
        st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
    gc.collect()  # outside the timed region (the collector is off)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cyc = 0
    for _ in range(steps):
        _, inf = st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
        cyc += inf.n_cycles
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    st.profile(True)
    for which in (0, 1):
        st.profile_read(which, reset=True)
    for _ in range(max(1, min(10, steps))):
        st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
    torch.cuda.synchronize()
    kern = {}
    for which, name in ((0, "down"), (1, "up")):
        ms, launches, cells = st.profile_read(which, reset=True)
        avg = ms / 1e3 / max(1, launches)
        # per-operation model (FP64, scheme 2, pinned) for nu sweeps per launch
        sweeps = nu1 if name == "down" else nu2
        model = (sweeps * (80.0 + 8.0) + (70.0 + 8.0 if name == "down" else 60.0 + 56.0 + 8.0))
        kern[name] = {"avg_launch_us": avg * 1e6, "launches": launches,
                      "tile": "%dx%d/%d" % st.tile_shape(0, which),
                      "model_bytes_per_cell": model,
                      "achieved_GBps": model * cells / avg / 1e9 if launches else None}
    st.profile(False)
    st.close()
    dom = max(kern, key=lambda k: kern[k]["avg_launch_us"])
    return {"time_steps_per_s": steps / el, "steps": steps, "vcycles_per_step": cyc / steps,
            "ms_per_vcycle": 1e3 * el / max(1, cyc),
            "unknowns_x_vcycles_per_s": 3.0 * m * n * cyc / el,
            "roofline": {"kernel": f"k_tile {dom} launch (general-index) on the 512x400 level",
                         "bound": "hbm", "achieved": kern[dom]["achieved_GBps"],
                         "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": (kern[dom]["achieved_GBps"] / HBM_PEAK_GBPS
                                  if kern[dom]["achieved_GBps"] else None)},
            "kernels": kern,
            "workload": "Sec. 4.6 sheared crystal, 512x400 periodic, eps=0.6, M=225, "
                        "h=4pi/(16sqrt3), s=0.025h^2, beta=0.2, scheme 2, FP64, pinning strips "
                        "(weight 2, height pi) with phi_hat sheared 4% of 2pi at the bottom, "
                        f"V({nu1},{nu2}) to 1e-10, coarsest 64x50 by 1 red-black sweep"
                        + ("" if energy else ", energies off")}


# Algorithmic bytes of one red-black half-sweep launch in three dimensions, per
# cell of the level (FP64, scheme 2): read u of every cell (24 B; the colour's
# own cells and all their neighbours), S and phi^k of the colour's cells
# (32 B x 1/2), write u of the colour's cells (24 B x 1/2).
HALF_SWEEP_3D_BYTES = 24.0 + 16.0 + 12.0


def bench_3d(api, inputs, torch, dev, steps, warmup, energy, N=128):
    """Three dimensions: scheme 2, FP64, N^3 periodic, h = pi/4, eps = 0.025,
    beta = 0.9, M = 1, dt = 0.05, phi0 = 0.07 + U[-0.05, 0.05] (seed 7),
    V(2,2) to 1e-10, energies every step.  Also the live timing of the finest
    level's half-sweep launches (the dominant kernel)."""
    prm = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2)
    phi0 = inputs.noise3(N, N, N, seed=7)
    st = api.Stepper3(N, N, N, api.Params(**prm), tol=1e-10, nu1=2, nu2=2, energy=energy)
    p_ = torch.from_numpy(phi0).to(dev)
    q_ = p_.clone()
    s_ = torch.zeros_like(p_)
    n_ = torch.empty_like(p_)
    for _ in range(warmup):
        st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
    gc.collect()  # outside the timed region (the collector is off)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cyc = 0
    for _ in range(steps):
        _, inf = st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
        cyc += inf.n_cycles
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    st.profile(True)
    st.profile_read(reset=True)
    for _ in range(2):
        st.step(p_, q_, s_, n_)
        q_, p_, n_ = p_, n_, q_
    torch.cuda.synchronize()
    ms, launches, cells = st.profile_read(reset=True)
    st.profile(False)
    st.close()
    avg = ms / 1e3 / max(1, launches)
    ach = HALF_SWEEP_3D_BYTES * cells / avg / 1e9 if launches else None
    return {"time_steps_per_s": steps / el, "steps": steps, "vcycles_per_step": cyc / steps,
            "ms_per_vcycle": 1e3 * el / max(1, cyc),
            "unknowns_x_vcycles_per_s": 3.0 * N ** 3 * cyc / el,
            "roofline": {"kernel": "k3_relax half-sweep launch on the finest level",
                         "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBPS if ach else None,
                         "bytes_per_launch": HALF_SWEEP_3D_BYTES * cells,
                         "avg_launch_us": avg * 1e6, "launches": launches},
            "workload": f"three dimensions, scheme 2, FP64, {N}^3 periodic, h=pi/4, eps=0.025, "
                        "beta=0.9, M=1, dt=0.05, 0.07 + U[-0.05,0.05] (seed 7), V(2,2) to 1e-10, "
                        "coarsest 2^3 by 2 red-black sweeps"
                        + ("" if energy else ", energies off")}


def bench_batch(api, inputs, torch, dev, steps, warmup):
    specs = inputs.batch(64)
    sims = [(sp.N, sp.N, api.Params(eps=sp.eps, beta=sp.beta, M=1.0, h=math.pi / 4, dt=0.05,
                                    scheme=2)) for sp in specs]
    t_create = time.perf_counter()
    # 3 FP32 cycles in a step's first outer iteration, 2 in later ones
    # (V(2,2) on every level, the cycle the byte model below counts)
    b = api.Batch(sims, nu1=2, nu2=2, tol=1e-10, precision=1, inner_cycles=3, inner_cycles_next=2)
    t_create = time.perf_counter() - t_create
    phi = [torch.from_numpy(sp.phi0).to(dev) for sp in specs]
    prev = [t.clone() for t in phi]
    psi = [torch.zeros_like(t) for t in phi]
    nxt = [torch.empty_like(t) for t in phi]
    cells = [sp.N * sp.N for sp in specs]

    def one():
        nonlocal phi, prev, nxt
        infos = b.step(phi, prev, psi, nxt, history=False)
        prev, phi, nxt = phi, nxt, prev
        return infos

    for _ in range(warmup):
        one()
    gc.collect()  # outside the timed region (the collector is off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0.0
    outer = 0
    for k in range(steps):
        infos = one()
        work += sum(3.0 * c * i.n_cycles for c, i in zip(cells, infos))
        outer += max(i.outer_iters for i in infos)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b.close()
    # FP32 V-cycles of all simulations against the per-operation byte model
    model_GBps = BATCH_FP32_VCYCLE_BYTES * work / 3.0 / el / 1e9
    return {"simulations": len(sims), "steps": steps, "sim_steps_per_s": len(sims) * steps / el,
            "batch_steps_per_s": steps / el, "cells": int(sum(cells)),
            "unknowns_x_fp32_vcycles_per_s": work / el,
            "roofline": {"basis": "340 B per cell per FP32 V(2,2) cycle (per-operation model), "
                                  "defect passes and set-up charged to the cycles",
                         "bound": "hbm", "achieved": model_GBps, "peak": HBM_PEAK_GBPS,
                         "unit": "GB/s", "frac": model_GBps / HBM_PEAK_GBPS},
            "max_outer_per_step": outer / steps, "create_s": t_create,
            "precision": "mixed (FP32 correction cycles, FP64 defect correction; 3 FP32 cycles "
                         "in a step's first outer iteration, 2 in later ones)",
            "sizes": {str(n): sum(1 for sp in specs if sp.N == n) for n in (128, 256, 512, 1024)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; run with --gpus 1 "
              "(the multi-GPU sharding of the step is a design, not a built path)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1208_2643_amd import _lib as L, api, inputs

    # Python's cyclic garbage collector stays off for the run, as timeit keeps
    # it off: a full collection pass over the interpreter's objects takes tens
    # of milliseconds and, landing inside a timed loop of ~1 ms steps, charged
    # itself to the GPU path now and then (one 37-50 ms pause in 100 steps
    # lowered a variant's rate by a quarter).  The step path allocates no
    # reference cycles; a collection runs before each timed region.
    gc.collect()
    gc.disable()

    if args.calib_copy:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the HBM byte counters (128 MiB read, 128 MiB written).
        a = torch.ones(16 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    N = args.N
    params = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2)
    tol = 1e-10
    phi0 = inputs.crystallites(N, N, params["h"], seed=2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    st = api.Stepper(N, N, api.Params(**params), tol=tol, nu1=2, nu2=2,
                     energy=0 if args.no_energy else 1)
    phi = torch.from_numpy(phi0).to(dev)
    prev = phi.clone()
    psi = torch.zeros_like(phi)
    nxt = torch.empty_like(phi)

    def one():
        nonlocal phi, prev, nxt
        _, info = st.step(phi, prev, psi, nxt)
        prev, phi, nxt = phi, nxt, prev
        return info

    for _ in range(args.warmup):
        one()
    cycles = []
    gc.collect()  # outside the timed region (the collector is off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = one()
        cycles.append(info.n_cycles)
        if (k + 1) % 50 == 0:
            print(f"[bench] {k + 1}/{args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_per_s = args.steps / elapsed
    total_cycles = int(sum(cycles))
    final_state = phi.clone()  # after warmup + steps, for the variants' comparison

    # Live per-kernel timing of the two finest-level launches (HIP events on
    # the library's stream), over a second timed region of the same workload.
    st.profile(True)
    for which in (0, 1):
        st.profile_read(which, reset=True)
    prof_steps = max(1, min(20, args.steps))
    for _ in range(prof_steps):
        one()
    torch.cuda.synchronize()
    timing = {}
    for which, name in ((0, "down"), (1, "up")):
        ms, launches, cells = st.profile_read(which, reset=True)
        timing[name] = (ms, launches, cells)
    st.profile(False)
    shapes = {name: "%dx%d/%d" % st.tile_shape(0, which)
              for which, name in ((0, "down"), (1, "up"))}
    dom = max(timing, key=lambda k: timing[k][0])
    ms, launches, cells = timing[dom]
    traffic = (MEASURED_TRAFFIC[dom].get(shapes[dom])
               if kernel_source_hash() == MEASURED_TRAFFIC["src"] else None)
    avg_s = ms / 1e3 / max(1, launches)
    achieved = MODEL_BYTES[dom] * cells / avg_s / 1e9 if launches else None
    compulsory = COMPULSORY_BYTES[dom] * cells / avg_s / 1e9 if launches else None
    kernels = {k: {"avg_launch_us": 1e3 * v[0] / max(1, v[1]), "launches": v[1], "tile": shapes[k],
                   "model_bytes_per_cell": MODEL_BYTES[k],
                   "compulsory_bytes_per_cell": COMPULSORY_BYTES[k]} for k, v in timing.items()}
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"MPFC second-order scheme, FP64, {N}x{N} periodic, h=pi/4, eps=0.025, "
                        "beta=0.9, M=1, dt=0.05, 0.07 liquid + 3 seeded crystallites (seed 2), "
                        "FAS V(2,2) to residual 1e-10, energies every step"
                        + (" (energies off)" if args.no_energy else ""),
            "grid": [N, N], "scheme": 2, "cycle": "V(2,2)", "tol": tol,
            "precision": "fp64", "guess": "extrapolated",
        },
        "roofline": {
            "kernel": f"k_tile {dom} launch on the finest level (fused red-black passes), "
                      f"tile {shapes[dom]}",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS if achieved else None,
            "traffic": traffic,
            "traffic_source": ("rocprofv3 FETCH_SIZE and WRITE_SIZE per launch of this tile "
                               "shape, scaled by a 128 MiB copy's readings, from a separate "
                               "run on these kernel sources (profiles/), not this run"
                               if traffic else "no counter reading for these kernel sources"),
            "measured_GBps": traffic / avg_s / 1e9 if traffic and launches else None,
            "frac_measured": traffic / avg_s / 1e9 / HBM_PEAK_GBPS if traffic and launches
                             else None,
            "achieved_basis": "algorithmic bytes: per-operation model of the launch's passes",
            "bytes_per_launch": MODEL_BYTES[dom] * cells,
            "avg_launch_us": avg_s * 1e6,
            "compulsory_GBps": compulsory,
            "frac_compulsory": compulsory / HBM_PEAK_GBPS if compulsory else None,
            "timed_steps": prof_steps,
            "kernels": kernels,
        },
        "extra": {
            "vcycles_per_step": total_cycles / args.steps,
            "unknowns_x_vcycles_per_s": 3.0 * N * N * total_cycles / elapsed,
            "ms_per_vcycle": 1e3 * elapsed / max(1, total_cycles),
            # whole V-cycle against the per-operation byte model (680 B per
            # finest cell, all levels and the stopping test), with the step's
            # set-up, psi update and energies charged to its cycles
            "vcycle_model_bytes": VCYCLE_MODEL_BYTES * N * N,
            "vcycle_frac_of_hbm_peak": VCYCLE_MODEL_BYTES * N * N * total_cycles / elapsed
                                       / 1e9 / HBM_PEAK_GBPS,
        },
    }
    # The same workload with mixed precision (FP32 correction cycles inside
    # FP64 defect correction), timed over its own region: the same warmup and
    # the same number of steps as the FP64 line, so that both cover the same
    # stretch of the trajectory (early steps need more cycles).
    if args.variants:
        out["variants"] = {"fp64": {"time_steps_per_s": steps_per_s,
                                    "vcycles_per_step": total_cycles / args.steps}}

        def same_workload(**opts):
            """The headline's protocol (warmup steps, then args.steps timed) in
            a fresh context with other solver options."""
            sv = api.Stepper(N, N, api.Params(**params), tol=tol, nu1=2, nu2=2,
                             energy=0 if args.no_energy else 1, **opts)
            p_, q_, s_ = (torch.from_numpy(phi0).to(dev), torch.from_numpy(phi0).to(dev),
                          torch.zeros_like(phi))
            n_ = torch.empty_like(phi)
            for _ in range(args.warmup):
                sv.step(p_, q_, s_, n_)
                q_, p_, n_ = p_, n_, q_
            gc.collect()  # outside the timed region (the collector is off)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            outer = cyc = 0
            for _ in range(args.steps):
                _, inf = sv.step(p_, q_, s_, n_)
                q_, p_, n_ = p_, n_, q_
                outer += inf.outer_iters
                cyc += inf.n_cycles
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            sv.close()
            d = float(torch.linalg.norm(p_ - final_state) / torch.linalg.norm(final_state))
            r = {"time_steps_per_s": args.steps / el, "steps": args.steps,
                 "speedup_vs_fp64": args.steps / el / steps_per_s,
                 "final_state_rel_l2_vs_fp64": d}
            if opts.get("precision") == 1:
                r.update(outer_per_step=outer / args.steps, fp32_vcycles_per_step=cyc / args.steps)
            else:
                r.update(vcycles_per_step=cyc / args.steps,
                         ms_per_vcycle=1e3 * el / max(1, cyc))
            return r

        # mixed precision: FP32 correction cycles inside FP64 defect correction
        # (three in the first outer iteration, which takes the defect of the
        # guess down to FP32's floor, two in each later one; V(1,1) on the
        # levels below the finest)
        mixed_opts = dict(inner_cycles=3, inner_cycles_next=2, inner_nu_coarse=1)
        out["variants"]["mixed"] = dict(**mixed_opts, **same_workload(precision=1, **mixed_opts))
        # App. B's smoother under-relaxed (omega = 0.9): same discrete solution,
        # fewer V-cycles per step; alone and with mixed precision
        out["variants"]["relaxed_smoother"] = dict(
            omega=RELAXED_OMEGA, **same_workload(omega=RELAXED_OMEGA))
        relaxed_mixed_opts = dict(omega=RELAXED_OMEGA, inner_cycles=2, inner_nu_coarse=1)
        out["variants"]["relaxed_mixed"] = dict(
            **relaxed_mixed_opts, **same_workload(precision=1, **relaxed_mixed_opts))
    # The same workload with Sec. 4.5's boundary conditions: periodic in x,
    # homogeneous Neumann in y (App. A), FP64, energies as above.
    if args.variants and args.bc_steps > 0:
        stb = api.Stepper(N, N, api.Params(**params, bc=L.MPFC_BC_NEUMANN_Y), tol=tol, nu1=2,
                          nu2=2, energy=0 if args.no_energy else 1)
        p_, q_, s_ = (torch.from_numpy(phi0).to(dev), torch.from_numpy(phi0).to(dev),
                      torch.zeros_like(phi))
        n_ = torch.empty_like(phi)
        for _ in range(args.warmup):
            stb.step(p_, q_, s_, n_)
            q_, p_, n_ = p_, n_, q_
        gc.collect()  # outside the timed region (the collector is off)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cyc = 0
        for _ in range(args.bc_steps):
            _, inf = stb.step(p_, q_, s_, n_)
            q_, p_, n_ = p_, n_, q_
            cyc += inf.n_cycles
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out["variants"]["neumann_y"] = {
            "time_steps_per_s": args.bc_steps / el, "steps": args.bc_steps,
            "vcycles_per_step": cyc / args.bc_steps,
            "workload": "as above with periodic x, homogeneous Neumann y boundaries"}
        stb.close()
    # The same workload with the pinning term of Sec. 4.6: weight 2 in strips
    # of 4 rows along the top and bottom, phi_hat the initial field.
    if args.variants and args.pin_steps > 0:
        W = torch.zeros_like(phi)
        W[:4] = 2.0
        W[-4:] = 2.0
        stp = api.Stepper(N, N, api.Params(**params), tol=tol, nu1=2, nu2=2,
                          energy=0 if args.no_energy else 1)
        stp.set_pinning(W, torch.from_numpy(phi0).to(dev))
        p_, q_, s_ = (torch.from_numpy(phi0).to(dev), torch.from_numpy(phi0).to(dev),
                      torch.zeros_like(phi))
        n_ = torch.empty_like(phi)
        for _ in range(args.warmup):
            stp.step(p_, q_, s_, n_)
            q_, p_, n_ = p_, n_, q_
        gc.collect()  # outside the timed region (the collector is off)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cyc = 0
        for _ in range(args.pin_steps):
            _, inf = stp.step(p_, q_, s_, n_)
            q_, p_, n_ = p_, n_, q_
            cyc += inf.n_cycles
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out["variants"]["pinned"] = {
            "time_steps_per_s": args.pin_steps / el, "steps": args.pin_steps,
            "vcycles_per_step": cyc / args.pin_steps,
            "workload": "as above with the pinning term (weight 2 in 4-row strips top and "
                        "bottom, phi_hat = initial field)"}
        stp.close()
    # Sec. 4.6's sheared crystal on its 512 x 400 grid (general grid sides).
    if args.variants and args.shear_steps > 0:
        # V(1,0) is the fastest cycle here (the collective smoother is close to
        # its stability limit at these parameters); V(2,2) as the headline's
        out["variants"]["sheared_crystal_512x400"] = bench_sheared(
            api, inputs, torch, dev, args.shear_steps, args.warmup, 0 if args.no_energy else 1,
            1, 0)
        out["variants"]["sheared_crystal_512x400_v22"] = bench_sheared(
            api, inputs, torch, dev, max(1, args.shear_steps // 2), args.warmup,
            0 if args.no_energy else 1, 2, 2)
    # The three-dimensional extension of the step at 128^3.
    if args.variants and args.steps_3d > 0:
        out["variants"]["three_d_128"] = bench_3d(api, inputs, torch, dev, args.steps_3d,
                                                  args.warmup, 0 if args.no_energy else 1)
    # 2048^2 with mixed precision (FP32 correction cycles inside FP64 defect
    # correction) against FP64 on the same input (seed 3).
    if args.variants and args.big_steps > 0:
        out["variants"]["mixed_2048"] = bench_big(api, inputs, torch, dev, params, tol,
                                                  args.big_steps, args.warmup)
    # Learned initial guess (the committed trained network) against the
    # extrapolated guess on the same evaluation input: 1024^2, the parameters
    # above, crystallites from seed 5, `learned_steps` steps each.
    if args.variants and args.learned_steps > 0:
        out["variants"]["learned"] = bench_learned(api, inputs, torch, dev, params, tol,
                                                   args.learned_steps, args.warmup, N)
    # Batched workload: 64 independent simulations, sizes uniform over
    # {128, ..., 1024}^2, eps / mean phi / beta drawn per simulation, seeded
    # noise, mixed precision, all advanced together by shared launches.
    if args.variants and args.batch_steps > 0:
        out["variants"]["batch64"] = bench_batch(api, inputs, torch, dev, args.batch_steps,
                                                 args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, phi0, tol, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
