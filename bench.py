#!/usr/bin/env python3
"""Benchmark of the MI355X reaction + SDC stage (one JSON line on stdout).

Workload: TT06 epicardial model on a 100x100x100 slab (1,000,000 vertices),
rest + U(-1, 1) mV, planar stimulus on the x = 0 face for 2 ms, fixed
diffusion current N(0, 0.5^2); dt = 0.02 ms, 500 steps per launch, 3
Gauss-Lobatto nodes, 3 sweeps, Newton tol 1e-10.  One benchmark "step" is
one whole pass of that workload: a single fused launch advancing every vertex
through all 500 time steps from the initial state (the state buffer is
restored by a device copy before each pass).  Measured in mixed precision
(the reported value) and in plain fp64 on the same GPU.

Reported: vertex-steps/s over the timed passes (wall clock, inputs resident
in HBM), kernel time from HIP events on the launch stream, the roofline
fraction of the dominant kernel (algorithmic flops from the per-evaluation
operation counts below and the Newton iterations the launch took), the
mixed-vs-fp64 difference on the full field, the serving latency of the
continuous-batching loop on the seeded request trace, and the CPU oracle
timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-serving] [--no-cpu]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

# Operation counts per evaluation of the TT06 model (forward-mode
# differentiation on the compile-time Jacobian pattern; printed by
# `python -m oracle.opcount`, checked against it by the CPU tests).
TT06_FLOPS = {"F": 553, "FJ": 1250, "solve": 362, "resolve": 155}
LR91_FLOPS = {"F": 232, "FJ": 465, "solve": 75, "resolve": 40}
# Rush-Larsen evaluations (work feeding the outputs the kernel keeps)
TT06_RL_FLOPS = {"gate_step_first": 568, "gate_step": 335, "core_FJ": 572, "core_solve": 174}
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}   # MI355X vector fp64 / fp32 (published)
HBM_PEAK_GBS = 8000.0
# Operation counts by kind (same source as above): the transcendental kinds
# and divisions of one F and one F+J evaluation, and the pivot reciprocals of
# one static solve (one per state).
TT06_KINDS = {"F": {"div": 72, "mul": 245, "add": 178, "exp": 52, "log": 4, "expm1": 1, "sqrt": 1},
              "FJ": {"div": 77, "mul": 813, "add": 302, "exp": 52, "log": 4, "expm1": 1, "sqrt": 1}}
TT06_N, TT06_N64 = 19, 6

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2510_27447_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sdc_kernel_tt06_slab1e6_500steps.txt")
STATE_BYTES = {"fp64": 19 * 8 * 1_000_000, "mixed": (6 * 8 + 13 * 4) * 1_000_000}


def kernel_source_hash():
    """Hash of the sources and compile flags of the step kernels, which the
    traffic counters belong to: the step translation units (kernels_*.hip), the
    headers they include and the build's flags; the stencil, elliptic,
    multigrid and control sources are not part of those kernels."""
    h = hashlib.sha1()
    for fn in sorted(os.listdir(CSRC)):
        if (fn.startswith("kernels_") and fn.endswith(".hip")) or fn in (
                "sdc_kernel.h", "dual.h", "sparse_solve.h", "kernel_ops.h", "kernel_ops_impl.h",
                "model_lr91.h", "model_tt06.h", "model_test.h"):
            h.update(fn.encode())
            with open(os.path.join(CSRC, fn), "rb") as f:
                h.update(f.read())
    # the compile flags (not the source list, which other kernels extend)
    from paper_2510_27447_amd import build as B
    flags = [f.replace(ROOT, ".") for f in B.FLAGS]  # include paths relative to the repository
    h.update(repr((B.ARCH, flags, sorted(B.OPT.items()), sorted(B.EXTRA.items()))).encode())
    return h.hexdigest()[:16]


SHORT_FLAGS = ("--no-serving", "--no-cpu", "--no-ros2", "--no-rl", "--no-diffusion",
               "--no-bidomain", "--no-c4", "--no-micro")


def step_kernel_args(name):
    """The template arguments of a step kernel's name in a rocprofv3 record,
    e.g. 'sdc_kernel<ionic::TT06, ionic::Mixed, 3, 0, 1>' -> ['ionic::TT06',
    'ionic::Mixed', '3', '0', '1'] (model, precision, nodes, predictor, and
    wavefronts per SIMD where the name carries it); None for other kernels."""
    if "sdc_kernel<" not in name:
        return None
    inner = name.split("sdc_kernel<", 1)[1].split(">", 1)[0]
    return [a.strip() for a in inner.split(",")]


def is_tt06_newton_step(name):
    args = step_kernel_args(name)
    return args is not None and "TT06" in args[0] and args[3] == "0"


def traffic_from_counters(fetch_csv, write_csv):
    """HBM bytes per launch of the step kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) of `bench.py --steps 1 --warmup 0`.
    Each counter is scaled by what it reads for the state-restore copies of the
    same run (__amd_rocclr_copyBuffer of a known number of bytes)."""
    out = {}
    for counter, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = list(csv.DictReader(open(path)))
        kern = {}
        copies = []
        for r in rows:
            v = float(r["Counter_Value"]) * 1024.0
            name = r["Kernel_Name"]
            if "sdc_kernel" in name:
                # the TT06 Newton kernels (predictor 0)
                if not is_tt06_newton_step(name):
                    continue
                # the first dispatch of each precision: the Newton tol 1e-10 pass
                kern.setdefault("fp64" if "Fp64" in name else "mixed", v)
            elif "copyBuffer" in name and v > 1e6:
                copies.append(v)
        # the two largest copy sizes are the fp64 and mixed state restores
        factors = []
        for prec, nbytes in STATE_BYTES.items():
            near = [c for c in copies if 0.3 * nbytes < c < 1.5 * nbytes]
            near_fp64 = prec == "fp64"
            if near:
                pick = max(near) if near_fp64 else min(near)
                factors.append(nbytes / pick)
        scale = float(np.median(factors))
        for prec, v in kern.items():
            out.setdefault(prec, {})[counter] = v * scale
            out[prec][counter + "_scale"] = scale
    return out


def write_traffic_file(fetch_csv, write_csv):
    t = traffic_from_counters(fetch_csv, write_csv)
    short = "python3 bench.py --steps 1 --warmup 0 " + " ".join(SHORT_FLAGS)
    lines = ["# HBM traffic of sdc_kernel<TT06, *, 3, Newton>, TT06 slab 1e6 vertices x 500 steps, "
             "per launch",
             "# commands (repository root, MI355X):",
             "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/fetch -o fetch -- "
             + short,
             "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/write -o write -- "
             + short,
             "#   python3 bench.py --traffic-from <fetch csv> <write csv>",
             "# counters scaled by their reading for the state-restore copy (known bytes)",
             "source_hash: %s" % kernel_source_hash()]
    for prec in ("fp64", "mixed"):
        d = t[prec]
        lines.append("%s_fetch_bytes: %.6e" % (prec, d["fetch"]))
        lines.append("%s_write_bytes: %.6e" % (prec, d["write"]))
        lines.append("%s_fetch_scale: %.4f" % (prec, d["fetch_scale"]))
        lines.append("%s_write_scale: %.4f" % (prec, d["write_scale"]))
        lines.append("%s_algorithmic_bytes: %.6e" % (prec, 2 * STATE_BYTES[prec] + 16 * 1_000_000))
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(prec):
    """Per-launch HBM bytes (fetch + write) recorded for the current kernel sources, or None."""
    try:
        kv = dict(l.split(": ", 1) for l in open(TRAFFIC_FILE).read().splitlines()
                  if l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("source_hash") != kernel_source_hash():
        return None
    return float(kv[prec + "_fetch_bytes"]) + float(kv[prec + "_write_bytes"])


def flops_per_launch(ev, n_states, vertex_steps, M, K, newton_iters):
    F_evals = vertex_steps * K * (M - 2)   # F(X_n) comes from the first Newton evaluation
    FJ = newton_iters + vertex_steps * K * (M - 1)
    return (F_evals * ev["F"] + FJ * (ev["FJ"] + ev["solve"]) + newton_iters * 6 * n_states
            + vertex_steps * K * ((M - 1) * M * 2 + (M - 1) * 3) * n_states)


def flops_per_launch_ros2(ev, n_states, vertex_steps, M, K):
    """ROS2 predictor: per sub-interval one F+J evaluation with its elimination,
    one F evaluation, one second solve and 12 flops of stage arithmetic per
    state; sweeps as above but F(X_n) comes from the first stage."""
    per_sub = ev["FJ"] + ev["solve"] + ev["F"] + ev["resolve"] + 12 * n_states
    sweeps = (K * (M - 2) * ev["F"] + K * (M - 1) * (ev["FJ"] + ev["solve"])
              + K * ((M - 1) * M * 2 + (M - 1) * 3) * n_states)
    return vertex_steps * ((M - 1) * per_sub + sweeps)


def flops_per_launch_rl(ev, rl, n_states, n_core, vertex_steps, M, K, newton_iters):
    """Rush-Larsen predictor: gating-state evaluations (the first gives F(X_n)),
    7 flops per gating state and sub-interval, per core Newton iteration the
    core evaluation, core solve and 6 flops per core state; sweeps as above."""
    gates = n_states - n_core
    per_step = rl["gate_step_first"] + (M - 2) * rl["gate_step"] + (M - 1) * 7 * gates
    sweeps = (K * (M - 2) * ev["F"] + K * (M - 1) * (ev["FJ"] + ev["solve"])
              + K * ((M - 1) * M * 2 + (M - 1) * 3) * n_states)
    return (vertex_steps * (per_step + sweeps)
            + newton_iters * (rl["core_FJ"] + rl["core_solve"] + 6 * n_core))


def work_split(vertex_steps, M, K, newton_iters, precision, ev=TT06_FLOPS, kinds=TT06_KINDS,
               n=TT06_N, n64=TT06_N64):
    """Algorithmic work of one Newton-predictor launch split by the unit that
    executes it (the t_min decomposition W64/P64 + W32/P32 + Wtr/Ptr).

    fp64 path: Wtr = the exp/log/expm1 calls (software sequences in double),
    W64 = every other flop (divisions, square roots and pivot reciprocals
    count one each).  Mixed path: Wtr = every exp, log, expm1, sqrt,
    division and pivot reciprocal of the fp32 evaluations and solves (each one
    hardware transcendental instruction), W32 = their adds and multiplies,
    W64 = the Newton residuals and the SDC quadrature and residuals (formed in
    double) and the updates of the n64 double-held states; the updates of the
    fp32 states and the stop tests are W32."""
    F_evals = vertex_steps * K * (M - 2)
    FJ_evals = newton_iters + vertex_steps * K * (M - 1)
    solve_rcp = n
    solve_arith = ev["solve"] - solve_rcp
    sw_nodes = vertex_steps * K * (M - 1)
    if precision == "fp64":
        tr = lambda c: c["exp"] + c["log"] + c["expm1"]
        wtr = F_evals * tr(kinds["F"]) + FJ_evals * tr(kinds["FJ"])
        total = flops_per_launch(ev, n, vertex_steps, M, K, newton_iters)
        return {"W64": total - wtr, "W32": 0.0, "Wtr": wtr}
    tr = lambda c: c["exp"] + c["log"] + c["expm1"] + c["sqrt"] + c["div"]
    ar = lambda c: c["add"] + c["mul"]
    wtr = F_evals * tr(kinds["F"]) + FJ_evals * (tr(kinds["FJ"]) + solve_rcp)
    w32 = (F_evals * ar(kinds["F"]) + FJ_evals * (ar(kinds["FJ"]) + solve_arith)
           + newton_iters * (2 * n + (n - n64)) + sw_nodes * (n - n64))
    w64 = newton_iters * (3 * n + n64) + sw_nodes * ((2 * M + 2) * n + n64)
    return {"W64": w64, "W32": w32, "Wtr": wtr}


def t_min(split, precision, rates):
    """Lower bound on a launch's time from its work split and unit rates
    (flop/s for P64 and P32, operations/s for the transcendentals)."""
    ptr = rates["exp64"] if precision == "fp64" else rates["trans32"]
    return split["W64"] / rates["P64"] + split["W32"] / rates["P32"] + split["Wtr"] / ptr


def state_bytes_per_vertex(precision):
    return 19 * 8 if precision == "fp64" else 6 * 8 + 13 * 4


VERTEX_ORDER = ("4 x 4 x 4 blocks of the grid per wavefront in the mixed Newton and "
                "Rush-Larsen kernels (ionic_set_vertex_order)")


def grid_order(sim, w, predictor="newton"):
    """The slab and spiral runs with the Newton and Rush-Larsen predictors process
    their vertices in 4 x 4 x 4 blocks of the grid per wavefront (their Newton
    loops then diverge less within a wavefront); ROS2 has no Newton loop and keeps
    the identity order, which spares it the gather.  The results are the same bit
    for bit in any order."""
    from paper_2510_27447_amd import workloads as W
    if len(w.grid) == 3 and predictor != "ros2":
        sim.set_vertex_order(W.blocked_order(*w.grid))


def run_pass_set(I, torch, w, steps, warmup, predictor="newton", sample=None, rates=None):
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    sim.set_predictor(predictor)
    grid_order(sim, w, predictor)
    stim = torch.as_tensor(w.i_stim).cuda()
    diff = torch.as_tensor(w.i_diff).cuda()
    init = sim.state.clone()
    stream = torch.cuda.current_stream()

    def one_pass():
        sim.state.copy_(init)
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, stim, w.stim_t_on, w.stim_t_off,
                 diff, stream=stream)

    for _ in range(warmup):
        one_pass()
    torch.cuda.synchronize()
    I.ionic_reset_stats(sim.handle)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        sim.state.copy_(init)
        starts[k].record(stream)
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, stim, w.stim_t_on, w.stim_t_off,
                 diff, stream=stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    st = sim.stats()
    X = sim.readback()
    V = X[0]
    Xs = X[:, sample] if sample is not None else None
    del X
    sim.close()
    vsteps = w.n * w.n_steps
    iters = st["newton_iters"] / steps
    if predictor == "newton":
        flops = flops_per_launch(TT06_FLOPS, 19, vsteps, w.n_nodes, w.n_sweeps, iters)
    elif predictor == "rush_larsen":
        flops = flops_per_launch_rl(TT06_FLOPS, TT06_RL_FLOPS, 19, 6, vsteps, w.n_nodes,
                                    w.n_sweeps, iters)
    else:
        flops = flops_per_launch_ros2(TT06_FLOPS, 19, vsteps, w.n_nodes, w.n_sweeps)
    kavg = float(np.mean(kernel_ms)) / 1e3
    achieved = flops / kavg / 1e12
    bytes_launch = w.n * (2 * state_bytes_per_vertex(w.precision) + 2 * 8)  # state r/w, stim, diff
    tmin = None
    if predictor == "newton":
        split = work_split(vsteps, w.n_nodes, w.n_sweeps, iters, w.precision)
        tmin = {"W64_per_vertex_step": split["W64"] / vsteps,
                "W32_per_vertex_step": split["W32"] / vsteps,
                "Wtr_per_vertex_step": split["Wtr"] / vsteps}
        if rates:
            # published vector peaks; no figure is published for the transcendental
            # unit or the software fp64 exp, so both variants take the measured rate
            spec = {"P64": 78.6e12, "P32": 157.3e12, "trans32": rates["trans32"],
                    "exp64": rates["exp64"]}
            ts, tm = t_min(split, w.precision, spec), t_min(split, w.precision, rates)
            tmin.update({"t_min_spec_ms": ts * 1e3, "frac_spec": round(ts / kavg, 4),
                         "t_min_measured_ms": tm * 1e3, "frac_measured": round(tm / kavg, 4)})
    return {
        "newton_tol": w.newton_tol if w.precision == "fp64" else max(w.newton_tol, 1e-6),
        "t_min": tmin,
        "X_sample": Xs,
        "value": vsteps * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "kernel_ms": float(np.mean(kernel_ms)),
        "kernel_ms_all": [round(x, 3) for x in kernel_ms],
        "newton_iters_per_solve": st["newton_iters"] / max(1, st["newton_solves"]),
        "newton_it_max": st["newton_it_max"],
        "n_nonconverged": st["n_nonconverged"],
        "n_nonfinite": st["n_nonfinite"],
        "algorithmic_flops_per_launch": flops,
        "roofline": {
            "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[w.precision],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[w.precision], 4),
            "traffic": read_traffic(w.precision) if predictor == "newton" else None,
        },
        "traffic_algorithmic_bytes": bytes_launch,
        "hbm_gbs_algorithmic": bytes_launch / kavg / 1e9,
        "V": V,
    }


def run_adaptive(I, torch, w, err_tol, t_end, dt_max, dt_init=0.01):
    """The paper's scheme with adaptive steps over [0, t_end] on the same slab:
    ROS2 predictor, 2 nodes, 1 correction, one step size for all vertices.
    One untimed run, then one timed run from the same initial state."""
    sim = I.Simulation(w.model, w.x0, precision=w.precision)
    stim = torch.as_tensor(w.i_stim).cuda()
    diff = torch.as_tensor(w.i_diff).cuda()
    init = sim.state.clone()
    stream = torch.cuda.current_stream()

    def run():
        sim.state.copy_(init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sim.adaptive(0.0, t_end, dt_init, dt_max, err_tol, n_nodes=2, n_sweeps=1,
                         i_stim=stim, stim_t_on=w.stim_t_on, stim_t_off=w.stim_t_off,
                         i_diff=diff, stream=stream)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    run()
    I.ionic_reset_stats(sim.handle)
    r, wall = run()
    st = sim.stats()
    V = sim.readback()[0]
    sim.close()
    attempts = r["accepted"] + r["rejected"]
    flops = flops_per_launch_ros2(TT06_FLOPS, 19, w.n * attempts, 2, 1)
    achieved = flops / wall / 1e12
    return {
        "err_tol": err_tol, "t_end_ms": t_end, "dt_max_ms": dt_max,
        "accepted": r["accepted"], "rejected": r["rejected"], "reached": r["reached"],
        "wall_s": wall, "simulated_ms_per_s": t_end / wall,
        "vertex_steps_per_s": w.n * r["accepted"] / wall,
        "mean_dt_ms": t_end / max(1, r["accepted"]),
        "alu_tflops_wall": round(achieved, 3),
        "frac_of_peak_wall": round(achieved / PEAK_TFLOPS[w.precision], 4),
        "n_nonfinite": st["n_nonfinite"],
        "V": V,
    }


def run_reaction_diffusion(I, torch, w, steps, warmup, h=0.01, sigma=0.75e-3):
    """The slab as tissue: per time step the Q1 diffusion current of the V field
    (h = 0.01 cm, the monodomain sigma of the paper's sigma_i = sigma_e = 1.5e-3)
    is held over one reaction step -- 500 diffusion launches and 500 one-step
    reaction launches per pass; stimulus -100 on the first five x-planes for
    2 ms.  Also times the diffusion kernel alone."""
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    grid_order(sim, w)
    # a one-plane stimulus drains into the tissue; five planes start a planar wave
    stim_np = np.where(np.arange(w.n) % w.grid[0] < 5, -100.0, 0.0)
    stim = torch.as_tensor(stim_np).cuda()
    work = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    grid = I.make_grid(*w.grid, h=h, sigma=sigma)
    init = sim.state.clone()
    stream = torch.cuda.current_stream()

    def one_pass():
        sim.state.copy_(init)
        I.reaction_diffusion_step(sim.handle, grid, 0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps,
                                  work, stim, w.stim_t_on, w.stim_t_off, stream=stream)

    for _ in range(warmup):
        one_pass()
    torch.cuda.synchronize()
    I.ionic_reset_stats(sim.handle)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.stats()
    V = sim.readback()[0]
    # diffusion kernel alone, 200 launches between two events
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(200):
        I.ionic_diffusion_current(sim.handle, grid, work, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dk = e0.elapsed_time(e1) / 200 / 1e3
    sim.close()
    n_act = int(np.sum(V > 0.0))
    bytes_diff = w.n * 16                      # V read once, I_diff written once
    vsteps = w.n * w.n_steps
    iters = st["newton_iters"] / steps
    flops = (flops_per_launch(TT06_FLOPS, 19, vsteps, w.n_nodes, w.n_sweeps, iters)
             + vsteps * 27 * 2)                # the stencil: 27 products and sums per node
    per_pass = wall / steps
    return {
        "value": vsteps * steps / wall,
        "ms_per_pass": per_pass * 1e3,
        "newton_iters_per_solve": st["newton_iters"] / max(1, st["newton_solves"]),
        "alu_tflops_wall": round(flops / per_pass / 1e12, 3),
        "frac_of_peak_wall": round(flops / per_pass / 1e12 / PEAK_TFLOPS[w.precision], 4),
        "diffusion_kernel_us": dk * 1e6,
        "diffusion_roofline": {"bound": "hbm", "achieved": round(bytes_diff / dk / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(bytes_diff / dk / 1e9 / HBM_PEAK_GBS, 4)},
        "vertices_depolarised_at_end": n_act,
    }


def run_bidomain(I, torch, w, n_steps=100, rtol=1e-8, max_iter=2000, h=0.01, sigma=1.5e-3):
    """The slab with the partitioned step of Algorithm 2 (one pass per step): the
    elliptic equation for u by Jacobi-preconditioned CG (warm start, rtol 1e-8),
    then the current -M_L^{-1} A_i (v + u) held over one reaction step; the
    paper's sigma_i = sigma_e = 1.5e-3 in every direction, stimulus on the first
    five x-planes.  One untimed pass, one timed pass of n_steps steps; then the
    time of one CG iteration from 100 iterations at rtol 0."""
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    grid_order(sim, w)
    stim = torch.as_tensor(np.where(np.arange(w.n) % w.grid[0] < 5, -100.0, 0.0)).cuda()
    grid = I.make_bidomain_grid(*w.grid, h=h, sigma_i=(sigma,) * 3, sigma_e=(sigma,) * 3)
    wb = I.ionic_elliptic_work_bytes(*w.grid, max_iter)
    work = torch.zeros(wb, dtype=torch.uint8, device="cuda")
    u = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    idiff = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    init = sim.state.clone()
    stream = torch.cuda.current_stream()

    def one_pass():
        sim.state.copy_(init)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = I.reaction_bidomain_step(sim.handle, grid, 0.0, w.dt, n_steps, w.n_nodes,
                                        w.n_sweeps, u, work, wb, idiff, stim, w.stim_t_on,
                                        w.stim_t_off, rtol=rtol, max_iter=max_iter, stream=stream)
        torch.cuda.synchronize()
        return info, time.perf_counter() - t0

    one_pass()
    info, wall = one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    I.ionic_elliptic_solve(sim.handle, grid, u, work, wb, rtol=0.0, max_iter=100, stream=stream)
    cg_iter = (time.perf_counter() - t0) / 100
    sim.close()
    return {
        "steps": n_steps, "ms_per_step": wall / n_steps * 1e3,
        "value": w.n * n_steps / wall,
        "cg_iterations_per_step": info["cg_iterations"] / n_steps,
        "cg_converged": info["converged"], "cg_rtol": rtol,
        "cg_iteration_ms": cg_iter * 1e3,
        "elliptic_share": min(1.0, info["cg_iterations"] * cg_iter / wall),
    }


def valu_mix(csv_paths, n_steps=500):
    """Instruction mix of the Newton step kernels from rocprofv3 --pmc runs of
    `bench.py --steps 1 --warmup 0` (the first dispatch of each precision: the
    Newton tol 1e-10 pass), per wave and time step, as a markdown table."""
    counts = {}
    for path in csv_paths:
        seen = {}
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if not is_tt06_newton_step(name):
                continue
            prec = "fp64" if "Fp64" in name else "mixed"
            d = seen.setdefault(prec, r["Dispatch_Id"])
            if r["Dispatch_Id"] != d:
                continue
            c = counts.setdefault(prec, {})
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    cols = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
            "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64",
            "SQ_INSTS_VALU_CVT", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64", "SQ_INSTS_SALU",
            "SQ_INSTS_LDS", "SQ_INSTS_VMEM"]
    lines = ["| counter (per wave and step) | " + " | ".join(sorted(counts)) + " |",
             "|---|" + "---|" * len(counts)]
    for col in cols + ["other VALU"]:
        vals = []
        for prec in sorted(counts):
            c = counts[prec]
            waves = c.get("SQ_WAVES", 15625.0)
            if col == "other VALU":
                typed = sum(c.get(k, 0.0) for k in cols[1:12])
                v = c.get("SQ_INSTS_VALU", 0.0) - typed
            else:
                v = c.get(col, float("nan"))
            vals.append("%.0f" % (v / waves / n_steps))
        lines.append("| %s | %s |" % (col.replace("SQ_INSTS_", ""), " | ".join(vals)))
    for prec in sorted(counts):
        c = counts[prec]
        if "SQ_ACTIVE_INST_VALU" in c and "SQ_BUSY_CYCLES" in c:
            lines.append("")
            # SQ_ACTIVE_INST_VALU counts quad-cycles
            lines.append("%s: 4 SQ_ACTIVE_INST_VALU / SQ_INSTS_VALU = %.2f cycles per wave64 VALU "
                         "instruction" % (prec, 4 * c["SQ_ACTIVE_INST_VALU"] / c["SQ_INSTS_VALU"]))
    print("\n".join(lines))
    return counts


def trace_overlap(trace_csv, skip=0):
    """Concurrency of the step kernels of different classes (cell model x
    precision) in a rocprofv3 kernel trace (--kernel-trace, CSV): the time
    during which at least one step kernel runs, the time during which kernels
    of two or more classes run at once, and the same per class pair.  The
    first `skip` step-kernel dispatches (in start order) are left out."""
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    iv = []
    for r in rows:
        name = r.get("Kernel_Name", "")
        if "sdc_kernel" not in name:
            continue
        if skip > 0:
            skip -= 1
            continue
        cls = ("TT06" if "TT06" in name else "LR91" if "LR91" in name else "test",
               "fp64" if "Fp64" in name else "mixed")
        iv.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), cls,
                   r.get("Queue_Id", r.get("Stream_Id", "?"))))
    events = sorted([(a, 1, c) for a, b, c, q in iv] + [(b, -1, c) for a, b, c, q in iv])
    running = {}
    busy = multi = 0
    pair = {}
    last = None
    for t, d, c in events:
        if last is not None and running:
            dt = t - last
            live = [k for k, v in running.items() if v > 0]
            if live:
                busy += dt
            if len(live) >= 2:
                multi += dt
                key = " + ".join("%s/%s" % k for k in sorted(live))
                pair[key] = pair.get(key, 0) + dt
        running[c] = running.get(c, 0) + d
        if running[c] == 0:
            del running[c]
        last = t
    per_class = {}
    for a, b, c, q in iv:
        k = "%s/%s" % c
        per_class.setdefault(k, [0, 0.0, set()])
        per_class[k][0] += 1
        per_class[k][1] += (b - a) * 1e-9
        per_class[k][2].add(q)
    out = {"step_kernel_dispatches": len(iv), "busy_s": busy * 1e-9,
           "two_or_more_classes_s": multi * 1e-9,
           "overlap_fraction_of_busy": multi / busy if busy else 0.0,
           "kernel_time_sum_s": sum((b - a) for a, b, c, q in iv) * 1e-9,
           "per_class": {k: {"dispatches": v[0], "kernel_s": round(v[1], 4),
                             "queues": sorted(v[2])} for k, v in sorted(per_class.items())},
           "concurrent_sets_s": {k: round(v * 1e-9, 4) for k, v in
                                 sorted(pair.items(), key=lambda kv: -kv[1])[:8]}}
    print(json.dumps(out, indent=1))
    return out


def microbench(torch):
    """Measured rates of the units the step kernels are bound by
    (libionic_microbench.so; best of three launches each)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2510_27447_amd", "_lib", "libionic_microbench.so")
    if not os.path.exists(path):
        raise RuntimeError("%s is missing: build it with __graft_entry__.build()" % path)
    mb = ctypes.CDLL(path)
    mb.ionic_mb_run.restype = ctypes.c_int
    mb.ionic_mb_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.c_void_p, ctypes.c_size_t]
    threads = 1 << 21                       # 8 waves per SIMD on every compute unit
    copy_threads = 1 << 28                  # 2 GiB read + 2 GiB written
    buf = torch.empty(2 * copy_threads * 8, dtype=torch.uint8, device="cuda")
    tests = [("fma64_tflops", 0, threads, 20000, 1e12), ("fma32_tflops", 1, threads, 20000, 1e12),
             ("v_exp_f32_gops", 2, threads, 8000, 1e9), ("expf_gops", 3, threads, 8000, 1e9),
             ("exp_f64_gops", 4, threads, 1000, 1e9), ("copy_gbs", 5, copy_threads, 1, 1e9)]
    out = {}
    for name, which, n, iters, unit in tests:
        best = None
        for _ in range(3):
            sec, ops = ctypes.c_double(), ctypes.c_double()
            rc = mb.ionic_mb_run(which, n, iters, ctypes.byref(sec), ctypes.byref(ops),
                                 buf.data_ptr(), buf.numel())
            if rc != 0:
                raise RuntimeError("microbenchmark %s failed: hip error %d" % (name, rc))
            r = ops.value / sec.value
            best = r if best is None or r > best else best
        out[name] = round(best / unit, 2)
    del buf
    torch.cuda.synchronize()
    return out


def run_bidomain_implicit(I, torch, w, n_steps=10, dt=0.05, h=0.01, sigma=1.5e-3,
                          inner_tol=1e-6, rtol=1e-8, max_iter=2000, precision="fp64", ref_V=None):
    """Algorithm 2 in full on the slab (reaction_bidomain_implicit_step): per
    step, inner passes of the elliptic solve and ROS2 + one correction with the
    parabolic term inside the stages, at the paper's largest step dt = 0.05 ms
    (beyond the explicit limit h^2 / (2 sigma_i) = 0.033 ms at h = 0.01 cm),
    stimulus on the first five x-planes for 1 ms.  One untimed run of 2 steps,
    then one timed run of n_steps from the same state.  precision: the handle's
    layout (mixed: F, J and the eliminations in float); with ref_V (the V of the
    fp64 run) the max and RMS of the V difference relative to max|ref_V|.  The
    returned "_V" is the final V (for the caller, not the JSON line)."""
    sim = I.Simulation(w.model, w.x0, precision=precision)
    stim = torch.as_tensor(np.where(np.arange(w.n) % w.grid[0] < 5, -100.0, 0.0)).cuda()
    g = I.make_bidomain_grid(*w.grid, h=h, sigma_i=(sigma,) * 3, sigma_e=(sigma,) * 3)
    wb = I.ionic_implicit_work_bytes(w.model, *w.grid, max_iter)
    work = torch.zeros(wb, dtype=torch.uint8, device="cuda")
    ewb = I.ionic_elliptic_work_bytes(*w.grid, max_iter)
    ework = torch.zeros(ewb, dtype=torch.uint8, device="cuda")
    u = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    I.ionic_elliptic_solve(sim.handle, g, u, ework, ewb, rtol=rtol, max_iter=max_iter,
                           stream=stream)
    init, u_init = sim.state.clone(), u.clone()

    def run(steps):
        sim.state.copy_(init)
        u.copy_(u_init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = I.reaction_bidomain_implicit_step(sim.handle, g, 0.0, dt, steps, u, work, wb, stim,
                                                 0.0, 1.0, elliptic_rtol=rtol, krylov_rtol=rtol,
                                                 inner_tol=inner_tol, max_inner=40,
                                                 max_iter=max_iter, stream=stream)
        torch.cuda.synchronize()
        return info, time.perf_counter() - t0

    run(2)
    info, wall = run(n_steps)
    V = sim.readback(count=None)[0]
    sim.close()
    levels = I.ionic_multigrid_levels(*w.grid)
    out = {
        "precision": precision,
        "steps": n_steps, "dt_ms": dt, "ms_per_step": wall / n_steps * 1e3,
        "value": w.n * n_steps / wall,
        "inner_passes_per_step": info["inner_passes"] / n_steps, "inner_max": info["inner_max"],
        "inner_tol": inner_tol, "converged": info["converged"],
        "cg_iterations_per_pass": info["cg_iterations"] / info["inner_passes"],
        "krylov_iterations_per_solve": info["krylov_iterations"] / (3 * info["inner_passes"]),
        "krylov_max": info["krylov_max"], "rtol": rtol,
        "multigrid_levels": levels,
        "launches_per_cycle": 4 * levels - 3 if levels else 0,
        "coarse_level_launches_per_cycle": 4 * levels - 7 if levels else 0,
        "V_range_mV": [float(np.min(V)), float(np.max(V))],
        "_V": V,
    }
    if ref_V is not None:
        d = np.abs(V - ref_V) / np.max(np.abs(ref_V))
        out["V_error_vs_fp64"] = {"max": float(d.max()), "rms": float(np.sqrt(np.mean(d * d)))}
    return out


def cpu_workers():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(w, per_worker, seed=11):
    """Vertices of the workload the CPU baseline runs: a few on the stimulated
    face, the rest uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cpu_workers() * per_worker
    stim = np.nonzero(w.i_stim)[0]
    idx = np.concatenate([rng.choice(stim, 16, replace=False),
                          rng.choice(np.setdiff1d(np.arange(w.n), stim), n - 16, replace=False)])
    return np.sort(idx)


def cpu_baseline(w, idx):
    """The oracle (fp64 numpy, one thread per worker process, one worker per
    available core up to 16) on disjoint vertex subsets of the same workload,
    all 500 steps.  Throughput = sampled vertex-steps / the slowest worker's
    time.  Also returns the oracle's final states of the sampled vertices."""
    from oracle.pool import advance_parallel
    s = w.subset(idx)
    k = cpu_workers()
    X, secs, wall = advance_parallel("TT06", s.x0, s.i_stim, s.i_diff, k, dt=s.dt,
                                     n_steps=s.n_steps, n_nodes=s.n_nodes, n_sweeps=s.n_sweeps,
                                     stim_on=s.stim_t_on, stim_off=s.stim_t_off,
                                     tol=s.newton_tol, maxit=s.newton_maxit)
    slowest = max(secs)
    vs = len(idx) * s.n_steps
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"value": vs / slowest, "unit": "vertex-steps/s", "cores": k, "kind": "oracle",
            "threads_per_process": 1, "nproc": nproc, "os_cpu_count": os.cpu_count(),
            "cpu_model": cpu_model(),
            "sample": "%d vertices of the C2/C3 slab (16 on the stimulated face) x %d steps, "
                      "fp64 numpy oracle, %d processes x 1 thread, slowest %.1f s (wall %.1f s)"
                      % (len(idx), s.n_steps, k, slowest, wall)}, X


def state_errors(Xg, Xo, names):
    """Max and RMS per state of |GPU - oracle|, relative to the state's max |oracle|."""
    out = {}
    for i, nm in enumerate(names):
        sc = max(float(np.max(np.abs(Xo[i]))), 1e-300)
        d = np.abs(Xg[i] - Xo[i])
        out[nm] = {"max": float(np.max(d) / sc), "rms": float(np.sqrt(np.mean(d * d)) / sc)}
    return out


def run_c1(I, torch):
    """C1, the plain LR91 method in fp64: 4096 vertices (64 x 64), 1000 steps of
    0.02 ms, 3 nodes, 2 sweeps, in one fused launch; one untimed pass, then one
    timed pass from the same state.  64 workgroups: a quarter of the compute
    units hold one wavefront each, so this is a latency figure, not a
    throughput one."""
    from paper_2510_27447_amd import workloads as W
    w = W.c1_lr91()
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    stim = torch.as_tensor(w.i_stim).cuda()
    init = sim.state.clone()
    stream = torch.cuda.current_stream()

    def one():
        sim.state.copy_(init)
        I.ionic_reset_stats(sim.handle)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, stim, w.stim_t_on, w.stim_t_off,
                 None, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one()
    secs = one()
    st = sim.stats()
    sim.close()
    return {"value": w.n * w.n_steps / secs, "kernel_ms": secs * 1e3, "vertices": w.n,
            "steps": w.n_steps, "workgroups": (w.n + 63) // 64,
            "newton_iters_per_solve": st["newton_iters"] / max(1, st["newton_solves"]),
            "n_nonfinite": st["n_nonfinite"], "newton_tol": w.newton_tol}


def run_c4(I, torch, precision):
    """One pass of the 8e6-vertex spiral (1000 steps of dt 0.01 ms, 4 nodes, 3
    sweeps, the diffusion input redrawn every 50 steps: 20 launches), with all
    20 input fields resident before the timed region."""
    from paper_2510_27447_amd import workloads as W
    w = W.c4_tt06_spiral(precision=precision)
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    grid_order(sim, w)
    I.ionic_gates_to_steady_state(sim.handle)
    diffs = [torch.as_tensor(d).cuda() for d in w.i_diff_series]
    n, n_steps = w.n, w.n_steps
    del w.x0, w.i_diff_series
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    I.ionic_reset_stats(sim.handle)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    done, k = 0, 0
    while done < n_steps:
        chunk = min(w.diff_period, n_steps - done)
        sim.step(done * w.dt, w.dt, chunk, w.n_nodes, w.n_sweeps, None, 0.0, 0.0, diffs[k],
                 stream=stream)
        done += chunk
        k += 1
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.stats()
    sim.close()
    del diffs
    vs = n * n_steps
    return {"value": vs / wall, "kernel_s": e0.elapsed_time(e1) / 1e3, "wall_s": wall,
            "launches": k, "newton_iters_per_solve": st["newton_iters"] / max(1, st["newton_solves"]),
            "n_nonfinite": st["n_nonfinite"], "n_nonconverged": st["n_nonconverged"],
            "newton_tol": 1e-10 if precision == "fp64" else 1e-6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--no-ros2", action="store_true")
    ap.add_argument("--no-rl", action="store_true")
    ap.add_argument("--no-diffusion", action="store_true")
    ap.add_argument("--no-bidomain", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--cpu-per-worker", type=int, default=256,
                    help="vertices per CPU worker of the oracle baseline (500 steps each)")
    ap.add_argument("--adaptive-tol", type=float, default=1e-3)
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--trace-overlap", metavar="KERNEL_TRACE_CSV",
                    help="print the class overlap of the step kernels in a rocprofv3 kernel "
                         "trace and exit")
    ap.add_argument("--valu-from", nargs="+", metavar="PMC_CSV",
                    help="print the instruction mix of the step kernels from rocprofv3 --pmc "
                         "runs and exit")
    ap.add_argument("--trace-skip", type=int, default=0,
                    help="with --trace-overlap: leave out the first N step-kernel dispatches")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic_file(*args.traffic_from)
        return
    if args.valu_from:
        valu_mix(args.valu_from)
        return
    if args.trace_overlap:
        trace_overlap(args.trace_overlap, args.trace_skip)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus 1): the reaction stage would shard by vertex "
              "ranges with no exchange, and only figures on a single MI355X are measured and "
              "reported.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_27447_amd import ionic as I
    from paper_2510_27447_amd import workloads as W

    I.lib()
    rates = None
    micro = None
    if not args.no_micro:
        print("[bench] unit-rate microbenchmarks", file=sys.stderr, flush=True)
        micro = microbench(torch)
        rates = {"P64": micro["fma64_tflops"] * 1e12, "P32": micro["fma32_tflops"] * 1e12,
                 "trans32": micro["v_exp_f32_gops"] * 1e9, "exp64": micro["exp_f64_gops"] * 1e9}
        print("[bench] %s" % micro, file=sys.stderr, flush=True)
    sample = cpu_sample(W.c2_tt06(), args.cpu_per_worker)
    res = {}
    for prec in ("fp64", "mixed"):
        w = W.c2_tt06(precision=prec)
        print("[bench] %s: %d vertices x %d steps, %d passes" % (w.name, w.n, w.n_steps, args.steps),
              file=sys.stderr, flush=True)
        res[prec] = run_pass_set(I, torch, w, args.steps, args.warmup, sample=sample, rates=rates)
        print("[bench] %s: %.3e vertex-steps/s, kernel %.1f ms" % (prec, res[prec]["value"],
              res[prec]["kernel_ms"]), file=sys.stderr, flush=True)
    Vf, Vm = res["fp64"].pop("V"), res["mixed"].pop("V")
    # like for like: the fp64 kernel at the mixed path's Newton tolerance
    w = W.c2_tt06(precision="fp64")
    w.newton_tol = 1e-6
    print("[bench] fp64 at Newton tol 1e-6", file=sys.stderr, flush=True)
    f6 = run_pass_set(I, torch, w, args.steps, args.warmup)
    f6.pop("V")
    fp64_tol6 = {k: f6[k] for k in ("value", "kernel_ms", "newton_iters_per_solve", "newton_tol")}

    def verr(V):
        return {"max": float(np.max(np.abs(V - Vf)) / np.max(np.abs(Vf))),
                "rms": float(np.sqrt(np.mean((V - Vf) ** 2)) / np.max(np.abs(Vf)))}

    mixed_err = verr(Vm)

    ros2 = None
    if not args.no_ros2:
        # the paper's own scheme: ROS2 predictor + one trapezoidal correction, over the
        # same 10 ms of the same slab; V compared with the fp64 Newton run (3 nodes,
        # 3 sweeps, order 4) at the end
        ros2 = {"fixed": {}, "adaptive": {}}
        for prec in ("mixed", "fp64"):
            w = W.c2_tt06(precision=prec)
            w.n_nodes, w.n_sweeps = 2, 1
            print("[bench] ros2 fixed %s" % prec, file=sys.stderr, flush=True)
            r = run_pass_set(I, torch, w, args.steps, args.warmup, predictor="ros2")
            r["V_error_vs_fp64_newton"] = verr(r.pop("V"))
            ros2["fixed"][prec] = {k: r[k] for k in ("value", "kernel_ms", "roofline",
                                                     "V_error_vs_fp64_newton", "n_nonfinite")}
        for prec in ("mixed", "fp64"):
            w = W.c2_tt06(precision=prec)
            print("[bench] ros2 adaptive %s" % prec, file=sys.stderr, flush=True)
            a = run_adaptive(I, torch, w, args.adaptive_tol, w.n_steps * w.dt, 0.05)
            a["V_error_vs_fp64_newton"] = verr(a.pop("V"))
            ros2["adaptive"][prec] = a

    rl = None
    if not args.no_rl:
        # the headline workload (3 nodes, 3 sweeps) with the Rush-Larsen predictor
        rl = {}
        for prec in ("mixed", "fp64"):
            w = W.c2_tt06(precision=prec)
            print("[bench] rush-larsen %s" % prec, file=sys.stderr, flush=True)
            r = run_pass_set(I, torch, w, args.steps, args.warmup, predictor="rush_larsen")
            r["V_error_vs_fp64_newton"] = verr(r.pop("V"))
            rl[prec] = {k: r[k] for k in ("value", "kernel_ms", "roofline", "newton_iters_per_solve",
                                          "V_error_vs_fp64_newton", "n_nonfinite")}

    rd = None
    if not args.no_diffusion:
        w = W.c2_tt06(precision="mixed")
        print("[bench] reaction-diffusion mixed", file=sys.stderr, flush=True)
        rd = run_reaction_diffusion(I, torch, w, args.steps, args.warmup)

    bido = None
    if not args.no_bidomain:
        w = W.c2_tt06(precision="mixed")
        print("[bench] partitioned bidomain mixed", file=sys.stderr, flush=True)
        bido = run_bidomain(I, torch, w)
        w = W.c2_tt06(precision="fp64")
        print("[bench] partitioned bidomain, parabolic term implicit, fp64", file=sys.stderr,
              flush=True)
        bido["implicit"] = run_bidomain_implicit(I, torch, w)
        print("[bench] implicit: %.1f ms per step" % bido["implicit"]["ms_per_step"],
              file=sys.stderr, flush=True)
        print("[bench] partitioned bidomain, parabolic term implicit, mixed", file=sys.stderr,
              flush=True)
        w = W.c2_tt06(precision="mixed")
        bido["implicit_mixed"] = run_bidomain_implicit(I, torch, w, precision="mixed",
                                                       ref_V=bido["implicit"]["_V"])
        print("[bench] implicit mixed: %.1f ms per step" % bido["implicit_mixed"]["ms_per_step"],
              file=sys.stderr, flush=True)
        bido["implicit"].pop("_V")
        bido["implicit_mixed"].pop("_V")

    serving = None
    if not args.no_serving:
        from paper_2510_27447_amd import serve
        print("[bench] serving trace: %d requests" % args.serving_requests, file=sys.stderr, flush=True)
        serving = serve.run_trace(W.c5_trace(n_requests=args.serving_requests), verbose=True)

    print("[bench] C1 LR91 fp64, 4096 vertices x 1000 steps", file=sys.stderr, flush=True)
    c1 = run_c1(I, torch)

    c4 = None
    if not args.no_c4:
        c4 = {}
        for prec in ("fp64", "mixed"):
            print("[bench] C4 spiral 8e6 vertices x 1000 steps, %s" % prec, file=sys.stderr,
                  flush=True)
            c4[prec] = run_c4(I, torch, prec)
            print("[bench] C4 %s: %.3e vertex-steps/s" % (prec, c4[prec]["value"]),
                  file=sys.stderr, flush=True)

    cpu = None
    oracle_errors = None
    if not args.no_cpu:
        print("[bench] cpu baseline: oracle on %d sampled vertices" % len(sample), file=sys.stderr,
              flush=True)
        cpu, Xo = cpu_baseline(W.c2_tt06(), sample)
        from paper_2510_27447_amd.workloads import STATE_NAMES
        names = STATE_NAMES["TT06"]
        oracle_errors = {
            "sample": "the %d vertices of the CPU baseline, after 500 steps" % len(sample),
            "mixed": state_errors(res["mixed"]["X_sample"], Xo, names),
            "fp64": state_errors(res["fp64"]["X_sample"], Xo, names),
        }
    for prec in ("fp64", "mixed"):
        res[prec].pop("X_sample")

    m = res["mixed"]
    out = {
        "metric": "TT06 vertex-steps/s, mixed vs FP64 at stated error; serving p50/p99 latency",
        "value": m["value"],
        "unit": "vertex-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "TT06-epi 100x100x100 slab (1e6 vertices), 500 steps of dt 0.02 ms per "
                        "pass, 3 Gauss-Lobatto nodes, 3 SDC sweeps, Newton tol 1e-10 requested "
                        "(the mixed path stops at max(tol, 1e-6)); value = mixed precision (fp32 "
                        "F/J/solve, fp64 V/Ca/Na/K/residual); fp64 alongside at 1e-10 and 1e-6",
            "n_vertices": 1_000_000, "steps_per_pass": 500, "dt_ms": 0.02, "nodes": 3, "sweeps": 3,
            "seed": 0, "vertex_order": VERTEX_ORDER,
        },
        "kernel_ms": m["kernel_ms"],
        "newton_tol": m["newton_tol"],
        "fp64": {k: res["fp64"][k] for k in ("value", "ms_per_step", "kernel_ms", "roofline",
                                            "t_min", "newton_iters_per_solve", "n_nonconverged",
                                            "newton_tol")},
        "fp64_at_mixed_tol": fp64_tol6,
        "mixed_speedup_vs_fp64": m["value"] / res["fp64"]["value"],
        "mixed_speedup_vs_fp64_same_tol": m["value"] / fp64_tol6["value"],
        "mixed_vs_fp64_V_error": mixed_err,
        "error_vs_oracle": oracle_errors,
        "newton_iters_per_solve": m["newton_iters_per_solve"],
        "roofline": m["roofline"],
        "t_min": m["t_min"],
        "microbench": micro,
        "c1_lr91": c1,
        "c4_spiral": c4,
        "traffic_algorithmic_bytes": m["traffic_algorithmic_bytes"],
        "hbm_gbs_algorithmic": m["hbm_gbs_algorithmic"],
        "cpu_baseline": cpu,
        "serving": serving,
        "ros2_sdc": ros2,
        "rush_larsen": rl,
        "reaction_diffusion": rd,
        "bidomain": bido,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
